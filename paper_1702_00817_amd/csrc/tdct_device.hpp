// Device-side building blocks of the codec, written for gfx950.
//
// The 1-D butterflies are templates on the value type so that one source
// serves three instantiations: packed int16 pairs (two blocks per lane on the
// encoder), int32 (the decoder) and a host-side counting type that checks
// the operation count of Table 1 (14 additions, no multiplication, no shift).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdct {

// |row i of T|^2 = 2^kA[i]: the diagonal D of Section 2 has d_i^2 = 2^-kA[i].
constexpr int kA[8] = {3, 1, 2, 1, 3, 1, 2, 1};

// Power of two that folds D^2 into the quantiser at the integer scale 64:
// W_ij = Y_ij << kShift(i, j), kShift = 6 - a_i - a_j in 0..4.
__host__ __device__ constexpr int kShift(int i, int j) { return 6 - kA[i] - kA[j]; }

// ---- 8-point transforms (Section 2) -----------------------------------------
//
// Forward, X = T x. Folding the fast algorithm's sign flips into operand order
// leaves seven sums and seven differences:
//   s_k = x_k + x_{7-k} (k < 4); X0 = (s0 + s3) + (s1 + s2), X4 = (s0 + s3) - (s1 + s2),
//   X2 = s0 - s3, X6 = s2 - s1, X1 = x0 - x7, X3 = x5 - x2, X5 = x6 - x1, X7 = x4 - x3.
template <typename V>
__host__ __device__ __forceinline__ void fwd8(V& x0, V& x1, V& x2, V& x3, V& x4, V& x5, V& x6,
                                              V& x7) {
    V s0 = x0 + x7, s1 = x1 + x6, s2 = x2 + x5, s3 = x3 + x4;
    V d0 = x0 - x7, d1 = x6 - x1, d2 = x5 - x2, d3 = x4 - x3;
    V e0 = s0 + s3, e1 = s1 + s2;
    x0 = e0 + e1;
    x4 = e0 - e1;
    x2 = s0 - s3;
    x6 = s2 - s1;
    x1 = d0;
    x3 = d2;
    x5 = d1;
    x7 = d3;
}

// Inverse direction, x = T^t X (the factors of T are symmetric, so this is
// the same graph run backwards), again 14 additions:
//   u = X0 + X4, v = X0 - X4, p = u + X2, m = u - X2, a = v - X6, b = v + X6,
//   x0 = p + X1, x7 = p - X1, x3 = m - X7, x4 = m + X7,
//   x1 = a - X5, x6 = a + X5, x2 = b - X3, x5 = b + X3.
template <typename V>
__host__ __device__ __forceinline__ void inv8(V& x0, V& x1, V& x2, V& x3, V& x4, V& x5, V& x6,
                                              V& x7) {
    V u = x0 + x4, v = x0 - x4;
    V p = u + x2, m = u - x2, a = v - x6, b = v + x6;
    V X1 = x1, X3 = x3, X5 = x5, X7 = x7;
    x0 = p + X1;
    x7 = p - X1;
    x3 = m - X7;
    x4 = m + X7;
    x1 = a - X5;
    x6 = a + X5;
    x2 = b - X3;
    x5 = b + X3;
}

// Row pass then column pass on an 8x8 array in registers (v[8*r + c]).
template <typename V>
__host__ __device__ __forceinline__ void fwd8x8(V* v) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
        fwd8(v[8 * r + 0], v[8 * r + 1], v[8 * r + 2], v[8 * r + 3], v[8 * r + 4], v[8 * r + 5],
             v[8 * r + 6], v[8 * r + 7]);
#pragma unroll
    for (int c = 0; c < 8; ++c)
        fwd8(v[c], v[8 + c], v[16 + c], v[24 + c], v[32 + c], v[40 + c], v[48 + c], v[56 + c]);
}

template <typename V>
__host__ __device__ __forceinline__ void inv8x8(V* v) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
        inv8(v[8 * i + 0], v[8 * i + 1], v[8 * i + 2], v[8 * i + 3], v[8 * i + 4], v[8 * i + 5],
             v[8 * i + 6], v[8 * i + 7]);
#pragma unroll
    for (int c = 0; c < 8; ++c)
        inv8(v[c], v[8 + c], v[16 + c], v[24 + c], v[32 + c], v[40 + c], v[48 + c], v[56 + c]);
}

// ---- zigzag scan (Section 3) ------------------------------------------------
//
// Built by walking the block the way a JPEG scanner does: step up-right along
// even anti-diagonals and down-left along odd ones, turning at the edges.
struct Zigzag {
    int8_t order[64];  // rank -> 8 i + j
    int8_t rank[64];   // 8 i + j -> rank
};

__host__ __device__ constexpr Zigzag make_zigzag() {
    Zigzag z{};
    int i = 0, j = 0;
    for (int n = 0; n < 64; ++n) {
        z.order[n] = (int8_t)(8 * i + j);
        z.rank[8 * i + j] = (int8_t)n;
        if (((i + j) & 1) == 0) {  // moving up-right
            if (j == 7) ++i;
            else if (i == 0) ++j;
            else { --i; ++j; }
        } else {                   // moving down-left
            if (i == 7) ++j;
            else if (j == 0) ++i;
            else { ++i; --j; }
        }
    }
    return z;
}

constexpr Zigzag kZigzag = make_zigzag();

// ---- quantiser --------------------------------------------------------------
//
// q = round-half-away(W / Q) with W = y * 2^s, evaluated as one fma whose
// addend is M = 1.5 * 2^23:
//   t = fma(float(y), r, M),  r = fl32(2^s / Q * (1 + 2^-20)),
// t is M + y r rounded once to the nearest integer (|y r| < 2^22, so the
// result lies in (2^23, 2^24), where floats are spaced by exactly 1), and the
// integer is q = bits(t) - bits(M). Since bits(M) = 0x4B400000 has zero low
// halves, the low 16 bits of t are q itself, ready to pack.
// Why the rounding is exact: the relative bias 2^-20 on r moves every exact
// tie z = W / Q = k + 1/2 away from zero by about |z| 2^-20, more than the
// rounding of r (2^-24 relative), so ties round away from zero; every other z
// lies at least 1 / (2Q) from a half-integer while the bias and r's rounding
// stay below |z| 1.1e-6 <= 0.0091 / Q for |W| <= 8192, so no such z is pushed
// onto or across one (and y r itself is never a half-integer: it would have
// to be one of these two cases). A position outside the zonal set has r = 0,
// t = M and q = 0. The host test sweeps every (y, s, Q) of the encoder's
// domain against the exact rational rounding.
constexpr float kRoundMagic = 12582912.0f;  // 1.5 * 2^23
constexpr uint32_t kRoundMagicBits = 0x4B400000u;

__host__ __device__ __forceinline__ uint32_t quant_bits(int y, float r) {
    return __builtin_bit_cast(uint32_t, fmaf((float)y, r, kRoundMagic));
}

__host__ __device__ __forceinline__ int quant_int(int y, float r) {
    return (int)(quant_bits(y, r) - kRoundMagicBits);
}

// Bias of the round trips' fp32 decoder half, added to W''_00 = q Q / 64 at
// position (0, 0): every output becomes S / 64 + 128 + 1/128, which rounds to
// nearest as floor((S + 32) / 64) + 128 (the fraction of S / 64 is a multiple
// of 1/64, so the value is never a tie).
constexpr float kPixelBiasF = 128.0f + 1.0f / 128.0f;

// Host-side constant for position (i, j): r as above, or 0 if masked.
inline float quant_recip(int Q, int s, bool kept) {
    if (!kept) return 0.0f;
    double v = (double)(1 << s) / (double)Q * (1.0 + 0x1p-20);
    return (float)v;
}

// ---- per-launch and per-image descriptors ----------------------------------

// Quantiser constants of one table: encoder reciprocals (zonal mask folded,
// natural order) and decoder multipliers.
struct QConst {
    float r[64];
    int32_t Q[64];
    float qs[64];  // Q / 64 in fp32: multipliers of the round trips' fp32 decoder half
};

enum : int32_t { OP_ENCODE = 0, OP_DECODE = 1, OP_ROUNDTRIP = 2, OP_ENCODE_I8ZZ = 3, OP_FORWARD = 4,
                 // internal: a round trip whose coefficients never leave the registers
                 OP_ROUNDTRIP_NC = 5 };

// Flags describing which load/store widths an image allows.
enum : int32_t {
    F_SRC8 = 1,    // src and src_stride 8-byte aligned
    F_DST8 = 4,    // dst and dst_stride 8-byte aligned
    F_COEF = 8     // coefficients are written (ROUNDTRIP)
};

struct ImgDesc {
    const uint8_t* src;
    uint8_t* dst;
    void* coef;
    int64_t src_stride;
    int64_t dst_stride;
    int64_t nblk;   // blocks in the image
    int32_t nbx;    // blocks per row
    int32_t op;
    int32_t qidx;   // QConst index
    int32_t flags;
};

// A tile is the run of blocks one wave handles in one step: up to 128
// consecutive blocks (raster order) of one image for encoder-side ops, 64 for
// the decoder and for the int32 forward transform (whose 4-byte output takes
// two LDS staging rounds per 64 blocks).
struct Tile {
    uint32_t img;
    uint32_t first_lo;  // first block index, split to keep the table 16-byte friendly
    uint32_t first_hi;
    uint32_t count;
};

constexpr int kEncTileBlocks = 128;
constexpr int kDecTileBlocks = 64;

__host__ __device__ inline int tile_blocks(int op) {
    return (op == OP_DECODE || op == OP_FORWARD) ? kDecTileBlocks : kEncTileBlocks;
}

// Workgroups are dealt to the XCDs in turn (workgroup b runs on XCD
// b mod kXcds). xcd_order(b, n) is the place workgroup b takes in the tile
// order when each XCD's workgroups work through one contiguous range of
// tiles: XCD x's workgroups get x's range in launch order. A bijection on
// [0, n), also when n is not a multiple of kXcds (the first n mod kXcds
// XCDs get one workgroup more).
constexpr uint32_t kXcds = 8;
__host__ __device__ inline uint32_t xcd_order(uint32_t b, uint32_t n) {
    const uint32_t xcd = b % kXcds, slot = b / kXcds;
    const uint32_t per = (n + kXcds - 1) / kXcds, tall = n % kXcds ? n % kXcds : kXcds;
    return xcd < tall ? xcd * per + slot : tall * per + (xcd - tall) * (per - 1) + slot;
}

}  // namespace tdct
