// Per-wave tile code of the codec for gfx950, shared by the batch kernels and
// the resident serving kernel: coefficient staging through LDS, pixel loads
// and stores, the encoder tile (two blocks per lane as packed int16 pairs)
// and the decoder tile (one block per lane in int32).
//
// Thread mapping. Every lane owns whole 8x8 blocks, so both 1-D passes of
// the separable transform (Section 3) run in registers without cross-lane
// traffic:
//  * encoder-side ops: a lane owns blocks first + l and first + 64 + l of its
//    wave-tile and keeps pixel (r, c) of both as one packed int16 pair, so
//    every v_pk_add/v_pk_sub does the butterfly of Section 2 for both blocks
//    (the whole 2-D forward transform costs 1.75 VALU ops per pixel).
//    Unshifted pixels keep every intermediate within 16 bits (|sum| <= 64 *
//    255), and the level shift -128 moves only the DC term (rows 1..7 of T
//    sum to zero), by -8192;
//  * the decoder: a lane owns one block in int32, because with Q <= 4095 an
//    arbitrary int16 input needs 32-bit intermediates.
// A wave-tile is up to 128 (encoder) or 64 (decoder) consecutive blocks of
// one image; rows of 64 consecutive blocks are contiguous, so pixel-side
// accesses of a wave cover whole 512-byte runs of a row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tdct_device.hpp"

namespace tdct {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s16x2 as_s16x2(uint32_t v) { return __builtin_bit_cast(s16x2, v); }

// Streaming accesses: every byte is touched once, so loads and stores carry
// the non-temporal hint and do not displace other data in L2 / MALL.
__device__ __forceinline__ v4u ld_nt4(const void* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const v4u*>(p));
}
__device__ __forceinline__ v2u ld_nt2(const void* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const v2u*>(p));
}
__device__ __forceinline__ void st_nt4(void* p, v4u v) {
    __builtin_nontemporal_store(v, reinterpret_cast<v4u*>(p));
}
__device__ __forceinline__ void st_nt2(void* p, v2u v) {
    __builtin_nontemporal_store(v, reinterpret_cast<v2u*>(p));
}

// Output stores that write through L2 to memory (agent-scope coherent, sc1)
// and carry the streaming hint (nt). Each XCD has its own L2, so ordinary
// stores of one wave become visible to other XCDs and to copy engines only
// once that L2 is written back; a wave that stores this way makes its outputs
// visible device-wide as soon as its stores complete (s_waitcnt vmcnt(0)),
// without writing back the whole L2 of its XCD.
constexpr int kBufSc1 = 16;                    // cache-policy bits: sc1
constexpr int kBufSc1Nt = kBufSc1 | 2;         // sc1, nt
constexpr uint32_t kBufRsrcWord3 = 0x00020000u;  // raw buffer, gfx9 family
// An 8-byte pixel-row store at any address (a buffer store would need a
// wave-uniform base within 4 GiB of every lane's row). No builtin gives a
// global store both sc1 and nt, so the instruction is written out; it takes
// no output register, and the count-off's s_waitcnt vmcnt(0) covers it like
// any other store. (Measured on a burst of decode requests: 1607-1728 Gpx/s
// with sc1 nt pixel stores and sc1 coefficient loads, 1210-1256 with sc1
// stores and sc1 nt loads.)
__device__ __forceinline__ void st_wt2(void* p, v2u v) {
    asm volatile("global_store_dwordx2 %0, %1, off sc1 nt" ::"v"(p), "v"(v) : "memory");
}
__device__ __forceinline__ void st_wt1(uint8_t* p, uint8_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Loads that never return a stale L2 line (sc1): what another agent (a copy
// engine, a kernel on another XCD) wrote to memory before the load is seen.
// A kernel that keeps running while its inputs change between requests reads
// them this way instead of invalidating its XCD's whole L2. They carry no
// streaming hint: with it, both the pixel-row loads and the coefficient-run
// loads ran slower in the resident kernel.
__device__ __forceinline__ v2u ld_wt2(const void* p) {
    return __builtin_bit_cast(v2u, __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ uint32_t ld_wt1(const uint8_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// 16-byte load at base + off (base wave-uniform, off per lane, in bytes);
// lanes with off >= limit read zero.
__device__ __forceinline__ v4u ld_wt4(const void* base, uint32_t off, uint32_t limit) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)limit, (int)kBufRsrcWord3);
    return __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, kBufSc1));
}

// 16-byte store at base + off (base wave-uniform, off per lane, both in
// bytes); lanes with off >= limit store nothing.
__device__ __forceinline__ void st_wt4(void* base, uint32_t off, uint32_t limit, v4u v) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)limit, (int)kBufRsrcWord3);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, kBufSc1Nt);
}

// Pixel-plane (and output) access policy, a compile-time parameter of the
// tile code. PX_STREAM and PX_CACHED are the batch kernels' pixel cache
// policies (below). PX_COHERENT reads every input with coherent loads
// (ld_wt*) and writes every output -- pixels and coefficients -- through L2
// (st_wt*), for kernels whose waves report finished outputs, and take new
// inputs, while the kernel keeps running.
enum { PX_STREAM = 0, PX_CACHED = 1, PX_COHERENT = 2 };

// Pixel-plane accesses under the cache policy a launch picks. Streaming
// (PX_STREAM) marks them non-temporal, as above. Cached ones are ordinary
// accesses that stay in L2 until evicted: where a tile's pixel rows end
// inside a 128-byte line (image widths that are not multiples of 128, and
// tile boundaries inside a row) the neighbouring tile fills the rest of that
// line, and with both halves meeting in one L2 the line reaches HBM once,
// whole. Coefficient runs are whole lines and always stream.
template <int PC>
__device__ __forceinline__ v2u ld_px(const void* p) {
    if constexpr (PC == PX_CACHED)
        return *reinterpret_cast<const v2u*>(p);
    else if constexpr (PC == PX_COHERENT)
        return ld_wt2(p);
    else
        return ld_nt2(p);
}
template <int PC>
__device__ __forceinline__ void st_px(void* p, v2u v) {
    if constexpr (PC == PX_CACHED)
        *reinterpret_cast<v2u*>(p) = v;
    else if constexpr (PC == PX_COHERENT)
        st_wt2(p, v);
    else
        st_nt2(p, v);
}

// A pointer the compiler cannot place in an address space (read from a
// table in memory or from LDS) is generic, and generic accesses become FLAT
// instructions, which also count against the LDS counter: every LDS fence of
// the tile code would then wait for the wave's outstanding global stores.
// Rebuilding it as a global-space pointer gives global instructions.
template <class T>
__device__ __forceinline__ T* global_ptr(T* p) {
    typedef __attribute__((address_space(1))) T GT;
    return (T*)(GT*)(uintptr_t)p;
}

// An image descriptor whose plane and coefficient pointers are global-space.
__device__ __forceinline__ ImgDesc global_desc(ImgDesc d) {
    d.src = global_ptr(d.src);
    d.dst = global_ptr(d.dst);
    d.coef = global_ptr(d.coef);
    return d;
}

// LDS writes of this wave complete before its following LDS reads (and the
// compiler keeps LDS accesses on their side of this point).
__device__ __forceinline__ void lds_fence() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Pack two int32 values (known to fit 16 bits) into one dword, low first.
__device__ __forceinline__ uint32_t pack16(int lo, int hi) {
    return __builtin_amdgcn_perm((uint32_t)hi, (uint32_t)lo, 0x05040100u);
}

// Pack four values in [0, 255] into one dword, first in the low byte.
__device__ __forceinline__ uint32_t pack8(int b0, int b1, int b2, int b3) {
    uint32_t lo = __builtin_amdgcn_perm((uint32_t)b1, (uint32_t)b0, 0x0c0c0400u);
    uint32_t hi = __builtin_amdgcn_perm((uint32_t)b3, (uint32_t)b2, 0x04000c0cu);
    return lo | hi;
}

// ---- coefficient-side staging through LDS ------------------------------------
//
// Every lane owns whole blocks, so the coefficients of one of its blocks form
// CPL consecutive 16-byte chunks (CPL = 8: an int16 block; CPL = 4: an int8
// block) of the contiguous run that 64 consecutive blocks occupy. Direct
// stores would make every instruction touch 64 chunks CPL * 16 bytes apart.
// Instead the wave writes its chunks to its own LDS slice and reads them back
// so that instruction k moves chunks 64k .. 64k + 63, i.e. 1 KB of
// consecutive bytes (and the reverse for the decoder's loads). Chunk m of
// lane L sits at slot CPL * L + (m ^ swz(L)); the XOR puts any 8 and any 16
// consecutive lanes of both access patterns on distinct 16-byte bank groups,
// whether the LDS has 32 or 64 four-byte banks.
template <int CPL>
__device__ __forceinline__ uint32_t swz(uint32_t L) {
    return CPL == 8 ? ((L ^ (L >> 3)) & 7u) : (((L >> 1) ^ (L >> 2)) & 3u);
}

// Stores the run of 64 * CPL chunks (only its first nchunks) from lane-owned
// chunks: chunk m of lane L goes to dst[STRIDE * L + m]. With STRIDE = CPL
// the run is contiguous; with STRIDE = 2 * CPL it is one half of each of 64
// blocks of 2 * CPL chunks (an int32 block in two rounds), and every store
// instruction still writes whole runs of CPL * 16 bytes.
template <int CPL, int STRIDE = CPL, int PC = PX_STREAM>
__device__ __forceinline__ void stage_out(v4u* wl, const v4u (&mine)[CPL], uint32_t nchunks,
                                          v4u* dst, uint32_t lane) {
    static_assert(PC != PX_COHERENT || STRIDE == CPL, "coherent stores of contiguous runs only");
#pragma unroll
    for (int m = 0; m < CPL; ++m) wl[CPL * lane + ((uint32_t)m ^ swz<CPL>(lane))] = mine[m];
    lds_fence();
    // CPL divides 64, so chunk 64 k + lane belongs to lane 64 k / CPL +
    // lane / CPL and, for a strided run, sits at one per-lane base plus a
    // constant per k.
    v4u* base = dst + STRIDE * (lane / CPL) + lane % CPL;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const uint32_t c = 64u * k + lane;
        const uint32_t L = c / CPL, m = c % CPL;
        const v4u v = wl[CPL * L + (m ^ swz<CPL>(L))];
        if constexpr (PC == PX_COHERENT)
            st_wt4(dst, 16u * c, 16u * nchunks, v);  // the range check drops c >= nchunks
        else if (c < nchunks) {
            if constexpr (STRIDE == CPL)
                st_nt4(dst + c, v);
            else
                st_nt4(base + (64 / CPL) * STRIDE * k, v);
        }
    }
    asm volatile("" ::: "memory");
}

// Loads the run of 512 chunks at src (only its first nchunks; the rest read
// as zero): chunk 64 k + lane into tmp[k].
template <int PC = PX_STREAM>
__device__ __forceinline__ void stage_load(const v4u* src, uint32_t nchunks, uint32_t lane,
                                           v4u (&tmp)[8]) {
    if constexpr (PC == PX_COHERENT) {
#pragma unroll
        for (int k = 0; k < 8; ++k) tmp[k] = ld_wt4(src, 16u * (64u * k + lane), 16u * nchunks);
    } else if (nchunks == 512) {
#pragma unroll
        for (int k = 0; k < 8; ++k) tmp[k] = ld_nt4(src + 64u * k + lane);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t c = 64u * k + lane;
            tmp[k] = c < nchunks ? ld_nt4(src + c) : (v4u){0u, 0u, 0u, 0u};
        }
    }
}

// Hands every lane the 8 chunks of its own int16 block from a loaded run.
__device__ __forceinline__ void stage_swap(v4u* wl, const v4u (&tmp)[8], uint32_t lane,
                                           v4u (&mine)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t c = 64u * k + lane;
        const uint32_t L = c >> 3, m = c & 7u;
        wl[8 * L + (m ^ swz<8>(L))] = tmp[k];
    }
    lds_fence();
#pragma unroll
    for (int m = 0; m < 8; ++m) mine[m] = wl[8 * lane + ((uint32_t)m ^ swz<8>(lane))];
    asm volatile("" ::: "memory");
}

// ---- pixel side ---------------------------------------------------------------

template <int PC>
__device__ __forceinline__ void load_rows8(const uint8_t* p, int64_t stride, int flags,
                                           uint32_t (&R)[8][2]) {
    if (flags & F_SRC8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const v2u v = ld_px<PC>(p + r * stride);
            R[r][0] = v.x;
            R[r][1] = v.y;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint8_t* q = p + r * stride;
            if constexpr (PC == PX_COHERENT) {
                R[r][0] = ld_wt1(q) | (ld_wt1(q + 1) << 8) | (ld_wt1(q + 2) << 16) | (ld_wt1(q + 3) << 24);
                R[r][1] = ld_wt1(q + 4) | (ld_wt1(q + 5) << 8) | (ld_wt1(q + 6) << 16) | (ld_wt1(q + 7) << 24);
            } else {
                R[r][0] = (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16) |
                          ((uint32_t)q[3] << 24);
                R[r][1] = (uint32_t)q[4] | ((uint32_t)q[5] << 8) | ((uint32_t)q[6] << 16) |
                          ((uint32_t)q[7] << 24);
            }
        }
    }
}

template <int PC>
__device__ __forceinline__ void store_rows8(uint8_t* p, int64_t stride, int flags,
                                            const uint32_t (&R)[8][2]) {
    if (flags & F_DST8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) st_px<PC>(p + r * stride, (v2u){R[r][0], R[r][1]});
    } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            uint8_t* q = p + r * stride;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if constexpr (PC == PX_COHERENT) {
                    st_wt1(q + c, (uint8_t)(R[r][0] >> (8 * c)));
                    st_wt1(q + 4 + c, (uint8_t)(R[r][1] >> (8 * c)));
                } else {
                    q[c] = (uint8_t)(R[r][0] >> (8 * c));
                    q[4 + c] = (uint8_t)(R[r][1] >> (8 * c));
                }
            }
        }
    }
}

__device__ __forceinline__ int64_t block_offset(int64_t stride, uint32_t nbx, uint32_t b) {
    const uint32_t by = b / nbx;
    const uint32_t bx = b - by * nbx;
    return (int64_t)(8 * by) * stride + 8 * bx;
}

// ---- decoder core ----------------------------------------------------------

// Inverse transform of one block of dequantised coefficients W'_ij (natural
// order) into 8 rows of 8 pixels: floor((S + 32) / 64) + 128, clamped.
__device__ __forceinline__ void reconstruct(int (&W)[64], uint32_t (&px)[8][2]) {
    // +32 rounds floor((S + 32) / 64); +8192 = 64 * 128 undoes the level
    // shift. Column 0 of T^t is all ones, so adding both to W'_00 adds them
    // to every S_rc.
    W[0] += 32 + 8192;
    inv8x8(W);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        int p[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) p[c] = min(max(W[8 * r + c] >> 6, 0), 255);
        px[r][0] = pack8(p[0], p[1], p[2], p[3]);
        px[r][1] = pack8(p[4], p[5], p[6], p[7]);
    }
}

// The decoder half of a round trip, in fp32. There q comes from the encoder,
// so |q Q| <= |W| + Q / 2 < 10240 and W'' = q Q / 64 is a multiple of 1/64 of
// magnitude below 160. Every value of the inverse transform is a signed sum of
// at most 16 of the 64 inputs (each column of T has four nonzeros) plus the
// bias c = 128 + 1/128 folded into W''_00 (which reaches every output, column 0
// of T^t being all ones): a multiple of 1/128 below 2560 + 129 in magnitude,
// far under 2^24 units of 1/128, so each fp32 addition (and each multiply
// folded into one as an FMA) is exact and the result is S / 64 + c exactly,
// S = T^t W' T.
// With y = (S + 32) / 64 + 128, whose fraction f is a multiple of 1/64, the
// result is z = y - 63/128 = floor(y) + (f - 63/128), and |f - 63/128| < 1/2:
// rounding z to the nearest integer gives floor(y), never from a tie. The
// hardware conversion to u8 rounds to nearest and saturates to [0, 255], so
// one instruction per pixel yields clamp(floor((S + 32) / 64) + 128), packed.
// (The general decoder keeps int32: an arbitrary int16 q times Q up to 4095
// leaves fp32's exact range.) The bias kPixelBiasF is in tdct_device.hpp.

__device__ __forceinline__ void reconstruct_f(float (&W)[64], uint32_t (&px)[8][2]) {
    W[0] += kPixelBiasF;
    inv8x8(W);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float* w = &W[8 * r + 4 * h];
            uint32_t p = __builtin_amdgcn_cvt_pk_u8_f32(w[0], 0u, 0u);
            p = __builtin_amdgcn_cvt_pk_u8_f32(w[1], 1u, p);
            p = __builtin_amdgcn_cvt_pk_u8_f32(w[2], 2u, p);
            px[r][h] = __builtin_amdgcn_cvt_pk_u8_f32(w[3], 3u, p);
        }
    }
}

// Round-trip decoder half from int16 coefficients the encoder just made (32
// dwords, natural order, two per dword): W'' = q (Q / 64), exact in fp32.
template <class QC>
__device__ __forceinline__ void decode_block_rt(const uint32_t (&qp)[32], const QC& qc,
                                                uint32_t (&px)[8][2]) {
    float W[64];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        W[2 * k] = (float)(int)(short)(qp[k] & 0xffffu) * qc.qs[2 * k];
        W[2 * k + 1] = (float)((int)qp[k] >> 16) * qc.qs[2 * k + 1];
    }
    reconstruct_f(W, px);
}

// Dequantise + inverse transform of one block whose int16 coefficients sit in
// 32 dwords (natural order, two per dword), producing 8 rows of 8 pixels.
template <class QC>
__device__ __forceinline__ void decode_block(const uint32_t (&qp)[32], const QC& qc,
                                             uint32_t (&px)[8][2]) {
    int W[64];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        // |q| <= 2^15 and Q <= 4095 fit the 24-bit multiplier exactly.
        W[2 * k] = __mul24((int)(short)(qp[k] & 0xffffu), qc.Q[2 * k]);
        W[2 * k + 1] = __mul24((int)qp[k] >> 16, qc.Q[2 * k + 1]);
    }
    reconstruct(W, px);
}

// ---- encoder tile ------------------------------------------------------------
//
// Lane l owns blocks first + l (a) and first + 64 + l (b) of the tile. The
// rows of 64 consecutive blocks are contiguous, so each pixel load covers a
// 512-byte run, and the coefficients of all a-blocks (then all b-blocks) are
// one contiguous 8 KB run for the staged stores.

// Raw pixel rows of an encoder tile as loaded: rows of block first + l (A)
// and of block first + 64 + l (B).
struct EncPixels {
    uint32_t A[8][2], B[8][2];
};

template <int PC = PX_STREAM>
__device__ __forceinline__ void enc_load(const ImgDesc& d, uint32_t first, uint32_t count,
                                         uint32_t lane, EncPixels& P) {
    const bool va = lane < count, vb = lane + 64u < count;
    const uint32_t nbx = (uint32_t)d.nbx;
    const uint32_t ba = first + lane, bb = ba + 64u;
    if (count == (uint32_t)kEncTileBlocks && (d.flags & F_SRC8)) {
        const uint8_t* pa = d.src + block_offset(d.src_stride, nbx, ba);
        const uint8_t* pb = d.src + block_offset(d.src_stride, nbx, bb);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const v2u x = ld_px<PC>(pa + r * d.src_stride);
            const v2u y = ld_px<PC>(pb + r * d.src_stride);
            P.A[r][0] = x.x;
            P.A[r][1] = x.y;
            P.B[r][0] = y.x;
            P.B[r][1] = y.y;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) P.A[r][0] = P.A[r][1] = P.B[r][0] = P.B[r][1] = 0x80808080u;
        if (va)
            load_rows8<PC>(d.src + block_offset(d.src_stride, nbx, ba), d.src_stride, d.flags, P.A);
        if (vb)
            load_rows8<PC>(d.src + block_offset(d.src_stride, nbx, bb), d.src_stride, d.flags, P.B);
    }
}

// A hook the tile code calls once its inputs are consumed and before its
// stores (a caller walking several tiles loads the next one's inputs there).
struct NoPrefetch {
    __device__ void operator()() const {}
};

// Codes the tile whose pixels are in P.
template <int OP, int PC = PX_STREAM, class QC, class PF>
__device__ __forceinline__ void enc_tile(const ImgDesc& d, const QC& qc, uint32_t first,
                                         uint32_t count, uint32_t lane, v4u* wl, EncPixels& P,
                                         PF&& prefetch) {
    const bool va = lane < count, vb = lane + 64u < count;
    const uint32_t nbx = (uint32_t)d.nbx;
    const uint32_t ba = first + lane, bb = ba + 64u;
    const auto& A = P.A;
    const auto& B = P.B;

    // Pixel (r, c) of both blocks as a packed (a, b) int16 pair.
    s16x2 v[64];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t k = (uint32_t)(c & 3);
            const uint32_t sel = k | (0x0cu << 8) | ((4u + k) << 16) | (0x0cu << 24);
            v[8 * r + c] = as_s16x2(__builtin_amdgcn_perm(B[r][c >> 2], A[r][c >> 2], sel));
        }
    }
    prefetch();
    fwd8x8(v);
    v[0] -= (s16x2){8192, 8192};

    // Blocks in the a and b halves; a tile of at most 64 blocks skips the
    // b half's staging round.
    const uint32_t na = min(count, 64u), nb = count > 64u ? count - 64u : 0u;
    if constexpr (OP == OP_FORWARD) {
        // int32 Y, natural order: 16 chunks per block, staged as the first
        // and then the second half of every block.
        v4u* out = reinterpret_cast<v4u*>(d.coef) + (int64_t)first * 16;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            v4u ma[8], mb[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int k = 32 * h + 4 * m;
                ma[m] = (v4u){(uint32_t)(int)v[k].x, (uint32_t)(int)v[k + 1].x,
                              (uint32_t)(int)v[k + 2].x, (uint32_t)(int)v[k + 3].x};
                mb[m] = (v4u){(uint32_t)(int)v[k].y, (uint32_t)(int)v[k + 1].y,
                              (uint32_t)(int)v[k + 2].y, (uint32_t)(int)v[k + 3].y};
            }
            stage_out<8, 16>(wl, ma, 8 * na, out + 8 * h, lane);
            if (nb) stage_out<8, 16>(wl, mb, 8 * nb, out + 1024 + 8 * h, lane);
        }
    } else if constexpr (OP == OP_ENCODE_I8ZZ) {
        // int8, zigzag order: 64 bytes (4 chunks) per block.
        v4u ma[4], mb[4];
#pragma unroll
        for (int n = 0; n < 64; n += 16) {
            uint32_t wa[4], wb[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                int a4[4], b4[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = kZigzag.order[n + 4 * g + t];
                    // t's bits grow with q, so saturating them saturates q;
                    // the low byte is then q's two's-complement byte.
                    a4[t] = (int)(min(max(quant_bits(v[k].x, qc.r[k]), kRoundMagicBits - 128u),
                                      kRoundMagicBits + 127u) & 0xffu);
                    b4[t] = (int)(min(max(quant_bits(v[k].y, qc.r[k]), kRoundMagicBits - 128u),
                                      kRoundMagicBits + 127u) & 0xffu);
                }
                wa[g] = pack8(a4[0], a4[1], a4[2], a4[3]);
                wb[g] = pack8(b4[0], b4[1], b4[2], b4[3]);
            }
            ma[n / 16] = (v4u){wa[0], wa[1], wa[2], wa[3]};
            mb[n / 16] = (v4u){wb[0], wb[1], wb[2], wb[3]};
        }
        v4u* out = reinterpret_cast<v4u*>(d.coef) + (int64_t)first * 4;
        stage_out<4, 4, PC>(wl, ma, 4 * na, out, lane);
        if (nb) stage_out<4, 4, PC>(wl, mb, 4 * nb, out + 256, lane);
    } else if constexpr (OP == OP_ROUNDTRIP_NC) {
        // Encode and decode without storing coefficients. The rounding float
        // t is M + q exactly (an integer in [2^23, 2^24)), so t - M is q as an
        // fp32 value and (t - M) (Q / 64) is the fp32 decoder's input.
        uint32_t px[8][2];
        if (va) {
            float W[64];
#pragma unroll
            for (int k = 0; k < 64; ++k)
                W[k] = (__builtin_bit_cast(float, quant_bits(v[k].x, qc.r[k])) - kRoundMagic) *
                       qc.qs[k];
            reconstruct_f(W, px);
            store_rows8<PC>(d.dst + block_offset(d.dst_stride, nbx, ba), d.dst_stride, d.flags, px);
        }
        if (vb) {
            float W[64];
#pragma unroll
            for (int k = 0; k < 64; ++k)
                W[k] = (__builtin_bit_cast(float, quant_bits(v[k].y, qc.r[k])) - kRoundMagic) *
                       qc.qs[k];
            reconstruct_f(W, px);
            store_rows8<PC>(d.dst + block_offset(d.dst_stride, nbx, bb), d.dst_stride, d.flags, px);
        }
    } else {
        // OP_ENCODE / OP_ROUNDTRIP: int16 coefficients, natural order.
        uint32_t qa[32], qb[32];
#pragma unroll
        for (int k = 0; k < 64; k += 2) {
            qa[k / 2] = pack16((int)quant_bits(v[k].x, qc.r[k]), (int)quant_bits(v[k + 1].x, qc.r[k + 1]));
            qb[k / 2] = pack16((int)quant_bits(v[k].y, qc.r[k]), (int)quant_bits(v[k + 1].y, qc.r[k + 1]));
        }
        const bool write_coef = (OP == OP_ENCODE) || (d.flags & F_COEF);
        if (write_coef) {
            v4u* out = reinterpret_cast<v4u*>(d.coef) + (int64_t)first * 8;
            v4u m8[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) m8[m] = (v4u){qa[4 * m], qa[4 * m + 1], qa[4 * m + 2], qa[4 * m + 3]};
            stage_out<8, 8, PC>(wl, m8, 8 * na, out, lane);
            if (nb) {
#pragma unroll
                for (int m = 0; m < 8; ++m)
                    m8[m] = (v4u){qb[4 * m], qb[4 * m + 1], qb[4 * m + 2], qb[4 * m + 3]};
                stage_out<8, 8, PC>(wl, m8, 8 * nb, out + 512, lane);
            }
        }
        if constexpr (OP == OP_ROUNDTRIP) {
            uint32_t px[8][2];
            if (va) {
                decode_block_rt(qa, qc, px);
                store_rows8<PC>(d.dst + block_offset(d.dst_stride, nbx, ba), d.dst_stride, d.flags, px);
            }
            if (vb) {
                decode_block_rt(qb, qc, px);
                store_rows8<PC>(d.dst + block_offset(d.dst_stride, nbx, bb), d.dst_stride, d.flags, px);
            }
        }
    }
}

template <int OP, int PC = PX_STREAM, class QC>
__device__ __forceinline__ void enc_tile(const ImgDesc& d, const QC& qc, uint32_t first,
                                         uint32_t count, uint32_t lane, v4u* wl) {
    EncPixels P;
    enc_load<PC>(d, first, count, lane, P);
    enc_tile<OP, PC>(d, qc, first, count, lane, wl, P, NoPrefetch());
}

// ---- decoder tile -----------------------------------------------------------
//
// Lane l owns block first + l.

// The tile's coefficients as loaded: 16-byte chunk 64 k + l of the tile's run
// in element k of lane l.
struct DecChunks {
    v4u c[8];
};

template <int PC = PX_STREAM>
__device__ __forceinline__ void dec_load(const ImgDesc& d, uint32_t first, uint32_t count,
                                         uint32_t lane, DecChunks& C) {
    stage_load<PC>(reinterpret_cast<const v4u*>(d.coef) + (int64_t)first * 8, 8 * count, lane, C.c);
}

// Decodes lane's block from its 8 chunks and stores its pixels.
template <int PC = PX_STREAM, class QC>
__device__ __forceinline__ void dec_finish(const ImgDesc& d, const QC& qc, uint32_t first,
                                           uint32_t lane, const v4u (&mine)[8]) {
    uint32_t qp[32];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        qp[4 * m] = mine[m].x;
        qp[4 * m + 1] = mine[m].y;
        qp[4 * m + 2] = mine[m].z;
        qp[4 * m + 3] = mine[m].w;
    }
    uint32_t px[8][2];
    decode_block(qp, qc, px);
    const uint32_t b = first + lane;
    store_rows8<PC>(d.dst + block_offset(d.dst_stride, (uint32_t)d.nbx, b), d.dst_stride, d.flags,
                        px);
}

template <int PC = PX_STREAM, class QC, class PF>
__device__ __forceinline__ void dec_tile(const ImgDesc& d, const QC& qc, uint32_t first,
                                         uint32_t count, uint32_t lane, v4u* wl, DecChunks& C,
                                         PF&& prefetch) {
    v4u mine[8];
    stage_swap(wl, C.c, lane, mine);
    prefetch();
    if (lane >= count) return;
    dec_finish<PC>(d, qc, first, lane, mine);
}

template <int PC = PX_STREAM, class QC>
__device__ __forceinline__ void dec_tile(const ImgDesc& d, const QC& qc, uint32_t first,
                                         uint32_t count, uint32_t lane, v4u* wl) {
    v4u tmp[8], mine[8];
    stage_load(reinterpret_cast<const v4u*>(d.coef) + (int64_t)first * 8, 8 * count, lane, tmp);
    stage_swap(wl, tmp, lane, mine);
    if (lane >= count) return;
    dec_finish<PC>(d, qc, first, lane, mine);
}

template <int OP, int PC = PX_STREAM, class QC>
__device__ __forceinline__ void run_tile(const ImgDesc& d, const QC& qc, uint32_t first,
                                         uint32_t count, uint32_t lane, v4u* wl) {
    if constexpr (OP == OP_DECODE)
        dec_tile<PC>(d, qc, first, count, lane, wl);
    else
        enc_tile<OP, PC>(d, qc, first, count, lane, wl);
}

// LDS bytes one wave needs for a set of ops (bit i = op i).
__host__ __device__ constexpr uint32_t lds_wave_bytes(int ops) {
    return (ops & ((1 << OP_ENCODE) | (1 << OP_ROUNDTRIP) | (1 << OP_DECODE) | (1 << OP_FORWARD)))
               ? 8192u
           : (ops & (1 << OP_ENCODE_I8ZZ)) ? 4096u
                                           : 0u;
}

}  // namespace tdct
