// Host-side instantiation of the library's device building blocks, for the
// CPU test suite: the same header the kernels use, compiled for the host.
// It lets the tests count the operations of one 8-point pass (Table 1), run
// the butterflies over exhaustive inputs, and sweep the quantiser over its
// whole domain without a GPU.
#include <stdint.h>

#include "tdct_device.hpp"

namespace {

struct Counts {
    int add = 0, sub = 0, neg = 0, mul = 0, shift = 0;
};
thread_local Counts g;

struct Op {
    int64_t v;
};
inline Op operator+(Op a, Op b) { ++g.add; return {a.v + b.v}; }
inline Op operator-(Op a, Op b) { ++g.sub; return {a.v - b.v}; }
inline Op operator-(Op a) { ++g.neg; return {-a.v}; }
inline Op operator*(Op a, Op b) { ++g.mul; return {a.v * b.v}; }
inline Op operator<<(Op a, int s) { ++g.shift; return {a.v << s}; }
inline Op operator>>(Op a, int s) { ++g.shift; return {a.v >> s}; }

}  // namespace

extern "C" {

// counts[0..4] = additions, subtractions, negations, multiplications, shifts
// of one 8-point pass (inverse = 0: T x, 1: T^t x), or of the whole 8x8
// block transform (block = 1).
void hc_count(int32_t inverse, int32_t block, int32_t counts[5]) {
    g = Counts{};
    Op v[64];
    for (int k = 0; k < 64; ++k) v[k] = Op{k};
    if (block) {
        if (inverse) tdct::inv8x8(v);
        else tdct::fwd8x8(v);
    } else {
        if (inverse) tdct::inv8(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
        else tdct::fwd8(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
    }
    counts[0] = g.add;
    counts[1] = g.sub;
    counts[2] = g.neg;
    counts[3] = g.mul;
    counts[4] = g.shift;
}

// n vectors of 8 in, 8 out each: the butterfly on int64.
void hc_apply8(const int64_t* in, int64_t* out, int64_t n, int32_t inverse) {
    for (int64_t k = 0; k < n; ++k) {
        int64_t x[8];
        for (int t = 0; t < 8; ++t) x[t] = in[8 * k + t];
        if (inverse) tdct::inv8(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7]);
        else tdct::fwd8(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7]);
        for (int t = 0; t < 8; ++t) out[8 * k + t] = x[t];
    }
}

// n blocks of 64: the 2-D butterfly transform (row pass, then column pass).
void hc_apply8x8(const int64_t* in, int64_t* out, int64_t n, int32_t inverse) {
    for (int64_t k = 0; k < n; ++k) {
        int64_t x[64];
        for (int t = 0; t < 64; ++t) x[t] = in[64 * k + t];
        if (inverse) tdct::inv8x8(x);
        else tdct::fwd8x8(x);
        for (int t = 0; t < 64; ++t) out[64 * k + t] = x[t];
    }
}

void hc_zigzag(int32_t order[64]) {
    for (int k = 0; k < 64; ++k) order[k] = tdct::kZigzag.order[k];
}

void hc_shifts(int32_t s[64]) {
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) s[8 * i + j] = tdct::kShift(i, j);
}

// q for every y in [y0, y0 + n) at shift s and divisor Q, exactly as the
// kernels compute it.
void hc_quant(int32_t Q, int32_t s, int32_t y0, int32_t n, int32_t* out) {
    const float r = tdct::quant_recip(Q, s, true);
    for (int32_t k = 0; k < n; ++k) out[k] = tdct::quant_int(y0 + k, r);
}

// The int8 path's saturation on the raw bits and the int16 path's low half:
// out8[k] = the byte the encoder stores, out16[k] = the halfword it stores.
void hc_quant_lanes(int32_t Q, int32_t s, int32_t y0, int32_t n, int8_t* out8, int16_t* out16) {
    const float r = tdct::quant_recip(Q, s, true);
    for (int32_t k = 0; k < n; ++k) {
        uint32_t b = tdct::quant_bits(y0 + k, r);
        uint32_t c = b < tdct::kRoundMagicBits - 128u ? tdct::kRoundMagicBits - 128u
                   : (b > tdct::kRoundMagicBits + 127u ? tdct::kRoundMagicBits + 127u : b);
        out8[k] = (int8_t)(uint8_t)(c & 0xffu);
        out16[k] = (int16_t)(uint16_t)(b & 0xffffu);
    }
}

// out[b] = the tile-order place of workgroup b of n under the XCD remap.
void hc_xcd_order(uint32_t n, uint32_t* out) {
    for (uint32_t b = 0; b < n; ++b) out[b] = tdct::xcd_order(b, n);
}

// The round trips' fp32 decoder half on the host, for n blocks of W' = q Q
// (int32, natural order): W'' = W' / 64 with the pixel bias at (0, 0), the
// library's inverse butterflies in fp32, the values before the conversion to
// u8 (out), and the pixels that conversion makes -- round to nearest, ties to
// even, saturated to [0, 255] (pix).
void hc_inverse_f32(const int32_t* wq, int64_t n, float* out, uint8_t* pix) {
    for (int64_t b = 0; b < n; ++b) {
        float W[64];
        for (int k = 0; k < 64; ++k) W[k] = (float)wq[64 * b + k] * (1.0f / 64.0f);
        W[0] += tdct::kPixelBiasF;
        tdct::inv8x8(W);
        for (int k = 0; k < 64; ++k) {
            out[64 * b + k] = W[k];
            const float r = __builtin_nearbyintf(W[k]);
            pix[64 * b + k] = (uint8_t)(r < 0.0f ? 0.0f : r > 255.0f ? 255.0f : r);
        }
    }
}

}  // extern "C"
