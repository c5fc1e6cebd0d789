/*
 * CPU oracle for the 14-addition approximate-DCT block codec
 * (Bayer and Cintra, "DCT-like Transform for Image Compression Requires
 * 14 Additions Only").
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this library. The product path (the HIP
 * library) never links, loads or calls it, and this file includes nothing
 * from the product sources.
 *
 * What it computes is the plain definition, written out as dense loops:
 *   - the paper's fast algorithm reaches T*x exactly over the integers, so
 *     the oracle uses the dense 8x8 matrix T (Section 2) and never the
 *     sparse factorisation;
 *   - the 2-D block transform of Section 3 applies T to the rows and the
 *     columns of every 8x8 block: Y = T * X * T^t, X = block - 128;
 *   - the diagonal scaling D of Section 2 enters only as D^2, merged into
 *     the quantiser: W_ij = 64 * d_i^2 * d_j^2 * Y_ij, with d_i^2 = 1 / |row i
 *     of T|^2, an exact integer multiple of Y_ij;
 *   - q_ij = round-half-away-from-zero(W_ij / Q_ij) on the exact rational;
 *   - zonal coding (Section 3): coefficients whose zigzag rank is >= keep
 *     are set to zero;
 *   - reconstruction (Section 3): W'_ij = q_ij * Q_ij, S = T^t * W' * T and
 *     pixel = clamp(floor((S + 32) / 64) + 128, 0, 255).
 * The integer conventions (level shift, the scale 64, both rounding rules,
 * the clamp) are not fixed by the paper; the oracle takes the readings
 * written out above. Every accumulator is 64-bit, so nothing here can
 * overflow.
 *
 * Block (bx, by) of a w x h plane covers rows 8*by..8*by+7 and columns
 * 8*bx..8*bx+7; blocks are numbered in raster order b = by * (w/8) + bx and
 * block b's 64 coefficients live at out[b*64 + 8*i + j], i = vertical and
 * j = horizontal frequency. Functions take a block range [blk0, blk0+nblk)
 * so that a caller may split one plane over threads; each writes only the
 * outputs of its own blocks.
 */
#include <stdint.h>
#include <stdlib.h>

/* The 8x8 matrix T of Section 2, entries in {0, +1, -1}. */
static const int T[8][8] = {
    {1, 1, 1, 1, 1, 1, 1, 1},
    {1, 0, 0, 0, 0, 0, 0, -1},
    {1, 0, 0, -1, -1, 0, 0, 1},
    {0, 0, -1, 0, 0, 1, 0, 0},
    {1, -1, -1, 1, 1, -1, -1, 1},
    {0, -1, 0, 0, 0, 0, 1, 0},
    {0, -1, 1, 0, 0, 1, -1, 0},
    {0, 0, 0, -1, 1, 0, 0, 0},
};

/* |row i of T|^2 = 1 / d_i^2 (Section 2: D = diag(|row i|^-1) makes D*T
 * orthogonal). */
static int64_t row_norm2(int i) {
    int64_t s = 0;
    for (int j = 0; j < 8; ++j) s += (int64_t)T[i][j] * T[i][j];
    return s;
}

/* 64 * d_i^2 * d_j^2 as an exact integer (64 / (|row i|^2 |row j|^2)). */
static int64_t wscale(int i, int j) {
    return 64 / (row_norm2(i) * row_norm2(j));
}

/* Zigzag scan of an 8x8 block (Section 3, the JPEG sequence): walk the
 * anti-diagonals d = i + j = 0..14; on an odd diagonal the row index i
 * increases (start at (0, d) or the top edge), on an even one it
 * decreases. order[rank] = 8*i + j. */
static void zigzag_order(int order[64]) {
    int rank = 0;
    for (int d = 0; d <= 14; ++d) {
        if (d % 2 == 1) {
            for (int i = 0; i <= d; ++i) {
                int j = d - i;
                if (i < 8 && j < 8) order[rank++] = 8 * i + j;
            }
        } else {
            for (int i = d; i >= 0; --i) {
                int j = d - i;
                if (i < 8 && j < 8) order[rank++] = 8 * i + j;
            }
        }
    }
}

static void zigzag_rank(int rank_of[64]) {
    int order[64];
    zigzag_order(order);
    for (int r = 0; r < 64; ++r) rank_of[order[r]] = r;
}

/* floor(a / b) for b > 0, written out for negative a. */
static int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b) != 0 && (a < 0)) q -= 1;
    return q;
}

/* ---- exported helpers (constants, for the oracle's own checks) -------- */

void oracle_get_T(int32_t out[64]) {
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) out[8 * i + j] = T[i][j];
}

void oracle_get_wscale(int32_t out[64]) {
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) out[8 * i + j] = (int32_t)wscale(i, j);
}

void oracle_get_zigzag(int32_t order_out[64]) {
    int order[64];
    zigzag_order(order);
    for (int r = 0; r < 64; ++r) order_out[r] = order[r];
}

/* round-half-away-from-zero of the rational W / Q, Q >= 1:
 * sign(W) * floor((2|W| + Q) / (2Q)). */
int64_t oracle_round_div(int64_t W, int64_t Q) {
    int64_t a = W < 0 ? -W : W;
    int64_t m = (2 * a + Q) / (2 * Q);
    return W < 0 ? -m : m;
}

/* out[k] = round-half-away(W[k] / Q) for k < n. */
void oracle_round_div_array(const int64_t* W, int64_t n, int64_t Q, int64_t* out) {
    for (int64_t k = 0; k < n; ++k) out[k] = oracle_round_div(W[k], Q);
}

/* 1-D: y = T * x (transpose = 0) or y = T^t * x (transpose = 1). */
void oracle_apply_T(const int64_t x[8], int64_t y[8], int32_t transpose) {
    for (int k = 0; k < 8; ++k) {
        int64_t s = 0;
        for (int n = 0; n < 8; ++n)
            s += (transpose ? T[n][k] : T[k][n]) * x[n];
        y[k] = s;
    }
}

/* Y = T * X * T^t on an arbitrary integer block (row-major X[r][c]). */
void oracle_forward_block(const int64_t X[64], int64_t Y[64]) {
    int64_t M[64];
    /* M = T * X : M[i][c] = sum_r T[i][r] X[r][c] */
    for (int i = 0; i < 8; ++i)
        for (int c = 0; c < 8; ++c) {
            int64_t s = 0;
            for (int r = 0; r < 8; ++r) s += T[i][r] * X[8 * r + c];
            M[8 * i + c] = s;
        }
    /* Y = M * T^t : Y[i][j] = sum_c M[i][c] T[j][c] */
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            int64_t s = 0;
            for (int c = 0; c < 8; ++c) s += M[8 * i + c] * T[j][c];
            Y[8 * i + j] = s;
        }
}

/* S = T^t * W * T on an arbitrary integer block (the inverse of Section 3
 * without the 1/64 scale). */
void oracle_inverse_block(const int64_t W[64], int64_t S[64]) {
    int64_t M[64];
    /* M = T^t * W : M[r][j] = sum_i T[i][r] W[i][j] */
    for (int r = 0; r < 8; ++r)
        for (int j = 0; j < 8; ++j) {
            int64_t s = 0;
            for (int i = 0; i < 8; ++i) s += T[i][r] * W[8 * i + j];
            M[8 * r + j] = s;
        }
    /* S = M * T : S[r][c] = sum_j M[r][j] T[j][c] */
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 8; ++c) {
            int64_t s = 0;
            for (int j = 0; j < 8; ++j) s += M[8 * r + j] * T[j][c];
            S[8 * r + c] = s;
        }
}

/* ---- plane-level codec ------------------------------------------------ */

static void load_block(const uint8_t* src, int64_t stride, int32_t w, int64_t b,
                       int64_t X[64]) {
    int64_t nbx = w / 8;
    int64_t by = b / nbx, bx = b % nbx;
    const uint8_t* p = src + (8 * by) * stride + 8 * bx;
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 8; ++c) X[8 * r + c] = (int64_t)p[r * stride + c] - 128;
}

/* Y (int32, unscaled) for blocks [blk0, blk0 + nblk). */
void oracle_forward(const uint8_t* src, int64_t stride, int32_t w, int32_t h,
                    int64_t blk0, int64_t nblk, int32_t* Y) {
    (void)h;
    int64_t X[64], Yb[64];
    for (int64_t b = blk0; b < blk0 + nblk; ++b) {
        load_block(src, stride, w, b, X);
        oracle_forward_block(X, Yb);
        for (int k = 0; k < 64; ++k) Y[b * 64 + k] = (int32_t)Yb[k];
    }
}

/* q for one block from its unscaled Y: W = 64 d_i^2 d_j^2 Y, rounded
 * quotient by Q, zonal mask by zigzag rank. */
static void quantise_block(const int64_t Y[64], const uint16_t Q[64], int32_t keep,
                           const int rank_of[64], int64_t q[64]) {
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            int k = 8 * i + j;
            int64_t W = Y[k] * wscale(i, j);
            q[k] = rank_of[k] < keep ? oracle_round_div(W, Q[k]) : 0;
        }
}

/* Fused forward + quantise: int16 coefficients, natural (i, j) order. */
void oracle_quantise(const uint8_t* src, int64_t stride, int32_t w, int32_t h,
                     const uint16_t Q[64], int32_t keep, int64_t blk0, int64_t nblk,
                     int16_t* out) {
    (void)h;
    int rank_of[64];
    zigzag_rank(rank_of);
    int64_t X[64], Y[64], q[64];
    for (int64_t b = blk0; b < blk0 + nblk; ++b) {
        load_block(src, stride, w, b, X);
        oracle_forward_block(X, Y);
        quantise_block(Y, Q, keep, rank_of, q);
        for (int k = 0; k < 64; ++k) out[b * 64 + k] = (int16_t)q[k];
    }
}

/* Forward + quantise with int8 saturation, stored in zigzag order:
 * out[b*64 + rank] = clamp(q[order[rank]], -128, 127). */
void oracle_quantise_i8_zigzag(const uint8_t* src, int64_t stride, int32_t w, int32_t h,
                               const uint16_t Q[64], int64_t blk0, int64_t nblk,
                               int8_t* out) {
    (void)h;
    int rank_of[64], order[64];
    zigzag_rank(rank_of);
    zigzag_order(order);
    int64_t X[64], Y[64], q[64];
    for (int64_t b = blk0; b < blk0 + nblk; ++b) {
        load_block(src, stride, w, b, X);
        oracle_forward_block(X, Y);
        quantise_block(Y, Q, 64, rank_of, q);
        for (int r = 0; r < 64; ++r) {
            int64_t v = q[order[r]];
            if (v > 127) v = 127;
            if (v < -128) v = -128;
            out[b * 64 + r] = (int8_t)v;
        }
    }
}

/* Dequantise + inverse for one block: 8x8 pixels into dst (row stride). */
static void reconstruct_block(const int16_t* qb, const uint16_t Q[64], uint8_t* dst,
                              int64_t dst_stride) {
    int64_t Wp[64], S[64];
    for (int k = 0; k < 64; ++k) Wp[k] = (int64_t)qb[k] * (int64_t)Q[k];
    oracle_inverse_block(Wp, S);
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 8; ++c) {
            int64_t v = floor_div(S[8 * r + c] + 32, 64) + 128;
            if (v < 0) v = 0;
            if (v > 255) v = 255;
            dst[r * dst_stride + c] = (uint8_t)v;
        }
}

/* Fused dequantise + inverse: int16 coefficients -> uint8 plane. */
void oracle_inverse(const int16_t* q, const uint16_t Q[64], int32_t w, int32_t h,
                    int64_t blk0, int64_t nblk, uint8_t* dst, int64_t dst_stride) {
    (void)h;
    int64_t nbx = w / 8;
    for (int64_t b = blk0; b < blk0 + nblk; ++b) {
        int64_t by = b / nbx, bx = b % nbx;
        reconstruct_block(q + b * 64, Q, dst + (8 * by) * dst_stride + 8 * bx, dst_stride);
    }
}
