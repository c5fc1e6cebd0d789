// HIP kernels of the codec for gfx950 (CDNA4), and the plain C-ABI calls.
// The per-wave tile code lives in tdct_tiles.hpp.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "tdct.h"
#include "tdct_device.hpp"
#include "tdct_internal.hpp"
#include "tdct_tiles.hpp"

namespace tdct {

// ---- kernels -----------------------------------------------------------------

// One image, quantiser constants in the kernel arguments. Wave w handles
// tiles w, w + nwaves, ... of the image, each of `tb` blocks (at most the
// op's tile size).
template <int OP, int PC>
__global__ __launch_bounds__(256) void plain_kernel(const ImgDesc d, const QConst qc,
                                                    uint32_t ntiles, uint32_t tb) {
    extern __shared__ v4u lds[];
    v4u* wl = lds + (threadIdx.x >> 6) * (lds_wave_bytes(1 << OP) / 16);
    const uint32_t wpg = blockDim.x >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * wpg + (threadIdx.x >> 6));
    const uint32_t nwaves = gridDim.x * wpg;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t nblk = (uint32_t)d.nblk;
    for (uint32_t t = wave; t < ntiles; t += nwaves) {
        const uint32_t first = t * tb;
        const uint32_t count = min(tb, nblk - first);
        run_tile<OP, PC>(d, qc, first, count, lane, wl);
    }
}

// Many images: tiles come from a table; each tile names its image, whose
// descriptor and quantiser constants are read with scalar loads (the tile is
// image-uniform, so they are the same for the whole wave). OPS is the set of
// ops the plan contains; single-op plans get a kernel with just that path.
// CACHED selects the pixel-plane cache policy (ld_px / st_px).
template <int OPS, bool CACHED>
__global__ __launch_bounds__(512) void batch_kernel(const Tile* __restrict__ tiles,
                                                     const ImgDesc* __restrict__ imgs,
                                                     const QConst* __restrict__ qcs,
                                                     uint32_t ntiles, uint32_t tile_waves,
                                                     uint32_t xcd_remap) {
    extern __shared__ v4u lds[];
    v4u* wl = lds + (threadIdx.x >> 6) * (lds_wave_bytes(OPS) / 16);
    const uint32_t wpg = blockDim.x >> 6;
    const uint32_t group = xcd_remap ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(group * wpg + (threadIdx.x >> 6));
    const uint32_t nwaves = gridDim.x * wpg;
    const uint32_t lane = threadIdx.x & 63;
    // A wave takes `tile_waves` consecutive tiles per step.
    for (uint32_t t0 = wave * tile_waves; t0 < ntiles; t0 += nwaves * tile_waves) {
        const uint32_t tend = min(t0 + tile_waves, ntiles);
        for (uint32_t t = t0; t < tend; ++t) {
            const Tile tl = tiles[t];
            const ImgDesc d = global_desc(imgs[tl.img]);
            const QConst& qc = qcs[d.qidx];
            const int op = (OPS & (OPS - 1)) == 0 ? __builtin_ctz(OPS) : d.op;
            switch (op) {
                case OP_ENCODE:
                    if constexpr ((OPS >> OP_ENCODE) & 1)
                        run_tile<OP_ENCODE, CACHED>(d, qc, tl.first_lo, tl.count, lane, wl);
                    break;
                case OP_DECODE:
                    if constexpr ((OPS >> OP_DECODE) & 1)
                        run_tile<OP_DECODE, CACHED>(d, qc, tl.first_lo, tl.count, lane, wl);
                    break;
                case OP_ROUNDTRIP:
                    if constexpr ((OPS >> OP_ROUNDTRIP) & 1)
                        run_tile<OP_ROUNDTRIP, CACHED>(d, qc, tl.first_lo, tl.count, lane, wl);
                    break;
                case OP_ENCODE_I8ZZ:
                    if constexpr ((OPS >> OP_ENCODE_I8ZZ) & 1)
                        run_tile<OP_ENCODE_I8ZZ, CACHED>(d, qc, tl.first_lo, tl.count, lane, wl);
                    break;
                case OP_ROUNDTRIP_NC:
                    if constexpr ((OPS >> OP_ROUNDTRIP_NC) & 1)
                        run_tile<OP_ROUNDTRIP_NC, CACHED>(d, qc, tl.first_lo, tl.count, lane, wl);
                    break;
                default:
                    if constexpr ((OPS >> OP_FORWARD) & 1)
                        run_tile<OP_FORWARD, CACHED>(d, qc, tl.first_lo, tl.count, lane, wl);
                    break;
            }
        }
    }
}

// Sum of squared differences; one 64-bit atomic per workgroup.
__global__ __launch_bounds__(256) void sse_kernel(const uint8_t* a, int64_t as, const uint8_t* b,
                                                  int64_t bs, int32_t w, int32_t h,
                                                  unsigned long long* out) {
    unsigned long long acc = 0;
    const int64_t n = (int64_t)w * h;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / w, x = i - y * w;
        const int dd = (int)a[y * as + x] - (int)b[y * bs + x];
        acc += (unsigned long long)(dd * dd);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += part[k];
        atomicAdd(out, s);
    }
}

__global__ void zero_u64(unsigned long long* p) { *p = 0ull; }

// ---- host side ---------------------------------------------------------------

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(what, e);
        return TDCT_EDEVICE;
    }
    return TDCT_OK;
}

int validate_plane(const void* p, int64_t stride, int32_t w, int32_t h) {
    if (w <= 0 || h <= 0 || (w & 7) || (h & 7) || w > TDCT_MAX_SIDE || h > TDCT_MAX_SIDE)
        return TDCT_EDIM;
    if (!p || stride < w) return TDCT_EINVAL;
    return TDCT_OK;
}

int validate_q(const tdct_qtable* Q) {
    if (!Q) return TDCT_EINVAL;
    for (int k = 0; k < 64; ++k)
        if (Q->q[k] < 1 || Q->q[k] > TDCT_QMAX) return TDCT_EQTAB;
    return TDCT_OK;
}

void make_qconst(const tdct_qtable* Q, int keep, QConst* out) {
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * i + j;
            const int q = Q ? Q->q[k] : 1;
            out->r[k] = quant_recip(q, kShift(i, j), kZigzag.rank[k] < keep);
            out->Q[k] = q;
            out->qs[k] = (float)q / 64.0f;  // exact: q < 2^12
        }
}

int image_flags(const ImgDesc& d) {
    int f = 0;
    const uintptr_t s = (uintptr_t)d.src, t = (uintptr_t)d.dst;
    if (d.src && (s % 8 == 0) && (d.src_stride % 8 == 0)) f |= F_SRC8;
    if (d.dst && (t % 8 == 0) && (d.dst_stride % 8 == 0)) f |= F_DST8;
    return f;
}

// Dynamic LDS above 64 KB per workgroup has to be enabled per kernel.
template <typename K>
static int allow_lds(K kernel, uint32_t bytes) {
    if (bytes <= 65536) return TDCT_OK;
    // initialised once, thread-safely, by the first caller
    static const int device_max = [] {
        int dev = 0, m = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&m, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return 65536;
        return m;
    }();
    if ((int)bytes > device_max) return TDCT_EINVAL;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
        set_error("dynamic LDS attribute", e);
        return TDCT_EDEVICE;
    }
    return TDCT_OK;
}

// SIMDs of the current device (4 per CU), cached per thread and device.
static uint32_t device_simds() {
    thread_local int dev_cached = -1;
    thread_local uint32_t simds = 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (dev != dev_cached) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            return 1024;
        dev_cached = dev;
        simds = 4u * (uint32_t)cus;
    }
    return simds;
}

// One wave per workgroup and one tile per wave, so that the few waves of a
// small image spread over as many CUs as there are waves. An encoder-side
// tile (two blocks per lane) shrinks to 64 blocks while 128-block tiles
// would leave SIMDs without a wave: each wave then does half the serial
// work (one block per lane) and there are twice as many of them.
// Pixel accesses of a plain call: cached for planes up to kPlainCachedPx
// pixels, streaming above. Measured with back-to-back calls over rotating
// sources: below about 4 Mpx cached accesses took the encoder and decoder
// 3-9 % faster (1000x1000 and 2040x1528; such planes sit in the 256 MB MALL
// between producer and consumer, and rows that end inside a 128-byte line
// meet their neighbour tile's part in L2), while from 4096x4096 up they were
// as fast for the encoder and 5-8 % slower for the decoder.
constexpr int64_t kPlainCachedPx = 4 << 20;

template <int OP>
static int launch_plain(const ImgDesc& d, const QConst& qc, hipStream_t stream) {
    uint32_t tb = (uint32_t)tile_blocks(OP);
    if (tb > 64 && (uint64_t)(d.nblk + tb - 1) / tb < device_simds()) tb = 64;
    const uint32_t ntiles = (uint32_t)((d.nblk + tb - 1) / tb);
    const uint32_t lds = lds_wave_bytes(1 << OP);
    if (d.nblk * 64 <= kPlainCachedPx)
        hipLaunchKernelGGL((plain_kernel<OP, PX_CACHED>), dim3(ntiles), dim3(64), lds, stream, d, qc, ntiles, tb);
    else
        hipLaunchKernelGGL((plain_kernel<OP, PX_STREAM>), dim3(ntiles), dim3(64), lds, stream, d, qc, ntiles, tb);
    return check_launch("plain kernel launch");
}

int launch_plain_op(int op, const ImgDesc& d, const QConst& qc, hipStream_t stream) {
    switch (op) {
        case OP_ENCODE: return launch_plain<OP_ENCODE>(d, qc, stream);
        case OP_DECODE: return launch_plain<OP_DECODE>(d, qc, stream);
        case OP_ROUNDTRIP: return launch_plain<OP_ROUNDTRIP>(d, qc, stream);
        case OP_ENCODE_I8ZZ: return launch_plain<OP_ENCODE_I8ZZ>(d, qc, stream);
        case OP_FORWARD: return launch_plain<OP_FORWARD>(d, qc, stream);
        case OP_ROUNDTRIP_NC: return launch_plain<OP_ROUNDTRIP_NC>(d, qc, stream);
    }
    return TDCT_EINVAL;
}

template <int OPS>
static int launch_batch_ops(const Tile* tiles, const ImgDesc* imgs, const QConst* qcs,
                            uint32_t ntiles, const tdct_tune& tune, int num_cus,
                            hipStream_t stream) {
    const uint32_t wpg = (uint32_t)tune.waves_per_group;
    const uint32_t tw = (uint32_t)tune.tile_waves;
    const uint32_t steps = (ntiles + tw - 1) / tw;
    uint32_t grid = (uint32_t)num_cus * (uint32_t)tune.groups_per_cu;
    const uint32_t need = (steps + wpg - 1) / wpg;
    if (grid > need) grid = need;
    if (grid == 0) grid = 1;
    const uint32_t lds = wpg * lds_wave_bytes(OPS);
    auto kernel = tune.pixel_cache ? batch_kernel<OPS, true> : batch_kernel<OPS, false>;
    int st = allow_lds(kernel, lds);
    if (st) return st;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(64 * wpg), lds, stream, tiles, imgs, qcs, ntiles, tw,
                       (uint32_t)(tune.xcd_remap != 0));
    return check_launch("batch kernel launch");
}

uint32_t batch_lds_bytes(int ops, int waves_per_group) {
    return (uint32_t)waves_per_group * lds_wave_bytes(ops);
}

int launch_batch(const Tile* tiles, const ImgDesc* imgs, const QConst* qcs, uint32_t ntiles,
                 int ops, const tdct_tune& tune, int num_cus, hipStream_t stream) {
    if (ntiles == 0) return TDCT_OK;
    constexpr int E = 1 << OP_ENCODE, D = 1 << OP_DECODE, R = 1 << OP_ROUNDTRIP,
                  Z = 1 << OP_ENCODE_I8ZZ, F = 1 << OP_FORWARD, N = 1 << OP_ROUNDTRIP_NC;
    switch (ops) {
        case N: return launch_batch_ops<N>(tiles, imgs, qcs, ntiles, tune, num_cus, stream);
        case E: return launch_batch_ops<E>(tiles, imgs, qcs, ntiles, tune, num_cus, stream);
        case D: return launch_batch_ops<D>(tiles, imgs, qcs, ntiles, tune, num_cus, stream);
        case R: return launch_batch_ops<R>(tiles, imgs, qcs, ntiles, tune, num_cus, stream);
        case Z: return launch_batch_ops<Z>(tiles, imgs, qcs, ntiles, tune, num_cus, stream);
        case F: return launch_batch_ops<F>(tiles, imgs, qcs, ntiles, tune, num_cus, stream);
        case E | D: return launch_batch_ops<E | D>(tiles, imgs, qcs, ntiles, tune, num_cus, stream);
        default:
            return launch_batch_ops<E | D | R | Z | F | N>(tiles, imgs, qcs, ntiles, tune, num_cus,
                                                           stream);
    }
}

int fill_desc(int op, const uint8_t* src, int64_t src_stride, int32_t w, int32_t h, void* coef,
              uint8_t* dst, int64_t dst_stride, int32_t qidx, bool write_coef, ImgDesc* d) {
    d->src = src;
    d->dst = dst;
    d->coef = coef;
    d->src_stride = src_stride;
    d->dst_stride = dst_stride;
    d->nbx = w / 8;
    d->nblk = (int64_t)(w / 8) * (h / 8);
    d->op = (op == OP_ROUNDTRIP && !write_coef) ? OP_ROUNDTRIP_NC : op;
    d->qidx = qidx;
    d->flags = image_flags(*d) | (write_coef ? F_COEF : 0);
    return TDCT_OK;
}

}  // namespace tdct

using namespace tdct;

static int coef_aligned(const void* p) { return p && ((uintptr_t)p % 16 == 0); }

extern "C" {

int tdct_forward(const uint8_t* src, int64_t src_stride, int32_t w, int32_t h, int32_t* coef,
                 void* stream) {
    int st = validate_plane(src, src_stride, w, h);
    if (st) return st;
    if (!coef_aligned(coef)) return TDCT_EINVAL;
    ImgDesc d;
    fill_desc(OP_FORWARD, src, src_stride, w, h, coef, nullptr, 0, 0, false, &d);
    QConst qc;
    make_qconst(nullptr, 64, &qc);
    return launch_plain_op(OP_FORWARD, d, qc, (hipStream_t)stream);
}

int tdct_quantise(const uint8_t* src, int64_t src_stride, int32_t w, int32_t h,
                  const tdct_qtable* Q, int32_t keep, int16_t* q, void* stream) {
    int st = validate_plane(src, src_stride, w, h);
    if (st) return st;
    if ((st = validate_q(Q))) return st;
    if (!coef_aligned(q) || keep < 1 || keep > 64) return TDCT_EINVAL;
    ImgDesc d;
    fill_desc(OP_ENCODE, src, src_stride, w, h, q, nullptr, 0, 0, true, &d);
    QConst qc;
    make_qconst(Q, keep, &qc);
    return launch_plain_op(OP_ENCODE, d, qc, (hipStream_t)stream);
}

int tdct_inverse(const int16_t* q, const tdct_qtable* Q, int32_t w, int32_t h, uint8_t* dst,
                 int64_t dst_stride, void* stream) {
    int st = validate_plane(dst, dst_stride, w, h);
    if (st) return st;
    if ((st = validate_q(Q))) return st;
    if (!coef_aligned(q)) return TDCT_EINVAL;
    ImgDesc d;
    fill_desc(OP_DECODE, nullptr, 0, w, h, const_cast<int16_t*>(q), dst, dst_stride, 0, false, &d);
    QConst qc;
    make_qconst(Q, 64, &qc);
    return launch_plain_op(OP_DECODE, d, qc, (hipStream_t)stream);
}

int tdct_roundtrip(const uint8_t* src, int64_t src_stride, int32_t w, int32_t h,
                   const tdct_qtable* Q, int32_t keep, int16_t* q_or_null, uint8_t* dst,
                   int64_t dst_stride, void* stream) {
    int st = validate_plane(src, src_stride, w, h);
    if (st) return st;
    if ((st = validate_plane(dst, dst_stride, w, h))) return st;
    if ((st = validate_q(Q))) return st;
    if (keep < 1 || keep > 64) return TDCT_EINVAL;
    if (q_or_null && !coef_aligned(q_or_null)) return TDCT_EINVAL;
    ImgDesc d;
    fill_desc(OP_ROUNDTRIP, src, src_stride, w, h, q_or_null, dst, dst_stride, 0,
              q_or_null != nullptr, &d);
    QConst qc;
    make_qconst(Q, keep, &qc);
    return launch_plain_op(d.op, d, qc, (hipStream_t)stream);
}

int tdct_quantise_i8_zigzag(const uint8_t* src, int64_t src_stride, int32_t w, int32_t h,
                            const tdct_qtable* Q, int8_t* out, void* stream) {
    int st = validate_plane(src, src_stride, w, h);
    if (st) return st;
    if ((st = validate_q(Q))) return st;
    if (!coef_aligned(out)) return TDCT_EINVAL;
    ImgDesc d;
    fill_desc(OP_ENCODE_I8ZZ, src, src_stride, w, h, out, nullptr, 0, 0, true, &d);
    QConst qc;
    make_qconst(Q, 64, &qc);
    return launch_plain_op(OP_ENCODE_I8ZZ, d, qc, (hipStream_t)stream);
}

int tdct_sse(const uint8_t* a, int64_t a_stride, const uint8_t* b, int64_t b_stride, int32_t w,
             int32_t h, uint64_t* sse_dev, void* stream) {
    int st = validate_plane(a, a_stride, w, h);
    if (st) return st;
    if ((st = validate_plane(b, b_stride, w, h))) return st;
    if (!sse_dev) return TDCT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, s, (unsigned long long*)sse_dev);
    const int64_t n = (int64_t)w * h;
    int64_t grid = (n + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(sse_kernel, dim3((uint32_t)grid), dim3(256), 0, s, a, a_stride, b, b_stride,
                       w, h, (unsigned long long*)sse_dev);
    return check_launch("sse kernel launch");
}


}  // extern "C"
