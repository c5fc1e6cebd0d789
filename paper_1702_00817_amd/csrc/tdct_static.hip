// The batch form for callers that cannot allocate device memory.
//
// tdct_batch_run_static does the work of tdct_batch_plan + tdct_batch_run in
// one call without a plan object and without any allocation: the plan's
// tables (tiles, image descriptors, quantiser constants) are built in a
// host buffer of static storage and copied into `scratch`, a file-scope
// device array of kStaticTableBytes that each GPU the library runs on holds
// until the process ends. The persistent batch kernel then reads them from
// there, exactly as it reads a plan's tables.
//
// In host code `scratch` names a host-side stand-in, not the array: its
// device address is looked up once per device, with that device current
// (hipGetSymbolAddress), and only that address is used afterwards.
//
// Sharing: every call on one GPU uses that GPU's array, which keeps the last
// call's tables. A call's copy and its kernel are ordered on the caller's
// stream, so calls on one stream follow each other safely; calls that
// overlap on one GPU (other streams, other threads) race: a later copy can
// overwrite tables an earlier kernel still reads. Nothing in the array has
// to start at zero: every byte a kernel reads is written by its own call.
// The call is not for stream capture: its copy reads g_stage, which the
// next call rewrites.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "tdct.h"
#include "tdct_device.hpp"
#include "tdct_internal.hpp"

// The device array (one per GPU the library runs on).
static __device__ __align__(256) unsigned char scratch[TDCT_STATIC_TABLE_BYTES];

namespace tdct {
namespace {

constexpr size_t kStaticTableBytes = (size_t)TDCT_STATIC_TABLE_BYTES;

// Host-side staging of the tables, also the storage of the overlap check;
// static storage, used under g_mu. A copy from pageable host memory is
// performed synchronously, so the buffer is free again when the copy call
// returns.
alignas(256) unsigned char g_stage[kStaticTableBytes];
std::mutex g_mu;

// Per device: the array's device address and the compute units.
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices];
int g_num_cus[kMaxDevices];

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Looks the array up on the current device (once per device). g_mu held.
int device_setup(int* dev_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("static tables: device", e);
        return TDCT_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error_text("static tables: device index out of range");
        return TDCT_EDEVICE;
    }
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        int cus = 0;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess || !p || cus <= 0) {
            set_error("static tables: address of the device array", e);
            return TDCT_EDEVICE;
        }
        g_num_cus[dev] = cus;
        g_scratch_dev[dev] = p;
    }
    *dev_out = dev;
    return TDCT_OK;
}

}  // namespace
}  // namespace tdct

using namespace tdct;

extern "C" int tdct_batch_run_static(const tdct_image_desc* imgs, int32_t n,
                                     const tdct_qtable* qtabs, int32_t nq,
                                     const tdct_tune* tune_or_null, void* stream) {
    if (n < 0 || (n > 0 && !imgs) || nq < 0 || (nq > 0 && !qtabs)) return TDCT_EINVAL;
    tdct_tune tune;
    int st = normalise_tune(tune_or_null, &tune);
    if (st) return st;
    for (int32_t k = 0; k < nq; ++k)
        if ((st = validate_q(&qtabs[k]))) return st;
    for (int32_t i = 0; i < n; ++i)
        if ((st = validate_image(imgs[i], nq))) return st;
    if (n == 0) return TDCT_OK;
    // descriptors and constants alone (one of each per image) must fit
    const size_t desc_bytes = up256((size_t)n * sizeof(ImgDesc));
    const size_t qc_bytes = (size_t)n * sizeof(QConst);
    if (desc_bytes + qc_bytes > kStaticTableBytes || 3 * (size_t)n * sizeof(Span) > kStaticTableBytes) {
        set_error_text("static tables: more images than the device array holds");
        return TDCT_ENOMEM;
    }

    std::lock_guard<std::mutex> lk(g_mu);
    // the overlap check keeps its spans in the staging buffer
    Span* in = reinterpret_cast<Span*>(g_stage);
    if ((st = check_no_overlap(imgs, n, in, in + n))) return st;
    int dev = 0;
    if ((st = device_setup(&dev))) return st;

    // Layout: tiles | descriptors | constants, parts 256-byte aligned.
    ImgDesc* descs = reinterpret_cast<ImgDesc*>(g_stage);  // placed after the tiles below
    int ops = 0;
    // descriptors first at the start, to count the tiles (moved after them)
    for (int32_t i = 0; i < n; ++i) {
        const tdct_image_desc& im = imgs[i];
        fill_desc(im.op, im.src, im.src_stride, im.w, im.h, im.coef, im.dst, im.dst_stride, i,
                  im.op == TDCT_OP_ROUNDTRIP && im.coef != nullptr, &descs[i]);
        ops |= 1 << descs[i].op;
    }
    const int64_t ntiles = plan_tiles(descs, n, g_num_cus[dev], nullptr);
    const size_t tile_bytes = up256((size_t)ntiles * sizeof(Tile));
    const size_t total = tile_bytes + desc_bytes + qc_bytes;
    if (ntiles >= 0xffffffffll || total > kStaticTableBytes) {
        set_error_text("static tables: the batch's tables exceed the device array");
        return TDCT_ENOMEM;
    }
    // move the descriptors behind the tiles, then write tiles and constants
    memmove(g_stage + tile_bytes, g_stage, (size_t)n * sizeof(ImgDesc));
    descs = reinterpret_cast<ImgDesc*>(g_stage + tile_bytes);
    plan_tiles(descs, n, g_num_cus[dev], reinterpret_cast<Tile*>(g_stage));
    QConst* qcs = reinterpret_cast<QConst*>(g_stage + tile_bytes + desc_bytes);
    for (int32_t i = 0; i < n; ++i) {
        const tdct_image_desc& im = imgs[i];
        const int keep = (im.op == TDCT_OP_ENCODE || im.op == TDCT_OP_ROUNDTRIP) ? im.keep : 64;
        make_qconst(im.op == TDCT_OP_FORWARD ? nullptr : &qtabs[im.qtab], keep, &qcs[i]);
    }

    char* d = (char*)g_scratch_dev[dev];
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d, g_stage, total, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        set_error("static tables: upload", e);
        return TDCT_EDEVICE;
    }
    return launch_batch(reinterpret_cast<const Tile*>(d), reinterpret_cast<const ImgDesc*>(d + tile_bytes),
                        reinterpret_cast<const QConst*>(d + tile_bytes + desc_bytes), (uint32_t)ntiles, ops,
                        tune, g_num_cus[dev], s);
}
