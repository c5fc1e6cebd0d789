// Host-side interfaces shared by the plain calls, the batch planner and the
// server (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <string>

#include "tdct.h"
#include "tdct_device.hpp"

namespace tdct {

void set_error(const char* what, hipError_t e);
void set_error_text(const char* what);

// Diagnostics on stderr, one line each, by level: 1 errors (everything
// set_error records), 2 plans, autotuning, the autotune cache and server
// lifecycle, 3 every server batch. The level comes from $TDCT_LOG (0 when
// unset) or tdct_log_level.
int log_level();
void log_line(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
#define TDCT_LOG(level, ...)                                                       \
    do {                                                                           \
        if (::tdct::log_level() >= (level)) ::tdct::log_line((level), __VA_ARGS__); \
    } while (0)

// Runs the body of a C-ABI call: a host allocation failure (or any other C++
// exception) becomes a status code, so no exception crosses the ABI.
template <class F>
int abi_call(F&& body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        set_error_text("host memory allocation failed");
        return TDCT_ENOMEM;
    } catch (...) {
        set_error_text("unexpected host error");
        return TDCT_EDEVICE;
    }
}
int check_launch(const char* what);
int validate_plane(const void* p, int64_t stride, int32_t w, int32_t h);
int validate_q(const tdct_qtable* Q);
void make_qconst(const tdct_qtable* Q, int keep, QConst* out);
int image_flags(const ImgDesc& d);
int fill_desc(int op, const uint8_t* src, int64_t src_stride, int32_t w, int32_t h, void* coef,
              uint8_t* dst, int64_t dst_stride, int32_t qidx, bool write_coef, ImgDesc* d);
int launch_plain_op(int op, const ImgDesc& d, const QConst& qc, hipStream_t stream);
// Whether a launch whose work makes `full_tiles` tiles of the ops' own size
// (128 blocks for encoder-side ops, 64 for the decoder) should cut
// encoder-side work into 64-block tiles instead: true while there would be
// fewer tiles, hence waves, than the device has SIMDs (4 per CU). Each wave
// then does half the serial work (one block per lane) and twice as many
// SIMDs take part.
inline bool shrink_tiles(int64_t full_tiles, int num_cus) {
    return full_tiles < 4 * (int64_t)num_cus;
}
// A launch shape with zero fields replaced by the defaults (one wave per
// workgroup, a full grid, one tile per step); TDCT_EINVAL if a field is out
// of range. `in` may be null (all defaults).
int normalise_tune(const tdct_tune* in, tdct_tune* out);
// The image-uniform tiles of a batch of filled descriptors (64-block
// encoder-side tiles when shrink_tiles says so): returns their number and,
// when `out` is not null, writes them there.
int64_t plan_tiles(const ImgDesc* imgs, int32_t n, int num_cus, Tile* out);
// Checks of one batch image against the plan's nq Q tables (status code).
int validate_image(const tdct_image_desc& im, int32_t nq);
// Byte span [lo, hi) an image reads or writes.
struct Span {
    uintptr_t lo, hi;
};
// A batch is run more than once (graph replays, autotuning) or in one launch
// whose tiles run in any order, so no image may write bytes that any image
// reads: TDCT_EINVAL if an input span (plane rows from src to the end of the
// last row, or a decoder's coefficient run) meets an output span. `in` and
// `out` are caller storage for n and 2 n spans (no allocation here).
int check_no_overlap(const tdct_image_desc* imgs, int32_t n, Span* in, Span* out);
// ops: bit i set when op i occurs in the tiles (selects the kernel instance).
int launch_batch(const Tile* tiles, const ImgDesc* imgs, const QConst* qcs, uint32_t ntiles,
                 int ops, const tdct_tune& tune, int num_cus, hipStream_t stream);
// LDS bytes per workgroup of the batch kernel for an op set and launch shape.
uint32_t batch_lds_bytes(int ops, int waves_per_group);

// Autotune cache (tdct_tunecache.cpp): the device's architecture name
// (gfx950), whether every pixel plane of a batch is 128-byte aligned in
// address, width and stride, a batch's class key, and lookups and stores
// (no-ops while the cache is off).
int device_arch(std::string* out);
bool pixels_aligned(const ImgDesc* imgs, size_t n);
std::string tune_key(const std::string& arch, int ops, int64_t tiles, bool aligned);
bool tune_cache_get(const std::string& key, tdct_tune* out);
bool tune_cache_nearest(const std::string& arch, int ops, int64_t tiles, bool aligned, tdct_tune* out);
void tune_cache_put(const std::string& key, const tdct_tune& t);

struct ResidentArgs;
// Workgroups of the resident kernel that fit on the device at once.
int resident_capacity(int num_cus, int* groups);
// One front wave plus `workers` worker waves, after rewinding the ticket
// cursors when `rewind` (every launch but the first).
int launch_resident(const ResidentArgs& a, int workers, bool rewind, hipStream_t stream);

}  // namespace tdct
