// Batch form: many images of uneven sizes in one persistent launch.
//
// Planning (host): the int64 prefix sum of blocks per image gives every
// image its global block range; each image is cut into wave-tiles (128
// blocks for encoder-side ops, 64 for the decoder) that never straddle two
// images, so everything a wave needs besides pixels -- the image descriptor
// and the quantiser constants -- is uniform across the wave and comes from
// scalar loads. The tables (tiles, descriptors, constants) live in one device
// allocation the plan owns. A run is one launch of the persistent kernel;
// the graph variant captures that launch once and replays it.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <new>
#include <utility>
#include <vector>

#include "tdct.h"
#include "tdct_internal.hpp"

using namespace tdct;

struct tdct_plan {
    std::vector<ImgDesc> imgs;
    std::vector<QConst> qcs;
    std::vector<Tile> tiles;
    std::vector<int64_t> blk_off;  // prefix sum of blocks, n + 1 entries
    void* dev = nullptr;
    size_t dev_bytes = 0;
    Tile* tiles_d = nullptr;
    ImgDesc* imgs_d = nullptr;
    QConst* qcs_d = nullptr;
    tdct_tune tune{};
    int ops = 0;  // bit i set when some image uses op i
    int num_cus = 0;
    int64_t pixels = 0;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t capture_stream = nullptr;
};

// One wave per workgroup and one tile per wave over a full grid: a small
// plan's waves land on as many CUs as there are waves, and on large plans
// the autotuner's pick is a full grid too.
static tdct_tune default_tune() {
    tdct_tune t{};
    t.waves_per_group = 1;
    t.groups_per_cu = 4096;
    t.tile_waves = 1;
    return t;
}

int tdct::normalise_tune(const tdct_tune* in, tdct_tune* out) {
    tdct_tune t = default_tune();
    if (in) {
        if (in->waves_per_group) t.waves_per_group = in->waves_per_group;
        if (in->groups_per_cu) t.groups_per_cu = in->groups_per_cu;
        if (in->tile_waves) t.tile_waves = in->tile_waves;
        t.xcd_remap = in->xcd_remap;
        t.pixel_cache = in->pixel_cache;
    }
    const int w = t.waves_per_group;
    if (!(w == 1 || w == 2 || w == 4 || w == 8)) return TDCT_EINVAL;
    if (t.groups_per_cu < 1 || t.groups_per_cu > 4096) return TDCT_EINVAL;
    if (!(t.tile_waves == 1 || t.tile_waves == 2 || t.tile_waves == 4)) return TDCT_EINVAL;
    if (t.xcd_remap != 0 && t.xcd_remap != 1) return TDCT_EINVAL;
    if (t.pixel_cache != 0 && t.pixel_cache != 1) return TDCT_EINVAL;
    *out = t;
    return TDCT_OK;
}

// Image-uniform tiles from each image's block range, 64-block encoder-side
// tiles when the batch is too small to fill the device.
int64_t tdct::plan_tiles(const ImgDesc* imgs, int32_t n, int num_cus, Tile* out) {
    int64_t full_tiles = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t tb = tile_blocks(imgs[i].op);
        full_tiles += (imgs[i].nblk + tb - 1) / tb;
    }
    const bool small = shrink_tiles(full_tiles, num_cus);
    int64_t k = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t nb = imgs[i].nblk;
        const int tb = small ? kDecTileBlocks : tile_blocks(imgs[i].op);
        if (!out) {
            k += (nb + tb - 1) / tb;
            continue;
        }
        for (int64_t f = 0; f < nb; f += tb, ++k) {
            Tile& t = out[k];
            t.img = (uint32_t)i;
            t.first_lo = (uint32_t)f;
            t.first_hi = (uint32_t)(f >> 32);
            t.count = (uint32_t)std::min<int64_t>(tb, nb - f);
        }
    }
    return k;
}

int tdct::validate_image(const tdct_image_desc& im, int32_t nq) {
    switch (im.op) {
        case TDCT_OP_ENCODE:
        case TDCT_OP_ROUNDTRIP:
            if (im.keep < 1 || im.keep > 64) return TDCT_EINVAL;
            break;
        case TDCT_OP_DECODE:
        case TDCT_OP_ENCODE_I8ZZ:
        case TDCT_OP_FORWARD:
            break;
        default:
            return TDCT_EINVAL;
    }
    if (im.op != TDCT_OP_FORWARD && (im.qtab < 0 || im.qtab >= nq)) return TDCT_EINVAL;
    int st;
    if (im.op != TDCT_OP_DECODE) {
        if ((st = validate_plane(im.src, im.src_stride, im.w, im.h))) return st;
    }
    if (im.op == TDCT_OP_DECODE || im.op == TDCT_OP_ROUNDTRIP) {
        if ((st = validate_plane(im.dst, im.dst_stride, im.w, im.h))) return st;
    } else if (im.w <= 0 || im.h <= 0 || (im.w & 7) || (im.h & 7)) {
        return TDCT_EDIM;
    }
    const bool need_coef = im.op != TDCT_OP_ROUNDTRIP;
    if (need_coef && !im.coef) return TDCT_EINVAL;
    if (im.coef && ((uintptr_t)im.coef % 16)) return TDCT_EINVAL;
    return TDCT_OK;
}

namespace {

Span plane_span(const void* p, int64_t stride, int32_t w, int32_t h) {
    const uintptr_t a = (uintptr_t)p;
    return {a, a + (uintptr_t)((int64_t)(h - 1) * stride + w)};
}

Span coef_span(const void* p, int64_t nblk, int64_t bytes_per_coef) {
    const uintptr_t a = (uintptr_t)p;
    return {a, a + (uintptr_t)(nblk * 64 * bytes_per_coef)};
}

}  // namespace

// Sorts the output spans by start and turns each end into the furthest end
// among the spans up to it; an input span [lo, hi) then meets an output span
// exactly when the last output starting before hi reaches past lo.
int tdct::check_no_overlap(const tdct_image_desc* imgs, int32_t n, Span* in, Span* out) {
    size_t nin = 0, nout = 0;
    for (int32_t i = 0; i < n; ++i) {
        const tdct_image_desc& im = imgs[i];
        const int64_t nblk = (int64_t)(im.w / 8) * (im.h / 8);
        switch (im.op) {
            case TDCT_OP_DECODE:
                in[nin++] = coef_span(im.coef, nblk, 2);
                out[nout++] = plane_span(im.dst, im.dst_stride, im.w, im.h);
                break;
            case TDCT_OP_ROUNDTRIP:
                in[nin++] = plane_span(im.src, im.src_stride, im.w, im.h);
                out[nout++] = plane_span(im.dst, im.dst_stride, im.w, im.h);
                if (im.coef) out[nout++] = coef_span(im.coef, nblk, 2);
                break;
            default:
                in[nin++] = plane_span(im.src, im.src_stride, im.w, im.h);
                out[nout++] = coef_span(im.coef, nblk,
                                        im.op == TDCT_OP_ENCODE ? 2 : im.op == TDCT_OP_FORWARD ? 4 : 1);
                break;
        }
    }
    std::sort(out, out + nout, [](const Span& a, const Span& b) { return a.lo < b.lo; });
    for (size_t k = 1; k < nout; ++k) out[k].hi = std::max(out[k].hi, out[k - 1].hi);
    for (size_t i = 0; i < nin; ++i) {
        const Span& s = in[i];
        const size_t k = (size_t)(std::lower_bound(out, out + nout, s.hi,
                                                   [](const Span& a, uintptr_t v) { return a.lo < v; }) -
                                  out);
        if (k && out[k - 1].hi > s.lo) return TDCT_EINVAL;
    }
    return TDCT_OK;
}

namespace {

void free_graph(tdct_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

int run(tdct_plan* p, hipStream_t s) {
    return launch_batch(p->tiles_d, p->imgs_d, p->qcs_d, (uint32_t)p->tiles.size(), p->ops,
                        p->tune, p->num_cus, s);
}

}  // namespace

extern "C" {

int tdct_batch_plan(const tdct_image_desc* imgs, int32_t n, const tdct_qtable* qtabs, int32_t nq,
                    const tdct_tune* tune_or_null, tdct_plan** out) {
    return abi_call([&]() -> int {
        if (!out || n < 0 || (n > 0 && !imgs) || nq < 0 || (nq > 0 && !qtabs)) return TDCT_EINVAL;
        *out = nullptr;
        tdct_tune tune;
        int st = normalise_tune(tune_or_null, &tune);
        if (st) return st;
        for (int32_t k = 0; k < nq; ++k)
            if ((st = validate_q(&qtabs[k]))) return st;
        for (int32_t i = 0; i < n; ++i)
            if ((st = validate_image(imgs[i], nq))) return st;
        {
            std::vector<Span> in((size_t)n), out(2 * (size_t)n);
            if ((st = check_no_overlap(imgs, n, in.data(), out.data()))) return st;
        }

        // freed with everything it holds on any early return
        std::unique_ptr<tdct_plan, void (*)(tdct_plan*)> p(new (std::nothrow) tdct_plan(),
                                                           tdct_plan_free);
        if (!p) return TDCT_ENOMEM;
        p->tune = tune;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) {
            set_error("device query", e);
            return TDCT_EDEVICE;
        }

        // Quantiser constants per distinct (table, keep) pair.
        std::map<std::pair<int, int>, int> qindex;
        p->imgs.resize(n);
        p->blk_off.assign((size_t)n + 1, 0);
        for (int32_t i = 0; i < n; ++i) {
            const tdct_image_desc& im = imgs[i];
            const int keep = (im.op == TDCT_OP_ENCODE || im.op == TDCT_OP_ROUNDTRIP) ? im.keep : 64;
            const int qt = im.op == TDCT_OP_FORWARD ? -1 : im.qtab;
            auto key = std::make_pair(qt, keep);
            auto it = qindex.find(key);
            int qi;
            if (it == qindex.end()) {
                qi = (int)p->qcs.size();
                QConst qc;
                make_qconst(qt >= 0 ? &qtabs[qt] : nullptr, keep, &qc);
                p->qcs.push_back(qc);
                qindex.emplace(key, qi);
            } else {
                qi = it->second;
            }
            fill_desc(im.op, im.src, im.src_stride, im.w, im.h, im.coef, im.dst, im.dst_stride, qi,
                      im.op == TDCT_OP_ROUNDTRIP && im.coef != nullptr, &p->imgs[i]);
            p->blk_off[i + 1] = p->blk_off[i] + p->imgs[i].nblk;
            p->ops |= 1 << p->imgs[i].op;
            p->pixels += (int64_t)im.w * im.h;
        }
        if (p->qcs.empty()) {
            QConst qc;
            make_qconst(nullptr, 64, &qc);
            p->qcs.push_back(qc);
        }
        const int64_t ntiles = plan_tiles(p->imgs.data(), n, p->num_cus, nullptr);
        if (ntiles >= 0xffffffffll) return TDCT_EINVAL;
        p->tiles.resize((size_t)ntiles);
        plan_tiles(p->imgs.data(), n, p->num_cus, p->tiles.data());
        // One device allocation: tiles | descriptors | constants (256-B aligned parts).
        auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
        const size_t tb = up(p->tiles.size() * sizeof(Tile) + 16);
        const size_t ib = up(p->imgs.size() * sizeof(ImgDesc) + 16);
        const size_t qb = up(p->qcs.size() * sizeof(QConst));
        p->dev_bytes = tb + ib + qb;
        e = hipMalloc(&p->dev, p->dev_bytes);
        if (e != hipSuccess) {
            p->dev = nullptr;
            set_error("plan tables", e);
            return TDCT_ENOMEM;
        }
        char* base = (char*)p->dev;
        p->tiles_d = (Tile*)base;
        p->imgs_d = (ImgDesc*)(base + tb);
        p->qcs_d = (QConst*)(base + tb + ib);
        e = hipMemcpy(p->tiles_d, p->tiles.data(), p->tiles.size() * sizeof(Tile),
                      hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->imgs_d, p->imgs.data(), p->imgs.size() * sizeof(ImgDesc),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->qcs_d, p->qcs.data(), p->qcs.size() * sizeof(QConst),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            set_error("plan upload", e);
            return TDCT_EDEVICE;
        }
        TDCT_LOG(2, "plan: %d images, %lld blocks, %zu tiles, ops 0x%x, %zu table bytes, shape %d/%d/%d/%d/%d",
                 n, (long long)(p->blk_off.empty() ? 0 : p->blk_off.back()), p->tiles.size(), p->ops,
                 p->dev_bytes, p->tune.waves_per_group, p->tune.groups_per_cu, p->tune.tile_waves,
                 p->tune.xcd_remap, p->tune.pixel_cache);
        *out = p.release();
        return TDCT_OK;
    });
}

int tdct_batch_run(tdct_plan* p, void* stream) {
    if (!p) return TDCT_EINVAL;
    return run(p, (hipStream_t)stream);
}

int tdct_batch_graph(tdct_plan* p, void* stream) {
    if (!p) return TDCT_EINVAL;
    if (p->tiles.empty()) return TDCT_OK;  // an empty plan launches nothing
    hipError_t e;
    if (!p->exec) {
        if (!p->capture_stream) {
            e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                set_error("capture stream", e);
                return TDCT_EDEVICE;
            }
        }
        e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            set_error("begin capture", e);
            return TDCT_EDEVICE;
        }
        int st = run(p, p->capture_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p->capture_stream, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) {
            set_error("end capture", e);
            return TDCT_EDEVICE;
        }
        p->graph = g;
        e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            set_error("graph instantiate", e);
            free_graph(p);
            return TDCT_EDEVICE;
        }
    }
    e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("graph launch", e);
        return TDCT_EDEVICE;
    }
    return TDCT_OK;
}

int tdct_autotune(tdct_plan* p, void* stream, int32_t reps, tdct_tune* best) {
    return abi_call([&]() -> int {
        if (!p || reps < 1) return TDCT_EINVAL;
        if (p->tiles.empty()) {  // nothing to time: the plan keeps its shape
            if (best) *best = p->tune;
            return TDCT_OK;
        }
        // a shape stored for the plan's class: applied without timing
        std::string arch, key;
        int st0 = device_arch(&arch);
        if (st0) return st0;
        key = tune_key(arch, p->ops, (int64_t)p->tiles.size(), pixels_aligned(p->imgs.data(), p->imgs.size()));
        tdct_tune cached;
        if (tune_cache_get(key, &cached)) {
            free_graph(p);  // a captured graph holds the launch shape it was made with
            p->tune = cached;
            if (best) *best = cached;
            TDCT_LOG(2, "autotune: %s: cached shape %d/%d/%d/%d/%d", key.c_str(), cached.waves_per_group,
                     cached.groups_per_cu, cached.tile_waves, cached.xcd_remap, cached.pixel_cache);
            return TDCT_OK;
        }
        hipStream_t s = (hipStream_t)stream;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return TDCT_EDEVICE;
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return TDCT_EDEVICE;
        }
        const tdct_tune saved = p->tune;
        // One launch in shape t, timed with events on the plan's stream.
        auto time_one = [&](const tdct_tune& t, float* ms) -> int {
            p->tune = t;
            hipError_t e = hipEventRecord(e0, s);
            int st = TDCT_OK;
            if (e == hipSuccess && (st = run(p, s))) return st;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
            if (e != hipSuccess) {
                set_error("autotune timing", e);
                return TDCT_EDEVICE;
            }
            return TDCT_OK;
        };
        auto median = [](std::vector<float> v) {
            std::sort(v.begin(), v.end());
            return v[v.size() / 2];
        };
        struct Cand {
            tdct_tune t;
            float ms;
        };
        std::vector<Cand> cands;
        std::vector<std::vector<float>> finals;
        size_t k = 0;
        tdct_tune winner = saved;
        float winner_ms = 0;
        int st = TDCT_OK;
        int rounds = 0;
        // Stage 1: every launch shape (persistent grids of 1..16 resident waves
        // per CU, and a full grid where every wave takes tile_waves tiles and
        // exits; tiles in launch order or one contiguous range per XCD;
        // streaming or cached pixel accesses), one warm-up and `reps` timed
        // launches each.
        const int wpgs[] = {1, 2, 4, 8};
        const int gpcs[] = {1, 2, 4, 8, 16, 4096};
        const int tws[] = {1, 2};
        for (int cached = 0; cached < 2; ++cached)
            for (int remap = 0; remap < 2; ++remap)
                for (int wpg : wpgs)
                    for (int gpc : gpcs)
                        for (int tw : tws) {
                            // at most 32 waves per CU are resident
                            if (gpc < 4096 && wpg * gpc > 32) continue;
                            if (batch_lds_bytes(p->ops, wpg) > 160 * 1024) continue;
                            tdct_tune t{};
                            t.waves_per_group = wpg;
                            t.groups_per_cu = gpc;
                            t.tile_waves = tw;
                            t.xcd_remap = remap;
                            t.pixel_cache = cached;
                            float m = 0;
                            if ((st = time_one(t, &m))) goto done;  // warm-up
                            std::vector<float> ms;
                            for (int r = 0; r < reps; ++r) {
                                if ((st = time_one(t, &m))) goto done;
                                ms.push_back(m);
                            }
                            cands.push_back({t, median(ms)});
                        }
        // Stage 2: the four fastest again, round-robin over several rounds, so
        // that a drift of the clocks between candidates cannot pick the winner.
        // Launch times scatter by a few per cent while the best shapes differ
        // by about as much, so the rounds fill about 0.2 s of launches (at
        // least max(5, reps), at most 25).
        std::sort(cands.begin(), cands.end(),
                  [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
        k = std::min<size_t>(4, cands.size());
        finals.assign(k, {});
        rounds = std::max(5, reps);
        if (k) {
            const double per_round_ms = (double)k * std::max(cands[0].ms, 1e-3f);
            rounds = std::max(rounds, std::min(25, (int)(200.0 / per_round_ms)));
        }
        for (int r = 0; r < rounds; ++r)
            for (size_t c = 0; c < k; ++c) {
                float m = 0;
                if ((st = time_one(cands[c].t, &m))) goto done;
                finals[c].push_back(m);
            }
        if (k) {
            size_t b = 0;
            for (size_t c = 1; c < k; ++c)
                if (median(finals[c]) < median(finals[b])) b = c;
            winner = cands[b].t;
            winner_ms = median(finals[b]);
        }
    done:
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st) {
            p->tune = saved;
            return st;
        }
        free_graph(p);  // a captured graph holds the launch shape it was made with
        p->tune = winner;
        if (best) *best = winner;
        TDCT_LOG(2, "autotune: %s: %zu shapes timed, kept %d/%d/%d/%d/%d (median %.4f ms over %d rounds)",
                 key.c_str(), cands.size(), winner.waves_per_group, winner.groups_per_cu, winner.tile_waves,
                 winner.xcd_remap, winner.pixel_cache, (double)winner_ms, rounds);
        tune_cache_put(key, winner);
        return TDCT_OK;
    });
}

int tdct_plan_info_get(const tdct_plan* p, tdct_plan_info* out) {
    if (!p || !out) return TDCT_EINVAL;
    out->images = (int64_t)p->imgs.size();
    out->blocks = p->blk_off.empty() ? 0 : p->blk_off.back();
    out->tiles = (int64_t)p->tiles.size();
    out->pixels = p->pixels;
    out->table_bytes = (int64_t)p->dev_bytes;
    out->tune = p->tune;
    return TDCT_OK;
}

void tdct_plan_free(tdct_plan* p) {
    if (!p) return;
    free_graph(p);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->dev) (void)hipFree(p->dev);
    delete p;
}

int tdct_run_per_image(const tdct_image_desc* imgs, int32_t n, const tdct_qtable* qtabs, int32_t nq,
                       void* stream) {
    if (n < 0 || (n > 0 && !imgs) || nq < 0 || (nq > 0 && !qtabs)) return TDCT_EINVAL;
    int st;
    for (int32_t k = 0; k < nq; ++k)
        if ((st = validate_q(&qtabs[k]))) return st;
    for (int32_t i = 0; i < n; ++i)
        if ((st = validate_image(imgs[i], nq))) return st;
    for (int32_t i = 0; i < n; ++i) {
        const tdct_image_desc& im = imgs[i];
        const int keep = (im.op == TDCT_OP_ENCODE || im.op == TDCT_OP_ROUNDTRIP) ? im.keep : 64;
        QConst qc;
        make_qconst(im.op == TDCT_OP_FORWARD ? nullptr : &qtabs[im.qtab], keep, &qc);
        ImgDesc d;
        fill_desc(im.op, im.src, im.src_stride, im.w, im.h, im.coef, im.dst, im.dst_stride, 0,
                  im.op == TDCT_OP_ROUNDTRIP && im.coef != nullptr, &d);
        if ((st = launch_plain_op(d.op, d, qc, (hipStream_t)stream))) return st;
    }
    return TDCT_OK;
}

}  // extern "C"
