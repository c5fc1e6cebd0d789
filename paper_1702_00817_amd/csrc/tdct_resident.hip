// Resident serving kernel: a grid that stays on the GPU and takes requests
// from a queue in host-coherent memory (layout and protocol in
// tdct_resident.hpp).
//
// Workgroup 0 is the front wave: it polls the host's published count, copies
// each new job into device memory, cuts it into work items of one or more
// tiles and fills the job's entries of the item ring; the items of up to 32
// jobs taken in one pass are then published behind one release. Every other
// workgroup is one worker wave: it takes a ticket for the next item, waits
// until that item is published, copies the item's job into its LDS (unless
// it already holds that job), runs the encoder or decoder tiles of the item
// (the per-wave tile code of the batch kernel) and counts the item off. A
// wave that keeps getting items of one job counts them off together, before
// it waits, changes job or holds 8. The wave that finishes a job's last item
// writes the job's done flag into host memory with a system-scope release.
//
// Every wave has an exit that it always reaches: the front wave leaves when
// the host sets the stop bit, after idle_ticks without a new job or after
// life_ticks; workers leave once the front wave has left and their ticket
// (below) is beyond the last published item, or after twice life_ticks. The
// host relaunches the kernel when work arrives and no launch is live; the
// state in device memory carries over between launches.
//
// Synchronisation uses only vector memory operations: scoped atomic loads,
// stores and fetch-adds, plus fences; polling loads are relaxed, so an idle
// wave issues no cache maintenance. Job data written inside the kernel is
// read with lane-indexed loads and kept in LDS.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tdct.h"
#include "tdct_device.hpp"
#include "tdct_internal.hpp"
#include "tdct_resident.hpp"
#include "tdct_tiles.hpp"

namespace tdct {
namespace {

__device__ __forceinline__ uint64_t first_lane64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t ticks() { return (uint64_t)wall_clock64(); }

// Back-off between polls: `n` sleeps of 16 x 64 clocks each.
__device__ __forceinline__ void nap(uint32_t n) {
    for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(16);
}

// Reads a trivially copyable record from LDS into wave-uniform registers.
template <class T>
__device__ __forceinline__ T uniform_copy(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized record");
    T out;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(p);
    uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return out;
}

// Control flow in the protocol code below is kept wave-uniform: every lane
// issues the same loads and stores (same address, one request), and atomics
// take a lane-0-only operand instead of sitting behind a lane test. A
// `lane == 0` branch around an atomic would let the compiler route the other
// lanes around it and back into a polling loop whose exit only lane 0
// decides.

// Jobs the front wave copies in before it publishes their items together.
constexpr uint32_t kIngestBatch = 32;

__device__ void front_wave(const ResidentArgs& a, uint32_t lane, uint64_t t0) {
    uint64_t taken = first_lane64(__hip_atomic_load(&a.st->taken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    uint64_t items = first_lane64(__hip_atomic_load(&a.st->items_pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint32_t jmask = a.ring_jobs - 1, imask = a.ring_items - 1;
    // lanes past the job's last 16-byte chunk all handle that chunk (same
    // value, same place)
    const uint32_t k = lane < (uint32_t)kJobChunks ? lane : (uint32_t)kJobChunks - 1;
    // chunk holding base (x, y), ntiles (z), done_value (w); then item_tiles (x)
    constexpr uint32_t kCountChunk = (uint32_t)(offsetof(ResidentJob, base) / 16);
    constexpr uint32_t kItemChunk = (uint32_t)(offsetof(ResidentJob, item_tiles) / 16);
    static_assert(offsetof(ResidentJob, base) % 16 == 0 && offsetof(ResidentJob, item_tiles) % 16 == 0,
                  "fields the front wave patches start their chunks");
    uint64_t last = t0;
    while (true) {
        // relaxed: an idle poll costs no cache maintenance
        const uint64_t ctrl = first_lane64(__hip_atomic_load(a.ctrl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
        const uint64_t now = ticks();
        if ((ctrl & kCtrlStop) || now - t0 > a.life_ticks) break;
        const uint64_t pub = ctrl & ~kCtrlStop;
        if (taken < pub) {
            // the host wrote these jobs before raising the count
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            const uint32_t n = pub - taken < kIngestBatch ? (uint32_t)(pub - taken) : kIngestBatch;
            // items published and not yet handed out (negative while workers
            // wait): the tickets of all queues, one cursor per lane, summed
            // across the wave
            const uint32_t cq = lane < a.nq ? lane : a.nq - 1;
            uint64_t mine = __hip_atomic_load(&a.cursors[cq * kCursorStride], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
            mine = lane < a.nq ? mine : 0;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)mine, off);
                const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(mine >> 32), off);
                mine += ((uint64_t)hi << 32) | lo;
            }
            const uint64_t handed = first_lane64(mine);
            for (uint32_t j = 0; j < n; ++j) {
                const uint32_t slot = (uint32_t)(taken + j) & jmask;
                v4u c = reinterpret_cast<const v4u*>(a.ring + slot)[k];
                const uint32_t ntiles = (uint32_t)__shfl((int)c.z, (int)kCountChunk);
                const bool backlog = (int64_t)(items - handed) > (int64_t)a.workers;
                const uint32_t per = item_tiles(ntiles, a.workers, backlog);
                uint32_t nitems = (ntiles + per - 1) / per;
                nitems = nitems > a.ring_items ? a.ring_items : nitems;
                c.x = k == kCountChunk ? (uint32_t)items : (k == kItemChunk ? per : c.x);
                c.y = k == kCountChunk ? (uint32_t)(items >> 32) : c.y;
                reinterpret_cast<v4u*>(a.jobs + slot)[k] = c;
                // lanes past the last queue repeat its store (same value, same place)
                const uint32_t q = lane < a.nq ? lane : a.nq - 1;
                a.remaining[remaining_at(q, slot, a.ring_jobs)] = items_in_queue(items, nitems, q, a.nq);
                a.remaining[queues_left_at(slot, a.ring_jobs)] = nitems < a.nq ? nitems : a.nq;
                for (uint32_t i = lane; i < nitems; i += 64) a.item_slot[(uint32_t)(items + i) & imask] = slot;
                items += nitems;
            }
            // the job copies, counts and item entries before the items
            // become visible
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            taken += n;
            __hip_atomic_store(&a.st->taken, taken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.st->items_pub, items, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = now;
            continue;
        }
        if (now - last > a.idle_ticks) break;
        nap(1);
    }
    __hip_atomic_store(&a.st->stop_epoch, a.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Codes tiles [tile0, tile1) of one image. A lone worker wave is bound by
// memory latency, so while it codes a tile it already loads the next one's
// inputs (the tile code calls the hook once the current inputs are
// consumed and before its stores).
template <int OP>
__device__ __forceinline__ void code_item(const ImgDesc& d, const QConst& qc, uint32_t tile0,
                                          uint32_t tile1, uint32_t tb, uint32_t lane, v4u* wl) {
    if (tile0 >= tile1) return;
    const uint32_t nblk = (uint32_t)d.nblk;
    uint32_t first = tile0 * tb, count = min(tb, nblk - first);
    if constexpr (OP == OP_ENCODE) {
        EncPixels P;
        enc_load<PX_COHERENT>(d, first, count, lane, P);
        for (uint32_t tile = tile0; tile < tile1; ++tile) {
            const bool more = tile + 1 < tile1;
            const uint32_t nfirst = first + tb;
            const uint32_t ncount = more ? min(tb, nblk - nfirst) : 0u;
            enc_tile<OP_ENCODE, PX_COHERENT>(d, qc, first, count, lane, wl, P, [&]() {
                if (more) enc_load<PX_COHERENT>(d, nfirst, ncount, lane, P);
            });
            first = nfirst;
            count = ncount;
        }
    } else {
        DecChunks C;
        dec_load<PX_COHERENT>(d, first, count, lane, C);
        for (uint32_t tile = tile0; tile < tile1; ++tile) {
            const bool more = tile + 1 < tile1;
            const uint32_t nfirst = first + tb;
            const uint32_t ncount = more ? min(tb, nblk - nfirst) : 0u;
            dec_tile<PX_COHERENT>(d, qc, first, count, lane, wl, C, [&]() {
                if (more) dec_load<PX_COHERENT>(d, nfirst, ncount, lane, C);
            });
            first = nfirst;
            count = ncount;
        }
    }
}

// 1 once item t is published, 2 when the wave should leave holding t;
// `pub` receives the published count seen.
__device__ __forceinline__ uint32_t ticket_state(const ResidentArgs& a, uint64_t t, uint64_t t0, uint64_t& pub) {
    pub = first_lane64(__hip_atomic_load(&a.st->items_pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (pub > t) return 1;
    const uint32_t stop = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&a.st->stop_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (stop != a.epoch && ticks() - t0 <= 2 * a.life_ticks) return 0;
    // the front wave's last publication precedes its exit
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    pub = first_lane64(__hip_atomic_load(&a.st->items_pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    return pub > t ? 1 : 2;
}

// Waits until this wave's memory operations have completed; the compiler
// keeps memory accesses on their side of this point.
__device__ __forceinline__ void wait_stores() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0) expcnt(0) lgkmcnt(0)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Items a wave may code before it counts them off (while they belong to the
// same job and the next item is already published).
constexpr uint32_t kMaxPendingItems = 8;

__device__ void worker_wave(const ResidentArgs& a, uint32_t worker, uint32_t lane, uint64_t t0, v4u* wl,
                            v4u* jl) {
    const uint32_t imask = a.ring_items - 1;
    const uint32_t queue = worker & (a.nq - 1);
    uint64_t* const cursor = &a.cursors[queue * kCursorStride];
    const uint32_t k = lane < (uint32_t)kJobChunks ? lane : (uint32_t)kJobChunks - 1;
    // Items coded and not yet counted off, all of the job in pend_slot.
    uint32_t pend_slot = 0, pend_items = 0, pend_done = 0;
    auto count_off = [&]() {
        if (pend_items == 0) return;
        // The tile code wrote this wave's outputs through L2 (PX_COHERENT):
        // once the stores have completed they are visible device-wide and to
        // copy engines, so the count needs no L2 write-back, only the wait.
        wait_stores();
        const uint32_t left = __builtin_amdgcn_readfirstlane(__hip_atomic_fetch_add(
            &a.remaining[remaining_at(queue, pend_slot, a.ring_jobs)], lane == 0 ? 0u - pend_items : 0u,
            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        // the job's items of this queue are all coded: count the queue off
        const uint32_t queues = left != pend_items
                                    ? 0u
                                    : __builtin_amdgcn_readfirstlane(__hip_atomic_fetch_add(
                                          &a.remaining[queues_left_at(pend_slot, a.ring_jobs)],
                                          lane == 0 ? 0xffffffffu : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (queues == 1) {
            // Every other wave of the job completed its stores before its
            // count, and this count came after theirs: the job's outputs are
            // all in memory. The flag itself goes straight to host memory.
            wait_stores();
            __hip_atomic_store(&a.done[pend_slot], pend_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        pend_items = 0;
    };
    // The job held in LDS covers items [cur_base, cur_end); item indices are
    // unique, so a ticket in that range is another item of the same job.
    uint64_t cur_base = 0, cur_end = 0;
    ImgDesc d{};
    uint32_t ntiles = 0, per = 1, tb = kEncTileBlocks, done_value = 0, slot = 0;
    const ResidentJob* J = reinterpret_cast<const ResidentJob*>(jl);
    while (true) {
        // A ticket of this wave's queue names the next work item it codes
        // (ticket k of queue q is item k nq + q); taking one always succeeds,
        // and the wave then waits for that item to be published. A wave that
        // leaves holding an unpublished ticket loses it: before a relaunch
        // each cursor is rewound to its queue's first unpublished item.
        const uint64_t t = first_lane64(__hip_atomic_fetch_add(cursor, lane == 0 ? 1ull : 0ull, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT)) *
                               a.nq +
                           queue;
        uint64_t pub;
        uint32_t state = ticket_state(a, t, t0, pub);
        if (state != 1) {
            count_off();  // nothing else to do meanwhile
            uint32_t backoff = 1;
            while (state == 0) {
                // the next waves in the queue poll often; waves far down it
                // less
                const uint64_t ahead = t - pub;
                const uint32_t cap = ahead < 32 ? 2u : 8u;
                const uint32_t far = ahead > 32 * 32 ? 32u : (uint32_t)(ahead / 32);
                nap(backoff > far ? backoff : far);
                backoff = backoff < cap ? 2 * backoff : cap;
                state = ticket_state(a, t, t0, pub);
            }
            if (state == 2) break;
        }
        if (t < cur_base || t >= cur_end) {
            // A new job: item t's entry, the job copy and count were released
            // before the publication that covered t, and the job's inputs
            // were written before it was queued. All of them are read with
            // coherent loads (the entry and the job copy here, the inputs in
            // the tile code), which see memory as it is now even where this
            // XCD's L2 holds an older copy, so no acquire (an invalidate of
            // the whole L2) is needed per job.
            count_off();
            slot = __builtin_amdgcn_readfirstlane(__hip_atomic_load(&a.item_slot[(uint32_t)t & imask],
                                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) &
                   (a.ring_jobs - 1);
            jl[k] = ld_wt4(a.jobs + slot, 16u * k, (uint32_t)sizeof(ResidentJob));
            lds_fence();
            // the job's pointers came through LDS
            d = global_desc(uniform_copy(&J->d));
            cur_base = first_lane64(J->base);
            ntiles = __builtin_amdgcn_readfirstlane(J->ntiles);
            done_value = __builtin_amdgcn_readfirstlane(J->done_value);
            per = __builtin_amdgcn_readfirstlane(J->item_tiles);
            per = per ? per : 1;
            cur_end = cur_base + (ntiles + per - 1) / per;
            tb = (uint32_t)tile_blocks(d.op);
        }
        const uint64_t tmax = ((uint64_t)d.nblk + tb - 1) / tb;
        const uint32_t tile0 = (uint32_t)min((t - cur_base) * per, tmax);
        const uint32_t tile1 = (uint32_t)min((uint64_t)tile0 + per, min((uint64_t)ntiles, tmax));
        if (d.op == OP_ENCODE)
            code_item<OP_ENCODE>(d, J->qc, tile0, tile1, tb, lane, wl);
        else if (d.op == OP_DECODE)
            code_item<OP_DECODE>(d, J->qc, tile0, tile1, tb, lane, wl);
        pend_slot = slot;
        pend_done = done_value;
        if (++pend_items >= kMaxPendingItems) count_off();
    }
    count_off();
}

__global__ __launch_bounds__(64) void resident_kernel(const ResidentArgs a) {
    extern __shared__ v4u lds[];
    const uint32_t lane = threadIdx.x;
    const uint64_t t0 = ticks();
    if (blockIdx.x == 0)
        front_wave(a, lane, t0);
    else
        worker_wave(a, blockIdx.x - 1, lane, t0, lds, lds + kResidentStageBytes / 16);
}

// Before a relaunch, on the kernel's stream (so after the previous launch
// has ended): each queue's cursor goes back to its first item not yet
// published (tickets the exiting workers took beyond the published items
// were lost), or stays if it is behind that.
__global__ void resident_rewind(const ResidentArgs a) {
    const uint32_t q = threadIdx.x;
    if (q >= a.nq) return;
    const uint64_t pub = a.st->items_pub;
    const uint64_t first = pub > q ? (pub - q + a.nq - 1) / a.nq : 0;
    uint64_t* c = &a.cursors[q * kCursorStride];
    *c = *c < first ? *c : first;
}

}  // namespace

// Workgroups of the resident kernel that fit on the device at once.
int resident_capacity(int num_cus, int* groups) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, resident_kernel, 64,
                                                                kResidentLdsBytes);
    if (e != hipSuccess) {
        set_error("resident kernel occupancy", e);
        return TDCT_EDEVICE;
    }
    *groups = per_cu * num_cus;
    return TDCT_OK;
}

int launch_resident(const ResidentArgs& a, int workers, bool rewind, hipStream_t stream) {
    if (rewind) {
        hipLaunchKernelGGL(resident_rewind, dim3(1), dim3(64), 0, stream, a);
        const int st = check_launch("resident cursor rewind");
        if (st) return st;
    }
    hipLaunchKernelGGL(resident_kernel, dim3(1 + workers), dim3(64), kResidentLdsBytes, stream, a);
    return check_launch("resident kernel launch");
}

}  // namespace tdct
