// Memory layout shared by the resident serving kernel and its host side.
//
// The host publishes requests into a ring of jobs in host-coherent pinned
// memory and raises a published count; one front wave of the resident
// kernel polls that count over PCIe, copies each new job into device memory,
// cuts it into work items of one or more tiles (the same image-uniform
// tiles as the batch kernel) and publishes the items to the worker waves
// through a device-side item ring. Workers take items by ticket (a fetch-add
// on one of several device cursors: worker w draws from queue w mod nq, and
// ticket t of queue q is item t nq + q), wait for their ticket's item to be
// published and code it; the wave that finishes a job's last item raises the job's done flag in
// host-coherent memory, which the host polls. No HIP call is made per
// request.
#pragma once

#include <stdint.h>

#include "tdct_device.hpp"

namespace tdct {

// One request as the host writes it into the ring (and the device keeps it).
struct alignas(16) ResidentJob {
    ImgDesc d;           // qidx unused: the job carries its own constants
    QConst qc;
    uint64_t base;       // host: tiles published before the job; device copy: index
                         // of the job's first work item
    uint32_t ntiles;     // tiles of 128 (encoder ops) or 64 (decoder) blocks
    uint32_t done_value; // written to the job's done flag when it completes
    uint32_t item_tiles; // device copy: tiles per work item, chosen by the front wave
    uint32_t pad[3];
};
static_assert(sizeof(ResidentJob) % 16 == 0, "jobs are copied in 16-byte chunks");
constexpr int kJobChunks = (int)(sizeof(ResidentJob) / 16);
static_assert(kJobChunks <= 64, "one wave copies a job with one load per lane");

// The host's control word: requests published so far in the low 63 bits,
// bit 63 asks the kernel to exit.
constexpr uint64_t kCtrlStop = 1ull << 63;

// Device-side state; it outlives each launch of the kernel.
struct ResidentState {
    uint64_t taken;       // jobs copied in by the front wave (front wave only)
    uint64_t items_pub;   // work items published to the workers (front wave writes)
    uint32_t stop_epoch;  // epoch of the launch whose front wave has exited
    uint32_t pad[11];
};
static_assert(sizeof(ResidentState) == 64, "state is one 64-byte record");

// Ticket queues. One cursor on one address serialises every worker's
// fetch-add (about 0.1 us each on this part, device-wide): a job cut into
// thousands of items waited on that counter alone. Each queue's cursor has
// its own 256-byte line; cursor q counts the tickets of queue q handed out
// (it may run ahead of the items published).
constexpr uint32_t kMaxQueues = 32;
constexpr uint32_t kCursorStride = 32;  // uint64 words: 256 bytes
__host__ __device__ inline uint32_t resident_queues(uint32_t workers) {
    uint32_t q = 1;
    while (2 * q <= kMaxQueues && 2 * q <= workers) q *= 2;
    return q;
}

struct ResidentArgs {
    const uint64_t* ctrl;     // host-coherent: published count | stop bit
    const ResidentJob* ring;  // host-coherent: ring_jobs slots, job j in slot j % ring_jobs
    uint32_t* done;           // host-coherent: done flag of each slot
    ResidentState* st;        // device
    uint64_t* cursors;        // device: nq ticket cursors, kCursorStride words apart
    uint32_t* remaining;      // device: items not yet counted off, per queue and slot
                              // (remaining_at); then queues of the job not yet done, per
                              // slot (queues_left_at)
    ResidentJob* jobs;        // device: copies of the ring
    uint32_t* item_slot;      // device: item i belongs to the job in slot item_slot[i % ring_items]
    uint32_t ring_jobs;
    uint32_t ring_items;
    uint32_t epoch;           // distinct for every launch
    uint32_t workers;         // worker waves of the launch
    uint32_t nq;              // ticket queues (resident_queues(workers))
    uint32_t pad0;
    uint64_t idle_ticks;      // the front wave exits after this long without a new job
    uint64_t life_ticks;      // every wave exits after this long in any case
};

// Completion counters. A job's items are spread over the queues (item g is
// in queue g mod nq), and a worker only ever codes items of its own queue, so
// it counts them off on its queue's counter of the job; the worker that
// brings that counter to zero counts the queue off on the job's counter, and
// the one that brings that to zero completes the job. Each counter is
// touched by the workers of one queue (or by at most nq queues), not by every
// worker that coded part of a large job. Counters sit 64 bytes apart.
constexpr uint32_t kCounterStride = 16;  // uint32 words
__host__ __device__ inline uint64_t remaining_at(uint32_t q, uint32_t slot, uint32_t ring_jobs) {
    return ((uint64_t)q * ring_jobs + slot) * kCounterStride;
}
__host__ __device__ inline uint64_t queues_left_at(uint32_t slot, uint32_t ring_jobs) {
    return remaining_at(kMaxQueues, slot, ring_jobs);
}
__host__ __device__ inline uint64_t counter_words(uint32_t ring_jobs) {
    return queues_left_at(ring_jobs, ring_jobs);
}
// Items g in [first, first + n) with g mod nq == q (nq a power of two).
__host__ __device__ inline uint32_t items_in_queue(uint64_t first, uint32_t n, uint32_t q, uint32_t nq) {
    const uint32_t skip = (uint32_t)((q - (uint32_t)first) & (nq - 1));
    return skip >= n ? 0u : (n - 1 - skip) / nq + 1;
}

// Tiles per work item. While fewer items wait than there are workers, a job
// gets one-tile items until it has a tile per worker (so every worker can
// take part and a small job finishes soon), and about one item per worker
// above that: every item costs a ticket, and all workers taking their next
// ticket at once queue up on the cursors. Under a backlog every job gets
// 16-tile items: parallelism then comes from the queue, and the cursors are
// touched 16 times less often.
constexpr uint32_t kMaxItemTiles = 16;
__host__ __device__ inline uint32_t item_tiles(uint32_t ntiles, uint32_t workers, bool backlog) {
    if (backlog) return ntiles < kMaxItemTiles ? (ntiles ? ntiles : 1) : kMaxItemTiles;
    const uint32_t w = workers ? workers : 1;
    const uint32_t c = (ntiles + w - 1) / w;
    return c < 1 ? 1 : (c > kMaxItemTiles ? kMaxItemTiles : c);
}

// Bytes of LDS one wave of the resident kernel uses: coefficient staging
// for the encoder and decoder, then its copy of the current job.
constexpr uint32_t kResidentStageBytes = 8192;
constexpr uint32_t kResidentLdsBytes = kResidentStageBytes + (uint32_t)sizeof(ResidentJob);

}  // namespace tdct
