// Memory layout shared by the resident serving kernel and its host side.
//
// The host publishes requests into a ring of jobs in host-coherent pinned
// memory and raises a published count; one front wave of the resident
// kernel polls that count over PCIe, copies each new job into device memory,
// cuts it into work items of one or more tiles (the same image-uniform
// tiles as the batch kernel) and publishes the items to the worker waves
// through a device-side item ring. Workers take items by ticket (a fetch-add
// on a device cursor), wait for their ticket's item to be published and code
// it; the wave that finishes a job's last item raises the job's done flag in
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
    uint64_t cursor;      // tickets handed out to workers (may run ahead of items_pub)
    uint32_t stop_epoch;  // epoch of the launch whose front wave has exited
    uint32_t pad[9];
};
static_assert(sizeof(ResidentState) == 64, "state is one 64-byte record");

struct ResidentArgs {
    const uint64_t* ctrl;     // host-coherent: published count | stop bit
    const ResidentJob* ring;  // host-coherent: ring_jobs slots, job j in slot j % ring_jobs
    uint32_t* done;           // host-coherent: done flag of each slot
    ResidentState* st;        // device
    uint32_t* remaining;      // device: tiles not yet finished, per slot
    ResidentJob* jobs;        // device: copies of the ring
    uint32_t* item_slot;      // device: item i belongs to the job in slot item_slot[i % ring_items]
    uint32_t ring_jobs;
    uint32_t ring_items;
    uint32_t epoch;           // distinct for every launch
    uint32_t workers;         // worker waves of the launch
    uint64_t idle_ticks;      // the front wave exits after this long without a new job
    uint64_t life_ticks;      // every wave exits after this long in any case
};

// Tiles per work item. While fewer items wait than there are workers, a job
// gets one-tile items until it has two tiles per worker (so every worker can
// take part and a small job finishes soon), and proportionally larger ones
// above that. Under a backlog every job gets 16-tile items: parallelism then
// comes from the queue, and the ticket counter, one atomic on one address
// per item, is touched 16 times less often.
constexpr uint32_t kMaxItemTiles = 16;
__host__ __device__ inline uint32_t item_tiles(uint32_t ntiles, uint32_t workers, bool backlog) {
    if (backlog) return ntiles < kMaxItemTiles ? (ntiles ? ntiles : 1) : kMaxItemTiles;
    const uint32_t c = ntiles / (2 * (workers ? workers : 1));
    return c < 1 ? 1 : (c > kMaxItemTiles ? kMaxItemTiles : c);
}

// Bytes of LDS one wave of the resident kernel uses: coefficient staging
// for the encoder and decoder, then its copy of the current job.
constexpr uint32_t kResidentStageBytes = 8192;
constexpr uint32_t kResidentLdsBytes = kResidentStageBytes + (uint32_t)sizeof(ResidentJob);

}  // namespace tdct
