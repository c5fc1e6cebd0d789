/*
 * tdct: an MI355X (gfx950) block codec built on the 8-point approximate DCT
 * of Bayer and Cintra, "DCT-like Transform for Image Compression Requires 14
 * Additions Only".
 *
 * The transform (Section 2) is the 8x8 matrix T with entries in {0, +1, -1};
 * its fast algorithm needs 14 additions, no multiplications and no shifts
 * (Section 2, Table 1). Images are split into 8x8 blocks that are transformed
 * along rows and columns (Section 3). This library runs that 2-D transform as
 * an integer codec on row-major uint8 planes:
 *
 *   encode  X = block - 128, Y = T X T^t,
 *           W_ij = Y_ij * 2^(6 - a_i - a_j)      (a = 3,1,2,1,3,1,2,1: the
 *                                                 diagonal D of Section 2
 *                                                 enters only as D^2, merged
 *                                                 into quantisation),
 *           q_ij = round-half-away(W_ij / Q_ij),
 *           q_ij = 0 where the zigzag rank of (i, j) is >= keep (zonal
 *           coding of Section 3);
 *   decode  W'_ij = q_ij Q_ij,  S = T^t W' T,
 *           pixel = clamp(floor((S + 32) / 64) + 128, 0, 255)
 *           (the inverse transform of Section 3 with the scale 64 removed).
 *
 * Everything is integer and exact: one correct output exists for any input.
 *
 * Conventions for every entry point:
 *  - Data pointers are DEVICE pointers owned by the caller; the plain calls
 *    allocate nothing.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *    stream) and return once the work is enqueued.
 *  - Errors are returned as tdct_status codes; no exception crosses the ABI.
 *    TDCT_EDEVICE means a HIP runtime call failed; tdct_last_error() then
 *    returns its text for the calling thread. A call that runs out of host
 *    memory returns TDCT_ENOMEM (and leaves nothing half-built).
 *  - Planes: w and h are positive multiples of 8 (TDCT_EDIM otherwise),
 *    at most 65536 each, the row stride in bytes is >= w. Any pixel pointer
 *    and stride are accepted; 8- and 16-byte aligned ones take faster loads.
 *  - Coefficients: block b = by * (w / 8) + bx (raster order) holds its 64
 *    coefficients contiguously at [b * 64 + 8 i + j], i = vertical and
 *    j = horizontal frequency (int16 or int32), or at [b * 64 + rank] in
 *    zigzag order (int8). Coefficient pointers must be 16-byte aligned
 *    (TDCT_EINVAL otherwise).
 *  - Quantisation tables hold Q_ij in natural (i, j) order, each in
 *    [1, 4095] (TDCT_EQTAB otherwise); this range keeps every intermediate of
 *    the decoder inside int32 for any int16 input.
 *  - Plain calls are reentrant; plans and servers are used from one thread
 *    at a time unless stated.
 */
#ifndef TDCT_H
#define TDCT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TDCT_OK = 0,
    TDCT_EINVAL = -1,    /* null pointer, stride < w, misaligned coefficients, bad keep/op */
    TDCT_EDIM = -2,      /* w or h not a positive multiple of 8, or above 65536 */
    TDCT_EQTAB = -3,     /* a Q entry outside [1, 4095] */
    TDCT_ENOMEM = -4,    /* device or host allocation failed, or a request larger than the budget */
    TDCT_EDEVICE = -5,   /* a HIP runtime call failed (see tdct_last_error) */
    TDCT_EBUSY = -6,     /* result not ready yet, or the server is shutting down */
    TDCT_ENOTFOUND = -7  /* unknown or already released ticket */
} tdct_status;

#define TDCT_QMAX 4095
#define TDCT_MAX_SIDE 65536

typedef struct {
    uint16_t q[64]; /* Q_ij at [8 i + j] */
} tdct_qtable;

/* ---- plain calls: one image ------------------------------------------ */

/* Forward transform only (Section 3's 2-D block transform of T, Section 2):
 * coef[b*64 + 8i + j] = Y_ij = (T (X - 128) T^t)_ij, int32, unscaled. */
int tdct_forward(const uint8_t* src, int64_t src_stride, int32_t w, int32_t h, int32_t* coef,
                 void* stream);

/* Fused forward + quantise (encode): q[b*64 + 8i + j] = q_ij as defined
 * above, with zonal retention of the first `keep` zigzag coefficients
 * (1..64; 64 keeps all). */
int tdct_quantise(const uint8_t* src, int64_t src_stride, int32_t w, int32_t h,
                  const tdct_qtable* Q, int32_t keep, int16_t* q, void* stream);

/* Fused dequantise + inverse (decode) of any int16 coefficients into a
 * uint8 plane (dst rows of w bytes at dst_stride). */
int tdct_inverse(const int16_t* q, const tdct_qtable* Q, int32_t w, int32_t h, uint8_t* dst,
                 int64_t dst_stride, void* stream);

/* Encode then decode in one pass: dst = decode(encode(src)). The
 * coefficients are also written to q_or_null unless it is NULL (then they
 * never leave the registers). src and dst may be the same plane. */
int tdct_roundtrip(const uint8_t* src, int64_t src_stride, int32_t w, int32_t h,
                   const tdct_qtable* Q, int32_t keep, int16_t* q_or_null, uint8_t* dst,
                   int64_t dst_stride, void* stream);

/* Encode with int8 saturation (clamp to [-128, 127] after rounding), stored
 * in zigzag order: out[b*64 + rank] (64 bytes per block, no zonal mask). */
int tdct_quantise_i8_zigzag(const uint8_t* src, int64_t src_stride, int32_t w, int32_t h,
                            const tdct_qtable* Q, int8_t* out, void* stream);

/* Sum of squared differences of two uint8 planes (for PSNR / MSE, the
 * figures of merit of Section 3), exact, written to *sse_dev (a device
 * uint64). */
int tdct_sse(const uint8_t* a, int64_t a_stride, const uint8_t* b, int64_t b_stride, int32_t w,
             int32_t h, uint64_t* sse_dev, void* stream);

/* Diagnostics: the HBM ceilings the codec kernels are measured against.
 * One launch streams `units` 16-byte units with the access mix of `kind`
 * and no arithmetic, non-temporal like the codec:
 *   COPY  src[units] -> dst[units]          (2 x 16 B per unit)
 *   READ  src[units], dst receives 16 B     (16 B per unit)
 *   WRITE dst[units]                        (16 B per unit)
 *   R1W2  src[units] -> dst[u] and dst[units + u] (48 B per unit; the encoder's 1:2 mix)
 *   R2W1  src[u] and src[units + u] -> dst[units] (48 B per unit; the decoder's 2:1 mix)
 *   R1W3  src[units] -> dst[u], dst[units + u], dst[2 units + u] (64 B per unit; the
 *         1:3 mix of a round trip that writes coefficients: 1 B in, 2 + 1 B out per pixel)
 * COPY at 1:1 is also the mix of the int8 zigzag encoder (1 B in, 1 B out per sample).
 * Device pointers, 16-byte aligned, sized as above. */
enum { TDCT_PROBE_COPY = 0, TDCT_PROBE_READ = 1, TDCT_PROBE_WRITE = 2, TDCT_PROBE_R1W2 = 3,
       TDCT_PROBE_R2W1 = 4, TDCT_PROBE_R1W3 = 5 };
int tdct_stream_probe(int32_t kind, const void* src, void* dst, int64_t units, void* stream);

const char* tdct_strerror(int status);
const char* tdct_last_error(void);
/* Diagnostics on stderr, one line per event, prefixed "[tdct <level>]":
 * 1 errors (every failure tdct_last_error reports), 2 plans, autotune
 * outcomes, the autotune cache and server lifecycle (create, resident
 * launches, final statistics at destroy), 3 every server batch. The level
 * starts at $TDCT_LOG (0, silent, when unset). Sets the level when
 * level >= 0 (above 3 means 3) and returns the previous one; a negative
 * argument only queries. */
int tdct_log_level(int level);

/* ---- batch form: many images of uneven sizes in one persistent launch -- */

enum {
    TDCT_OP_ENCODE = 0,      /* src -> int16 coef */
    TDCT_OP_DECODE = 1,      /* int16 coef -> dst */
    TDCT_OP_ROUNDTRIP = 2,   /* src -> dst, int16 coef too if coef != NULL */
    TDCT_OP_ENCODE_I8ZZ = 3, /* src -> int8 zigzag coef */
    TDCT_OP_FORWARD = 4      /* src -> int32 Y */
};

typedef struct {
    int32_t op;   /* TDCT_OP_* */
    int32_t w, h; /* positive multiples of 8 */
    int32_t qtab; /* index into the plan's Q tables (ignored by FORWARD) */
    int32_t keep; /* 1..64 (ENCODE, ROUNDTRIP); ignored otherwise */
    int32_t reserved;
    const uint8_t* src;
    int64_t src_stride;
    void* coef; /* device, 16-byte aligned; element type per op */
    uint8_t* dst;
    int64_t dst_stride;
} tdct_image_desc;

/* Launch shape of the persistent kernel. Zero fields take the defaults:
 * one wave per workgroup, a full grid (groups_per_cu 4096: the grid is
 * capped at one wave per tile step), one tile per step, no XCD remap,
 * streaming pixel accesses. */
typedef struct {
    int32_t waves_per_group; /* 1, 2, 4 or 8 (64-lane waves per workgroup) */
    int32_t groups_per_cu;   /* workgroups per compute unit; grid = CUs * this, capped at the
                                workgroups needed for one tile step per wave */
    int32_t tile_waves;      /* consecutive wave-tiles one wave takes per step (1, 2, 4) */
    int32_t xcd_remap;       /* 0 or 1: workgroup b runs on XCD b mod 8; with 1, the
                                workgroups of each XCD take one contiguous range of tiles */
    int32_t pixel_cache;     /* 0 or 1: pixel-plane loads and stores are non-temporal (0) or
                                ordinary cached accesses (1); coefficients always stream.
                                Only speed differs, never the output */
} tdct_tune;

typedef struct {
    int64_t images;
    int64_t blocks;
    int64_t tiles;
    int64_t pixels;
    int64_t table_bytes; /* device bytes held by the plan's tables */
    tdct_tune tune;      /* launch shape in use */
} tdct_plan_info;

typedef struct tdct_plan tdct_plan;

/* Build a plan: validates every image, computes the int64 prefix sum of
 * blocks per image and the image-uniform tile list, and uploads both with
 * the per-table quantiser constants to device tables the plan owns.
 * Image descriptors and tables are copied; device buffers they name must
 * stay valid while the plan is run. A plan may run many times (graph
 * replays, the autotuner's candidates), so no image may write bytes that
 * any image of the plan reads: TDCT_EINVAL if the span an image reads (its
 * plane rows from src to the last row's end, or a decoder's coefficient run)
 * meets the span any image writes (an in-place round trip, or a decode of
 * coefficients another image of the plan encodes). */
int tdct_batch_plan(const tdct_image_desc* imgs, int32_t n, const tdct_qtable* qtabs,
                    int32_t nq, const tdct_tune* tune_or_null, tdct_plan** out);

/* One persistent launch over every tile of the plan on `stream` (a plan of
 * no images launches nothing; run, graph and autotune return TDCT_OK). */
int tdct_batch_run(tdct_plan* plan, void* stream);

/* Same work as tdct_batch_run, through a hipGraph captured on the first
 * call (on `stream`) and replayed afterwards. */
int tdct_batch_graph(tdct_plan* plan, void* stream);

/* Times candidate launch shapes on the plan (reps launches each, after one
 * warm-up), then times the four fastest again in turn over max(5, reps)
 * rounds or more (up to 25, about 0.2 s of launches), keeps the one with the
 * lowest median in the plan and returns it in *best. With the autotune cache
 * on (below), a shape stored for the plan's class is applied instead, with no
 * launch, and a newly timed winner is stored. Outputs are overwritten
 * with the same bytes by every candidate (a plan's outputs never overlap its
 * inputs, see tdct_batch_plan). */
int tdct_autotune(tdct_plan* plan, void* stream, int32_t reps, tdct_tune* best);

/* Autotune cache (process-wide). tdct_tune_cache_open(path) loads the JSON
 * file at `path` (a missing file is an empty cache; NULL or "" turns the
 * cache off; TDCT_EINVAL, cache off, for a file not in the cache's format)
 * and replaces the environment's choice: without a call, the first use of the
 * cache opens the file named by $TDCT_TUNE_CACHE, if set. While the cache is
 * on, tdct_autotune first looks up the plan's class -- device architecture,
 * the library's source hash, op set, size class floor(log2(tiles)) and
 * whether every pixel plane's
 * address, width and stride are multiples of 128 bytes -- and on a hit applies
 * the stored shape without timing anything; on a miss it times candidates as
 * below and stores the winner, rewriting the file (through a temporary file
 * and a rename; entries other processes stored in the file meanwhile are
 * kept, this process's winning on the same class). Servers created with tune_cache = 1 launch each batch in the
 * shape stored for its class, or for the nearest size class within a factor
 * of 4 (tdct_server_cfg). The file holds one object:
 * {"format": "tdct-autotune-1", "entries": {"gfx950/src=<hash>/ops=1/tiles=17/aligned=1":
 * [waves_per_group, groups_per_cu, tile_waves, xcd_remap, pixel_cache], ...}}.
 * Write failures leave the file as it was and are counted. */
typedef struct {
    int32_t on;       /* 1 while a cache file is open */
    int32_t reserved;
    int64_t entries;  /* classes held */
    int64_t hits, misses, stores, write_errors; /* tdct_autotune, since the cache was opened */
    int64_t batch_hits, batch_misses;          /* server batch launches (tune_cache = 1) */
} tdct_tune_cache_stats;
int tdct_tune_cache_open(const char* path);
int tdct_tune_cache_info(tdct_tune_cache_stats* out);

int tdct_plan_info_get(const tdct_plan* plan, tdct_plan_info* out);
void tdct_plan_free(tdct_plan* plan);

/* Per-image launches of the same work (one plain call per image in order,
 * on `stream`), the baseline the batch form is compared with. */
int tdct_run_per_image(const tdct_image_desc* imgs, int32_t n, const tdct_qtable* qtabs,
                       int32_t nq, void* stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the work
 * of tdct_batch_plan + tdct_batch_run in one call, with no plan object and
 * no allocation. The tables go into a fixed device array of
 * TDCT_STATIC_TABLE_BYTES (16 MiB) that the library holds on each GPU it
 * runs on until the process ends: 16 B per tile (128 blocks of encoder-side
 * work, 64 of decoder or int32-forward work) plus 64 + 768 B per image, each
 * part rounded up to 256 B. Tables that do not fit return TDCT_ENOMEM before
 * any device work: about 19,000 images, or 8.6 Gpx of encoding in one call.
 * Arguments, checks and other errors as for tdct_batch_plan. The tables are
 * built in host memory of static storage and copied from there, which HIP
 * performs synchronously with respect to the host; then the kernel is queued
 * on `stream`. Every call on one GPU shares that GPU's array: calls on one
 * stream are ordered, but calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller. Not for stream
 * capture: the table copy reads the library's static host buffer, which the
 * next call overwrites, so a captured graph could replay another call's
 * tables. */
#define TDCT_STATIC_TABLE_BYTES (16 << 20)
int tdct_batch_run_static(const tdct_image_desc* imgs, int32_t n, const tdct_qtable* qtabs,
                          int32_t nq, const tdct_tune* tune_or_null, void* stream);

/* ---- serving form ------------------------------------------------------ */

typedef struct {
    int64_t budget_bytes;  /* device arena for request outputs (admission limit) */
    int32_t streams;       /* batches that may be in flight at once (1..16) */
    int32_t max_batch;     /* requests per batch, at most */
    int32_t max_wait_us;   /* a batch launches when a stream is free and either the
                              queue holds max_batch requests or the oldest waited this long.
                              0: no window; a free stream then takes its share of the
                              admitted requests, ceil(admitted / streams) up to max_batch,
                              so requests the free streams can take one by one launch
                              alone and batches form under a backlog */
    int32_t batching;      /* 1 = continuous batching into the persistent kernel;
                              0 = one plain launch per request (comparison mode) */
    int64_t max_batch_px;  /* a batch stops growing once it holds this many pixels, so
                              small requests do not wait for a huge one (0 = no cap) */
    tdct_tune tune;        /* launch shape of batch launches (zero fields: one wave per
                              workgroup, one tile per wave; out of range: TDCT_EINVAL) */
    int32_t fake_device_us; /* > 0: no GPU at all -- outputs live in host memory and a
                               batch "completes" this many microseconds after launch
                               (exercises admission and batching on a CPU) */
    int32_t fake_fail_every; /* fake device only: n > 0: every n-th batch fails when it
                                completes; n < 0: every |n|-th batch fails partway through
                                its launch, after its work was queued (0 = never). A batch
                                whose launch fails gives its memory back only once the work
                                it queued has drained */
    /* Resident mode (resident = 1): no launch per batch. Requests go into a
     * queue in host-coherent pinned memory that a resident kernel polls; its
     * front wave copies each request to the device and cuts it into work
     * items of one or more tiles, its worker waves take items from a
     * device-side ring and code them, and the wave that finishes a request's
     * last item raises the request's done flag in host memory, which the
     * scheduler polls. Submitting a request publishes it at once from the
     * submitting thread. The kernel exits after resident_idle_us without a
     * new request (and after one second in any case) and is relaunched by
     * the next one; while requests are live, the next launch is queued behind
     * the running one before its second ends. streams, max_batch,
     * max_wait_us, batching, max_batch_px and tune are unused; host_io
     * requests are refused (TDCT_EINVAL). With fake_device_us > 0 a host
     * thread plays the kernel's part of the protocol. */
    int32_t resident;
    int32_t resident_workers; /* worker waves (0: four per compute unit; clamped to what
                                 fits on the device at once) */
    int32_t resident_idle_us; /* 0: 20000 */
    int32_t resident_jobs;    /* queue slots, rounded up to a power of two (0: 1024,
                                 at most 65536); a request holds its slot until done */
    int32_t resident_tiles;   /* work-item ring slots, rounded up to a power of two
                                 (0: 2^21, at most 2^24); a request with more tiles
                                 than this (blocks / 128 encoding, blocks / 64
                                 decoding; an item holds one or more tiles) is
                                 refused with TDCT_ENOMEM */
    int32_t resident_reserved;
    int32_t tune_cache;       /* 1: each batch launch takes the autotune cache's shape for
                                 its class (nearest size class within a factor of 4), when
                                 the cache holds one; otherwise `tune` */
    int32_t idle_poll_us;     /* the scheduler polls (completions, arrivals) this long after the
                                 last activity before it sleeps until the next submit (0: 2000;
                                 at most 10^7). A request submitted to a sleeping scheduler is
                                 launched by the submitting thread at once, but its completion
                                 is seen only once the scheduler's thread has woken: polling
                                 longer spends a host core to keep that wake-up out of the
                                 latency at low request rates */
} tdct_server_cfg;

typedef struct {
    int32_t op;      /* TDCT_OP_ENCODE or TDCT_OP_DECODE */
    int32_t w, h;
    int32_t keep;    /* ENCODE only */
    const void* input; /* uint8 plane (ENCODE) or int16 coefficients (DECODE); device memory,
                          or pinned host memory when host_io */
    int64_t in_stride; /* ENCODE: bytes per row */
    tdct_qtable Q;
    int32_t host_io;   /* 0: device-resident input, output left in the arena.
                          1: the input is copied host -> device into the arena and the output
                          device -> host into host_output, on the request's stream, before the
                          request completes (the arena holds both copies meanwhile) */
    int32_t reserved;
    void* host_output; /* host_io: pinned host buffer of the output's size */
} tdct_request;

typedef struct {
    int32_t status;       /* TDCT_OK done, TDCT_EBUSY pending, < 0 failed */
    int32_t batch_size;   /* requests in the launch that served it (resident mode: requests
                             in the queue when it was published, itself included) */
    void* output;         /* device, in the arena: int16 [w*h/64][64] or uint8 [h][w]
                             (host_io: the caller's host_output) */
    int64_t output_bytes;
    double submit_us;     /* host clock, microseconds since server start */
    double done_us;       /* completion observed on the host */
} tdct_result;

typedef struct {
    int64_t submitted, completed, failed, rejected;
    int64_t batches;      /* launches (resident mode: launches of the resident kernel) */
    int64_t pixels_done;
    int64_t arena_bytes_in_use, arena_high_water;
    double busy_us;       /* wall time with at least one batch in flight */
    double p50_us, p99_us, p999_us, mean_us; /* latency, submit -> completion observed */
    double mean_batch;
} tdct_stats;

typedef struct tdct_server tdct_server;

int tdct_server_create(const tdct_server_cfg* cfg, tdct_server** out);
/* Queues a request (never blocks on the GPU). TDCT_ENOMEM if its output
 * alone exceeds the budget; otherwise it waits for arena space in FIFO
 * order. */
int tdct_server_submit(tdct_server* s, const tdct_request* req, uint64_t* ticket);
/* Non-blocking status; TDCT_ENOTFOUND for unknown tickets. */
int tdct_server_poll(tdct_server* s, uint64_t ticket, tdct_result* out);
/* Blocks until the request completes (or fails). */
int tdct_server_wait(tdct_server* s, uint64_t ticket, tdct_result* out);
/* Returns the request's output memory to the arena; the ticket is gone. */
int tdct_server_release(tdct_server* s, uint64_t ticket);
/* Blocks until every submitted request has completed. */
int tdct_server_drain(tdct_server* s);
int tdct_server_stats(tdct_server* s, tdct_stats* out);
/* Text of the last HIP error the scheduler met ("" if none). */
const char* tdct_server_last_error(tdct_server* s);
/* Stops the server: requests in flight finish, requests still waiting for
 * memory fail, then everything is freed. No other call on the server may
 * run concurrently with or after it (a thread blocked in tdct_server_wait
 * must have returned first). */
void tdct_server_destroy(tdct_server* s);

/* Open-loop replay: request k is submitted at arrival_us[k] after the call
 * starts (host clock); outputs are released as they complete unless
 * keep_outputs (then the caller releases the tickets, and TDCT_ENOMEM is
 * returned up front when all outputs together exceed the budget).
 * latency_us[k] receives submit -> completion; status[k] the final status;
 * batch_size[k] the requests in the launch that served it (as in
 * tdct_result). Output arrays may be NULL. Returns after every request has
 * completed. */
int tdct_server_replay(tdct_server* s, const tdct_request* reqs, const double* arrival_us,
                       int32_t n, int32_t keep_outputs, uint64_t* tickets_out,
                       double* latency_us, int32_t* status, int32_t* batch_size);

#ifdef __cplusplus
}
#endif

#endif /* TDCT_H */
