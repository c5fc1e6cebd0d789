/*
 * Seeded synthetic image generators (input data only; no codec arithmetic).
 *
 * A "blob field" plane is the sum of N isotropic 2-D Gaussian blobs
 *   A_k * exp(-((x - cx_k)^2 + (y - cy_k)^2) / (2 sigma_k^2))
 * with cx ~ U[0, fw), cy ~ U[0, fh), sigma ~ U[8, 64] px, A ~ U[0, 255],
 * evaluated in float64, rounded to the nearest integer, plus integer noise
 * uniform in [-amp, amp], clipped to [0, 255]. Blob parameters come from a
 * splitmix64 stream seeded with blob_seed; the noise of pixel (x, y) is a
 * counter-based hash of (noise_seed, y * w + x), so any sub-rectangle can be
 * regenerated on its own and the result does not depend on the thread count.
 *
 * A plane may show a window of a larger field (fw x fh) shifted by (ox, oy)
 * and scaled by `scale` (0.5 gives the half-resolution chroma view of the
 * same field), which is how moving video frames are made.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t splitmix64(uint64_t* s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double unif01(uint64_t* s) { return (double)(splitmix64(s) >> 11) * 0x1.0p-53; }

static int32_t noise_at(uint64_t noise_seed, uint64_t idx, int32_t amp) {
    if (amp <= 0) return 0;
    uint64_t s = noise_seed ^ (idx * 0xD1B54A32D192ED03ull);
    uint64_t r = splitmix64(&s) >> 32;               /* uniform in [0, 2^32) */
    return (int32_t)((r * (uint64_t)(2 * amp + 1)) >> 32) - amp;
}

typedef struct {
    int32_t nb;
    double cx[64], cy[64], sg[64], A[64];
} blobs_t;

static void draw_blobs(blobs_t* b, uint64_t seed, int32_t nblobs, int32_t fw, int32_t fh,
                       double scale) {
    uint64_t s = seed;
    b->nb = nblobs > 64 ? 64 : nblobs;
    for (int k = 0; k < b->nb; ++k) {
        b->cx[k] = unif01(&s) * fw * scale;
        b->cy[k] = unif01(&s) * fh * scale;
        b->sg[k] = (8.0 + 56.0 * unif01(&s)) * scale;
        b->A[k] = 255.0 * unif01(&s);
    }
}

/* Rows [y0, y1) of one plane. gx: [nb][w], gy: [nb][h] precomputed. The
 * blob sum runs over k in ascending order for every pixel. */
static void fill_rows(uint8_t* out, int64_t stride, int32_t w, const blobs_t* b,
                      const double* gx, const double* gy, int32_t h, int32_t y0, int32_t y1,
                      uint64_t noise_seed, int32_t amp) {
    double* acc = (double*)malloc(sizeof(double) * (size_t)w + 8);
    for (int32_t y = y0; y < y1; ++y) {
        uint8_t* row = out + (int64_t)y * stride;
        for (int32_t x = 0; x < w; ++x) acc[x] = 0.0;
        for (int k = 0; k < b->nb; ++k) {
            const double ay = b->A[k] * gy[(int64_t)k * h + y];
            const double* g = gx + (int64_t)k * w;
            for (int32_t x = 0; x < w; ++x) acc[x] += ay * g[x];
        }
        for (int32_t x = 0; x < w; ++x) {
            int32_t v = (int32_t)nearbyint(acc[x]) + noise_at(noise_seed, (uint64_t)y * (uint64_t)w + x, amp);
            row[x] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
        }
    }
    free(acc);
}

static void tables(const blobs_t* b, int32_t w, int32_t h, int32_t ox, int32_t oy, double* gx,
                   double* gy) {
    for (int k = 0; k < b->nb; ++k) {
        double inv = 1.0 / (2.0 * b->sg[k] * b->sg[k]);
        for (int32_t x = 0; x < w; ++x) {
            double d = (double)(x + ox) - b->cx[k];
            gx[(int64_t)k * w + x] = exp(-d * d * inv);
        }
        for (int32_t y = 0; y < h; ++y) {
            double d = (double)(y + oy) - b->cy[k];
            gy[(int64_t)k * h + y] = exp(-d * d * inv);
        }
    }
}

typedef struct {
    uint8_t* out;
    int64_t stride;
    int32_t w, h;
    const blobs_t* b;
    const double *gx, *gy;
    uint64_t noise_seed;
    int32_t amp;
    int32_t y0, y1;
} rows_job;

static void* rows_worker(void* p) {
    rows_job* j = (rows_job*)p;
    fill_rows(j->out, j->stride, j->w, j->b, j->gx, j->gy, j->h, j->y0, j->y1, j->noise_seed, j->amp);
    return NULL;
}

/* One plane, rows split over nthreads threads. */
void synth_blob_plane(uint8_t* out, int64_t stride, int32_t w, int32_t h, uint64_t blob_seed,
                      int32_t nblobs, int32_t fw, int32_t fh, double scale, int32_t ox, int32_t oy,
                      uint64_t noise_seed, int32_t amp, int32_t nthreads) {
    blobs_t b;
    draw_blobs(&b, blob_seed, nblobs, fw, fh, scale);
    double* gx = (double*)malloc(sizeof(double) * (size_t)b.nb * (size_t)w + 8);
    double* gy = (double*)malloc(sizeof(double) * (size_t)b.nb * (size_t)h + 8);
    tables(&b, w, h, ox, oy, gx, gy);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > h) nthreads = h;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    rows_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        rows_job j = {out, stride, w, h, &b, gx, gy, noise_seed, amp,
                      (int32_t)((int64_t)h * t / nthreads), (int32_t)((int64_t)h * (t + 1) / nthreads)};
        jobs[t] = j;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, rows_worker, &jobs[t]);
    rows_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(gx);
    free(gy);
}

/* Many independent images (each its own field and seed), packed in one
 * buffer at the given byte offsets; images are handed to threads from a
 * shared counter. */
typedef struct {
    uint8_t* base;
    const int64_t *off, *stride;
    const int32_t *w, *h;
    const uint64_t* seed;
    int32_t n, nblobs, amp;
    int32_t next;
    pthread_mutex_t mu;
} batch_job;

static void* batch_worker(void* p) {
    batch_job* J = (batch_job*)p;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int32_t i = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (i >= J->n) break;
        blobs_t b;
        int32_t w = J->w[i], h = J->h[i];
        draw_blobs(&b, J->seed[i], J->nblobs, w, h, 1.0);
        double* gx = (double*)malloc(sizeof(double) * (size_t)b.nb * (size_t)w + 8);
        double* gy = (double*)malloc(sizeof(double) * (size_t)b.nb * (size_t)h + 8);
        tables(&b, w, h, 0, 0, gx, gy);
        fill_rows(J->base + J->off[i], J->stride[i], w, &b, gx, gy, h, 0, h,
                  J->seed[i] ^ 0xA5A5A5A55A5A5A5Aull, J->amp);
        free(gx);
        free(gy);
    }
    return NULL;
}

void synth_blob_batch(uint8_t* base, const int64_t* off, const int64_t* stride, const int32_t* w,
                      const int32_t* h, const uint64_t* seed, int32_t n, int32_t nblobs,
                      int32_t amp, int32_t nthreads) {
    batch_job J;
    J.base = base; J.off = off; J.stride = stride; J.w = w; J.h = h; J.seed = seed;
    J.n = n; J.nblobs = nblobs; J.amp = amp; J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, batch_worker, &J);
    batch_worker(&J);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
}

/* Rounded blob field of a whole canvas (no noise), clipped to [-16, 272]:
 * clipping this far outside [0, 255] cannot change any final pixel, since the
 * noise added later is at most 16 in magnitude. Identical values to
 * synth_blob_plane for the same field, window and scale. */
typedef struct {
    int16_t* out;
    int32_t w, h;
    const blobs_t* b;
    const double *gx, *gy;
    int32_t y0, y1;
} field_job;

static void* field_worker(void* p) {
    field_job* j = (field_job*)p;
    double* acc = (double*)malloc(sizeof(double) * (size_t)j->w + 8);
    for (int32_t y = j->y0; y < j->y1; ++y) {
        for (int32_t x = 0; x < j->w; ++x) acc[x] = 0.0;
        for (int k = 0; k < j->b->nb; ++k) {
            const double ay = j->b->A[k] * j->gy[(int64_t)k * j->h + y];
            const double* g = j->gx + (int64_t)k * j->w;
            for (int32_t x = 0; x < j->w; ++x) acc[x] += ay * g[x];
        }
        int16_t* row = j->out + (int64_t)y * j->w;
        for (int32_t x = 0; x < j->w; ++x) {
            int32_t v = (int32_t)nearbyint(acc[x]);
            row[x] = (int16_t)(v < -16 ? -16 : (v > 272 ? 272 : v));
        }
    }
    free(acc);
    return NULL;
}

void synth_blob_field(int16_t* out, int32_t w, int32_t h, uint64_t blob_seed, int32_t nblobs,
                      int32_t fw, int32_t fh, double scale, int32_t nthreads) {
    blobs_t b;
    draw_blobs(&b, blob_seed, nblobs, fw, fh, scale);
    double* gx = (double*)malloc(sizeof(double) * (size_t)b.nb * (size_t)w + 8);
    double* gy = (double*)malloc(sizeof(double) * (size_t)b.nb * (size_t)h + 8);
    tables(&b, w, h, 0, 0, gx, gy);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > h) nthreads = h;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    field_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        field_job j = {out, w, h, &b, gx, gy, (int32_t)((int64_t)h * t / nthreads),
                       (int32_t)((int64_t)h * (t + 1) / nthreads)};
        jobs[t] = j;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, field_worker, &jobs[t]);
    field_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(gx);
    free(gy);
}

/* Window (ox, oy) of a precomputed field plus per-pixel noise. */
typedef struct {
    const int16_t* field;
    int32_t fw;
    int32_t ox, oy;
    uint8_t* out;
    int64_t stride;
    int32_t w;
    uint64_t noise_seed;
    int32_t amp;
    int32_t y0, y1;
} window_job;

static void* window_worker(void* p) {
    window_job* j = (window_job*)p;
    for (int32_t y = j->y0; y < j->y1; ++y) {
        const int16_t* src = j->field + (int64_t)(y + j->oy) * j->fw + j->ox;
        uint8_t* row = j->out + (int64_t)y * j->stride;
        for (int32_t x = 0; x < j->w; ++x) {
            int32_t v = src[x] + noise_at(j->noise_seed, (uint64_t)y * (uint64_t)j->w + x, j->amp);
            row[x] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
        }
    }
    return NULL;
}

void synth_window(const int16_t* field, int32_t fw, int32_t ox, int32_t oy, uint8_t* out,
                  int64_t stride, int32_t w, int32_t h, uint64_t noise_seed, int32_t amp,
                  int32_t nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > h) nthreads = h;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    window_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        window_job j = {field, fw, ox, oy, out, stride, w, noise_seed, amp,
                        (int32_t)((int64_t)h * t / nthreads), (int32_t)((int64_t)h * (t + 1) / nthreads)};
        jobs[t] = j;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, window_worker, &jobs[t]);
    window_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
}
