/*
 * synth.c - seeded synthetic dedispersed blocks for the single-pulse search.
 *
 * Input generation only: this file holds none of the search's arithmetic
 * (no medians, no boxcars, no S/N). Both the CPU oracle and the HIP path are
 * fed from the arrays it writes.
 *
 * Random numbers come from Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), a counter-based
 * generator: block = philox(counter, key). Every value therefore depends only
 * on (seed, stream, purpose, row, sample index), never on thread count or on
 * the order in which rows are generated.
 *
 * Noise is an integer Gaussian: round(N(mu, sigma^2)) drawn by inverse CDF
 * over a fixed-point table of cumulative probabilities for offsets in
 * [-8 sigma, +8 sigma] (the tails beyond are clamped; their mass is ~1e-15).
 * A sinusoidal drift round(A sin(2 pi t / P)) (t = global sample index) is
 * added after rounding, so every sample is an exact integer stored in FP32.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define PH_M0 0xD2E7470EE14C6C93ULL
#define PH_M1 0xCA5A826395121157ULL
#define PH_W0 0x9E3779B97F4A7C15ULL
#define PH_W1 0xBB67AE8584CAA73BULL

/* Philox4x64 with 10 rounds, as published (Random123 reference parameters). */
void synth_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += PH_W0; k1 += PH_W1; }
        u128 p0 = (u128)PH_M0 * x0;
        u128 p1 = (u128)PH_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Batch helper for Python: n consecutive blocks starting at ctr (ctr[0]
 * incremented per block), 4 words each. */
void synth_philox_blocks(const uint64_t ctr[4], const uint64_t key[2], int64_t n, uint64_t* out)
{
    uint64_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    for (int64_t i = 0; i < n; ++i) {
        synth_philox4x64(c, key, out + 4 * i);
        c[0] += 1;
    }
}

/* ---- integer Gaussian table ------------------------------------------- */

typedef struct {
    int32_t kmin;         /* offset of entry 0 (= -half) */
    int32_t nent;         /* 2*half + 1 entries */
    uint64_t* cdf;        /* cdf[j] = floor(2^64 * P(round(Z) <= kmin + j)), last = UINT64_MAX */
    int32_t* guide;       /* guide[h] = first j with cdf[j] > (h << 48) */
} ig_table;

static int ig_build(ig_table* t, double sigma)
{
    int32_t half = (int32_t)ceil(8.0 * sigma);
    if (half < 1) half = 1;
    t->kmin = -half;
    t->nent = 2 * half + 1;
    t->cdf = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)t->nent);
    t->guide = (int32_t*)malloc(sizeof(int32_t) * 65536);
    if (!t->cdf || !t->guide) return -1;
    for (int32_t j = 0; j < t->nent; ++j) {
        long double z = ((long double)(t->kmin + j) + 0.5L) / ((long double)sigma * sqrtl(2.0L));
        long double p = 0.5L * erfcl(-z);           /* P(Z < k + 1/2) = P(round(Z) <= k) */
        long double f = ldexpl(p, 64);
        uint64_t c;
        if (f >= 18446744073709551615.0L) c = UINT64_MAX;
        else if (f <= 0.0L) c = 0;
        else c = (uint64_t)f;
        t->cdf[j] = c;
    }
    t->cdf[t->nent - 1] = UINT64_MAX;
    int32_t j = 0;
    for (int32_t h = 0; h < 65536; ++h) {
        uint64_t lo = (uint64_t)h << 48;
        while (j < t->nent - 1 && t->cdf[j] <= lo) ++j;
        t->guide[h] = j;
    }
    return 0;
}

static void ig_free(ig_table* t) { free(t->cdf); free(t->guide); }

static inline int32_t ig_draw(const ig_table* t, uint64_t u)
{
    int32_t j = t->guide[u >> 48];
    while (j < t->nent - 1 && u >= t->cdf[j]) ++j;
    return t->kmin + j;
}

/* ---- noise + drift fill ------------------------------------------------ */

typedef struct {
    float* out;            /* [nrow][nsamp], row stride = ld */
    int64_t nrow, nsamp, ld;
    int64_t row0;          /* global row index of out row 0 (counter word 1) */
    int64_t t0;            /* global sample index of out column 0 */
    uint64_t seed, stream; /* Philox key */
    double mu, sigma;
    double drift_amp;      /* drift amplitude in sample units (0 = none) */
    int64_t drift_period;
} synth_fill_args;

typedef struct {
    const synth_fill_args* a;
    const ig_table* tab;
    const int32_t* drift;  /* drift[t mod period] */
    int64_t r_begin, r_end;
} fill_job;

#define PURPOSE_NOISE 0x4E4F495345ULL /* "NOISE" */

static void* fill_worker(void* p)
{
    fill_job* jb = (fill_job*)p;
    const synth_fill_args* a = jb->a;
    const uint64_t key[2] = {a->seed, a->stream};
    const int32_t mu = (int32_t)llround(a->mu);
    for (int64_t r = jb->r_begin; r < jb->r_end; ++r) {
        float* row = a->out + r * a->ld;
        int64_t t = a->t0;
        int64_t tend = a->t0 + a->nsamp;
        int64_t col = 0;
        while (t < tend) {
            /* one Philox block covers the four samples sharing t >> 2 */
            uint64_t ctr[4] = {(uint64_t)(t >> 2), (uint64_t)(a->row0 + r), PURPOSE_NOISE, 0};
            uint64_t w[4];
            synth_philox4x64(ctr, key, w);
            for (int q = (int)(t & 3); q < 4 && t < tend; ++q, ++t, ++col) {
                int32_t v = mu + ig_draw(jb->tab, w[q]);
                if (jb->drift) {
                    int64_t ph = t % a->drift_period;
                    if (ph < 0) ph += a->drift_period;
                    v += jb->drift[ph];
                }
                row[col] = (float)v;
            }
        }
    }
    return NULL;
}

/* Fill out[nrow][nsamp] with integer Gaussian noise plus drift.
 * Returns 0, or -1 on allocation failure / bad arguments. */
int synth_fill_noise(const synth_fill_args* a, int nthreads)
{
    if (!a || !a->out || a->nrow < 0 || a->nsamp < 0 || a->ld < a->nsamp || a->sigma <= 0.0)
        return -1;
    if (a->nrow == 0 || a->nsamp == 0) return 0;
    ig_table tab;
    if (ig_build(&tab, a->sigma)) { ig_free(&tab); return -1; }
    int32_t* drift = NULL;
    if (a->drift_amp != 0.0 && a->drift_period > 0) {
        drift = (int32_t*)malloc(sizeof(int32_t) * (size_t)a->drift_period);
        if (!drift) { ig_free(&tab); return -1; }
        const double two_pi = 6.283185307179586476925286766559;
        for (int64_t p = 0; p < a->drift_period; ++p) {
            double v = a->drift_amp * sin(two_pi * (double)p / (double)a->drift_period);
            drift[p] = (int32_t)floor(v + 0.5);
        }
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > a->nrow) nthreads = (int)a->nrow;
    pthread_t th[256];
    int created[256];
    fill_job jobs[256];
    int64_t per = (a->nrow + nthreads - 1) / nthreads;
    for (int i = 0; i < nthreads; ++i) {
        jobs[i].a = a; jobs[i].tab = &tab; jobs[i].drift = drift;
        jobs[i].r_begin = (int64_t)i * per < a->nrow ? (int64_t)i * per : a->nrow;
        jobs[i].r_end = jobs[i].r_begin + per < a->nrow ? jobs[i].r_begin + per : a->nrow;
        created[i] = 0;
        if (i > 0 && jobs[i].r_begin < jobs[i].r_end)
            created[i] = pthread_create(&th[i], NULL, fill_worker, &jobs[i]) == 0;
    }
    fill_worker(&jobs[0]);
    for (int i = 1; i < nthreads; ++i) {
        if (created[i]) pthread_join(th[i], NULL);
        else fill_worker(&jobs[i]);   /* empty range, or thread creation failed */
    }
    free(drift);
    ig_free(&tab);
    return 0;
}

/* Expose one table lookup for tests of the inverse-CDF sampler. */
int synth_int_gauss(double sigma, const uint64_t* u, int64_t n, int32_t* out)
{
    ig_table tab;
    if (sigma <= 0.0 || ig_build(&tab, sigma)) return -1;
    for (int64_t i = 0; i < n; ++i) out[i] = ig_draw(&tab, u[i]);
    ig_free(&tab);
    return 0;
}
