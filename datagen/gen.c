/*
 * Seeded synthetic inputs shared by the tests, the oracle checks and the
 * benchmark.  This file holds no part of the scan/lookup method: it only
 * draws column values and row IDs.
 *
 * Random numbers come from the SplitMix64 sequence (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) used as a
 * counter-based generator: draw i of stream `seed` is mix(seed + (i+1)*gamma).
 * Every value therefore depends only on (seed, row index), never on how rows
 * are split across threads.
 *
 * Zipf(s, N) ranks k in [1, N] with P(k) proportional to k^-s:
 *   - N <= 2^24: inverse CDF over an explicit cumulative table;
 *   - larger N : rejection-inversion (Hoermann & Derflinger, "Rejection-
 *     inversion to generate variates from monotone discrete distributions",
 *     ACM TOMACS 6(3), 1996);
 *   - s == 0   : uniform.
 * Rank k maps to a value either by a seeded bijection on [0, 2^w)
 * ("scatter": frequent values land anywhere in the domain) or by k-1
 * ("sorted": frequent values are the smallest ones).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* draw `ctr` of stream `seed` */
static inline uint64_t draw(uint64_t seed, uint64_t ctr) {
    return mix64(seed + (ctr + 1) * GAMMA);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double draw_unit(uint64_t seed, uint64_t ctr) {
    return (double)(draw(seed, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

uint64_t dg_draw_u64(uint64_t seed, uint64_t ctr) { return draw(seed, ctr); }

/* ---- rank -> value bijection on [0, 2^w) -------------------------------- */
typedef struct {
    uint32_t w;
    uint64_t mask, add, mul1, mul2;
    uint32_t sh;
} perm_t;

static perm_t perm_make(uint32_t w, uint64_t seed) {
    perm_t p;
    p.w = w;
    p.mask = (w >= 64) ? ~0ULL : ((1ULL << w) - 1);
    p.add = draw(seed ^ 0x5EEDULL, 0) & p.mask;
    p.mul1 = (draw(seed ^ 0x5EEDULL, 1) | 1ULL) & p.mask;
    p.mul2 = (draw(seed ^ 0x5EEDULL, 2) | 1ULL) & p.mask;
    if (p.mul1 == 0) p.mul1 = 1;
    if (p.mul2 == 0) p.mul2 = 1;
    p.sh = (w + 1) / 2;
    if (p.sh == 0) p.sh = 1;
    return p;
}

/* add, odd multiply and x ^= x >> sh are each invertible modulo 2^w */
static inline uint64_t perm_apply(const perm_t* p, uint64_t x) {
    x = (x + p->add) & p->mask;
    x = (x * p->mul1) & p->mask;
    x ^= x >> p->sh;
    x = (x * p->mul2) & p->mask;
    x ^= x >> p->sh;
    return x & p->mask;
}

uint64_t dg_perm(uint32_t w, uint64_t seed, uint64_t x) {
    perm_t p = perm_make(w, seed);
    return perm_apply(&p, x);
}

/* ---- Zipf by rejection-inversion ---------------------------------------- */
typedef struct {
    double s, n;
    double h_x1, h_n, skip;
} zri_t;

/* (exp(x)-1)/x, accurate near 0 */
static double expm1_over_x(double x) {
    if (fabs(x) > 1e-8) return expm1(x) / x;
    return 1.0 + x * 0.5 * (1.0 + x / 3.0 * (1.0 + 0.25 * x));
}
/* log(1+x)/x, accurate near 0 */
static double log1p_over_x(double x) {
    if (fabs(x) > 1e-8) return log1p(x) / x;
    return 1.0 - x * (0.5 - x * (1.0 / 3.0 - 0.25 * x));
}
/* h(x) = x^-s */
static double zh(const zri_t* z, double x) { return exp(-z->s * log(x)); }
/* H(x) = integral of h: (x^(1-s) - 1) / (1 - s), or log(x) when s == 1 */
static double zH(const zri_t* z, double x) {
    double lx = log(x);
    return expm1_over_x((1.0 - z->s) * lx) * lx;
}
/* inverse of H */
static double zHinv(const zri_t* z, double y) {
    double t = y * (1.0 - z->s);
    if (t < -1.0) t = -1.0;
    return exp(log1p_over_x(t) * y);
}
static zri_t zri_make(double s, double n) {
    zri_t z;
    z.s = s;
    z.n = n;
    z.h_x1 = zH(&z, 1.5) - 1.0;
    z.h_n = zH(&z, n + 0.5);
    z.skip = 2.0 - zHinv(&z, zH(&z, 2.5) - zh(&z, 2.0));
    return z;
}
static uint64_t zri_sample(const zri_t* z, uint64_t seed, uint64_t row) {
    for (uint64_t a = 0;; ++a) {
        double u01 = draw_unit(seed, (row << 12) | (a & 0xFFF));
        double u = z->h_n + u01 * (z->h_x1 - z->h_n);
        double x = zHinv(z, u);
        double kd = floor(x + 0.5);
        if (kd < 1.0) kd = 1.0;
        if (kd > z->n) kd = z->n;
        if (kd - x <= z->skip || u >= zH(z, kd + 0.5) - zh(z, kd)) return (uint64_t)kd;
    }
}

/* ---- threaded fill ------------------------------------------------------- */
typedef struct {
    uint32_t* out;
    uint64_t lo, hi, seed, nvals;
    uint32_t w;
    int mapping;   /* 0 scatter, 1 sorted */
    int method;    /* 0 uniform, 1 table, 2 rejection-inversion */
    const double* cdf;
    const uint32_t* guide;   /* guide[b] = first index with cdf > b / ng */
    uint64_t ng;
    zri_t zri;
    perm_t perm;
} job_t;

static void* fill_worker(void* arg) {
    job_t* j = (job_t*)arg;
    for (uint64_t i = j->lo; i < j->hi; ++i) {
        uint64_t k; /* 1-based rank */
        if (j->method == 0) {
            k = 1 + (uint64_t)(((__uint128_t)draw(j->seed, i << 12) * j->nvals) >> 64);
        } else if (j->method == 1) {
            double u = draw_unit(j->seed, i << 12);
            /* first idx with cdf[idx] > u, searched between the guide entries of
               the bucket of u (the same index a search of the whole table finds) */
            uint64_t b = (uint64_t)(u * (double)j->ng);
            if (b >= j->ng) b = j->ng - 1;
            while (b > 0 && (double)b / (double)j->ng > u) --b;
            while (b + 1 < j->ng && (double)(b + 1) / (double)j->ng <= u) ++b;
            uint64_t lo = j->guide[b], hi = j->guide[b + 1];
            while (lo < hi) {
                uint64_t mid = (lo + hi) >> 1;
                if (j->cdf[mid] > u) hi = mid; else lo = mid + 1;
            }
            k = lo + 1;
        } else {
            k = zri_sample(&j->zri, j->seed, i);
        }
        uint64_t v = (j->mapping == 1) ? (k - 1) : perm_apply(&j->perm, k - 1);
        j->out[i] = (uint32_t)v;
    }
    return NULL;
}

/*
 * n values of Zipf(s) over N = 2^w ranks (w in [1, 32]).
 * Returns 0 on success, -1 on bad arguments or allocation failure.
 */
int dg_zipf_u32(uint32_t* out, uint64_t n, uint32_t w, double s, uint64_t seed,
                int mapping, uint32_t nthreads) {
    if (w < 1 || w > 32 || s < 0.0 || (n && !out)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    uint64_t nv = 1ULL << w;
    job_t base;
    memset(&base, 0, sizeof(base));
    base.out = out;
    base.seed = seed;
    base.nvals = nv;
    base.w = w;
    base.mapping = mapping;
    base.perm = perm_make(w, seed);
    double* cdf = NULL;
    uint32_t* guide = NULL;
    if (s == 0.0) {
        base.method = 0;
    } else if (w <= 24) {
        base.method = 1;
        cdf = (double*)malloc(sizeof(double) * nv);
        if (!cdf) return -1;
        /* sum small terms first for accuracy, then normalise */
        double tot = 0.0;
        for (uint64_t k = nv; k >= 1; --k) tot += pow((double)k, -s);
        double acc = 0.0;
        for (uint64_t k = 1; k <= nv; ++k) {
            acc += pow((double)k, -s);
            cdf[k - 1] = acc / tot;
        }
        cdf[nv - 1] = 2.0; /* guard: every u < 1 lands inside */
        base.cdf = cdf;
        /* guide table: bucket b of [0, 1) starts its search at the first index
           whose cdf exceeds b / ng; the last entry closes the final bucket */
        base.ng = nv < (1ULL << 22) ? nv : (1ULL << 22);
        guide = (uint32_t*)malloc(sizeof(uint32_t) * (base.ng + 1));
        if (!guide) {
            free(cdf);
            return -1;
        }
        uint64_t idx = 0;
        for (uint64_t b = 0; b < base.ng; ++b) {
            while (cdf[idx] <= (double)b / (double)base.ng) ++idx;
            guide[b] = (uint32_t)idx;
        }
        guide[base.ng] = (uint32_t)(nv - 1);
        base.guide = guide;
    } else {
        base.method = 2;
        base.zri = zri_make(s, (double)nv);
    }
    pthread_t th[256];
    job_t jobs[256];
    int threaded[256];
    uint64_t chunk = (n + nthreads - 1) / nthreads;
    for (uint32_t t = 0; t < nthreads; ++t) {
        threaded[t] = 0;
        jobs[t] = base;
        jobs[t].lo = (uint64_t)t * chunk;
        jobs[t].hi = jobs[t].lo + chunk;
        if (jobs[t].lo > n) jobs[t].lo = n;
        if (jobs[t].hi > n) jobs[t].hi = n;
        if (jobs[t].lo == jobs[t].hi) continue;
        if (pthread_create(&th[t], NULL, fill_worker, &jobs[t]) == 0)
            threaded[t] = 1;
        else
            fill_worker(&jobs[t]); /* no thread available: run inline */
    }
    for (uint32_t t = 0; t < nthreads; ++t)
        if (threaded[t]) pthread_join(th[t], NULL);
    free(cdf);
    free(guide);
    return 0;
}

/* m integers uniform in [0, bound), stream `seed` (e.g. row IDs) */
int dg_uniform_u32(uint32_t* out, uint64_t m, uint64_t bound, uint64_t seed) {
    if (bound == 0 || bound > (1ULL << 32) || (m && !out)) return -1;
    for (uint64_t i = 0; i < m; ++i)
        out[i] = (uint32_t)(((__uint128_t)draw(seed, i) * bound) >> 64);
    return 0;
}
