/*
 * Seeded synthetic temporal edge streams.
 *
 * This module produces the inputs that both the GPU library and the CPU
 * oracle consume. It contains no part of the walk method itself: only a
 * counter-based hash RNG, a bounded Zipf sampler, uniform integers and
 * Poisson / Markov-modulated Poisson arrival times.
 *
 * Every output element i is a pure function of (seed, stream, i), so results
 * do not depend on the number of threads. Prefix sums of arrival gaps are
 * done in 2^-20 fixed point on int64, which is associative, so they are also
 * independent of chunking.
 *
 * RNG: the SplitMix64 finaliser (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) applied to a mixed counter.
 * The walk method's own RNG (Philox) is deliberately not used here.
 *
 * Zipf: rejection-inversion for monotone discrete distributions
 * (Hormann and Derflinger, ACM TOMACS 6(3), 1996), written here from the
 * method's description: sample a continuous variate from the integral of the
 * hat x^-s by inversion, round to the nearest integer k, and accept when the
 * variate falls inside the part of k's hat interval whose area equals k^-s.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t rnd64(uint64_t seed, uint64_t stream, uint64_t i) {
    uint64_t k = mix64(seed * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL);
    k = mix64(k ^ (stream * 0xD1B54A32D192ED03ULL));
    return mix64(k + i * 0x9E3779B97F4A7C15ULL);
}

/* uniform double in (0,1): 52 random bits, centred in their cell */
static inline double unit_open(uint64_t x) {
    return ((double)(x >> 12) * 2.0 + 1.0) * 0x1.0p-53;
}

/* floor(x * n / 2^64) */
static inline uint64_t scale64(uint64_t x, uint64_t n) {
    return (uint64_t)(((unsigned __int128)x * n) >> 64);
}

/* ---- bounded Zipf by rejection-inversion ---------------------------------- */

typedef struct {
    double s, one_minus_s;
    double lo, hi;      /* integer support [lo, hi], lo >= 1 */
    double area_lo, area_hi;
} zipf_t;

/* exp(t)-1 over t, continuous at 0 */
static double expm1_over(double t) { return fabs(t) > 1e-8 ? expm1(t) / t : 1.0 + 0.5 * t; }
/* log(1+t) over t, continuous at 0 */
static double log1p_over(double t) { return fabs(t) > 1e-8 ? log1p(t) / t : 1.0 - 0.5 * t; }

/* antiderivative of x^-s that vanishes at x = 1 */
static double zipf_H(const zipf_t* z, double x) {
    double l = log(x);
    return l * expm1_over(z->one_minus_s * l);
}
/* inverse of zipf_H */
static double zipf_Hinv(const zipf_t* z, double y) {
    return exp(y * log1p_over(z->one_minus_s * y));
}
static double zipf_h(const zipf_t* z, double x) { return exp(-z->s * log(x)); }

static void zipf_init(zipf_t* z, double s, double lo, double hi) {
    z->s = s;
    z->one_minus_s = 1.0 - s;
    z->lo = lo;
    z->hi = hi;
    z->area_lo = zipf_H(z, lo + 0.5) - zipf_h(z, lo);
    z->area_hi = zipf_H(z, hi + 0.5);
}

/* draw #attempt for sample i uses counter i on a per-attempt stream */
static int64_t zipf_draw(const zipf_t* z, uint64_t seed, uint64_t stream, uint64_t i) {
    for (uint64_t attempt = 0;; ++attempt) {
        double u01 = (double)(rnd64(seed, stream + (attempt << 40), i) >> 11) * 0x1.0p-53;
        double y = z->area_hi + u01 * (z->area_lo - z->area_hi);
        double x = zipf_Hinv(z, y);
        double k = floor(x + 0.5);
        if (k < z->lo) k = z->lo;
        if (k > z->hi) k = z->hi;
        if (y >= zipf_H(z, k + 0.5) - zipf_h(z, k)) return (int64_t)k;
    }
}

/* rank (0-based) -> node id: an affine bijection of [0, V) */
typedef struct { uint64_t V, a, b; } perm_t;

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

static void perm_init(perm_t* p, uint64_t V, uint64_t seed) {
    p->V = V;
    if (V <= 1) { p->a = 1; p->b = 0; return; }
    uint64_t a = (0x9E3779B97F4A7C15ULL ^ mix64(seed + 17)) % V;
    for (;; ++a) {
        a %= V;
        if (a != 0 && gcd_u64(a, V) == 1) break;
    }
    p->a = a;
    p->b = mix64(seed + 99) % V;
}

static inline uint64_t perm_apply(const perm_t* p, uint64_t r) {
    return (uint64_t)(((unsigned __int128)p->a * r + p->b) % p->V);
}

/*
 * Node ids for samples [start, start+n) of one endpoint stream.
 * s <= 0: uniform over [0, V). Otherwise Zipf(s) over ranks k0+1 .. k0+V
 * (k0 > 0 gives the Zipf-Mandelbrot law), rank mapped to an id through the
 * bijection keyed by perm_seed (use the same perm_seed for src and dst so that
 * hubs both send and receive).
 */
void synth_nodes(uint64_t seed, uint64_t stream, int64_t start, int64_t n, int64_t V,
                 double s, double k0, uint64_t perm_seed, int32_t* out) {
    if (n <= 0) return;
    if (s <= 0.0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            out[i] = (int32_t)scale64(rnd64(seed, stream, (uint64_t)(start + i)), (uint64_t)V);
        return;
    }
    zipf_t z;
    zipf_init(&z, s, k0 + 1.0, k0 + (double)V);
    perm_t p;
    perm_init(&p, (uint64_t)V, perm_seed);
    int64_t ik0 = (int64_t)k0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = zipf_draw(&z, seed, stream, (uint64_t)(start + i));
        out[i] = (int32_t)perm_apply(&p, (uint64_t)(k - ik0 - 1));
    }
}

/* Exact Zipf probability mass over ranks, for testing the sampler. */
void synth_zipf_pmf(int64_t V, double s, double k0, double* pmf) {
    double tot = 0.0;
    for (int64_t k = 0; k < V; ++k) { pmf[k] = pow(k0 + 1.0 + (double)k, -s); tot += pmf[k]; }
    for (int64_t k = 0; k < V; ++k) pmf[k] /= tot;
}

/* rank of a node id under the bijection (inverse map), for testing */
int64_t synth_perm_apply(int64_t V, uint64_t perm_seed, int64_t rank) {
    perm_t p;
    perm_init(&p, (uint64_t)V, perm_seed);
    return (int64_t)perm_apply(&p, (uint64_t)rank);
}

/* uniform int64 in [lo, hi) for samples [start, start+n) */
void synth_uniform_i64(uint64_t seed, uint64_t stream, int64_t start, int64_t n, int64_t lo,
                       int64_t hi, int64_t* out) {
    uint64_t span = (uint64_t)(hi - lo);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = lo + (int64_t)scale64(rnd64(seed, stream, (uint64_t)(start + i)), span);
}

/*
 * Sorted arrival times of a (Markov-modulated) Poisson stream.
 * Edge j (global index start+i) has state segment g with seg_start[g] <= j <
 * seg_start[g+1]; its gap is Exp(seg_mean[g]) in 2^-20 fixed point. The
 * running fixed-point sum continues from *acc (updated on return) and the
 * timestamp is ts0 + floor(sum / 2^20).
 */
void synth_poisson_ts(uint64_t seed, uint64_t stream, int64_t start, int64_t n, int32_t nseg,
                      const int64_t* seg_start, const double* seg_mean, int64_t ts0,
                      int64_t* acc, int64_t* out) {
    if (n <= 0) return;
    /* gaps first (parallel), then an integer prefix sum in fixed chunks */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = start + i;
        int32_t lo = 0, hi = nseg - 1; /* last segment with seg_start <= j */
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) / 2;
            if (seg_start[mid] <= j) lo = mid; else hi = mid - 1;
        }
        double u = unit_open(rnd64(seed, stream, (uint64_t)j));
        double g = -seg_mean[lo] * log(u) * 1048576.0;
        out[i] = (int64_t)g;
    }
    const int64_t CH = 1 << 20;
    int64_t nch = (n + CH - 1) / CH;
    int64_t* part = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nch + 1));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) {
        int64_t s = 0, e = (c + 1) * CH < n ? (c + 1) * CH : n;
        for (int64_t i = c * CH; i < e; ++i) s += out[i];
        part[c + 1] = s;
    }
    part[0] = *acc;
    for (int64_t c = 0; c < nch; ++c) part[c + 1] += part[c];
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) {
        int64_t s = part[c], e = (c + 1) * CH < n ? (c + 1) * CH : n;
        for (int64_t i = c * CH; i < e; ++i) {
            s += out[i];
            out[i] = ts0 + (s >> 20);
        }
    }
    *acc = part[nch];
    free(part);
}

/* raw generator words, for tests of determinism */
void synth_raw(uint64_t seed, uint64_t stream, int64_t start, int64_t n, uint64_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = rnd64(seed, stream, (uint64_t)(start + i));
}

int synth_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
