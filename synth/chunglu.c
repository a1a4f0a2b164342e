/*
 * Seeded synthetic bipartite graphs for tests and benchmarks.
 *
 * This file only draws inputs: node ids, edge pairs and edge weights. It holds
 * none of the similarity method's arithmetic, so the FP64 oracle and the GPU
 * library can both consume its output without sharing any method code.
 *
 * Model: a bipartite Chung-Lu graph. Node i of a side gets expected-degree
 * weight (i+1)^(-1/(gamma-1)); ids are then shuffled so id order carries no
 * degree information. Each edge draws its U endpoint and its V endpoint
 * independently from those weights (Walker alias tables); repeated (u,v)
 * pairs are rejected until exactly n_e distinct pairs exist, which are
 * returned in draw order (unsorted).
 *
 * Weights: kind 0 = integers uniform on 1..10 (exact in FP32 and FP64);
 * kind 1 = exp(N(0,1)) drawn in FP64 (Box-Muller) and rounded to FP32, so the
 * FP64 value equals an FP32 value exactly.
 *
 * PRNG: xoshiro256** (Blackman and Vigna) seeded through splitmix64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t* x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t* r) {
    uint64_t* s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
}

static void rng_seed(rng_t* r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

/* uniform double in [0,1) with 53 random bits */
static double rng_unif(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0,n) by rejection (no modulo bias) */
static uint64_t rng_below(rng_t* r, uint64_t n) {
    uint64_t lim = UINT64_MAX - (UINT64_MAX % n);
    uint64_t x;
    do { x = rng_next(r); } while (x >= lim);
    return x % n;
}

typedef struct { double* prob; int32_t* alias; int32_t n; } alias_t;

/* Vose's alias method over weights p[0..n) */
static int alias_build(alias_t* a, const double* p, int32_t n) {
    a->n = n;
    a->prob = (double*)malloc(sizeof(double) * (size_t)n);
    a->alias = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* small = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* large = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double* q = (double*)malloc(sizeof(double) * (size_t)n);
    if (!a->prob || !a->alias || !small || !large || !q) return -1;
    double tot = 0.0;
    for (int32_t i = 0; i < n; ++i) tot += p[i];
    int32_t ns = 0, nl = 0;
    for (int32_t i = 0; i < n; ++i) {
        q[i] = p[i] * (double)n / tot;
        if (q[i] < 1.0) small[ns++] = i; else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        int32_t s = small[--ns], l = large[--nl];
        a->prob[s] = q[s];
        a->alias[s] = l;
        q[l] = (q[l] + q[s]) - 1.0;
        if (q[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl > 0) { int32_t l = large[--nl]; a->prob[l] = 1.0; a->alias[l] = l; }
    while (ns > 0) { int32_t s = small[--ns]; a->prob[s] = 1.0; a->alias[s] = s; }
    free(small); free(large); free(q);
    return 0;
}

static int32_t alias_draw(const alias_t* a, rng_t* r) {
    int32_t i = (int32_t)rng_below(r, (uint64_t)a->n);
    return rng_unif(r) < a->prob[i] ? i : a->alias[i];
}

static void alias_free(alias_t* a) { free(a->prob); free(a->alias); }

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 33)) * 0xff51afd7ed558ccdULL;
    z = (z ^ (z >> 33)) * 0xc4ceb9fe1a85ec53ULL;
    return z ^ (z >> 33);
}

/*
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 * out_u/out_v receive n_e ids, out_w n_e weights (FP64 holding FP32 or
 * integer values).
 */
int synth_chung_lu(int32_t n_u, int32_t n_v, int64_t n_e, double gamma,
                   int32_t weight_kind, uint64_t seed,
                   int32_t* out_u, int32_t* out_v, double* out_w) {
    if (n_u <= 0 || n_v <= 0 || n_e < 0 || gamma <= 1.0) return -1;
    if ((double)n_e > 0.5 * (double)n_u * (double)n_v) return -1;
    rng_t r;
    rng_seed(&r, seed);
    double expo = -1.0 / (gamma - 1.0);
    double* pu = (double*)malloc(sizeof(double) * (size_t)n_u);
    double* pv = (double*)malloc(sizeof(double) * (size_t)n_v);
    int32_t* perm_u = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_u);
    int32_t* perm_v = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_v);
    if (!pu || !pv || !perm_u || !perm_v) return -2;
    for (int32_t i = 0; i < n_u; ++i) pu[i] = pow((double)(i + 1), expo);
    for (int32_t i = 0; i < n_v; ++i) pv[i] = pow((double)(i + 1), expo);
    /* Fisher-Yates shuffles: rank i -> node id perm[i] */
    for (int32_t i = 0; i < n_u; ++i) perm_u[i] = i;
    for (int32_t i = n_u - 1; i > 0; --i) {
        int32_t j = (int32_t)rng_below(&r, (uint64_t)i + 1);
        int32_t t = perm_u[i]; perm_u[i] = perm_u[j]; perm_u[j] = t;
    }
    for (int32_t i = 0; i < n_v; ++i) perm_v[i] = i;
    for (int32_t i = n_v - 1; i > 0; --i) {
        int32_t j = (int32_t)rng_below(&r, (uint64_t)i + 1);
        int32_t t = perm_v[i]; perm_v[i] = perm_v[j]; perm_v[j] = t;
    }
    alias_t au, av;
    if (alias_build(&au, pu, n_u) || alias_build(&av, pv, n_v)) return -2;
    free(pu); free(pv);

    uint64_t cap = 1024;
    while (cap < (uint64_t)n_e * 2 + 16) cap <<= 1;
    uint64_t* table = (uint64_t*)calloc(cap, sizeof(uint64_t));
    if (!table) return -2;
    uint64_t mask = cap - 1;
    int64_t have = 0;
    while (have < n_e) {
        int32_t u = perm_u[alias_draw(&au, &r)];
        int32_t v = perm_v[alias_draw(&av, &r)];
        uint64_t key = (uint64_t)u * (uint64_t)n_v + (uint64_t)v + 1ULL; /* 0 = empty */
        uint64_t h = mix64(key) & mask;
        int fresh = 1;
        while (table[h] != 0) {
            if (table[h] == key) { fresh = 0; break; }
            h = (h + 1) & mask;
        }
        if (!fresh) continue;
        table[h] = key;
        out_u[have] = u;
        out_v[have] = v;
        ++have;
    }
    free(table);
    alias_free(&au); alias_free(&av);
    free(perm_u); free(perm_v);

    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t e = 0; e < n_e; ++e) {
        if (weight_kind == 0) {
            out_w[e] = (double)(1 + (int)rng_below(&r, 10));
        } else {
            double u1 = rng_unif(&r), u2 = rng_unif(&r);
            if (u1 <= 0.0) u1 = 0x1.0p-53;
            double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
            out_w[e] = (double)(float)exp(z);
        }
    }
    return 0;
}
