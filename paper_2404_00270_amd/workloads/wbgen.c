/*
 * Seeded synthetic max-flow workloads.
 *
 * This module only produces input graphs (CSR with integer capacities plus a
 * source and a sink).  It contains none of the max-flow arithmetic: both the
 * CPU oracle and the HIP solver consume what it writes, and neither includes
 * it.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood 2014) seeds xoshiro256**
 * (Blackman and Vigna 2018); both are written here from their published
 * definitions.  Integers are drawn by rejection, doubles as (x >> 11) * 2^-53.
 *
 * Shapes follow the paper's evaluation workloads (section 4): small random
 * graphs, bipartite matching with a super-source and super-sink, a power-law
 * social-network-like graph (R-MAT), a vision-style grid cut, and a stream of
 * many small instances.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
    int32_t V;
    int64_t E;
    int64_t *rp;   /* [V+1] */
    int32_t *col;  /* [E]   */
    int32_t *cap;  /* [E]   */
    int32_t s, t;
} wbgen_graph;

/* ------------------------------------------------------------------ PRNG */
typedef struct { uint64_t s[4]; } xo256;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static void xo_seed(xo256 *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}
static inline uint64_t xo_next(xo256 *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl64(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}
/* uniform integer in [0, n) by rejection of the biased low range */
static inline uint64_t xo_below(xo256 *r, uint64_t n) {
    uint64_t thresh = (0 - n) % n;
    for (;;) {
        uint64_t x = xo_next(r);
        if (x >= thresh) return x % n;
    }
}
static inline double xo_unit(xo256 *r) { return (double)(xo_next(r) >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------ sorting helpers */
/* Stable LSD radix sort of 64-bit keys with a 64-bit payload, on the low
 * `bits` bits of the key. */
static int radix_sort_kv(uint64_t *key, uint64_t *val, int64_t n, int bits) {
    if (n <= 1) return 0;
    uint64_t *k2 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t *v2 = val ? (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n) : NULL;
    if (!k2 || (val && !v2)) { free(k2); free(v2); return -1; }
    const int D = 11;
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) << D);
    if (!cnt) { free(k2); free(v2); return -1; }
    uint64_t *ka = key, *kb = k2, *va = val, *vb = v2;
    int passes = 0;
    for (int sh = 0; sh < bits; sh += D) {
        memset(cnt, 0, sizeof(int64_t) << D);
        for (int64_t i = 0; i < n; i++) cnt[(ka[i] >> sh) & ((1u << D) - 1)]++;
        int64_t acc = 0;
        for (int d = 0; d < (1 << D); d++) { int64_t c = cnt[d]; cnt[d] = acc; acc += c; }
        for (int64_t i = 0; i < n; i++) {
            int64_t p = cnt[(ka[i] >> sh) & ((1u << D) - 1)]++;
            kb[p] = ka[i];
            if (va) vb[p] = va[i];
        }
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint64_t *tv = va; va = vb; vb = tv;
        passes++;
    }
    if (passes & 1) {
        memcpy(key, ka, sizeof(uint64_t) * (size_t)n);
        if (val) memcpy(val, va, sizeof(uint64_t) * (size_t)n);
    }
    free(cnt);
    free(k2);
    free(v2);
    return 0;
}

static int bits_for(uint64_t n) { int b = 1; while ((1ULL << b) < n) b++; return b; }

static int alloc_graph(wbgen_graph *g, int32_t V, int64_t E) {
    g->V = V; g->E = E;
    g->rp = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    g->cap = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    if (!g->rp || !g->col || !g->cap) return -1;
    return 0;
}

void wbgen_free(wbgen_graph *g) {
    if (!g) return;
    free(g->rp); free(g->col); free(g->cap);
    g->rp = NULL; g->col = NULL; g->cap = NULL;
}

/* Fill CSR from keys (u << vb | v) already sorted ascending. */
static void fill_csr_from_sorted(wbgen_graph *g, const uint64_t *key, int vb) {
    int64_t E = g->E;
    for (int64_t i = 0; i < E; i++) {
        uint32_t u = (uint32_t)(key[i] >> vb);
        g->col[i] = (int32_t)(key[i] & ((1ULL << vb) - 1));
        g->rp[u + 1]++;
    }
    for (int32_t v = 0; v < g->V; v++) g->rp[v + 1] += g->rp[v];
}

/* ----------------------------------------------- distinct uniform arcs */
/* E distinct arcs (u,v), u != v, endpoints uniform on [0,V); rows sorted by
 * column; capacities uniform on [cmin, cmax] drawn in CSR order. */
static int gen_distinct_uniform(xo256 *r, int32_t V, int64_t E, int32_t cmin, int32_t cmax,
                                wbgen_graph *g) {
    if (V < 2 || E < 0 || (double)E > (double)V * (double)(V - 1)) return -1;
    int vb = bits_for((uint64_t)V);
    /* open-addressing hash set of accepted keys */
    uint64_t hcap = 1; while (hcap < (uint64_t)E * 2 + 16) hcap <<= 1;
    uint64_t *tab = (uint64_t *)malloc(sizeof(uint64_t) * hcap);
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(E > 0 ? E : 1));
    if (!tab || !keys) { free(tab); free(keys); return -1; }
    memset(tab, 0xff, sizeof(uint64_t) * hcap);
    int64_t n = 0;
    while (n < E) {
        uint64_t u = xo_below(r, (uint64_t)V), v = xo_below(r, (uint64_t)V);
        if (u == v) continue;
        uint64_t k = (u << vb) | v;
        uint64_t h = (k * 0x9e3779b97f4a7c15ULL) & (hcap - 1);
        int dup = 0;
        while (tab[h] != UINT64_MAX) {
            if (tab[h] == k) { dup = 1; break; }
            h = (h + 1) & (hcap - 1);
        }
        if (dup) continue;
        tab[h] = k;
        keys[n++] = k;
    }
    free(tab);
    if (radix_sort_kv(keys, NULL, E, 2 * vb)) { free(keys); return -1; }
    if (alloc_graph(g, V, E)) { free(keys); return -1; }
    fill_csr_from_sorted(g, keys, vb);
    free(keys);
    uint64_t span = (uint64_t)((int64_t)cmax - cmin + 1);
    for (int64_t i = 0; i < E; i++) g->cap[i] = (int32_t)(cmin + (int64_t)xo_below(r, span));
    return 0;
}

/* Plain single max-flow: V vertices, E distinct uniform arcs, caps in
 * [cmin,cmax], s = 0, t = V-1. */
int wbgen_random(int32_t V, int64_t E, int32_t cmin, int32_t cmax, uint64_t seed, wbgen_graph *g) {
    memset(g, 0, sizeof(*g));
    xo256 r; xo_seed(&r, seed);
    if (gen_distinct_uniform(&r, V, E, cmin, cmax, g)) { wbgen_free(g); return -1; }
    g->s = 0; g->t = V - 1;
    return 0;
}

/* Adversarial small multigraph for tests: E arcs with uniform endpoints in
 * [0,V) (parallel arcs, antiparallel arcs and self-loops all allowed), caps
 * uniform on [0, cmax].  s = 0, t = V-1.  Rows keep generation order. */
int wbgen_multi(int32_t V, int64_t E, int32_t cmax, uint64_t seed, wbgen_graph *g) {
    memset(g, 0, sizeof(*g));
    if (V < 2 || E < 0 || cmax < 0) return -1;
    xo256 r; xo_seed(&r, seed);
    size_t nE = (size_t)(E > 0 ? E : 1);
    uint64_t *row = (uint64_t *)malloc(sizeof(uint64_t) * nE);
    uint64_t *idx = (uint64_t *)malloc(sizeof(uint64_t) * nE);
    int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * nE);
    int32_t *cp = (int32_t *)malloc(sizeof(int32_t) * nE);
    if (!row || !idx || !dst || !cp) { free(row); free(idx); free(dst); free(cp); return -1; }
    for (int64_t i = 0; i < E; i++) {
        row[i] = xo_below(&r, (uint64_t)V);
        dst[i] = (int32_t)xo_below(&r, (uint64_t)V);
        cp[i] = (int32_t)xo_below(&r, (uint64_t)cmax + 1);
        idx[i] = (uint64_t)i;
    }
    /* group by source row (stable: generation order kept inside a row) */
    if (radix_sort_kv(row, idx, E, bits_for((uint64_t)V)) || alloc_graph(g, V, E)) {
        free(row); free(idx); free(dst); free(cp); wbgen_free(g); return -1;
    }
    for (int64_t i = 0; i < E; i++) {
        g->col[i] = dst[idx[i]];
        g->cap[i] = cp[idx[i]];
        g->rp[row[i] + 1]++;
    }
    for (int32_t v = 0; v < V; v++) g->rp[v + 1] += g->rp[v];
    free(row); free(idx); free(dst); free(cp);
    g->s = 0; g->t = V - 1;
    return 0;
}

/* ------------------------------------------------- bipartite (Zipf right) */
/* L left + R right vertices; `narcs` left->right arcs with the left end
 * uniform and the right end drawn by inverse CDF from Zipf(expo) over ranks
 * 1..R (rank k is vertex L+k-1); super-source s = L+R feeds every left
 * vertex, every right vertex feeds super-sink t = L+R+1; all caps 1.
 * Parallel left->right arcs are kept (multigraph).  Rows sorted by column,
 * parallel arcs in sampling order. */
int wbgen_bipartite(int32_t L, int32_t R, int64_t narcs, double expo, uint64_t seed, wbgen_graph *g) {
    memset(g, 0, sizeof(*g));
    if (L < 1 || R < 1 || narcs < 0) return -1;
    xo256 r; xo_seed(&r, seed);
    double *cdf = (double *)malloc(sizeof(double) * (size_t)R);
    if (!cdf) return -1;
    double acc = 0.0;
    for (int32_t k = 1; k <= R; k++) { acc += pow((double)k, -expo); cdf[k - 1] = acc; }
    for (int32_t k = 0; k < R; k++) cdf[k] /= acc;
    int32_t V = L + R + 2;
    int vb = bits_for((uint64_t)V);
    int64_t E = narcs + L + R;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)E);
    uint64_t *ord = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)E);
    if (!keys || !ord) { free(cdf); free(keys); free(ord); return -1; }
    int64_t n = 0;
    for (int64_t i = 0; i < narcs; i++) {
        uint64_t u = xo_below(&r, (uint64_t)L);
        double x = xo_unit(&r);
        int32_t lo = 0, hi = R - 1;            /* first k with cdf[k] > x */
        while (lo < hi) { int32_t mid = lo + (hi - lo) / 2; if (cdf[mid] > x) hi = mid; else lo = mid + 1; }
        uint64_t v = (uint64_t)L + (uint64_t)lo;
        keys[n++] = (u << vb) | v;
    }
    uint64_t s = (uint64_t)(L + R), t = (uint64_t)(L + R + 1);
    for (int32_t u = 0; u < L; u++) keys[n++] = (s << vb) | (uint64_t)u;
    for (int32_t v = 0; v < R; v++) keys[n++] = ((uint64_t)(L + v) << vb) | t;
    for (int64_t i = 0; i < E; i++) ord[i] = (uint64_t)i;
    free(cdf);
    if (radix_sort_kv(keys, ord, E, 2 * vb)) { free(keys); free(ord); return -1; }
    free(ord);
    if (alloc_graph(g, V, E)) { free(keys); wbgen_free(g); return -1; }
    fill_csr_from_sorted(g, keys, vb);
    free(keys);
    for (int64_t i = 0; i < E; i++) g->cap[i] = 1;
    g->s = (int32_t)s; g->t = (int32_t)t;
    return 0;
}

/* ------------------------------------------------------------ R-MAT */
/* 2^scale vertices, ef * 2^scale samples; each sample takes `scale`
 * quadrant draws with probabilities (a, b, c, 1-a-b-c), most significant
 * bit first.  Vertex ids are then relabelled by a seeded Fisher-Yates
 * permutation; self-loops and duplicate arcs are dropped; caps uniform in
 * [cmin, cmax] in CSR order.  s = argmax out-degree, t = argmax in-degree
 * over v != s (ties: smallest id). */
int wbgen_rmat(int scale, int ef, double a, double b, double c, int32_t cmin, int32_t cmax,
               uint64_t seed, wbgen_graph *g) {
    memset(g, 0, sizeof(*g));
    if (scale < 1 || scale > 30 || ef < 1) return -1;
    xo256 r; xo_seed(&r, seed);
    int64_t n = (int64_t)1 << scale;
    int64_t ns = (int64_t)ef * n;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)ns);
    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    if (!keys || !perm) { free(keys); free(perm); return -1; }
    double ab = a + b, abc = a + b + c;
    for (int64_t i = 0; i < ns; i++) {
        uint64_t u = 0, v = 0;
        for (int l = 0; l < scale; l++) {
            double x = xo_unit(&r);
            uint64_t bu, bv;
            if (x < a) { bu = 0; bv = 0; }
            else if (x < ab) { bu = 0; bv = 1; }
            else if (x < abc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu; v = (v << 1) | bv;
        }
        keys[i] = (u << 32) | v;
    }
    for (int64_t i = 0; i < n; i++) perm[i] = (uint32_t)i;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)xo_below(&r, (uint64_t)(i + 1));
        uint32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    }
    int64_t m = 0;
    for (int64_t i = 0; i < ns; i++) {
        uint64_t u = perm[keys[i] >> 32], v = perm[keys[i] & 0xffffffffULL];
        if (u == v) continue;
        keys[m++] = (u << scale) | v;
    }
    free(perm);
    if (radix_sort_kv(keys, NULL, m, 2 * scale)) { free(keys); return -1; }
    int64_t E = 0;
    for (int64_t i = 0; i < m; i++) if (i == 0 || keys[i] != keys[i - 1]) keys[E++] = keys[i];
    if (alloc_graph(g, (int32_t)n, E)) { free(keys); wbgen_free(g); return -1; }
    fill_csr_from_sorted(g, keys, scale);
    int64_t *indeg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!indeg) { free(keys); wbgen_free(g); return -1; }
    for (int64_t i = 0; i < E; i++) indeg[g->col[i]]++;
    free(keys);
    uint64_t span = (uint64_t)((int64_t)cmax - cmin + 1);
    for (int64_t i = 0; i < E; i++) g->cap[i] = (int32_t)(cmin + (int64_t)xo_below(&r, span));
    int32_t s = 0; int64_t best = -1;
    for (int32_t v = 0; v < (int32_t)n; v++) { int64_t d = g->rp[v + 1] - g->rp[v]; if (d > best) { best = d; s = v; } }
    int32_t t = -1; best = -1;
    for (int32_t v = 0; v < (int32_t)n; v++) { if (v == s) continue; if (indeg[v] > best) { best = indeg[v]; t = v; } }
    free(indeg);
    g->s = s; g->t = t;
    return 0;
}

/* ---------------------------------------------------------- grid cut */
/* W x H 4-connected pixel grid, pixel id y*W + x, s = W*H, t = W*H + 1.
 * U_p uniform on [0,1) per pixel (pixel order).  S = U smoothed by a
 * separable Gaussian (sigma_s px, radius 3, clamp-to-edge), min-max
 * normalised to [0,1].  n-link cap in both directions between 4-neighbours:
 * round(255 * exp(-((S_p - S_q)/sigma)^2)).  t-links: cap(s->p) =
 * floor(256 U_p) (uniform on 0..255), cap(p->t) = 255 - cap(s->p). */
int wbgen_grid(int32_t W, int32_t H, double sigma, double sigma_s, uint64_t seed, wbgen_graph *g) {
    memset(g, 0, sizeof(*g));
    if (W < 1 || H < 1) return -1;
    xo256 r; xo_seed(&r, seed);
    int64_t P = (int64_t)W * H;
    double *U = (double *)malloc(sizeof(double) * (size_t)P);
    double *T = (double *)malloc(sizeof(double) * (size_t)P);
    double *S = (double *)malloc(sizeof(double) * (size_t)P);
    if (!U || !T || !S) { free(U); free(T); free(S); return -1; }
    for (int64_t p = 0; p < P; p++) U[p] = xo_unit(&r);
    const int RAD = 3;
    double w[2 * RAD + 1], ws = 0.0;
    for (int i = -RAD; i <= RAD; i++) { w[i + RAD] = exp(-(double)(i * i) / (2.0 * sigma_s * sigma_s)); ws += w[i + RAD]; }
    for (int i = 0; i <= 2 * RAD; i++) w[i] /= ws;
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            double acc = 0.0;
            for (int i = -RAD; i <= RAD; i++) {
                int32_t xx = x + i; if (xx < 0) xx = 0; if (xx >= W) xx = W - 1;
                acc += w[i + RAD] * U[(int64_t)y * W + xx];
            }
            T[(int64_t)y * W + x] = acc;
        }
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            double acc = 0.0;
            for (int i = -RAD; i <= RAD; i++) {
                int32_t yy = y + i; if (yy < 0) yy = 0; if (yy >= H) yy = H - 1;
                acc += w[i + RAD] * T[(int64_t)yy * W + x];
            }
            S[(int64_t)y * W + x] = acc;
        }
    double mn = S[0], mx = S[0];
    for (int64_t p = 1; p < P; p++) { if (S[p] < mn) mn = S[p]; if (S[p] > mx) mx = S[p]; }
    double rng = mx - mn;
    for (int64_t p = 0; p < P; p++) S[p] = rng > 0 ? (S[p] - mn) / rng : 0.0;
    free(T);
    int32_t V = (int32_t)(P + 2);
    int32_t s = (int32_t)P, t = (int32_t)(P + 1);
    int64_t nl = 2 * ((int64_t)(W - 1) * H + (int64_t)W * (H - 1));
    int64_t E = nl + 2 * P;
    if (alloc_graph(g, V, E)) { free(U); free(S); wbgen_free(g); return -1; }
    int64_t k = 0;
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int64_t p = (int64_t)y * W + x;
            g->rp[p] = k;
            int64_t nb[4]; int nn = 0;
            if (y > 0) nb[nn++] = p - W;
            if (x > 0) nb[nn++] = p - 1;
            if (x < W - 1) nb[nn++] = p + 1;
            if (y < H - 1) nb[nn++] = p + W;
            for (int i = 0; i < nn; i++) {
                double d = (S[p] - S[nb[i]]) / sigma;
                g->col[k] = (int32_t)nb[i];
                g->cap[k] = (int32_t)lround(255.0 * exp(-d * d));
                k++;
            }
            int32_t cs = (int32_t)floor(256.0 * U[p]);
            if (cs > 255) cs = 255;
            g->col[k] = t; g->cap[k] = 255 - cs; k++;
        }
    g->rp[s] = k;
    for (int64_t p = 0; p < P; p++) {
        int32_t cs = (int32_t)floor(256.0 * U[p]);
        if (cs > 255) cs = 255;
        g->col[k] = (int32_t)p; g->cap[k] = cs; k++;
    }
    g->rp[t] = k;
    g->rp[t + 1] = k;
    free(U); free(S);
    g->s = s; g->t = t;
    return (k == E) ? 0 : -1;
}

/* ----------------------------------------------------- batch instance */
/* Instance i of the batched stream: its own stream seeded with `seed`;
 * V = floor(vmin * (vmax/vmin)^u) (log-uniform), deg*V distinct uniform
 * arcs, caps uniform on [cmin, cmax], s = 0, t = V-1. */
int wbgen_batch_instance(int32_t vmin, int32_t vmax, int32_t deg, int32_t cmin, int32_t cmax,
                         uint64_t seed, wbgen_graph *g) {
    memset(g, 0, sizeof(*g));
    if (vmin < 2 || vmax < vmin) return -1;
    xo256 r; xo_seed(&r, seed);
    double u = xo_unit(&r);
    int32_t V = (int32_t)floor((double)vmin * pow((double)vmax / (double)vmin, u));
    if (V < vmin) V = vmin;
    if (V > vmax) V = vmax;
    int64_t E = (int64_t)deg * V;
    int64_t maxe = (int64_t)V * (V - 1);
    if (E > maxe) E = maxe;
    if (gen_distinct_uniform(&r, V, E, cmin, cmax, g)) { wbgen_free(g); return -1; }
    g->s = 0; g->t = V - 1;
    return 0;
}
