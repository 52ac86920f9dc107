/*
 * Seeded synthetic graph generators.
 *
 * This module holds no arithmetic of the sparsification method. It produces
 * the inputs that both the GPU library and the CPU oracle consume: weighted,
 * undirected, connected graphs as a canonical edge list (u < v, sorted by
 * (u, v), no duplicates; edge id = position), int32 node ids and FP64 weights.
 *
 * Draw order (fixed, so a seed names exactly one graph):
 *   1. topology draws (random families only), in the order documented per family;
 *   2. the edge list is canonicalised (sorted, de-duplicated);
 *   3. one weight per edge, drawn in canonical edge order.
 * All draws come from one xoshiro256** stream seeded through splitmix64(seed).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- RNG --- */
typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t res = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return res;
}
/* uniform in [0,1) with 53 random bits */
static double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
/* uniform integer in [0, n) (n > 0), multiply-shift with rejection (unbiased) */
static uint64_t rng_below(rng_t *r, uint64_t n) {
    uint64_t lim = (uint64_t)(-n) % n;
    for (;;) {
        uint64_t x = rng_next(r);
        __uint128_t p = (__uint128_t)x * n;
        if ((uint64_t)p >= lim) return (uint64_t)(p >> 64);
    }
}
static double rng_normal(rng_t *r) {
    /* Box-Muller, one value per call (the second is discarded). */
    double u1 = ((double)(rng_next(r) >> 11) + 0.5) * 0x1.0p-53;
    double u2 = rng_u01(r);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

/* ------------------------------------------------------- edge buffers --- */
typedef struct { int64_t n, m, cap; uint64_t *key; } ebuf_t; /* key = u<<32 | v, u<v */

static int eb_init(ebuf_t *b, int64_t cap) {
    b->n = 0; b->m = 0; b->cap = cap > 16 ? cap : 16;
    b->key = (uint64_t *)malloc((size_t)b->cap * sizeof(uint64_t));
    return b->key ? 0 : -1;
}
static int eb_push(ebuf_t *b, int64_t u, int64_t v) {
    if (u == v) return 0;
    if (u > v) { int64_t t = u; u = v; v = t; }
    if (b->m == b->cap) {
        int64_t nc = b->cap * 2;
        uint64_t *k = (uint64_t *)realloc(b->key, (size_t)nc * sizeof(uint64_t));
        if (!k) return -1;
        b->key = k; b->cap = nc;
    }
    b->key[b->m++] = ((uint64_t)u << 32) | (uint64_t)v;
    return 0;
}
static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}
/* sort + unique, in place */
static void eb_canon(ebuf_t *b) {
    if (b->m == 0) return;
    qsort(b->key, (size_t)b->m, sizeof(uint64_t), cmp_u64);
    int64_t w = 1;
    for (int64_t i = 1; i < b->m; i++)
        if (b->key[i] != b->key[w - 1]) b->key[w++] = b->key[i];
    b->m = w;
}

/* weight distributions */
enum { W_UNIFORM = 0, W_LOGUNIFORM10 = 1, W_LOGNORMAL = 2, W_CONST = 3 };
static double draw_w(rng_t *r, int kind, double a, double b) {
    switch (kind) {
    case W_UNIFORM: return a + (b - a) * rng_u01(r);               /* U[a,b) */
    case W_LOGUNIFORM10: return pow(10.0, a + (b - a) * rng_u01(r)); /* 10^U(a,b) */
    case W_LOGNORMAL: return exp(a + b * rng_normal(r));            /* exp(N(a, b^2)) */
    default: return a;                                              /* constant a */
    }
}

/* Output handed to the caller (freed with gen_free). */
typedef struct {
    int64_t n, m;
    int32_t *src, *dst;
    double *w;
} gen_graph;

static int finish(ebuf_t *b, int64_t n, rng_t *r, int wkind, double wa, double wb, gen_graph *out) {
    eb_canon(b);
    out->n = n; out->m = b->m;
    size_t mm = (size_t)(b->m > 0 ? b->m : 1);
    out->src = (int32_t *)malloc(mm * sizeof(int32_t));
    out->dst = (int32_t *)malloc(mm * sizeof(int32_t));
    out->w = (double *)malloc(mm * sizeof(double));
    if (!out->src || !out->dst || !out->w) { free(b->key); return -1; }
    for (int64_t e = 0; e < b->m; e++) {
        out->src[e] = (int32_t)(b->key[e] >> 32);
        out->dst[e] = (int32_t)(b->key[e] & 0xffffffffu);
        out->w[e] = draw_w(r, wkind, wa, wb);
    }
    free(b->key);
    return 0;
}

void gen_free(gen_graph *g) {
    if (!g) return;
    free(g->src); free(g->dst); free(g->w);
    g->src = g->dst = NULL; g->w = NULL;
}

/* 2-D 4-neighbour grid, node id = y*nx + x. */
int gen_grid2d(int64_t nx, int64_t ny, int wkind, double wa, double wb, uint64_t seed, gen_graph *out) {
    if (nx < 1 || ny < 1 || nx * ny > (1ll << 31) - 1) return -1;
    rng_t r; rng_seed(&r, seed);
    ebuf_t b; if (eb_init(&b, 2 * nx * ny)) return -1;
    for (int64_t y = 0; y < ny; y++)
        for (int64_t x = 0; x < nx; x++) {
            int64_t v = y * nx + x;
            if (x + 1 < nx) eb_push(&b, v, v + 1);
            if (y + 1 < ny) eb_push(&b, v, v + nx);
        }
    return finish(&b, nx * ny, &r, wkind, wa, wb, out);
}

/* 3-D 7-point mesh, node id = (z*ny + y)*nx + x. */
int gen_mesh3d(int64_t nx, int64_t ny, int64_t nz, int wkind, double wa, double wb, uint64_t seed, gen_graph *out) {
    if (nx < 1 || ny < 1 || nz < 1 || nx * ny * nz > (1ll << 31) - 1) return -1;
    rng_t r; rng_seed(&r, seed);
    ebuf_t b; if (eb_init(&b, 3 * nx * ny * nz)) return -1;
    for (int64_t z = 0; z < nz; z++)
        for (int64_t y = 0; y < ny; y++)
            for (int64_t x = 0; x < nx; x++) {
                int64_t v = (z * ny + y) * nx + x;
                if (x + 1 < nx) eb_push(&b, v, v + 1);
                if (y + 1 < ny) eb_push(&b, v, v + nx);
                if (z + 1 < nz) eb_push(&b, v, v + nx * ny);
            }
    return finish(&b, nx * ny * nz, &r, wkind, wa, wb, out);
}

/*
 * Power-grid-like circuit: side x side 4-neighbour grid plus
 * floor(frac * grid_edges) long-range edges. Topology draws, repeated until the
 * target count of distinct new edges is reached: u uniform over nodes, then
 * (dx, dy) uniform over the integer L1 ball of radius maxhops (rejection from the
 * square), rejected if |dx|+|dy| < 2, if u+(dx,dy) leaves the grid, or if the pair
 * was already drawn.
 */
int gen_grid2d_longrange(int64_t side, double frac, int64_t maxhops, int wkind, double wa, double wb,
                         uint64_t seed, gen_graph *out) {
    if (side < 2 || side * side > (1ll << 31) - 1 || maxhops < 2) return -1;
    rng_t r; rng_seed(&r, seed);
    int64_t n = side * side;
    int64_t mgrid = 2 * side * (side - 1);
    int64_t target = (int64_t)floor(frac * (double)mgrid);
    ebuf_t lr; if (eb_init(&lr, target + 16)) return -1;
    int64_t have = 0;
    while (have < target) {
        int64_t need = target - have;
        for (int64_t i = 0; i < need; i++) {
            for (;;) {
                int64_t u = (int64_t)rng_below(&r, (uint64_t)n);
                int64_t dx = (int64_t)rng_below(&r, (uint64_t)(2 * maxhops + 1)) - maxhops;
                int64_t dy = (int64_t)rng_below(&r, (uint64_t)(2 * maxhops + 1)) - maxhops;
                int64_t d = llabs(dx) + llabs(dy);
                if (d < 2 || d > maxhops) continue;
                int64_t ux = u % side, uy = u / side;
                int64_t vx = ux + dx, vy = uy + dy;
                if (vx < 0 || vx >= side || vy < 0 || vy >= side) continue;
                eb_push(&lr, u, vy * side + vx);
                break;
            }
        }
        eb_canon(&lr);
        have = lr.m;
    }
    ebuf_t b; if (eb_init(&b, mgrid + target)) { free(lr.key); return -1; }
    for (int64_t y = 0; y < side; y++)
        for (int64_t x = 0; x < side; x++) {
            int64_t v = y * side + x;
            if (x + 1 < side) eb_push(&b, v, v + 1);
            if (y + 1 < side) eb_push(&b, v, v + side);
        }
    for (int64_t i = 0; i < lr.m; i++) eb_push(&b, (int64_t)(lr.key[i] >> 32), (int64_t)(lr.key[i] & 0xffffffffu));
    free(lr.key);
    return finish(&b, n, &r, wkind, wa, wb, out);
}

/* union-find helpers (generator-local) */
static int64_t uf_find(int64_t *p, int64_t x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
}

/*
 * Random geometric graph: n0 uniform points in the unit square (x then y per
 * point), edge between points closer than r = sqrt(avgdeg / (pi * n0)); keep the
 * largest connected component (ties: the one holding the smallest point index),
 * renumbered in increasing original index.
 */
int gen_rgg(int64_t n0, double avgdeg, int wkind, double wa, double wb, uint64_t seed, gen_graph *out) {
    if (n0 < 2 || n0 > (1ll << 31) - 1) return -1;
    rng_t r; rng_seed(&r, seed);
    double *px = (double *)malloc((size_t)n0 * sizeof(double));
    double *py = (double *)malloc((size_t)n0 * sizeof(double));
    for (int64_t i = 0; i < n0; i++) { px[i] = rng_u01(&r); py[i] = rng_u01(&r); }
    double rad = sqrt(avgdeg / (3.14159265358979323846 * (double)n0));
    int64_t g = (int64_t)floor(1.0 / rad); if (g < 1) g = 1; if (g > 65536) g = 65536;
    int64_t ncell = g * g;
    int64_t *head = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    int64_t *next = (int64_t *)malloc((size_t)n0 * sizeof(int64_t));
    for (int64_t c = 0; c < ncell; c++) head[c] = -1;
    for (int64_t i = n0 - 1; i >= 0; i--) {
        int64_t cx = (int64_t)(px[i] * g), cy = (int64_t)(py[i] * g);
        if (cx >= g) cx = g - 1; if (cy >= g) cy = g - 1;
        int64_t c = cy * g + cx; next[i] = head[c]; head[c] = i;
    }
    ebuf_t b; if (eb_init(&b, (int64_t)(avgdeg * n0 / 2) + 16)) return -1;
    double r2 = rad * rad;
    for (int64_t i = 0; i < n0; i++) {
        int64_t cx = (int64_t)(px[i] * g), cy = (int64_t)(py[i] * g);
        if (cx >= g) cx = g - 1; if (cy >= g) cy = g - 1;
        for (int64_t oy = -1; oy <= 1; oy++)
            for (int64_t ox = -1; ox <= 1; ox++) {
                int64_t qx = cx + ox, qy = cy + oy;
                if (qx < 0 || qy < 0 || qx >= g || qy >= g) continue;
                for (int64_t j = head[qy * g + qx]; j >= 0; j = next[j]) {
                    if (j <= i) continue;
                    double ddx = px[i] - px[j], ddy = py[i] - py[j];
                    if (ddx * ddx + ddy * ddy < r2) eb_push(&b, i, j);
                }
            }
    }
    free(head); free(next); free(px); free(py);
    /* largest component */
    int64_t *par = (int64_t *)malloc((size_t)n0 * sizeof(int64_t));
    for (int64_t i = 0; i < n0; i++) par[i] = i;
    for (int64_t e = 0; e < b.m; e++) {
        int64_t a = uf_find(par, (int64_t)(b.key[e] >> 32)), c = uf_find(par, (int64_t)(b.key[e] & 0xffffffffu));
        if (a != c) { if (a < c) par[c] = a; else par[a] = c; }
    }
    int64_t *cnt = (int64_t *)calloc((size_t)n0, sizeof(int64_t));
    for (int64_t i = 0; i < n0; i++) cnt[uf_find(par, i)]++;
    int64_t best = 0;
    for (int64_t i = 0; i < n0; i++) if (cnt[i] > cnt[best]) best = i;
    int64_t *newid = cnt; /* reuse */
    int64_t nn = 0;
    for (int64_t i = 0; i < n0; i++) newid[i] = (uf_find(par, i) == best) ? nn++ : -1;
    int64_t w = 0;
    for (int64_t e = 0; e < b.m; e++) {
        int64_t u = (int64_t)(b.key[e] >> 32), v = (int64_t)(b.key[e] & 0xffffffffu);
        if (newid[u] >= 0 && newid[v] >= 0) b.key[w++] = ((uint64_t)newid[u] << 32) | (uint64_t)newid[v];
    }
    b.m = w;
    free(par); free(cnt);
    return finish(&b, nn, &r, wkind, wa, wb, out);
}

/*
 * Barabasi-Albert preferential attachment: a seed clique on m0+1 nodes, then each
 * new node v attaches to m0 distinct earlier nodes, each drawn uniformly from the
 * list of all edge endpoints so far (probability proportional to degree); a
 * repeated target is redrawn.
 */
int gen_ba(int64_t n, int64_t m0, int wkind, double wa, double wb, uint64_t seed, gen_graph *out) {
    if (m0 < 1 || n < m0 + 2 || n > (1ll << 31) - 1) return -1;
    rng_t r; rng_seed(&r, seed);
    int64_t medges = (m0 + 1) * m0 / 2 + (n - m0 - 1) * m0;
    int64_t *ends = (int64_t *)malloc((size_t)(2 * medges) * sizeof(int64_t));
    ebuf_t b; if (!ends || eb_init(&b, medges)) return -1;
    int64_t ne = 0;
    for (int64_t u = 0; u <= m0; u++)
        for (int64_t v = u + 1; v <= m0; v++) { eb_push(&b, u, v); ends[ne++] = u; ends[ne++] = v; }
    int64_t *tgt = (int64_t *)malloc((size_t)m0 * sizeof(int64_t));
    for (int64_t v = m0 + 1; v < n; v++) {
        int64_t got = 0, lim = ne;
        while (got < m0) {
            int64_t t = ends[rng_below(&r, (uint64_t)lim)];
            int dup = 0;
            for (int64_t i = 0; i < got; i++) if (tgt[i] == t) { dup = 1; break; }
            if (!dup) tgt[got++] = t;
        }
        for (int64_t i = 0; i < m0; i++) { eb_push(&b, tgt[i], v); ends[ne++] = tgt[i]; ends[ne++] = v; }
    }
    free(tgt); free(ends);
    return finish(&b, n, &r, wkind, wa, wb, out);
}

/* Cycle 0-1-...-(n-1)-0. */
int gen_cycle(int64_t n, int wkind, double wa, double wb, uint64_t seed, gen_graph *out) {
    if (n < 3) return -1;
    rng_t r; rng_seed(&r, seed);
    ebuf_t b; if (eb_init(&b, n)) return -1;
    for (int64_t v = 0; v < n; v++) eb_push(&b, v, (v + 1) % n);
    return finish(&b, n, &r, wkind, wa, wb, out);
}

/* Complete graph K_n. */
int gen_complete(int64_t n, int wkind, double wa, double wb, uint64_t seed, gen_graph *out) {
    if (n < 2 || n > 4096) return -1;
    rng_t r; rng_seed(&r, seed);
    ebuf_t b; if (eb_init(&b, n * (n - 1) / 2)) return -1;
    for (int64_t u = 0; u < n; u++)
        for (int64_t v = u + 1; v < n; v++) eb_push(&b, u, v);
    return finish(&b, n, &r, wkind, wa, wb, out);
}

/*
 * Random connected graph for property tests: a random spanning tree (node v>0
 * joins a uniform earlier node) plus `extra` uniform random pairs (duplicates and
 * self-loops dropped by canonicalisation).
 */
int gen_random_connected(int64_t n, int64_t extra, int wkind, double wa, double wb, uint64_t seed, gen_graph *out) {
    if (n < 2 || n > (1ll << 31) - 1) return -1;
    rng_t r; rng_seed(&r, seed);
    ebuf_t b; if (eb_init(&b, n + extra)) return -1;
    for (int64_t v = 1; v < n; v++) eb_push(&b, (int64_t)rng_below(&r, (uint64_t)v), v);
    for (int64_t i = 0; i < extra; i++) {
        int64_t u = (int64_t)rng_below(&r, (uint64_t)n), v = (int64_t)rng_below(&r, (uint64_t)n);
        eb_push(&b, u, v);
    }
    return finish(&b, n, &r, wkind, wa, wb, out);
}
