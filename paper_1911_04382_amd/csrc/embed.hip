// Spectral off-tree edge embedding on gfx950 (Sec. III-F of the paper):
// Philox start vectors (eq. 28), Laplacian products (eq. 1), the grounded tree
// solve and PCG on L_P that realise the generalized power iteration (eq. 29),
// and the per-edge Joule heat with FP64 Rayleigh-quotient sums (eqs. 2, 31, 35,
// 55, 61). None of these steps is a dense contraction: every kernel is bound by
// HBM traffic (or latency), so the design work is coalescing, fusion and the
// block -> XCD mapping, not MFMA.
#include <type_traits>

#include "embed.h"
#include "gram.h"
#include "kern.h"
#include "lap.h"
#include "profiler.h"

namespace grass {

namespace {

constexpr int kGaussBlocksMax = 2048;
constexpr bool kLapNTStore = true;    // the 16-byte-lane product stores y non-temporally
constexpr int kScoreBlocksMax = 4096;  // scoring grid cap (each block then walks several rounds)

// ------------------------------------------------------------ start vectors
// Philox4x64-10 of Salmon et al. (SC'11); counter (v, j, pass, 0), key (seed, 0).
__device__ __forceinline__ double philox_gauss(unsigned long long v, unsigned long long j, unsigned long long pass,
                                               unsigned long long seed) {
    unsigned long long c0 = v, c1 = j, c2 = pass, c3 = 0, k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        unsigned long long lo0 = 0xD2E7470EE14C6C93ull * c0, hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0);
        unsigned long long lo1 = 0xCA5A826395121157ull * c2, hi1 = __umul64hi(0xCA5A826395121157ull, c2);
        unsigned long long n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    double ua = ((double)(c0 >> 11) + 0.5) * 0x1.0p-53;
    double ub = ((double)(c1 >> 11) + 0.5) * 0x1.0p-53;
    return sqrt(-2.0 * log(ua)) * cos(6.283185307179586476925286766559 * ub);
}

template <int KP>
__global__ __launch_bounds__(kThreads) void k_gauss_sum(long long n, int k, unsigned long long seed, int pass,
                                                        double *__restrict__ part) {
    constexpr int G = kThreads / KP;
    __shared__ double sh[G][KP];
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double s = 0.0;
    if (j < k)
        for (long long v = (long long)blockIdx.x * G + g; v < n; v += (long long)gridDim.x * G)
            s += philox_gauss(v, j, pass, seed);
    sh[g][j] = s;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int q = 0; q < G; q++) t += sh[q][j];
        part[(long long)blockIdx.x * KP + j] = t;
    }
}

// Column sums of per-block partials (part[b * stride + offset + j]) in a fixed
// order: 1024 threads, thread (g, j) adds blocks g, g + G, ... with four
// interleaved accumulators, then the groups are combined in order.
template <int KP>
__global__ __launch_bounds__(kColThreads) void k_col_sum(const double *__restrict__ part, int nblk, int stride,
                                                         int offset, double scale, double *__restrict__ out) {
    // block c reduces partial blocks [c * chunk, (c + 1) * chunk) into out[c * KP + j]
    constexpr int G = kColThreads / KP;
    __shared__ double sh[G][KP];
    int chunk = (nblk + gridDim.x - 1) / gridDim.x;
    int lo = blockIdx.x * chunk, hi = min(nblk, lo + chunk);
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = lo + g;
    for (; b + 3 * G < hi; b += 4 * G) {
        a0 += part[(long long)b * stride + offset + j];
        a1 += part[(long long)(b + G) * stride + offset + j];
        a2 += part[(long long)(b + 2 * G) * stride + offset + j];
        a3 += part[(long long)(b + 3 * G) * stride + offset + j];
    }
    for (; b < hi; b += G) a0 += part[(long long)b * stride + offset + j];
    sh[g][j] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    for (int w = G / 2; w > 0; w >>= 1) {
        if (g < w) sh[g][j] += sh[g + w][j];
        __syncthreads();
    }
    if (g == 0) out[(long long)blockIdx.x * KP + j] = sh[0][j] * scale;
}

template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_gauss_write(long long n, int k, unsigned long long seed, int pass,
                                                          const double *__restrict__ mean, T *__restrict__ out) {
    constexpr int G = kThreads / KP;
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    if (j >= k) return;
    double mu = mean[j];
    for (long long v = (long long)blockIdx.x * G + g; v < n; v += (long long)gridDim.x * G)
        out[v * k + j] = (T)(philox_gauss(v, j, pass, seed) - mu);
}

// ------------------------------------------------------------ Laplacian
template <typename T, int KP, int E>
__global__ __launch_bounds__(kThreads) void k_lap(long long n, int k, const int *__restrict__ rowptr,
                                                  const int *__restrict__ col, const T *__restrict__ val,
                                                  const T *__restrict__ ltail, const int *__restrict__ ecol,
                                                  const T *__restrict__ eval, const int *__restrict__ edeg,
                                                  const T *__restrict__ x,
                                                  T *__restrict__ y, int root,
                                                  const unsigned long long *__restrict__ scale_from,
                                                  double *__restrict__ dot_part, int nblk) {
    constexpr int G = kThreads / KP;
    constexpr int NIT = LapShape<KP>::NIT;
    constexpr int RPB = G * NIT;
    __shared__ __align__(16) char lds[(kThreads / 64) * LapTile<T, KP, E>::SLICE];
    int b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= nblk) return;
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    T xo[NIT], yo[NIT];
    lap_tile<T, KP, E>((long long)b * RPB, n, k, rowptr, col, val, ltail, ecol, eval, edeg, x, y, root,
                       (T)pow2_scale(scale_from), lds, xo, yo);
    if (dot_part) {
        double dacc = 0.0;
#pragma unroll
        for (int it = 0; it < NIT; it++) dacc += (double)xo[it] * (double)yo[it];
        __shared__ double sh[G][KP];
        sh[g][j] = dacc;
        __syncthreads();
        if (g == 0) {
            double t = 0.0;
            for (int q = 0; q < G; q++) t += sh[q][j];
            dot_part[(long long)b * KP + j] = t;
        }
    }
}

// ------------------------------------------------------------ tree solve
// A tile with more extra light-child entries (third and later per node) than
// kHubEntries, or a node with more than kHubPerNode of them, sums them in parallel
// rounds; otherwise each node's lane group walks its own (two dependent loads each)
constexpr int kHubEntries = 32, kHubPerNode = 2;

// Tagged words: a 32-bit payload and a 32-bit tag in one 64-bit agent-scope atomic,
// so a reader that sees the tag it waits for also holds the data (no separate
// flag, no store-completion wait on the writer). A double takes two words.
template <typename T>
__device__ __forceinline__ void tag_put(unsigned long long *p, T v, unsigned tag) {
    const unsigned long long t = (unsigned long long)tag << 32;
    if constexpr (sizeof(T) == 4) {
        st_agent_u64(p, t | __float_as_uint(v));
    } else {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        st_agent_u64(p, t | (b & 0xffffffffull));
        st_agent_u64(p + 1, t | (b >> 32));
    }
}
// bounded spin until every word of the value carries `epoch` (tag >> 1); false on
// time-out
template <typename T>
__device__ __forceinline__ bool tag_get(const unsigned long long *p, unsigned epoch, T &v, unsigned &tag) {
    long long spin = 0;
    while (true) {
        const unsigned long long w0 = ld_agent_u64(p);
        const unsigned long long w1 = sizeof(T) == 8 ? ld_agent_u64(p + 1) : w0;
        if ((unsigned)(w0 >> 33) == (epoch & 0x7fffffffu) && (unsigned)(w1 >> 33) == (epoch & 0x7fffffffu)) {
            tag = (unsigned)(w0 >> 32);
            if constexpr (sizeof(T) == 4)
                v = __uint_as_float((unsigned)w0);
            else
                v = __longlong_as_double((long long)((w1 << 32) | (w0 & 0xffffffffull)));
            return true;
        }
        if (++spin > kSpinLimit) return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

// One sweep of the grounded tree solve over the heavy-light layout, all levels in
// one launch. Paths are contiguous segments of the layout (top to bottom):
//   UP   (reverse scan, segments start at path bottoms):
//        f[i] = y[perm i] + sum_{light children c} f[c] + f[i+1]   (subtree currents)
//   DOWN (forward scan, segments start at path tops):
//        x[perm i] = x[parent of top] + sum_{top..i} f / pw        (potentials)
// Tiles take an atomic ticket in processing order (UP: deepest level first,
// tiles in reverse; DOWN: root level first). A tile first waits for the tiles
// it depends on in other levels (precomputed lists: the tiles of its light
// children, or of its paths' parents), then scans, publishes its aggregate as
// tagged words (tag: sweep epoch and whether the tile holds a segment start),
// looks back within its level to the nearest tile holding a segment start (adding
// aggregates in a fixed order, so results never depend on timing), writes its
// outputs and stamps itself done. Every awaited tile holds a smaller ticket, so
// it is already running; every wait is bounded. Data another tile reads inside
// the same launch moves through agent-scope (XCD-coherent) loads and stores.
template <typename T, int KP, bool UP, bool HUB, bool GRAM>
__device__ __forceinline__ void sweep_tile(
    int tk, int nlev, const int *__restrict__ lvl_tile, int k, const int *__restrict__ perm,
    const uint8_t *__restrict__ flags,
    const int *__restrict__ ptop, const int *__restrict__ lc_ptr, const int *__restrict__ lc_pos,
    const int *__restrict__ lc_owner,
    const T *__restrict__ rpw, const T *__restrict__ yin, T *__restrict__ F, T *__restrict__ xout,
    unsigned long long *__restrict__ aggw, unsigned *__restrict__ done,
    const unsigned *__restrict__ epoch_ptr, const int *__restrict__ dep_ptr, const int *__restrict__ dep,
    int *__restrict__ ticket, unsigned *__restrict__ devflags, const T *__restrict__ rdot,
    double *__restrict__ dot_part, unsigned long long *__restrict__ absmax, int ntiles_total,
    const T *__restrict__ qz_q, double *__restrict__ qz_part, int *__restrict__ qz_cnt, double *__restrict__ qz_out,
    const double *__restrict__ beta_ginv, T *__restrict__ beta_out) {
    constexpr int RUNS = kSolveThreads / KP;
    constexpr int NPR = solve_npr(KP);
    constexpr int TN = RUNS * NPR;
    __shared__ int s_info[3];  // level's first tile, level's tile count, logical tile
    __shared__ T s_agg[RUNS][KP];
    __shared__ int s_hs[RUNS];
    __shared__ T s_excl[RUNS][KP];
    __shared__ int s_exhs[RUNS];
    __shared__ T s_carry[KP];
    __shared__ double s_red[RUNS][KP];
    __shared__ double s_max[kSolveThreads / 64];
    // per-position layout data, shared by the KP lanes of a run (index: scan order)
    __shared__ uint8_t s_fl[TN];
    __shared__ int s_vid[TN];  // node id (-1: padding)
    __shared__ int s_l0[TN];   // UP: first light child's position; DOWN: parent of a path top (-1: none)
    __shared__ int s_l1[TN];   // UP: second light child's position (-1: none)
    __shared__ int s_lcr[TN];  // UP: index in lc_pos of the third light child (rare), or -1
    __shared__ int s_lce[TN];
    __shared__ T s_rw[TN];     // DOWN: 1/parent weight
    // UP, tiles whose nodes have many light children (hubs): the tile's light-child
    // entries go through LDS in rounds of CH, all runs loading at once
    constexpr int HU = sizeof(T) == 4 ? 16 : 8, CH = RUNS * HU;
    __shared__ T s_ev[UP && HUB ? CH : 1][KP];  // per run: partial sums of its owner segments
    __shared__ int s_eo[UP && HUB ? CH : 1];    // owner (scan index) of each partial
    __shared__ int s_en[UP && HUB ? RUNS : 1];  // partials per run
    __shared__ int s_ex[4];  // UP: extra entries (third and later light children), tile's entry range, max per node

    const int tid = threadIdx.x;
    const int j = tid % KP, r = tid / KP;
    const unsigned epoch = epoch_ptr[0] + (UP ? 0u : 1u);
    if (tid == 0) {
        int acc = 0;
        s_ex[0] = 0;
        s_ex[3] = 0;
        s_info[0] = 0;
        s_info[1] = 1;
        s_info[2] = 0;
        for (int q = 0; q < nlev; q++) {
            int l = UP ? (nlev - 1 - q) : q;
            int f0 = lvl_tile[l], nt = lvl_tile[l + 1] - f0;
            if (tk < acc + nt) {
                int i = tk - acc;
                s_info[0] = f0;
                s_info[1] = nt;
                s_info[2] = UP ? (nt - 1 - i) : i;
                break;
            }
            acc += nt;
        }
    }
    __syncthreads();
    const int lvl_first = s_info[0], ntiles = s_info[1], lt = s_info[2];
    const long long gt = (long long)lvl_first + lt;
    const long long p0 = gt * TN;
    const bool act = j < k;

    // Everything that does not depend on other tiles is loaded first, so that the
    // critical path through the levels keeps a single memory hop per tile. The
    // layout data goes to LDS once per position (coalesced, unconditional loads
    // with clamped indices); each thread keeps only its column's values.
    T vals[NPR];
    const int d0 = dep_ptr[gt], d1 = dep_ptr[gt + 1];
    const int dep_first = dep[d0 + tid < d1 ? d0 + tid : 0];
    if (!UP) {
#pragma unroll
        for (int q = 0; q < NPR; q++) {
            const long long pos = p0 + r * NPR + q;
            const T f = F[act ? pos * k + j : 0];
            vals[q] = act ? f : (T)0;
        }
    }
    for (int i = tid; i < TN; i += kSolveThreads) {
        const long long pos = p0 + (UP ? (TN - 1 - i) : i);
        const uint8_t fl = flags[pos];
        s_fl[i] = fl;
        s_vid[i] = perm[pos];
        if (UP) {
            const int c0 = lc_ptr[pos], c1 = lc_ptr[pos + 1];
            const int l0 = lc_pos[c1 > c0 ? c0 : 0];
            const int l1 = lc_pos[c1 > c0 + 1 ? c0 + 1 : 0];
            s_l0[i] = c1 > c0 ? l0 : -1;
            s_l1[i] = c1 > c0 + 1 ? l1 : -1;
            s_lcr[i] = c1 > c0 + 2 ? c0 + 2 : -1;
            s_lce[i] = c1;
            if (c1 > c0 + 2) {
                atomicAdd(&s_ex[0], c1 - c0 - 2);
                atomicMax(&s_ex[3], c1 - c0 - 2);
            }
            if (i == TN - 1) s_ex[1] = c0;  // pos == p0
            if (i == 0) s_ex[2] = c1;       // pos == p0 + TN - 1
        } else {
            const int pt = ptop[pos];
            s_l0[i] = (fl & SEG_TOP) ? pt : -1;
            s_rw[i] = rpw[pos];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NPR; q++) {
        const int sidx = r * NPR + q;
        if (UP) {
            const int v = s_vid[sidx];
            const bool okv = act && v >= 0;
            const T y = yin[okv ? (long long)v * k + j : 0];
            vals[q] = okv ? y : (T)0;
        } else {
            vals[q] = vals[q] * s_rw[sidx];
        }
    }

    // cross-level dependencies (tiles of light children / of path parents)
    {
        int bad = 0;
        for (int d = d0 + tid; d < d1; d += kSolveThreads) {
            const unsigned *f = &done[d == d0 + tid ? dep_first : dep[d]];
            long long spin = 0;
            while (ld_agent_u32(f) != epoch) {
                if (++spin > kSpinLimit) {
                    bad = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (bad) atomicOr(devflags, DEVERR_SPIN);
    }
    __syncthreads();

    // the single dependent hop (all of a thread's loads in flight together:
    // clamped indices, then selects), then the run-local inclusive segmented scan
    {
        T h0[NPR], h1[NPR];
#pragma unroll
        for (int q = 0; q < NPR; q++) {
            const int sidx = r * NPR + q;
            const int l0 = s_l0[sidx], l1 = UP ? s_l1[sidx] : -1;
            const bool ok0 = act && l0 >= 0, ok1 = UP && act && l1 >= 0;
            const T a = ld_agent(UP ? &F[ok0 ? (long long)l0 * k + j : 0] : &xout[ok0 ? (long long)l0 * k + j : 0]);
            const T b = UP ? ld_agent(&F[ok1 ? (long long)l1 * k + j : 0]) : (T)0;
            h0[q] = ok0 ? a : (T)0;
            h1[q] = ok1 ? b : (T)0;
        }
#pragma unroll
        for (int q = 0; q < NPR; q++) {
            vals[q] += h0[q];
            vals[q] += h1[q];
        }
    }
    // many extra light children in this tile: per round every run loads HU entries of
    // the tile's (contiguous) light-child range, sums them per owner segment in
    // registers and leaves one partial per segment in LDS; each node's owner then
    // adds one partial per run its entries span (the last segment of the first run,
    // the first of the later ones). Fixed order: entries within a run, runs, rounds.
    const bool hub = UP && HUB && (s_ex[0] > kHubEntries || s_ex[3] > kHubPerNode);
    if (hub) {
        const int ea = s_ex[1], eb = s_ex[2];
        for (int base = ea; base < eb; base += CH) {
            int ch[HU], ow[HU];
#pragma unroll
            for (int u = 0; u < HU; u++) {
                const int e = base + r * HU + u;
                ch[u] = lc_pos[e < eb ? e : ea];
                ow[u] = lc_owner[e < eb ? e : ea];
            }
            T fv[HU];
#pragma unroll
            for (int u = 0; u < HU; u++) fv[u] = ld_agent(&F[act ? (long long)ch[u] * k + j : 0]);
            int nseg = 0, cur = -1;
            T acc = 0;
#pragma unroll
            for (int u = 0; u < HU; u++) {
                const int e = base + r * HU + u;
                // scan index of the owner (UP scans positions in reverse); -1 past the range
                const int os = e < eb ? (int)(p0 + TN - 1 - ow[u]) : -1;
                const int lr = os >= 0 ? s_lcr[os] : -1;
                const T x = (lr >= 0 && e >= lr) ? fv[u] : (T)0;
                if (u > 0 && os != cur) {
                    s_ev[r * HU + nseg][j] = acc;
                    if (j == 0) s_eo[r * HU + nseg] = cur;
                    nseg++;
                    acc = 0;
                }
                cur = os;
                acc += x;
            }
            s_ev[r * HU + nseg][j] = acc;
            if (j == 0) {
                s_eo[r * HU + nseg] = cur;
                s_en[r] = nseg + 1;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < NPR; q++) {
                const int sidx = r * NPR + q;
                const int lr = s_lcr[sidx];
                if (lr >= 0) {
                    const int lo = lr > base ? lr : base, hi = s_lce[sidx] < base + CH ? s_lce[sidx] : base + CH;
                    if (lo < hi) {
                        const int ra = (lo - base) / HU, rb = (hi - 1 - base) / HU;
                        if (ra == rb) {
                            for (int sl = 0; sl < s_en[ra]; sl++)
                                if (s_eo[ra * HU + sl] == sidx) vals[q] += s_ev[ra * HU + sl][j];
                        } else {
                            vals[q] += s_ev[ra * HU + s_en[ra] - 1][j];
                            for (int rr = ra + 1; rr <= rb; rr++) vals[q] += s_ev[rr * HU][j];
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    unsigned pre = 0;  // bit q: a segment starts at or before position q of this run
    bool seen = false;
    T acc = 0;
#pragma unroll
    for (int q = 0; q < NPR; q++) {
        const int sidx = r * NPR + q;
        T val = vals[q];
        if (UP && act && !hub) {
            const int c1 = s_lce[sidx];
            for (int c = s_lcr[sidx]; c >= 0 && c < c1; c++) val += ld_agent(&F[(long long)lc_pos[c] * k + j]);
        }
        const uint8_t fl = s_fl[sidx];
        const bool start = UP ? (fl & SEG_BOT) : (fl & SEG_TOP);
        if (start) {
            acc = 0;
            seen = true;
        }
        acc += val;
        vals[q] = acc;
        if (seen) pre |= 1u << q;
    }
    s_agg[r][j] = acc;
    if (j == 0) s_hs[r] = seen ? 1 : 0;
    __syncthreads();

    // cross-run exclusive scan per column, tile aggregate, publication, look-back
    if constexpr (RUNS <= 32) {
        // few runs (k >= 16): one thread per column walks them
        if (r == 0) {
            T carry = 0;
            int any = 0;
            for (int rr = 0; rr < RUNS; rr++) {
                s_excl[rr][j] = carry;
                if (j == 0) s_exhs[rr] = any;
                if (s_hs[rr]) carry = s_agg[rr][j];
                else carry += s_agg[rr][j];
                any |= s_hs[rr];
            }
            const unsigned tag = (epoch << 1) | (unsigned)any;
            constexpr int TW = sizeof(T) / 4;
            tag_put<T>(&aggw[(gt * KP + j) * TW], carry, tag);
        }
    } else {
        // many runs (small k): log-step segmented scan across runs, in place, pairs
        // (value, segment-start seen) combined as (b.f ? b.v : a.v + b.v, a.f | b.f)
        T vv = s_agg[r][j];
        int ff = s_hs[r];
        for (int dd = 1; dd < RUNS; dd <<= 1) {
            T pv = 0;
            int pf = 0;
            if (r >= dd) {
                pv = s_agg[r - dd][j];
                pf = s_hs[r - dd];
            }
            __syncthreads();
            if (r >= dd && !ff) vv = pv + vv;
            ff |= pf;
            s_agg[r][j] = vv;
            if (j == 0) s_hs[r] = ff;
            __syncthreads();
        }
        // exclusive value of run r: the inclusive one of run r - 1
        s_excl[r][j] = r > 0 ? s_agg[r - 1][j] : (T)0;
        if (j == 0) s_exhs[r] = r > 0 ? s_hs[r - 1] : 0;
        if (r == 0) {
            const int any = s_hs[RUNS - 1];
            const unsigned tag = (epoch << 1) | (unsigned)any;
            constexpr int TW = sizeof(T) / 4;
            tag_put<T>(&aggw[(gt * KP + j) * TW], s_agg[RUNS - 1][j], tag);
        }
    }
    // carry-in: the sum of the published aggregates of the tiles back to the nearest
    // one holding a segment start, nearest first; each step is one tagged load that
    // gives readiness, the start bit and the value together. The summation order
    // follows from the layout alone: deterministic.
    if (r == 0) {
        const uint8_t f0 = s_fl[0];
        const bool first_start = UP ? (f0 & SEG_BOT) : (f0 & SEG_TOP);
        constexpr int TW = sizeof(T) / 4;
        T cin = 0;
        if (!first_start) {
            const int npred = UP ? (ntiles - 1 - lt) : lt;  // tiles before this one in scan order
            int bad = 1;  // cleared when a tile holding a segment start is reached
            for (int back = 1; back <= npred; back++) {
                const long long pg = (long long)lvl_first + (UP ? (lt + back) : (lt - back));
                T val;
                unsigned tg;
                if (!tag_get<T>(&aggw[(pg * KP + j) * TW], epoch, val, tg)) break;
                cin += val;
                if (tg & 1u) {
                    bad = 0;
                    break;
                }
            }
            if (bad && j == 0) atomicOr(devflags, DEVERR_SPIN);
        }
        s_carry[j] = cin;
    }
    __syncthreads();

    // final values
    const T rc = s_exhs[r] ? s_excl[r][j] : (T)(s_carry[j] + s_excl[r][j]);
    double dacc = 0.0, mx = 0.0;
#pragma unroll
    for (int q = 0; q < NPR; q++) {
        const int sidx = r * NPR + q;
        const long long pos = p0 + (UP ? (TN - 1 - sidx) : sidx);
        const T out = ((pre >> q) & 1u) ? vals[q] : (T)(rc + vals[q]);
        const uint8_t fl = s_fl[sidx];
        if (UP) {
            if (act) {
                if (fl & SEG_TOP) st_agent(&F[pos * k + j], out);  // read by the parent's tile
                else F[pos * k + j] = out;
            }
        } else {
            const int v = s_vid[sidx];
            if (v >= 0 && act) {
                if (fl & SEG_LC) st_agent(&xout[(long long)v * k + j], out);  // a path parent's potential
                else xout[(long long)v * k + j] = out;
                if (rdot) dacc += (double)rdot[(long long)v * k + j] * (double)out;
                const double ao = fabs((double)out);
                mx = ao > mx ? ao : mx;
            }
            if constexpr (GRAM) vals[q] = (v >= 0 && act) ? out : (T)0;
        }
    }
    // completion stamp: all of this tile's stores are done before it is published
    wait_mem();
    __syncthreads();
    if (tid == 0) st_agent_u32(&done[gt], epoch);

    if constexpr (!UP && GRAM) {
        // after the stamp, off the path through the levels: this tile's share of the
        // Gram Q'x (rows of Q gathered by node id), reduced over all tiles in ticket
        // order
        constexpr int KK = KP * KP;
        __shared__ double s_gw[KK];
        T qv[NPR];
#pragma unroll
        for (int q = 0; q < NPR; q++) {
            const int v = s_vid[r * NPR + q];
            const bool ok = v >= 0 && act;
            const T x = qz_q[ok ? (long long)v * k + j : 0];
            qv[q] = ok ? x : (T)0;
        }
        BlockGram<T, KP> gq;
        gq.zero();
#pragma unroll
        for (int q = 0; q < NPR; q++) gq.add(qv[q], vals[q]);
        gq.flush(s_gw, qz_part + (long long)tk * KK);
        if (tail_reduce(qz_part, ntiles_total, KK, qz_cnt, s_gw, tk)) {
            if (beta_out) {
                // the k x k step that follows this Gram, by the block that holds the
                // total: beta = -G^-1 Q'x (G^-1 saved by the alpha step)
                for (int e = tid; e < KK; e += kSolveThreads) {
                    const int rr = e / KP, cc = e % KP;
                    double acc = 0.0;
                    if (rr < k && cc < k)
                        for (int p = 0; p < k; p++) acc -= beta_ginv[rr * KP + p] * s_gw[p * KP + cc];
                    beta_out[e] = (T)acc;
                }
            } else {
                for (int e = tid; e < KK; e += kSolveThreads) qz_out[e] = s_gw[e];
            }
        }
    }

    if (!UP) {
        if (dot_part) {
            s_red[r][j] = dacc;
            __syncthreads();
            if (r == 0) {
                double t = 0.0;
                for (int q = 0; q < RUNS; q++) t += s_red[q][j];
                dot_part[gt * KP + j] = t;
            }
        }
        if (absmax) {
            for (int off = 32; off >= 1; off >>= 1) {
                double o = __shfl_xor(mx, off, 64);
                mx = o > mx ? o : mx;
            }
            if ((tid & 63) == 0) s_max[tid >> 6] = mx;
            __syncthreads();
            if (tid == 0) {
                double m2 = 0.0;
                for (int w = 0; w < kSolveThreads / 64; w++) m2 = s_max[w] > m2 ? s_max[w] : m2;
                if (m2 > 0.0) atomicMax(absmax, (unsigned long long)__double_as_longlong(m2));
            }
        }
    }
}

template <typename T, int KP, bool UP, bool HUB, bool GRAM>
__global__ __launch_bounds__(kSolveThreads) void k_sweep(
    int ntiles_total, int nlev, const int *__restrict__ lvl_tile, int k, const int *__restrict__ perm,
    const uint8_t *__restrict__ flags, const int *__restrict__ ptop, const int *__restrict__ lc_ptr,
    const int *__restrict__ lc_pos, const int *__restrict__ lc_owner, const T *__restrict__ rpw,
    const T *__restrict__ yin, T *__restrict__ F, T *__restrict__ xout, unsigned long long *__restrict__ aggw,
    unsigned *__restrict__ done, const unsigned *__restrict__ epoch_ptr, const int *__restrict__ dep_ptr,
    const int *__restrict__ dep, int *__restrict__ ticket, unsigned *__restrict__ devflags,
    const T *__restrict__ rdot, double *__restrict__ dot_part, unsigned long long *__restrict__ absmax,
    const T *__restrict__ qz_q, double *__restrict__ qz_part, int *__restrict__ qz_cnt, double *__restrict__ qz_out,
    const double *__restrict__ beta_ginv, T *__restrict__ beta_out, const int *__restrict__ gate) {
    if (gate && *gate) return;
    __shared__ int s_tk;
    if (threadIdx.x == 0) s_tk = atomicAdd(ticket, 1);
    __syncthreads();
    const int tk = s_tk;
    if (tk >= ntiles_total) return;
    sweep_tile<T, KP, UP, HUB, GRAM>(tk, nlev, lvl_tile, k, perm, flags, ptop, lc_ptr, lc_pos, lc_owner, rpw, yin, F,
                                     xout, aggw, done, epoch_ptr, dep_ptr, dep, ticket, devflags, rdot, dot_part,
                                     absmax, ntiles_total, qz_q, qz_part, qz_cnt, qz_out, beta_ginv, beta_out);
}

// start of a solve: reset the sweep tickets and advance the device-side epoch by
// two (one per sweep), so stamps of earlier solves never match
__global__ void k_solve_begin(int *__restrict__ tickets, unsigned *__restrict__ epoch, const int *__restrict__ gate) {
    if (gate && *gate) return;
    if (threadIdx.x == 0) {
        tickets[0] = 0;
        tickets[1] = 0;
        epoch[0] += 2u;
    }
}

// ------------------------------------------------------------ scoring
// Edge heat w_pq sum_j (h_j[p] - h_j[q])^2 (eqs. 31, 35, 55) with the FP64
// per-vector sums over E and over P (eqs. 2, 4) and the largest heat off P.
// A lane group of KP lanes (lane j = vector j) takes KP consecutive edges per
// round: lane i loads edge i's endpoints, weight and mask byte (coalesced) into
// LDS. The group then works through the round in batches of SB edges: every
// lane gathers column j of both H rows of the batch's edges at once (no load
// waits on another), adds its FP64 terms to the column sums, and a
// reduce-scatter over log2(SB) lane bits followed by a plain reduction over the
// rest leaves each run of KP/SB lanes with the heat of one edge. Column sums add
// the edges in id order within a lane group, and the groups and blocks in index
// order: the result does not depend on timing.
template <typename T>
__device__ __forceinline__ T ld_u32off(const T *__restrict__ base, unsigned byte_off) {
    // element at a 32-bit byte offset (arrays under 4 GiB): the load then takes the
    // scalar-base plus 32-bit vector-offset form
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

template <typename T, int KP, bool WIDE>
__global__ __launch_bounds__(kThreads) void k_score(long long m, int k, int rounds, int nblk, const int *__restrict__ src,
                                                    const int *__restrict__ dst, const T *__restrict__ wT,
                                                    const uint8_t *__restrict__ mask, const T *__restrict__ H,
                                                    T *__restrict__ heat, double *__restrict__ part,
                                                    unsigned long long *__restrict__ hmax,
                                                    unsigned *__restrict__ devflags) {
    constexpr int G = kThreads / KP;
    constexpr int SB = KP < 16 ? KP : 16;  // edges per gather batch (8 -> 16: 104 -> 97 us on C2)
    constexpr int RUN = KP / SB;         // lanes that end with the same edge's heat
    __shared__ int s_p[G][KP], s_q[G][KP];
    __shared__ T s_w[G][KP], s_wp[G][KP];  // weight; weight if the edge is in P, else 0
    __shared__ double s_num[G][KP];
    __shared__ double s_den[G][KP];
    __shared__ double s_max[kThreads / 64];
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    const int jj = act ? j : 0;  // inactive lanes load a valid column and discard it
    // the edge of the batch whose heat this lane ends with: lane bits, high to low
    const int eb = j / RUN;
    double num = 0.0, den = 0.0, hm = 0.0;
    bool bad = false;
    // each XCD scores a contiguous eighth of the edges, so the rows of H that its
    // edges share stay in that XCD's L2
    const int b = xcd_block(blockIdx.x, gridDim.x);
    for (int r = 0; r < (b < nblk ? rounds : 0); r++) {
        const long long e0 = ((long long)b * rounds + r) * kThreads + (long long)g * KP;
        if (e0 >= m) break;  // uniform over the lane group
        {
            const long long e = e0 + j;
            const long long ee = e < m ? e : m - 1;
            const T w = e < m ? wT[ee] : (T)0;  // past m: no term, no heat
            s_p[g][j] = src[ee];
            s_q[g][j] = dst[ee];
            s_w[g][j] = w;
            s_wp[g][j] = mask[ee] ? w : (T)0;
        }
        // the group is part of one wave: its LDS writes are seen by its later reads
        __builtin_amdgcn_wave_barrier();
        // one batch in flight per wave: unrolled batches would hold every batch's
        // loads at once (160+ registers at KP = 32)
#pragma unroll 1
        for (int b0 = 0; b0 < KP; b0 += SB) {
            T hp[SB], hq[SB], v[SB];
#pragma unroll
            for (int i = 0; i < SB; i++) {
                const int pi = s_p[g][b0 + i], qi = s_q[g][b0 + i];
                if constexpr (WIDE) {
                    hp[i] = H[(long long)pi * k + jj];
                    hq[i] = H[(long long)qi * k + jj];
                } else {
                    hp[i] = ld_u32off(H, ((unsigned)pi * (unsigned)k + (unsigned)jj) * (unsigned)sizeof(T));
                    hq[i] = ld_u32off(H, ((unsigned)qi * (unsigned)k + (unsigned)jj) * (unsigned)sizeof(T));
                }
            }
#pragma unroll
            for (int i = 0; i < SB; i++) {
                const T di = act ? hp[i] - hq[i] : (T)0;
                const double dd = (double)di;
                num += (double)s_w[g][b0 + i] * dd * dd;
                den += (double)s_wp[g][b0 + i] * dd * dd;  // + 0 off P: the same sum
                v[i] = di * di;
            }
            // reduce-scatter: at offset o the lanes with bit o set keep the upper half
            // of the remaining slots (values first: a conditional of the elements
            // themselves would pick an address and index the array at run time)
#pragma unroll
            for (int o = KP / 2, c = SB / 2; c >= 1; o >>= 1, c >>= 1) {
                const bool hi = (j & o) != 0;
#pragma unroll
                for (int i = 0; i < c; i++) {
                    const T lo = v[i], up = v[i + c];
                    const T send = hi ? lo : up;
                    const T keep = hi ? up : lo;
                    v[i] = keep + __shfl_xor(send, o, KP);
                }
            }
            // then the plain sum over the RUN lanes that hold the same edge
#pragma unroll
            for (int o = RUN / 2; o >= 1; o >>= 1) v[0] += __shfl_xor(v[0], o, KP);
            const long long e = e0 + b0 + eb;
            if (j % RUN == 0 && e < m) {
                const T w = s_w[g][b0 + eb];
                const T h = w * v[0];
                if (heat) heat[e] = h;
                if (!__builtin_isfinite((double)h)) bad = true;
                if (s_wp[g][b0 + eb] == (T)0) hm = (double)h > hm ? (double)h : hm;  // off P (w > 0)
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    s_num[g][j] = num;
    s_den[g][j] = den;
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(hm, off, 64);
        hm = o > hm ? o : hm;
    }
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = hm;
    const bool anybad = __syncthreads_or(bad);
    if (g == 0) {
        double a = 0.0, c = 0.0;
        for (int q = 0; q < G; q++) {
            a += s_num[q][j];
            c += s_den[q][j];
        }
        if (b < nblk) {
            part[(long long)b * 2 * KP + j] = a;
            part[(long long)b * 2 * KP + KP + j] = c;
        }
    }
    if (threadIdx.x == 0) {
        double m2 = 0.0;
        for (int w = 0; w < kThreads / 64; w++) m2 = s_max[w] > m2 ? s_max[w] : m2;
        if (m2 > 0.0) atomicMax(hmax, (unsigned long long)__double_as_longlong(m2));
        if (anybad) atomicOr(devflags, DEVERR_NONFINITE);
    }
}

// The scorer with rows as 16-byte slices (k a power of two of at least W values,
// as k_lapv): a row group of LPR = k / W lanes takes 8 edges per round; lane c
// gathers the c-th slice of both endpoint rows of all 8 edges at once, adds its
// W columns' FP64 terms, and a reduce-scatter over the group's lanes (then a plain
// sum over any remaining lanes) leaves each lane with whole edges' heats.
// edges per row group and round: 8 for rows of 8 or more lanes, else 4 (C2, k = 32:
// 8 took 96 -> 85 us; C3, k = 16: 4 took 125 -> 110 us)
constexpr int scorev_sb(int lpr) { return lpr >= 8 ? 8 : 4; }
template <typename T, int KP>
struct ScoreV {
    static constexpr int W = V16<T>::W, LPR = KP / W, SB = scorev_sb(LPR);
    static constexpr int G = kThreads / LPR;                       // row groups per block
    static constexpr int RUN = LPR > SB ? LPR / SB : 1;            // lanes ending with one edge
    static constexpr int M = LPR < SB ? SB / LPR : 1;              // edges ending in one lane
    static constexpr int EPR = G * SB;                              // edges per block round
};
// TH: the type of the potentials read (T, or double for the FP64 solution of an L_P
// solve: each difference h_p - h_q is then taken in FP64 and rounded to T once,
// instead of differencing two rounded potentials); the geometry follows TH.
template <typename T, typename TH, int KP, bool WIDE>
__global__ __launch_bounds__(kThreads) void k_scorev(long long m, int rounds, int nblk, const int *__restrict__ src,
                                                     const int *__restrict__ dst, const T *__restrict__ wT,
                                                     const uint8_t *__restrict__ mask, const TH *__restrict__ H,
                                                     T *__restrict__ heat, double *__restrict__ part,
                                                     unsigned long long *__restrict__ hmax,
                                                     unsigned *__restrict__ devflags) {
    using S = ScoreV<TH, KP>;
    using V = typename V16<TH>::type;
    constexpr int W = S::W, LPR = S::LPR, SB = S::SB, G = S::G, RUN = S::RUN, M = S::M;
    __shared__ int s_p[G][SB], s_q[G][SB];
    __shared__ T s_w[G][SB], s_wp[G][SB];  // weight; weight if the edge is in P, else 0
    __shared__ double s_num[G][KP];
    __shared__ double s_den[G][KP];
    __shared__ double s_max[kThreads / 64];
    const int g = threadIdx.x / LPR, c = threadIdx.x % LPR;
    double num[W], den[W];
#pragma unroll
    for (int w = 0; w < W; w++) num[w] = den[w] = 0.0;
    double hm = 0.0;
    bool bad = false;
    const V *Hs = reinterpret_cast<const V *>(H);
    // each XCD scores a contiguous eighth of the edges, so the rows of H that its
    // edges share stay in that XCD's L2
    const int b = xcd_block(blockIdx.x, gridDim.x);
    for (int r = 0; r < (b < nblk ? rounds : 0); r++) {
        const long long e0 = ((long long)b * rounds + r) * S::EPR + (long long)g * SB;
        if (e0 >= m) break;  // uniform over the row group
#pragma unroll
        for (int i = c; i < SB; i += LPR) {
            // the edge arrays stream through once: non-temporal loads leave L2 to H
            const long long e = e0 + i, ee = e < m ? e : m - 1;
            const T w = e < m ? __builtin_nontemporal_load(&wT[ee]) : (T)0;  // past m: no term, no heat
            s_p[g][i] = __builtin_nontemporal_load(&src[ee]);
            s_q[g][i] = __builtin_nontemporal_load(&dst[ee]);
            s_w[g][i] = w;
            s_wp[g][i] = __builtin_nontemporal_load(&mask[ee]) ? w : (T)0;
        }
        __builtin_amdgcn_wave_barrier();  // the group is part of one wave
        V hp[SB], hq[SB];
#pragma unroll
        for (int i = 0; i < SB; i++) {
            if constexpr (WIDE) {
                hp[i] = Hs[(long long)s_p[g][i] * LPR + c];
                hq[i] = Hs[(long long)s_q[g][i] * LPR + c];
            } else {  // 32-bit byte offsets: no 64-bit address per load
                hp[i] = ld_u32off(Hs, ((unsigned)s_p[g][i] * (unsigned)LPR + (unsigned)c) * 16u);
                hq[i] = ld_u32off(Hs, ((unsigned)s_q[g][i] * (unsigned)LPR + (unsigned)c) * 16u);
            }
        }
        T sq[SB];
        T bn[W], bd[W];  // the batch's terms per column, added to the FP64 sums once
#pragma unroll
        for (int w = 0; w < W; w++) bn[w] = bd[w] = (T)0;
#pragma unroll
        for (int i = 0; i < SB; i++) {
            const V dv = hp[i] - hq[i];
            T acc = (T)0;
#pragma unroll
            for (int w = 0; w < W; w++) {
                const T dw = (T)dv[w];
                const T d2 = dw * dw;
                bn[w] += s_w[g][i] * d2;
                bd[w] += s_wp[g][i] * d2;  // + 0 off P: the same sum
                acc += d2;
            }
            sq[i] = acc;
        }
#pragma unroll
        for (int w = 0; w < W; w++) {
            num[w] += (double)bn[w];
            den[w] += (double)bd[w];
        }
        // reduce-scatter over the group's lanes: at offset o the lanes with bit o set
        // keep the upper half of the remaining slots (values first: a conditional of
        // the elements themselves would index the array at run time)
#pragma unroll
        for (int o = LPR / 2, cnt = SB / 2; o >= 1 && cnt >= M; o >>= 1, cnt >>= 1) {
            const bool hi = (c & o) != 0;
#pragma unroll
            for (int i = 0; i < cnt; i++) {
                const T lo = sq[i], up = sq[i + cnt];
                const T send = hi ? lo : up;
                const T keep = hi ? up : lo;
                sq[i] = keep + __shfl_xor(send, o, LPR);
            }
        }
#pragma unroll
        for (int o = RUN / 2; o >= 1; o >>= 1) sq[0] += __shfl_xor(sq[0], o, LPR);
        if (c % RUN == 0) {
#pragma unroll
            for (int mm = 0; mm < M; mm++) {
                const int i = (c / RUN) * M + mm;  // this lane's edge within the round
                const long long e = e0 + i;
                if (e < m) {
                    const T h = s_w[g][i] * sq[mm];
                    if (heat) heat[e] = h;
                    if (!__builtin_isfinite((double)h)) bad = true;
                    if (s_wp[g][i] == (T)0) hm = (double)h > hm ? (double)h : hm;  // off P (w > 0)
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int w = 0; w < W; w++) {
        s_num[g][c * W + w] = num[w];
        s_den[g][c * W + w] = den[w];
    }
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(hm, off, 64);
        hm = o > hm ? o : hm;
    }
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = hm;
    const bool anybad = __syncthreads_or(bad);
    if (threadIdx.x < KP && b < nblk) {
        const int j = threadIdx.x;
        double a = 0.0, d2 = 0.0;
        for (int q = 0; q < G; q++) {
            a += s_num[q][j];
            d2 += s_den[q][j];
        }
        part[(long long)b * 2 * KP + j] = a;
        part[(long long)b * 2 * KP + KP + j] = d2;
    }
    if (threadIdx.x == 0) {
        double m2 = 0.0;
        for (int w = 0; w < kThreads / 64; w++) m2 = s_max[w] > m2 ? s_max[w] : m2;
        if (m2 > 0.0) atomicMax(hmax, (unsigned long long)__double_as_longlong(m2));
        if (anybad) atomicOr(devflags, DEVERR_NONFINITE);
    }
}

template <int KP>
__global__ void k_lambda_max(double *__restrict__ red, int k) {
    if (threadIdx.x != 0) return;
    double best = 0.0;
    bool any = false;
    for (int j = 0; j < k; j++) {
        double nm = red[RED_NUM * kMaxK + j], dn = red[RED_DEN * kMaxK + j];
        if (dn > 0.0) {
            double r = nm / dn;
            if (!any || r > best) best = r;
            any = true;
        }
    }
    red[RED_LMAX * kMaxK] = best;
}

__global__ void k_lambda_min(long long n, const double *__restrict__ degG, const double *__restrict__ degP,
                             unsigned long long *__restrict__ slot) {
    __shared__ unsigned long long s_min[kThreads / 64];
    unsigned long long best = ~0ull;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x) {
        double r = degG[v] / degP[v];
        unsigned long long b = (unsigned long long)__double_as_longlong(r);
        best = b < best ? b : best;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        unsigned long long o = __shfl_xor(best, off, 64);
        best = o < best ? o : best;
    }
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = ~0ull;
        for (int w = 0; w < kThreads / 64; w++) b = s_min[w] < b ? s_min[w] : b;
        atomicMin(slot, b);
    }
}

// ------------------------------------------------------------ FP64 outer iteration
// r = b - L_P x in FP64 (difference form), grounded at root; r32 = r rounded to T,
// r64 (optional) = r
template <typename T, int KP, typename TB>
__global__ __launch_bounds__(kThreads) void k_resid64(long long n, int k, const int *__restrict__ prow,
                                                      const int *__restrict__ pcol, const double *__restrict__ pval,
                                                      const TB *__restrict__ b, const double *__restrict__ x,
                                                      T *__restrict__ r32, double *__restrict__ r64, int root,
                                                      double *__restrict__ part, int nblk) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    __shared__ double sh[G][KP];
    int bid = xcd_block(blockIdx.x, gridDim.x);
    if (bid >= nblk) return;
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double acc2 = 0.0;
    if (j < k) {
        long long r0 = (long long)bid * RPB;
        for (int i = g; i < RPB; i += G) {
            long long v = r0 + i;
            if (v >= n) break;
            double xv = x[v * k + j];
            double lx = 0.0;
            int pe = prow[v + 1];
            for (int p = prow[v]; p < pe; p++) lx += pval[p] * (xv - x[(long long)pcol[p] * k + j]);
            double rv = (v == root) ? 0.0 : (double)b[v * k + j] - lx;
            r32[v * k + j] = (T)rv;
            if (r64) r64[v * k + j] = rv;
            acc2 += rv * rv;
        }
    }
    sh[g][j] = acc2;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int q = 0; q < G; q++) t += sh[q][j];
        part[(long long)bid * KP + j] = t;
    }
}

// y = L_G x for x the FP64 solution of the previous step's L_P solve: differences
// and sums in FP64 with the FP64 edge weights, y rounded to T once and scaled by sc
// (a power of two). Differencing two FP32-rounded potentials of a smooth vector
// loses the digits that tell them apart; this product keeps them.
template <typename TY, int KP>
__global__ __launch_bounds__(kThreads) void k_lap_x64(long long n, int k, const int *__restrict__ rowptr,
                                                      const int *__restrict__ col, const int *__restrict__ ceid,
                                                      const double *__restrict__ w, const double *__restrict__ x,
                                                      TY *__restrict__ y,
                                                      const unsigned long long *__restrict__ scale_from,
                                                      int nblk) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    int bid = xcd_block(blockIdx.x, gridDim.x);
    if (bid >= nblk) return;
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    if (j >= k) return;
    const double sc = pow2_scale(scale_from);
    long long r0 = (long long)bid * RPB;
    for (int i = g; i < RPB; i += G) {
        long long v = r0 + i;
        if (v >= n) break;
        const int pb = rowptr[v], pe = rowptr[v + 1];
        if (pe - pb > kLongRow) continue;  // k_lap_x64_long writes this row
        const double xv = x[v * k + j];
        double acc = 0.0;
        for (int p = pb; p < pe; p++) acc += w[ceid[p]] * (xv - x[(long long)col[p] * k + j]);
        y[v * k + j] = (TY)(acc * sc);
    }
}

// The rows of y = L_G x64 longer than kLongRow entries (list lrow), one workgroup per
// row: lane groups take every G-th entry, and their FP64 sums are added in group
// order, so the result does not depend on timing.
template <int KP>
__global__ __launch_bounds__(kThreads) void k_lap_x64_long(int k, const int *__restrict__ rowptr,
                                                           const int *__restrict__ col, const int *__restrict__ ceid,
                                                           const double *__restrict__ w, const int *__restrict__ lrow,
                                                           const double *__restrict__ x, double *__restrict__ y,
                                                           const unsigned long long *__restrict__ scale_from) {
    constexpr int G = kThreads / KP, U = 4;
    __shared__ double s[G][KP];
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    const int v = lrow[blockIdx.x];
    const int p0 = rowptr[v], p1 = rowptr[v + 1];
    const double xv = x[act ? (long long)v * k + j : 0];
    double acc = 0.0;
    for (int p = p0 + g; p < p1; p += G * U) {
        int c[U], e[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int q = p + u * G < p1 ? p + u * G : p0;
            c[u] = col[q];
            e[u] = ceid[q];
        }
        double wv[U], xn[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            wv[u] = w[e[u]];
            xn[u] = x[act ? (long long)c[u] * k + j : 0];
        }
#pragma unroll
        for (int u = 0; u < U; u++) acc += p + u * G < p1 ? wv[u] * (xv - xn[u]) : 0.0;
    }
    s[g][j] = acc;
    __syncthreads();
    if (g == 0 && act) {
        double t = 0.0;
        for (int q = 0; q < G; q++) t += s[q][j];
        y[(long long)v * k + j] = t * pow2_scale(scale_from);
    }
}

// Flexible CG in FP64 around the working-precision block PCG (one recurrence per
// column): the block PCG returns z ~ L_P^-1 r; the direction is z made
// L_P-orthogonal to the previous one, and the step along it minimizes the energy
// norm of the error, so an inaccurate inner solve slows the iteration but cannot
// make it diverge. Reductions run over fixed row blocks, summed in index order.
//
// w = L_P z in FP64 (z in working precision, difference form, grounded at root);
// with adp, per-block partials of z'(A d_prev) per column
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_apply64(long long n, int k, const int *__restrict__ prow,
                                                      const int *__restrict__ pcol, const double *__restrict__ pval,
                                                      const T *__restrict__ z, double *__restrict__ w,
                                                      const double *__restrict__ adp, int root,
                                                      double *__restrict__ part, int nblk) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    __shared__ double sh[G][KP];
    int bid = xcd_block(blockIdx.x, gridDim.x);
    if (bid >= nblk) return;
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double acc = 0.0;
    if (j < k) {
        long long r0 = (long long)bid * RPB;
        for (int i = g; i < RPB; i += G) {
            long long v = r0 + i;
            if (v >= n) break;
            const double zv = (double)z[v * k + j];
            double lz = 0.0;
            const int pe = prow[v + 1];
            for (int p = prow[v]; p < pe; p++) lz += pval[p] * (zv - (double)z[(long long)pcol[p] * k + j]);
            if (v == root) lz = 0.0;
            w[v * k + j] = lz;
            if (adp) acc += zv * adp[v * k + j];
        }
    }
    sh[g][j] = acc;
    __syncthreads();
    if (g == 0 && adp) {
        double t = 0.0;
        for (int q = 0; q < G; q++) t += sh[q][j];
        part[(long long)bid * KP + j] = t;
    }
}

// d = z - beta d, Ad = w - beta Ad (beta per column; first: d = z, Ad = w, the
// previous direction not read); per-block partials of d'r (offset 0) and d'Ad
// (offset KP)
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_fcg64_dir(long long n, int k, int first, const double *__restrict__ beta,
                                                        const T *__restrict__ z, const double *__restrict__ w,
                                                        const double *__restrict__ r, double *__restrict__ d,
                                                        double *__restrict__ ad, double *__restrict__ part,
                                                        int nblk) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    __shared__ double s1[G][KP], s2[G][KP];
    int bid = xcd_block(blockIdx.x, gridDim.x);
    if (bid >= nblk) return;
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double dr = 0.0, dad = 0.0;
    if (j < k) {
        const double bj = beta[j];
        long long r0 = (long long)bid * RPB;
        for (int i = g; i < RPB; i += G) {
            long long v = r0 + i;
            if (v >= n) break;
            const long long o = v * k + j;
            const double dn = first ? (double)z[o] : (double)z[o] - bj * d[o];
            const double an = first ? w[o] : w[o] - bj * ad[o];
            d[o] = dn;
            ad[o] = an;
            dr += dn * r[o];
            dad += dn * an;
        }
    }
    s1[g][j] = dr;
    s2[g][j] = dad;
    __syncthreads();
    if (g == 0) {
        double a = 0.0, c = 0.0;
        for (int q = 0; q < G; q++) {
            a += s1[q][j];
            c += s2[q][j];
        }
        part[(long long)bid * 2 * KP + j] = a;
        part[(long long)bid * 2 * KP + KP + j] = c;
    }
}

// x += alpha d, r -= alpha Ad, r32 = r rounded to T, z = 0 (the inner solve's
// accumulator, cleared for the next one); per-block partials of r'r
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_fcg64_step(long long n, int k, const double *__restrict__ alpha,
                                                         const double *__restrict__ d, const double *__restrict__ ad,
                                                         double *__restrict__ x, double *__restrict__ r,
                                                         T *__restrict__ r32, T *__restrict__ z,
                                                         double *__restrict__ part, int nblk) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    __shared__ double sh[G][KP];
    int bid = xcd_block(blockIdx.x, gridDim.x);
    if (bid >= nblk) return;
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double rr = 0.0;
    if (j < k) {
        const double aj = alpha[j];
        long long r0 = (long long)bid * RPB;
        for (int i = g; i < RPB; i += G) {
            long long v = r0 + i;
            if (v >= n) break;
            const long long o = v * k + j;
            x[o] += aj * d[o];
            const double rn = r[o] - aj * ad[o];
            r[o] = rn;
            r32[o] = (T)rn;
            z[o] = (T)0;
            rr += rn * rn;
        }
    }
    sh[g][j] = rr;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int q = 0; q < G; q++) t += sh[q][j];
        part[(long long)bid * KP + j] = t;
    }
}

// FCG coefficients per column from reduced dots in red:
//   FIRST beta = 0; NEXT beta = z'Ad_prev / d_prev'Ad_prev; ALPHA alpha = d'r / d'Ad
//   (0 when d'Ad <= 0: a direction without energy adds nothing), d_prev'Ad_prev = d'Ad
enum : int { FC64_FIRST = 0, FC64_NEXT = 1, FC64_ALPHA = 2 };
__global__ void k_fcg64_coef(int k, int op, double *__restrict__ red) {
    const int j = threadIdx.x;
    if (j >= k) return;
    if (op == FC64_FIRST) {
        red[RED_FB * kMaxK + j] = 0.0;
    } else if (op == FC64_NEXT) {
        const double p = red[RED_DADP * kMaxK + j];
        red[RED_FB * kMaxK + j] = p > 0.0 ? red[RED_ZAD * kMaxK + j] / p : 0.0;
    } else {
        const double dad = red[RED_DAD * kMaxK + j];
        red[RED_FA * kMaxK + j] = dad > 0.0 ? red[RED_DR * kMaxK + j] / dad : 0.0;
        red[RED_DADP * kMaxK + j] = dad;
    }
}

template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_norm2(long long n, int k, const T *__restrict__ b, int root,
                                                    double *__restrict__ part) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    __shared__ double sh[G][KP];
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double acc = 0.0;
    if (j < k) {
        long long r0 = (long long)blockIdx.x * RPB;
        for (int i = g; i < RPB; i += G) {
            long long v = r0 + i;
            if (v >= n) break;
            if (v == root) continue;
            double x = (double)b[v * k + j];
            acc += x * x;
        }
    }
    sh[g][j] = acc;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int q = 0; q < G; q++) t += sh[q][j];
        part[(long long)blockIdx.x * KP + j] = t;
    }
}

template <typename T>
__global__ void k_x64_out(long long nk, const double *__restrict__ x64, T *__restrict__ out,
                          unsigned long long *__restrict__ absmax) {
    __shared__ double s_max[kThreads / 64];
    double mx = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x) {
        T o = (T)x64[i];
        out[i] = o;
        double a = fabs((double)o);
        mx = a > mx ? a : mx;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0 && absmax) {
        double m2 = 0.0;
        for (int w = 0; w < kThreads / 64; w++) m2 = s_max[w] > m2 ? s_max[w] : m2;
        if (m2 > 0.0) atomicMax(absmax, (unsigned long long)__double_as_longlong(m2));
    }
}

template <typename T>
__global__ void k_absmax(long long nk, const T *__restrict__ x, unsigned long long *__restrict__ absmax) {
    __shared__ double s_max[kThreads / 64];
    double mx = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x) {
        double a = fabs((double)x[i]);
        mx = a > mx ? a : mx;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m2 = 0.0;
        for (int w = 0; w < kThreads / 64; w++) m2 = s_max[w] > m2 ? s_max[w] : m2;
        if (m2 > 0.0) atomicMax(absmax, (unsigned long long)__double_as_longlong(m2));
    }
}


}  // namespace

// ============================================================= host side

static int lap_rows_per_block(int kp) { return (kThreads / kp) * lap_nit(kp); }
static int lap_blocks(const Dims &d) { return div_up(d.n, lap_rows_per_block(d.kp)); }

// a round of a scoring block is kThreads consecutive edges (KP per lane group)
// edges per block round: kThreads for the scalar scorer, ScoreV::EPR for the
// 16-byte-lane one (used when k is a power of two of at least 16 bytes); h64: the
// potentials read are FP64
static int score_epr(const Dims &d, bool h64 = false) {
    const int W = d.prec == 64 || h64 ? 2 : 4;
    if (d.k != d.kp || d.kp < W) return kThreads;
    return (kThreads / (d.kp / W)) * scorev_sb(d.kp / W);
}
static int score_rounds(const Dims &d, bool h64 = false) {
    return div_up(div_up(d.m, score_epr(d, h64)), kScoreBlocksMax);
}
static int score_blocks(const Dims &d, bool h64 = false) {
    return div_up(div_up(d.m, score_epr(d, h64)), score_rounds(d, h64));
}
static int gauss_blocks(const Dims &d) {
    return (int)std::min<long long>(kGaussBlocksMax, div_up(d.n, kThreads / d.kp));
}

template <typename T>
void plan_vecs(Arena &a, const Dims &d, Vecs<T> &v) {
    long long n = d.n, m = d.m, nk = n * d.k;
    v.wT = a.take<T>(m);
    v.cval = a.take<T>(2 * m);
    v.pval = a.take<T>(2 * m);
    // at most 2m / (kLongRow + 1) rows are longer than kLongRow
    const int lcap = (int)std::min<long long>(n, 2 * m / (kLongRow + 1) + 1);
    for (Ell<T> *e : {&v.eg, &v.ep}) {
        e->E = e == &v.eg ? kEllG : kEllP;
        e->col = a.take<int>(d.n * e->E);
        e->val = a.take<T>(d.n * e->E);
        e->deg = a.take<int>(d.n);
        e->cap = lcap;
        e->lcount = a.take<int>(1);
        e->lrow = a.take<int>(lcap);
        e->tail = a.take<T>((long long)lcap * d.k);
    }
    v.rpw = a.take<T>(d.Npad + 1);
    v.H = a.take<T>(nk);
    v.Y = a.take<T>(nk);
    v.F = a.take<T>((d.Npad + 1) * d.k);
    v.aggw = a.take<unsigned long long>(d.ntiles * d.kp * (long long)(sizeof(T) / 4));
    v.heat = a.take<T>(m);
    v.r = a.take<T>(nk);
    v.z = a.take<T>(nk);
    v.p = a.take<T>(nk);
    v.q = a.take<T>(nk);
    v.dx = a.take<T>(nk);
    v.x64 = a.take<double>(nk);
    v.r64 = a.take<double>(nk);
    v.d64 = a.take<double>(nk);
    v.ad64 = a.take<double>(nk);
    v.w64 = a.take<double>(nk);
    v.b64 = a.take<double>(nk);
    v.z64 = std::is_same<T, double>::value ? nullptr : a.take<double>(nk);
    long long parts = std::max<long long>({(long long)lap_blocks(d) + 8, (long long)vec_blocks(d) + 8, d.ntiles, 2ll * std::max(score_blocks(d), score_blocks(d, true)),
                                           (long long)gauss_blocks(d)});
    v.part = a.take<double>(parts * d.kp + 64);
    v.part2 = a.take<double>(64 * d.kp + 64);
    v.small = a.take<double>(7 * d.kp * d.kp + 64);  // G^-1, Gram input, right-hand-side basis
    v.smallT = a.take<T>(4 * d.kp * d.kp + 64);      // alpha, -alpha, beta, R^-1
    v.gpart = a.take<double>(bpcg_part_doubles(d));
    v.tcnt = a.take<int>(bpcg_counters(d));
    v.red = a.take<double>(RED_SLOTS * kMaxK);
    v.active = a.take<int>(kMaxK);
    v.loop = a.take<LoopCtl>(1);
    v.u64s = a.take<unsigned long long>(U_SLOTS);
}

template <typename T>
void start_vectors(const Dims &d, uint64_t seed, int pass, T *out, Vecs<T> &v, hipStream_t s) {
    int nb = gauss_blocks(d);
    double *mean = v.red + RED_MEAN * kMaxK;
    ProfScope ps(PK_START, (double)d.n * d.k * sizeof(T), s);
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL(k_gauss_sum<KP>, dim3(nb), dim3(kThreads), 0, s, d.n, d.k, (unsigned long long)seed, pass,
                           v.part);
        hipLaunchKernelGGL(k_col_sum<KP>, dim3(1), dim3(kColThreads), 0, s, v.part, nb, KP, 0, 1.0 / (double)d.n, mean);
        hipLaunchKernelGGL((k_gauss_write<T, KP>), dim3(nb), dim3(kThreads), 0, s, d.n, d.k, (unsigned long long)seed,
                           pass, mean, out);
    });
    GR_CHECK_LAUNCH();
}

template <typename T>
void lap_long(const Dims &d, const int *rowptr, const int *col, const T *val, const Ell<T> &ell, const T *x,
              hipStream_t s, const int *gate) {
    if (ell.nlong == 0) return;
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL((k_lap_long<T, KP>), dim3(ell.nlong), dim3(kThreads), 0, s, d.k, ell.E, rowptr, col, val,
                           ell.lrow, x, ell.tail, gate);
    });
    GR_CHECK_LAUNCH();
}

// y = L x with padded rows of width E: the 16-byte-lane kernel for rows of whole
// 16-byte slices (k a power of two), else the one-value-per-lane kernel
template <typename T, int KP, int E>
static void lap_launch(const Dims &d, const int *rowptr, const int *col, const T *val, const Ell<T> &ell, const T *x,
                       T *y, int root, const unsigned long long *scale_from, double *dot_part, int nb, hipStream_t s) {
    if constexpr (lapv_ok<T, KP>()) {
        if (d.k == KP && dot_part == nullptr) {
            constexpr int RPB = 4 * (64 / (KP / V16<T>::W));
            const int nv = div_up(d.n, RPB);
            hipLaunchKernelGGL((k_lapv<T, KP, E, kLapNTStore>), dim3(xcd_grid(nv)), dim3(256), 0, s, d.n, rowptr, col,
                               val, ell.tail, ell.col, ell.val, ell.deg, x, y, root, scale_from, nv);
            return;
        }
    }
    hipLaunchKernelGGL((k_lap<T, KP, E>), dim3(xcd_grid(nb)), dim3(kThreads), 0, s, d.n, d.k, rowptr, col, val,
                       ell.tail, ell.col, ell.val, ell.deg, x, y, root, scale_from, dot_part, nb);
}

template <typename T>
void lap_apply(const Dims &d, const int *rowptr, const int *col, const T *val, const Ell<T> &ell, const T *x, T *y,
               int root, const unsigned long long *scale_from, double *dot_part, hipStream_t s) {
    const int nb = lap_blocks(d);
    ProfScope ps(root < 0 ? PK_SPMM_G : PK_SPMM_P,
                 4.0 * (d.n + 1) + (double)(root < 0 ? 2 * d.m : d.p_nnz) * (4 + sizeof(T)) +
                     2.0 * d.n * d.k * sizeof(T),
                 s);
    lap_long<T>(d, rowptr, col, val, ell, x, s);
    KP_DISPATCH(d.kp, {
        switch (ell.E) {
        case 4: lap_launch<T, KP, 4>(d, rowptr, col, val, ell, x, y, root, scale_from, dot_part, nb, s); break;
        case 6: lap_launch<T, KP, 6>(d, rowptr, col, val, ell, x, y, root, scale_from, dot_part, nb, s); break;
        default: lap_launch<T, KP, 8>(d, rowptr, col, val, ell, x, y, root, scale_from, dot_part, nb, s); break;
        }
    });
    GR_CHECK_LAUNCH();
}

void lap_apply_x64(Topo &t, const Dims &d, const double *x64, double *y, const unsigned long long *scale_from,
                   const int *lrow, int nlong, hipStream_t s) {
    const int nbv = vec_blocks(d);
    ProfScope ps(PK_SPMM_G64, 4.0 * (d.n + 1) + 2.0 * d.m * 16 + (double)d.n * d.k * 16, s);
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL((k_lap_x64<double, KP>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k, t.rowptr,
                           t.col, t.ceid, t.w, x64, y, scale_from, nbv);
        if (nlong > 0)
            hipLaunchKernelGGL(k_lap_x64_long<KP>, dim3(nlong), dim3(kThreads), 0, s, d.k, t.rowptr, t.col, t.ceid,
                               t.w, lrow, x64, y, scale_from);
    });
    GR_CHECK_LAUNCH();
}

template <typename T>
void tree_solve(Topo &t, Vecs<T> &v, const Dims &d, const T *y, T *x, const T *rdot, double *dot_part,
                unsigned long long *absmax, hipStream_t s, const T *qz_q, double *qz_part, int *qz_cnt,
                double *qz_out, const double *beta_ginv, T *beta_out, const int *gate) {
    const int nt = (int)t.ntiles_used;
    const double vbytes = 2.0 * d.n * d.k * sizeof(T);
    hipLaunchKernelGGL(k_solve_begin, dim3(1), dim3(64), 0, s, t.tickets, t.epoch_dev, gate);
#define SWEEP_ARGS(TK, DP, DEP, RD, DOT, AM, QQ, QP, QC, QO, BG, BO)                                            \
    nt, t.nlev, t.lvl_tile, d.k, t.perm, t.flags, t.ptop, t.lc_ptr, t.lc_pos, t.lc_owner, v.rpw, y, v.F, x,        \
        v.aggw, t.done, t.epoch_dev, DP, DEP, TK, t.devflags, RD, DOT, AM, QQ, QP, QC, QO, BG, BO, gate
    KP_DISPATCH(d.kp, {
        {
            // y in, subtree sums out; per node: flags, perm, light-child pointers
            ProfScope ps(PK_TREE_UP, vbytes + 13.0 * d.n, s);
            // trees with nodes of many light children (hubs) take the variant that sums
            // them in parallel rounds; others keep the lighter kernel
            if (t.max_lc > 2 + kHubPerNode)
                hipLaunchKernelGGL((k_sweep<T, KP, true, true, false>), dim3(nt), dim3(kSolveThreads), 0, s,
                                   SWEEP_ARGS(t.tickets, t.dep_up_ptr, t.dep_up, (const T *)nullptr, (double *)nullptr,
                                              (unsigned long long *)nullptr, (const T *)nullptr, (double *)nullptr,
                                              (int *)nullptr, (double *)nullptr, (const double *)nullptr,
                                              (T *)nullptr));
            else
                hipLaunchKernelGGL((k_sweep<T, KP, true, false, false>), dim3(nt), dim3(kSolveThreads), 0, s,
                                   SWEEP_ARGS(t.tickets, t.dep_up_ptr, t.dep_up, (const T *)nullptr, (double *)nullptr,
                                              (unsigned long long *)nullptr, (const T *)nullptr, (double *)nullptr,
                                              (int *)nullptr, (double *)nullptr, (const double *)nullptr,
                                              (T *)nullptr));
        }
        {
            // subtree sums in, potentials out; per node: flags, perm, path top, 1/w;
            // with the fused Gram also the rows of Q
            const bool gram = UseMF<T, KP>::value && qz_q != nullptr;
            ProfScope ps(PK_TREE_DOWN, vbytes + (9.0 + sizeof(T)) * d.n + (gram ? (double)d.n * d.k * sizeof(T) : 0.0),
                         s);
            if (gram)
                hipLaunchKernelGGL((k_sweep<T, KP, false, false, UseMF<T, KP>::value>), dim3(nt), dim3(kSolveThreads),
                                   0, s,
                                   SWEEP_ARGS(t.tickets + 1, t.dep_dn_ptr, t.dep_dn, rdot, dot_part, absmax, qz_q,
                                              qz_part, qz_cnt, qz_out, beta_ginv, beta_out));
            else
                hipLaunchKernelGGL((k_sweep<T, KP, false, false, false>), dim3(nt), dim3(kSolveThreads), 0, s,
                                   SWEEP_ARGS(t.tickets + 1, t.dep_dn_ptr, t.dep_dn, rdot, dot_part, absmax,
                                              (const T *)nullptr, (double *)nullptr, (int *)nullptr,
                                              (double *)nullptr, (const double *)nullptr, (T *)nullptr));
        }
    });
#undef SWEEP_ARGS
    GR_CHECK_LAUNCH();
}

template <typename T>
void absmax_of(const Dims &d, const T *x, unsigned long long *slot, hipStream_t s) {
    long long nk = d.n * d.k;
    hipLaunchKernelGGL(k_absmax<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, x, slot);
    GR_CHECK_LAUNCH();
}

// Fixed-order column sums of per-block partials: one stage up to 2048 partials,
// else 64-block first stage into Vecs::part2, then one block.
template <typename T>
void col_sum(const Dims &d, Vecs<T> &v, const double *part, int nblk, int stride, int offset, double *out,
                    hipStream_t s) {
    KP_DISPATCH(d.kp, {
        if (nblk <= 2048) {
            hipLaunchKernelGGL(k_col_sum<KP>, dim3(1), dim3(kColThreads), 0, s, part, nblk, stride, offset, 1.0, out);
        } else {
            hipLaunchKernelGGL(k_col_sum<KP>, dim3(64), dim3(kColThreads), 0, s, part, nblk, stride, offset, 1.0,
                               v.part2);
            hipLaunchKernelGGL(k_col_sum<KP>, dim3(1), dim3(kColThreads), 0, s, v.part2, 64, KP, 0, 1.0, out);
        }
    });
    GR_CHECK_LAUNCH();
}

// max_j ||r_j|| / ||b_j|| from the squared norms in red[RED_RN] and red[RED_BN]
template <typename T>
static double worst_rel_resid(Vecs<T> &v, const Dims &d, hipStream_t s) {
    static_assert(RED_RN == RED_BN + 1, "norms of b and r are read together");
    double *bn = v.red + RED_BN * kMaxK;
    std::vector<double> hb(2 * kMaxK);
    GR_HIP(hipMemcpyAsync(hb.data(), bn, 2 * kMaxK * sizeof(double), hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    for (int j = 0; j < d.k; j++) {
        double bj = std::sqrt(hb[j]), rj = std::sqrt(hb[kMaxK + j]);
        require(std::isfinite(bj) && std::isfinite(rj), GRASS_ERR_NONFINITE,
                "a NaN or infinity appeared in an L_P solve (the working precision overflowed)");
        double rel = bj > 0 ? rj / bj : 0.0;
        worst = rel > worst ? rel : worst;
    }
    return worst;
}

template <typename T>
double true_residual(Topo &t, Vecs<T> &v, const Dims &d, const T *b, hipStream_t s, const double *b64) {
    const int nbv = vec_blocks(d);
    {
        ProfScope ps(PK_RESID64, 4.0 * (d.n + 1) + 12.0 * d.p_nnz + (double)d.n * d.k * (16 + 2 * sizeof(T)), s);
        KP_DISPATCH(d.kp, {
            if (b64)
                hipLaunchKernelGGL((k_resid64<T, KP, double>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k,
                                   t.prow, t.pcol, t.pval64, b64, v.x64, v.r, v.r64, 0, v.part, nbv);
            else
                hipLaunchKernelGGL((k_resid64<T, KP, T>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k, t.prow,
                                   t.pcol, t.pval64, b, v.x64, v.r, v.r64, 0, v.part, nbv);
        });
    }
    GR_CHECK_LAUNCH();
    col_sum<T>(d, v, v.part, nbv, d.kp, 0, v.red + RED_RN * kMaxK, s);
    return worst_rel_resid(v, d, s);
}

template <typename T>
double fcg_outer_step(Topo &t, Vecs<T> &v, const Dims &d, bool first, hipStream_t s, const double *z64) {
    const int nbv = vec_blocks(d);
    double *red = v.red;
    {
        ProfScope ps(PK_RESID64, 4.0 * (d.n + 1) + 12.0 * d.p_nnz + (double)d.n * d.k * (sizeof(T) + 56), s);
        KP_DISPATCH(d.kp, {
            // w = A z (with z'Ad_prev after the first step)
            const double *adp = first ? (const double *)nullptr : v.ad64;
            if (z64)
                hipLaunchKernelGGL((k_apply64<double, KP>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k,
                                   t.prow, t.pcol, t.pval64, z64, v.w64, adp, 0, v.part, nbv);
            else
                hipLaunchKernelGGL((k_apply64<T, KP>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k, t.prow,
                                   t.pcol, t.pval64, v.dx, v.w64, adp, 0, v.part, nbv);
            GR_CHECK_LAUNCH();
            if (!first) col_sum<T>(d, v, v.part, nbv, KP, 0, red + RED_ZAD * kMaxK, s);
            hipLaunchKernelGGL(k_fcg64_coef, dim3(1), dim3(kMaxK), 0, s, d.k, first ? (int)FC64_FIRST : (int)FC64_NEXT,
                               red);
            // d = z - beta d, Ad = w - beta Ad; d'r, d'Ad; alpha
            if (z64)
                hipLaunchKernelGGL((k_fcg64_dir<double, KP>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k,
                                   (int)first, red + RED_FB * kMaxK, z64, v.w64, v.r64, v.d64, v.ad64, v.part, nbv);
            else
                hipLaunchKernelGGL((k_fcg64_dir<T, KP>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k,
                                   (int)first, red + RED_FB * kMaxK, v.dx, v.w64, v.r64, v.d64, v.ad64, v.part, nbv);
            GR_CHECK_LAUNCH();
            col_sum<T>(d, v, v.part, nbv, 2 * KP, 0, red + RED_DR * kMaxK, s);
            col_sum<T>(d, v, v.part, nbv, 2 * KP, KP, red + RED_DAD * kMaxK, s);
            hipLaunchKernelGGL(k_fcg64_coef, dim3(1), dim3(kMaxK), 0, s, d.k, (int)FC64_ALPHA, red);
            // x += alpha d, r -= alpha Ad, r32 = r, z = 0; r'r
            hipLaunchKernelGGL((k_fcg64_step<T, KP>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k,
                               red + RED_FA * kMaxK, v.d64, v.ad64, v.x64, v.r64, v.r, v.dx, v.part, nbv);
            GR_CHECK_LAUNCH();
            col_sum<T>(d, v, v.part, nbv, KP, 0, red + RED_RN * kMaxK, s);
        });
    }
    return worst_rel_resid(v, d, s);
}

template <typename T>
SolveInfo pcg_solve(Topo &t, Vecs<T> &v, const Dims &d, const T *b, T *x, const grass_opts &o, hipStream_t s,
                    const double *b64, bool basis, bool single) {
    const long long nk = d.n * d.k;
    const int root = 0;
    const int nbv = vec_blocks(d);
    double *bn = v.red + RED_BN * kMaxK;
    if (single) {
        PcgParams pp;
        pp.rtol = o.pcg_rtol > 0 ? o.pcg_rtol : 1e-6;
        pp.itol = std::max(o.pcg_inner_rtol > 0 ? o.pcg_inner_rtol : 1e-2, pp.rtol);
        pp.max_it = o.pcg_max_iters > 0 ? o.pcg_max_iters : 8000;
        pp.basis = false;
        pp.single = true;
        // ||b||^2 per vector: the reference of the phase's convergence test
        KP_DISPATCH(d.kp, {
            hipLaunchKernelGGL((k_norm2<T, KP>), dim3(nbv), dim3(kThreads), 0, s, d.n, d.k, b, root, v.part);
        });
        GR_CHECK_LAUNCH();
        col_sum<T>(d, v, v.part, nbv, d.kp, 0, v.red + RED_RN * kMaxK, s);
        fill_T(v.dx, nk, (T)0, s);
        SolveInfo info = block_pcg<T>(t, v, d, b, pp, s, nullptr);
        // x is the working-precision solution itself
        GR_HIP(hipMemcpyAsync(x, v.dx, nk * sizeof(T), hipMemcpyDeviceToDevice, s));
        return info;
    }
    // ||b|| per vector (grounded rows)
    KP_DISPATCH(d.kp, {
        if (b64)
            hipLaunchKernelGGL((k_norm2<double, KP>), dim3(nbv), dim3(kThreads), 0, s, d.n, d.k, b64, root, v.part);
        else
            hipLaunchKernelGGL((k_norm2<T, KP>), dim3(nbv), dim3(kThreads), 0, s, d.n, d.k, b, root, v.part);
    });
    GR_CHECK_LAUNCH();
    col_sum<T>(d, v, v.part, nbv, d.kp, 0, bn, s);
    fill_f64(v.x64, nk, 0.0, s);
    fill_T(v.dx, nk, (T)0, s);
    PcgParams pp;
    pp.rtol = o.pcg_rtol > 0 ? o.pcg_rtol : 1e-6;
    pp.itol = o.pcg_inner_rtol > 0 ? o.pcg_inner_rtol : 1e-2;
    // a target looser than the inner phase's reduction ends that phase at the target
    pp.itol = std::max(pp.itol, pp.rtol);
    pp.max_it = o.pcg_max_iters > 0 ? o.pcg_max_iters : 8000;
    pp.max_repl = o.pcg_max_outer > 0 ? o.pcg_max_outer : 50;
    pp.basis = basis;
    SolveInfo info = block_pcg<T>(t, v, d, b, pp, s, b64);
    fill_u32(reinterpret_cast<unsigned *>(v.u64s + U_ABSMAX), 2, 0u, s);
    hipLaunchKernelGGL(k_x64_out<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, v.x64, x, v.u64s + U_ABSMAX);
    GR_CHECK_LAUNCH();
    return info;
}

template <typename T, typename TH, int KP>
static bool launch_scorev(Topo &t, Vecs<T> &v, const Dims &d, const TH *H, T *heat, int nb, hipStream_t s) {
    if constexpr (lapv_ok<TH, KP>()) {
        constexpr bool h64 = !std::is_same<T, TH>::value;
        if (d.k != KP) return false;
        if (ScoreV<TH, KP>::EPR != score_epr(d, h64)) throw Error(GRASS_ERR_DEVICE, "scorer round size mismatch");
        if ((unsigned long long)d.n * d.k * sizeof(TH) < (1ull << 32))
            hipLaunchKernelGGL((k_scorev<T, TH, KP, false>), dim3(xcd_grid(nb)), dim3(kThreads), 0, s, d.m,
                               score_rounds(d, h64), nb, t.src, t.dst, v.wT, t.mask, H, heat, v.part,
                               v.u64s + U_HMAX, t.devflags);
        else
            hipLaunchKernelGGL((k_scorev<T, TH, KP, true>), dim3(xcd_grid(nb)), dim3(kThreads), 0, s, d.m,
                               score_rounds(d, h64), nb, t.src, t.dst, v.wT, t.mask, H, heat, v.part,
                               v.u64s + U_HMAX, t.devflags);
        return true;
    }
    return false;
}

template <typename T>
void score_edges(Topo &t, Vecs<T> &v, const Dims &d, const T *H, T *heat, hipStream_t s, const double *H64) {
    const bool h64 = H64 != nullptr && !std::is_same<T, double>::value && d.k == d.kp && d.kp >= 2;
    int nb = score_blocks(d, h64);
    fill_u32(reinterpret_cast<unsigned *>(v.u64s + U_HMAX), 2, 0u, s);
    ProfScope ps(PK_SCORE, (double)d.m * (9 + 2 * sizeof(T)) + (double)d.n * d.k * (h64 ? 8 : sizeof(T)), s);
    KP_DISPATCH(d.kp, {
        bool vec = h64 ? launch_scorev<T, double, KP>(t, v, d, H64, heat, nb, s)
                       : launch_scorev<T, T, KP>(t, v, d, H, heat, nb, s);
        // 32-bit gather offsets while the n x k block is under 4 GiB
        if (vec) {
        } else if ((unsigned long long)d.n * d.k * sizeof(T) < (1ull << 32))
            hipLaunchKernelGGL((k_score<T, KP, false>), dim3(xcd_grid(nb)), dim3(kThreads), 0, s, d.m, d.k,
                               score_rounds(d), nb, t.src, t.dst, v.wT, t.mask, H, heat, v.part, v.u64s + U_HMAX, t.devflags);
        else
            hipLaunchKernelGGL((k_score<T, KP, true>), dim3(xcd_grid(nb)), dim3(kThreads), 0, s, d.m, d.k,
                               score_rounds(d), nb, t.src, t.dst, v.wT, t.mask, H, heat, v.part, v.u64s + U_HMAX, t.devflags);
        GR_CHECK_LAUNCH();
        col_sum<T>(d, v, v.part, nb, 2 * KP, 0, v.red + RED_NUM * kMaxK, s);
        col_sum<T>(d, v, v.part, nb, 2 * KP, KP, v.red + RED_DEN * kMaxK, s);
        hipLaunchKernelGGL(k_lambda_max<KP>, dim3(1), dim3(64), 0, s, v.red, d.k);
    });
    GR_CHECK_LAUNCH();
}

template <typename T>
PassScalars finish_estimates(Topo &t, Vecs<T> &v, const Dims &d, hipStream_t s) {
    fill_u32(reinterpret_cast<unsigned *>(v.u64s + U_LMIN), 2, 0xffffffffu, s);
    hipLaunchKernelGGL(k_lambda_min, dim3(grid_nk(d.n)), dim3(kThreads), 0, s, d.n, t.degG, t.degP,
                       v.u64s + U_LMIN);
    GR_CHECK_LAUNCH();
    double lmax = 0;
    unsigned long long u[U_SLOTS];
    GR_HIP(hipMemcpyAsync(&lmax, v.red + RED_LMAX * kMaxK, sizeof(double), hipMemcpyDeviceToHost, s));
    GR_HIP(hipMemcpyAsync(u, v.u64s, sizeof(u), hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
    PassScalars ps;
    ps.lambda_max = lmax;
    double lm, hm;
    std::memcpy(&lm, &u[U_LMIN], 8);
    std::memcpy(&hm, &u[U_HMAX], 8);
    ps.lambda_min = lm;
    ps.heat_max = hm;
    return ps;
}

#define INST(T)                                                                                                  \
    template void plan_vecs<T>(Arena &, const Dims &, Vecs<T> &);                                                \
    template void start_vectors<T>(const Dims &, uint64_t, int, T *, Vecs<T> &, hipStream_t);                    \
    template void lap_long<T>(const Dims &, const int *, const int *, const T *, const Ell<T> &, const T *,       \
                              hipStream_t, const int *);                                                      \
    template void lap_apply<T>(const Dims &, const int *, const int *, const T *, const Ell<T> &, const T *, T *, \
                               int,                                                                              \
                               const unsigned long long *, double *, hipStream_t);                               \
    template void tree_solve<T>(Topo &, Vecs<T> &, const Dims &, const T *, T *, const T *, double *,            \
                                unsigned long long *, hipStream_t, const T *, double *, int *, double *,         \
                                const double *, T *, const int *);                                               \
    template double true_residual<T>(Topo &, Vecs<T> &, const Dims &, const T *, hipStream_t, const double *);  \
    template double fcg_outer_step<T>(Topo &, Vecs<T> &, const Dims &, bool, hipStream_t, const double *);        \
    template SolveInfo pcg_solve<T>(Topo &, Vecs<T> &, const Dims &, const T *, T *, const grass_opts &,         \
                                    hipStream_t, const double *, bool, bool);                                    \
    template void score_edges<T>(Topo &, Vecs<T> &, const Dims &, const T *, T *, hipStream_t, const double *);  \
    template PassScalars finish_estimates<T>(Topo &, Vecs<T> &, const Dims &, hipStream_t);                      \
    template void absmax_of<T>(const Dims &, const T *, unsigned long long *, hipStream_t);               \
    template void col_sum<T>(const Dims &, Vecs<T> &, const double *, int, int, int, double *, hipStream_t);
INST(float)
INST(double)

}  // namespace grass
