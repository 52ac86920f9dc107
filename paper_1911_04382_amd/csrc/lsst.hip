// Low-stretch spanning tree on gfx950. The paper builds its sparsifier on a
// low-stretch spanning tree (Sec. III-A; it cites star and petal decompositions).
// This is the AKPW construction (Alon, Karp, Peleg, West 1995): edges fall into
// classes by the binary exponent of their weight (class 0 the heaviest), and
// round j clusters the current clusters over the edges of class <= j, adding one
// tree edge per cluster that joins another; the clustering is exponential
// start-time clustering (Miller, Peng, Xu 2013) with integer geometric shifts:
//  - cluster u starts at time kDmax - d_u, d_u the index of the first all-zero
//    3-bit group of the Philox4x64-10 output at counter (u, j, kDomain, 0), key
//    (seed, 0) (85 if none), so P(d_u >= k) = (7/8)^k;
//  - a cluster's center minimises hop distance + start time, the smaller id on
//    ties; it joins through the heaviest edge (FP32 weight) from a cluster of
//    that center one hop nearer, the smaller edge id on ties.
// The rule is evaluated as a breadth-first expansion over time steps: at step t
// an unclaimed cluster takes the smallest center among its own id (if it starts
// at t) and the centers of its neighbours claimed at step t - 1 (integer
// atomicMin), then the heaviest edge from that center (atomicMax of the FP32
// weight bits above the complemented edge id). Both choices are order-free, so
// the tree is the same on every run. Every step is a pass over the edges or the
// nodes (latency- and gather-bound, no contraction).
#include "lsst.h"

#include <climits>

#include "philox.h"

namespace grass {

int read_i32(const int *p, hipStream_t s);
void validate_graph(Topo &t, hipStream_t s);

namespace {

constexpr int kDmax = 85;                         // largest shift (85 groups of 3 bits)
constexpr unsigned long long kDomain = 0x4C535354;  // counter word 2: "LSST"
constexpr int kT = 256;

inline int blocks_for(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + kT - 1) / kT, 65536)); }
#define LS_STRIDE(i, n) \
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

// one atomic per wave: the wave's maximum / sum first
__device__ __forceinline__ int wave_max(int x) {
    for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ __forceinline__ int wave_sum(int x) {
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// counters: [0] largest ilogb(w), [1] largest class, [2] clusters, [3] active edges
__global__ void k_ls_exp(long long m, const double *__restrict__ w, int *__restrict__ cnt) {
    int mx = INT_MIN;
    LS_STRIDE(e, m) mx = max(mx, ilogb(w[e]));
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0 && mx != INT_MIN) atomicMax(&cnt[0], mx);
}

__global__ void k_ls_class(long long m, const double *__restrict__ w, int bits, int *__restrict__ cls,
                           int *__restrict__ cnt) {
    const int X = cnt[0];
    int mx = 0;
    LS_STRIDE(e, m) {
        const int c = (X - ilogb(w[e])) / bits;
        cls[e] = c;
        mx = max(mx, c);
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) atomicMax(&cnt[1], mx);
}

__global__ void k_ls_iota(long long n, int *__restrict__ cl) {
    LS_STRIDE(v, n) cl[v] = (int)v;
}

__global__ void k_ls_count(long long n, long long m, int j, const int *__restrict__ src, const int *__restrict__ dst,
                           const int *__restrict__ cls, const int *__restrict__ cl, int *__restrict__ cnt) {
    int nc = 0, na = 0;
    LS_STRIDE(v, n) nc += cl[v] == (int)v;
    LS_STRIDE(e, m) na += cls[e] <= j && cl[src[e]] != cl[dst[e]];
    nc = wave_sum(nc);
    na = wave_sum(na);
    if ((threadIdx.x & 63) == 0) {
        if (nc) atomicAdd(&cnt[2], nc);
        if (na) atomicAdd(&cnt[3], na);
    }
}

// start times of the round's clusters; clears the claim state
__global__ void k_ls_start(long long n, unsigned long long seed, int j, const int *__restrict__ cl,
                           int *__restrict__ start, int *__restrict__ owner, int *__restrict__ when,
                           int *__restrict__ bc, unsigned long long *__restrict__ bk) {
    LS_STRIDE(u, n) {
        owner[u] = -1;
        when[u] = -1;
        bc[u] = INT_MAX;
        bk[u] = 0;
        int st = -1;
        if (cl[u] == (int)u) {
            unsigned long long c[4] = {(unsigned long long)u, (unsigned long long)j, kDomain, 0};
            philox4x64_10(c, seed, 0);
            int d = kDmax;
            for (int g = 0; g < kDmax; g++) {
                int v = 0;
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    const int i = 3 * g + b;
                    v |= (int)((c[i >> 6] >> (i & 63)) & 1ull) << b;
                }
                if (v == 0) {
                    d = g;
                    break;
                }
            }
            st = kDmax - d;
        }
        start[u] = st;
    }
}

// offers: the smallest center among the neighbours claimed at t - 1 (and the own
// id of a cluster that starts at t)
__global__ void k_ls_offer(long long n, long long m, int j, int t, const int *__restrict__ src,
                           const int *__restrict__ dst, const int *__restrict__ cls, const int *__restrict__ cl,
                           const int *__restrict__ start, const int *__restrict__ owner,
                           const int *__restrict__ when, int *__restrict__ bc) {
    if (t > 0) {
        LS_STRIDE(e, m) {
            if (cls[e] > j) continue;
            const int a = cl[src[e]], b = cl[dst[e]];
            if (a == b) continue;
            if (when[a] == t - 1 && owner[b] < 0) atomicMin(&bc[b], owner[a]);
            if (when[b] == t - 1 && owner[a] < 0) atomicMin(&bc[a], owner[b]);
        }
    }
    LS_STRIDE(u, n) {
        if (start[u] == t && owner[u] < 0) atomicMin(&bc[u], (int)u);
    }
}

// the joining edge: heaviest FP32 weight from a cluster of the chosen center,
// smaller edge id on ties (one 64-bit key: weight bits over the complemented id)
__global__ void k_ls_edge(long long m, int j, int t, const int *__restrict__ src, const int *__restrict__ dst,
                          const double *__restrict__ w, const int *__restrict__ cls, const int *__restrict__ cl,
                          const int *__restrict__ owner, const int *__restrict__ when, const int *__restrict__ bc,
                          unsigned long long *__restrict__ bk) {
    LS_STRIDE(e, m) {
        if (cls[e] > j) continue;
        const int a = cl[src[e]], b = cl[dst[e]];
        if (a == b) continue;
        const unsigned long long key =
            ((unsigned long long)__float_as_uint((float)w[e]) << 32) | (0xFFFFFFFFull - (unsigned long long)e);
        if (when[a] == t - 1 && owner[b] < 0 && owner[a] == bc[b]) atomicMax(&bk[b], key);
        if (when[b] == t - 1 && owner[a] < 0 && owner[b] == bc[a]) atomicMax(&bk[a], key);
    }
}

__global__ void k_ls_claim(long long n, long long m, int t, int *__restrict__ owner, int *__restrict__ when,
                           int *__restrict__ bc, unsigned long long *__restrict__ bk, uint8_t *__restrict__ tree) {
    LS_STRIDE(u, n) {
        const int c = bc[u];
        if (c == INT_MAX || owner[u] >= 0) continue;
        owner[u] = c;
        when[u] = t;
        // a center offered by a neighbour always comes with its edge's key (> 0)
        const unsigned long long key = bk[u], e = 0xFFFFFFFFull - (key & 0xFFFFFFFFull);
        if (c != (int)u && key != 0 && e < (unsigned long long)m) tree[e] = 1;
        bc[u] = INT_MAX;
        bk[u] = 0;
    }
}

// clusters merge into their centers
__global__ void k_ls_contract(long long n, int *__restrict__ cl, const int *__restrict__ owner) {
    // every cluster claims itself by its start time at the latest, so owner >= 0
    LS_STRIDE(v, n) {
        const int o = owner[cl[v]];
        if (o >= 0) cl[v] = o;
    }
}

struct LsBufs {
    int *cls, *cl, *start, *owner, *when, *bc, *cnt;
    unsigned long long *bk;
};
LsBufs plan_ls(Arena &a, long long n, long long m) {
    LsBufs B;
    B.cls = a.take<int>(m);
    B.cl = a.take<int>(n);
    B.start = a.take<int>(n);
    B.owner = a.take<int>(n);
    B.when = a.take<int>(n);
    B.bc = a.take<int>(n);
    B.bk = a.take<unsigned long long>(n);
    B.cnt = a.take<int>(8);
    return B;
}

}  // namespace

size_t lsst_bytes(long long n, long long m) {
    Arena a;
    a.dry = true;
    (void)plan_ls(a, n, m);
    (void)a.take<unsigned>(4);  // validation flags
    return a.off + 256;
}

int low_stretch_tree(Topo &t, Arena &a, uint64_t seed, int class_bits, uint8_t *tree, hipStream_t s) {
    require(class_bits >= 1, GRASS_ERR_INVALID, "class_bits must be >= 1");
    const long long n = t.n, m = t.m;
    LsBufs B = plan_ls(a, n, m);
    const int be = blocks_for(m), bn = blocks_for(n), bb = blocks_for(std::max(n, m));
    int host[4];
    auto read4 = [&]() {
        GR_HIP(hipMemcpyAsync(host, B.cnt, sizeof(host), hipMemcpyDeviceToHost, s));
        GR_HIP(hipStreamSynchronize(s));
    };
    const int init[4] = {INT_MIN, 0, 0, 0};
    GR_HIP(hipMemcpyAsync(B.cnt, init, sizeof(init), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ls_exp, dim3(be), dim3(kT), 0, s, m, t.w, B.cnt);
    hipLaunchKernelGGL(k_ls_class, dim3(be), dim3(kT), 0, s, m, t.w, class_bits, B.cls, B.cnt);
    hipLaunchKernelGGL(k_ls_iota, dim3(bn), dim3(kT), 0, s, n, B.cl);
    fill_u8(tree, m, 0, s);
    GR_CHECK_LAUNCH();
    read4();
    const int maxc = host[1];
    int rounds = 0;
    for (int j = 0;; j++) {
        require(j <= maxc + 4096, GRASS_ERR_DEVICE, "low-stretch tree: rounds do not end");
        fill_i32(B.cnt + 2, 2, 0, s);
        hipLaunchKernelGGL(k_ls_count, dim3(bb), dim3(kT), 0, s, n, m, j, t.src, t.dst, B.cls, B.cl, B.cnt);
        GR_CHECK_LAUNCH();
        read4();
        const int nclusters = host[2], nactive = host[3];
        if (nclusters <= 1) break;
        if (nactive == 0) {
            require(j < maxc, GRASS_ERR_DISCONNECTED, "graph is disconnected");
            continue;
        }
        hipLaunchKernelGGL(k_ls_start, dim3(bn), dim3(kT), 0, s, n, (unsigned long long)seed, j, B.cl, B.start,
                           B.owner, B.when, B.bc, B.bk);
        for (int tt = 0; tt <= kDmax; tt++) {
            hipLaunchKernelGGL(k_ls_offer, dim3(bb), dim3(kT), 0, s, n, m, j, tt, t.src, t.dst, B.cls, B.cl, B.start,
                               B.owner, B.when, B.bc);
            if (tt > 0)
                hipLaunchKernelGGL(k_ls_edge, dim3(be), dim3(kT), 0, s, m, j, tt, t.src, t.dst, t.w, B.cls, B.cl,
                                   B.owner, B.when, B.bc, B.bk);
            hipLaunchKernelGGL(k_ls_claim, dim3(bn), dim3(kT), 0, s, n, m, tt, B.owner, B.when, B.bc, B.bk, tree);
        }
        hipLaunchKernelGGL(k_ls_contract, dim3(bn), dim3(kT), 0, s, n, B.cl, B.owner);
        GR_CHECK_LAUNCH();
        rounds++;
    }
    return rounds;
}

}  // namespace grass
