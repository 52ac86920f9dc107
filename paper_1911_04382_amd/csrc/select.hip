// Filtering and similarity check on gfx950 (eq. 58, Sec. IV-D steps 5-6):
// candidates = off-subgraph edges with heat >= theta * heat_max, ranked by heat
// descending then id ascending, then a greedy pass that skips an edge whose two
// endpoints were already marked by an accepted edge of this pass and stops at the
// per-pass budget.
#include "select.h"

namespace grass {

namespace {
#define GSTRIDE(i, n) for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)
inline int grid_for(long long n) { return (int)std::min<long long>(std::max<long long>(1, (n + 255) / 256), 65536); }

template <typename T>
__global__ void k_cand_flags(long long m, const uint8_t *__restrict__ mask, const T *__restrict__ heat, double thr,
                             int *__restrict__ flag) {
    GSTRIDE(e, m) flag[e] = (mask[e] == 0 && (double)heat[e] >= thr) ? 1 : 0;
}

__device__ __forceinline__ unsigned long long desc_key(float h) { return (unsigned long long)(~__float_as_uint(h)); }
__device__ __forceinline__ unsigned long long desc_key(double h) {
    return ~(unsigned long long)__double_as_longlong(h);
}

// scatter flagged edge ids to their compacted positions (id order kept) with
// their descending-heat sort keys
template <typename T>
__global__ void k_cand_scatter(long long m, const int *__restrict__ flag, const int *__restrict__ pos,
                               const T *__restrict__ heat, unsigned long long *__restrict__ keys, int *__restrict__ cand) {
    GSTRIDE(e, m) if (flag[e]) {
        int p = pos[e];
        keys[p] = desc_key(heat[e]);
        cand[p] = (int)e;
    }
}

template <typename T>
__global__ void k_heat_max(long long m, const uint8_t *__restrict__ mask, const T *__restrict__ heat,
                           unsigned long long *__restrict__ slot) {
    unsigned long long best = 0ull;
    GSTRIDE(e, m) if (mask[e] == 0) {
        double h = (double)heat[e];
        unsigned long long b = h > 0.0 ? (unsigned long long)__double_as_longlong(h) : 0ull;
        best = b > best ? b : best;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        unsigned long long o = __shfl_xor(best, off, 64);
        best = o > best ? o : best;
    }
    if ((threadIdx.x & 63) == 0 && best) atomicMax(slot, best);
}

template <typename T>
__global__ void k_scores(long long m, const uint8_t *__restrict__ mask, const T *__restrict__ heat, double hmax,
                         T *__restrict__ scores) {
    GSTRIDE(e, m) scores[e] = (mask[e] != 0 || !(hmax > 0.0)) ? (T)0 : (T)((double)heat[e] / hmax);
}

// The "mark set" of candidate e = (p, q): p, q, and with hops >= 1 the
// neighbours of p and q in G.
template <typename F>
__device__ __forceinline__ void for_marks(int p, int q, int hops, const int *__restrict__ rowptr,
                                          const int *__restrict__ col, F f) {
    f(p);
    f(q);
    if (hops >= 1) {
        for (int a = rowptr[p]; a < rowptr[p + 1]; a++) f(col[a]);
        for (int a = rowptr[q]; a < rowptr[q + 1]; a++) f(col[a]);
    }
}

constexpr int kGreedyThreads = 1024;

// Deterministic reservations, one workgroup: candidates are taken in windows of
// 1024 in rank order. In a round every undecided candidate reserves its mark set
// (owner[x] = min rank); a candidate whose two endpoints it owns has no undecided
// earlier candidate that could mark them, so it can be decided now, exactly as the
// sequential greedy would: it is similar iff both endpoints carry a mark of an
// earlier accepted candidate (mark[x] = min accepting rank). At least the first
// undecided candidate is decided per round, so every loop is bounded. owner[] and
// mark[] (INT_MAX when idle) are restored before the kernel ends.
__global__ __launch_bounds__(kGreedyThreads) void k_greedy(long long c, const int *__restrict__ cand,
                                                           const int *__restrict__ src, const int *__restrict__ dst,
                                                           const int *__restrict__ rowptr, const int *__restrict__ col,
                                                           int hops, long long budget, int *__restrict__ mark,
                                                           int *__restrict__ owner, uint8_t *__restrict__ acc,
                                                           uint8_t *__restrict__ mask, int *__restrict__ out) {
    __shared__ int s_wsum[kGreedyThreads / 64];
    __shared__ long long s_accepted;
    __shared__ long long s_processed;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) {
        s_accepted = 0;
        s_processed = 0;
    }
    __syncthreads();
    for (long long pos = 0; pos < c; pos += kGreedyThreads) {
        if (budget > 0 && s_accepted >= budget) break;
        long long i = pos + tid;
        bool valid = i < c;
        int e = valid ? cand[i] : 0;
        int p = valid ? src[e] : 0, q = valid ? dst[e] : 0;
        const int rank = (int)i;
        bool undecided = valid, take = false;
        for (;;) {
            bool was = undecided;
            if (undecided && hops >= 0)
                for_marks(p, q, hops, rowptr, col, [&](int x) { atomicMin(&owner[x], rank); });
            __syncthreads();
            bool now = false;
            if (undecided) {
                bool free_ = hops < 0 || (ld_agent_i32(&owner[p]) == rank && ld_agent_i32(&owner[q]) == rank);
                if (free_) {
                    bool similar = hops >= 0 && ld_agent_i32(&mark[p]) < rank && ld_agent_i32(&mark[q]) < rank;
                    take = !similar;
                    undecided = false;
                    now = true;
                }
            }
            __syncthreads();
            if (was && hops >= 0)
                for_marks(p, q, hops, rowptr, col, [&](int x) { st_agent_i32(&owner[x], INT_MAX); });
            if (now && take && hops >= 0)
                for_marks(p, q, hops, rowptr, col, [&](int x) { atomicMin(&mark[x], rank); });
            if (!__syncthreads_or(undecided)) break;
        }
        // budget: keep the first accepted candidates in rank order
        unsigned long long bal = __ballot(take);
        int before = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        if (lane == 0) s_wsum[wv] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < kGreedyThreads / 64; w++) {
            if (w < wv) woff += s_wsum[w];
            tot += s_wsum[w];
        }
        long long rnk = s_accepted + woff + before;
        bool keep = take && (budget <= 0 || rnk < budget);
        if (valid) acc[i] = take ? (keep ? 1 : 2) : 0;
        if (keep) mask[e] = 2;
        __syncthreads();
        if (tid == 0) {
            long long room = budget > 0 ? budget - s_accepted : (long long)tot;
            s_accepted += tot < room ? tot : room;
            s_processed = (pos + kGreedyThreads < c) ? pos + kGreedyThreads : c;
        }
        __syncthreads();
    }
    // restore the marks
    long long np = s_processed;
    for (long long i = tid; i < np; i += kGreedyThreads) {
        if (acc[i] && hops >= 0) {
            int e = cand[i];
            for_marks(src[e], dst[e], hops, rowptr, col, [&](int x) { st_agent_i32(&mark[x], INT_MAX); });
        }
    }
    if (tid == 0) {
        out[0] = (int)s_accepted;
        out[1] = (int)np;
    }
}
}  // namespace

void init_greedy_state(Topo &t, hipStream_t s) {
    fill_i32(t.greedy_mark, t.n, INT_MAX, s);
    fill_i32(t.greedy_owner, t.n, INT_MAX, s);
}

template <typename T>
SelectOut select_edges(Topo &t, const Dims &d, const T *heat, double theta, double heat_max, int sim_hops,
                       long long budget, T *scores, hipStream_t s) {
    SelectOut so;
    long long m = t.m;
    if (scores) {
        hipLaunchKernelGGL(k_scores<T>, dim3(grid_for(m)), dim3(256), 0, s, m, t.mask, heat, heat_max, scores);
        GR_CHECK_LAUNCH();
    }
    double thr = theta * heat_max;
    int *flag = t.tmpA, *posv = t.tmpB;
    hipLaunchKernelGGL(k_cand_flags<T>, dim3(grid_for(m)), dim3(256), 0, s, m, t.mask, heat, thr, flag);
    GR_CHECK_LAUNCH();
    int *total = t.scal_i + 20;
    scan_excl_i32(flag, posv, m, total, t.scan, s);
    int c = read_i32(total, s);
    so.candidates = c;
    if (c == 0) return so;
    int *cand = t.tmpA + m;  // tmpA holds >= 2m ints: flags in [0, m), candidates in [m, 2m)
    hipLaunchKernelGGL(k_cand_scatter<T>, dim3(grid_for(m)), dim3(256), 0, s, m, flag, posv, heat, t.keys, cand);
    GR_CHECK_LAUNCH();
    radix_sort_pairs(t.keys, cand, c, sizeof(T) == 4 ? 32 : 64, t.sort, s);
    int *out = t.scal_i + 24;
    hipLaunchKernelGGL(k_greedy, dim3(1), dim3(kGreedyThreads), 0, s, (long long)c, cand, t.src, t.dst, t.rowptr,
                       t.col, sim_hops, budget, t.greedy_mark, t.greedy_owner, t.cand_acc, t.mask, out);
    GR_CHECK_LAUNCH();
    int h[2];
    GR_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
    so.accepted = h[0];
    so.processed = h[1];
    return so;
}

template SelectOut select_edges<float>(Topo &, const Dims &, const float *, double, double, int, long long, float *,
                                       hipStream_t);
template SelectOut select_edges<double>(Topo &, const Dims &, const double *, double, double, int, long long,
                                        double *, hipStream_t);

template <typename T>
void normalized_scores(Topo &t, const T *heat, double heat_max, T *scores, hipStream_t s) {
    hipLaunchKernelGGL(k_scores<T>, dim3(grid_for(t.m)), dim3(256), 0, s, t.m, t.mask, heat, heat_max, scores);
    GR_CHECK_LAUNCH();
}
template <typename T>
double heat_max_off(Topo &t, const T *heat, hipStream_t s) {
    unsigned long long *slot = reinterpret_cast<unsigned long long *>(t.scal_i + 28);
    fill_u32(reinterpret_cast<unsigned *>(slot), 2, 0u, s);
    hipLaunchKernelGGL(k_heat_max<T>, dim3(grid_for(t.m)), dim3(256), 0, s, t.m, t.mask, heat, slot);
    GR_CHECK_LAUNCH();
    unsigned long long h = 0;
    GR_HIP(hipMemcpyAsync(&h, slot, 8, hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
    double v;
    std::memcpy(&v, &h, 8);
    return v;
}
template double heat_max_off<float>(Topo &, const float *, hipStream_t);
template double heat_max_off<double>(Topo &, const double *, hipStream_t);

template void normalized_scores<float>(Topo &, const float *, double, float *, hipStream_t);
template void normalized_scores<double>(Topo &, const double *, double, double *, hipStream_t);

}  // namespace grass
