// Spectral off-tree edge embedding on gfx950 (Sec. III-F of the paper):
// Philox start vectors (eq. 28), Laplacian products (eq. 1), the grounded tree
// solve and PCG on L_P that realise the generalized power iteration (eq. 29),
// and the per-edge Joule heat with FP64 Rayleigh-quotient sums (eqs. 2, 31, 35,
// 55, 61). None of these steps is a dense contraction: every kernel is bound by
// HBM traffic (or latency), so the design work is coalescing, fusion and the
// block -> XCD mapping, not MFMA.
#include "embed.h"

namespace grass {

#define KP_DISPATCH(kp, ...)                                                                    \
    switch (kp) {                                                                               \
    case 1: { constexpr int KP = 1; __VA_ARGS__; } break;                                       \
    case 2: { constexpr int KP = 2; __VA_ARGS__; } break;                                       \
    case 4: { constexpr int KP = 4; __VA_ARGS__; } break;                                       \
    case 8: { constexpr int KP = 8; __VA_ARGS__; } break;                                       \
    case 16: { constexpr int KP = 16; __VA_ARGS__; } break;                                     \
    case 32: { constexpr int KP = 32; __VA_ARGS__; } break;                                     \
    case 64: { constexpr int KP = 64; __VA_ARGS__; } break;                                     \
    default: throw Error(GRASS_ERR_INVALID, "k must be in 1..64");                              \
    }

namespace {

constexpr int kThreads = 256;
constexpr int kGaussBlocksMax = 2048;
constexpr int kRowsPerGroup = 16;   // Laplacian rows per lane group
constexpr int kEdgesPerGroup = 16;  // scored edges per lane group

// 8 XCDs: consecutive workgroup ids land on different XCDs; remap them so that each
// XCD works on one contiguous range of rows (its L2 then holds the neighbourhood).
__device__ __forceinline__ int xcd_block(int bid, int grid) {
    int per = grid >> 3;
    return (bid & 7) * per + (bid >> 3);
}
inline int xcd_grid(int nb) { return (nb + 7) / 8 * 8; }

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

template <int KP>
__global__ void k_col_sum(const double *__restrict__ part, int nblk, int stride, int offset, double scale,
                          double *__restrict__ out) {
    constexpr int G = kThreads / KP;
    __shared__ double sh[G][KP];
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double s = 0.0;
    for (int b = g; b < nblk; b += G) s += part[(long long)b * stride + offset + j];
    sh[g][j] = s;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int q = 0; q < G; q++) t += sh[q][j];
        out[j] = t * scale;
    }
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
__device__ __forceinline__ double pow2_scale(const unsigned long long *slot) {
    if (!slot) return 1.0;
    double mx = __longlong_as_double((long long)*slot);
    if (!(mx > 0.0) || !(mx < INFINITY)) return 1.0;
    return ldexp(1.0, -ilogb(mx));
}

template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_lap(long long n, int k, const int *__restrict__ rowptr,
                                                  const int *__restrict__ col, const T *__restrict__ val,
                                                  const T *__restrict__ x, T *__restrict__ y, int root,
                                                  const unsigned long long *__restrict__ scale_from,
                                                  double *__restrict__ dot_part, int nblk) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    int b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= nblk) return;
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const T sc = (T)pow2_scale(scale_from);
    double dacc = 0.0;
    long long r0 = (long long)b * RPB;
    if (j < k) {
        for (int i = g; i < RPB; i += G) {
            long long v = r0 + i;
            if (v >= n) break;
            T xv = x[v * k + j];
            T acc = 0;
            int pe = rowptr[v + 1];
            for (int p = rowptr[v]; p < pe; p++) {
                int u = col[p];
                acc += val[p] * (xv - x[(long long)u * k + j]);
            }
            acc *= sc;
            if (v == root) acc = 0;
            y[v * k + j] = acc;
            dacc += (double)xv * (double)acc;
        }
    }
    if (dot_part) {
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
// One heavy-light level of a sweep, as a segmented scan over the level's layout
// positions (paths are contiguous segments, top to bottom).
//   UP   (reverse scan, segments start at path bottoms):
//        f[i] = y[perm i] + sum_{light children c} f[c] + f[i+1]   (subtree currents)
//   DOWN (forward scan, segments start at path tops):
//        x[perm i] = x[parent of top] + sum_{top..i} f / pw        (potentials)
// A tile publishes its aggregate before looking back; its carry-in is the sum of
// the predecessors' aggregates back to the nearest tile holding a segment start,
// added in a fixed order, so results never depend on timing. Tiles take their
// index from an atomic ticket, so every awaited tile is already running; every
// wait is bounded.
template <typename T, int KP, bool UP>
__global__ __launch_bounds__(kThreads) void k_sweep(
    long long level_pos, int ntiles, long long tile_base, int k, const int *__restrict__ perm,
    const uint8_t *__restrict__ flags, const int *__restrict__ ptop, const int *__restrict__ lc_ptr,
    const int *__restrict__ lc_pos, const T *__restrict__ rpw, const T *__restrict__ yin, T *__restrict__ F,
    T *__restrict__ xout, T *__restrict__ agg, int *__restrict__ hs, unsigned *__restrict__ status, unsigned epoch,
    int *__restrict__ ticket, unsigned *__restrict__ devflags, const T *__restrict__ rdot, double *__restrict__ dot_part,
    unsigned long long *__restrict__ absmax) {
    constexpr int RUNS = kThreads / KP;
    constexpr int NPR = kSolveNPR;
    constexpr int TN = RUNS * NPR;
    __shared__ int s_tile;
    __shared__ T s_agg[RUNS][KP];
    __shared__ int s_hs[RUNS];
    __shared__ T s_excl[RUNS][KP];
    __shared__ int s_exhs[RUNS];
    __shared__ T s_carry[KP];
    __shared__ double s_red[RUNS][KP];
    __shared__ double s_max[kThreads / 64];

    const int tid = threadIdx.x;
    const int j = tid % KP, r = tid / KP;
    if (tid == 0) s_tile = atomicAdd(ticket, 1);
    __syncthreads();
    const int tk = s_tile;
    const int lt = UP ? (ntiles - 1 - tk) : tk;  // logical tile within the level
    const long long p0 = level_pos + (long long)lt * TN;
    const long long gt = tile_base + lt;
    const bool act = j < k;

    // load + run-local inclusive segmented scan (scan order index s -> position)
    T vals[NPR];
    bool pre[NPR];
    bool seen = false;
    T acc = 0;
#pragma unroll
    for (int q = 0; q < NPR; q++) {
        int sidx = r * NPR + q;
        long long pos = p0 + (UP ? (TN - 1 - sidx) : sidx);
        uint8_t fl = flags[pos];
        bool start = UP ? (fl & SEG_BOT) : (fl & SEG_TOP);
        T val = 0;
        if (act) {
            if (UP) {
                int v = perm[pos];
                if (v >= 0) val = yin[(long long)v * k + j];
                int c1 = lc_ptr[pos + 1];
                for (int c = lc_ptr[pos]; c < c1; c++) val += F[(long long)lc_pos[c] * k + j];
            } else {
                val = F[pos * k + j] * rpw[pos];
                if (fl & SEG_TOP) {
                    int pt = ptop[pos];
                    if (pt >= 0) val += xout[(long long)pt * k + j];
                }
            }
        }
        if (start) {
            acc = 0;
            seen = true;
        }
        acc += val;
        vals[q] = acc;
        pre[q] = seen;
    }
    s_agg[r][j] = acc;
    if (j == 0) s_hs[r] = seen ? 1 : 0;
    __syncthreads();

    // cross-run exclusive scan per column, tile aggregate, publication, look-back
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
        st_agent(&agg[gt * KP + j], carry);
        if (j == 0) st_agent_i32(&hs[gt], any);
        wait_mem();
        if (j == 0) st_agent_u32(&status[gt], epoch);
        // carry-in from predecessors (only needed when the first element is not a start)
        uint8_t f0 = flags[p0 + (UP ? (TN - 1) : 0)];
        bool first_start = UP ? (f0 & SEG_BOT) : (f0 & SEG_TOP);
        T cin = 0;
        if (!first_start) {
            int cnt = 0;
            int bad = 0;
            for (int back = 1; back <= lt + 1 && back <= ntiles; back++) {
                int plt = UP ? (lt + back) : (lt - back);
                if (plt < 0 || plt >= ntiles) {
                    bad = 1;
                    break;
                }
                long long pg = tile_base + plt;
                long long spin = 0;
                while (ld_agent_u32(&status[pg]) != epoch) {
                    if (++spin > kSpinLimit) {
                        bad = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (bad) break;
                cnt = back;
                if (ld_agent_i32(&hs[pg])) break;
            }
            if (bad && j == 0) atomicOr(devflags, DEVERR_SPIN);
            for (int back = cnt; back >= 1; back--) {
                long long pg = tile_base + (UP ? (lt + back) : (lt - back));
                cin += ld_agent(&agg[pg * KP + j]);
            }
        }
        s_carry[j] = cin;
    }
    __syncthreads();

    // final values
    T rc = s_exhs[r] ? s_excl[r][j] : (T)(s_carry[j] + s_excl[r][j]);
    double dacc = 0.0, mx = 0.0;
#pragma unroll
    for (int q = 0; q < NPR; q++) {
        int sidx = r * NPR + q;
        long long pos = p0 + (UP ? (TN - 1 - sidx) : sidx);
        T out = pre[q] ? vals[q] : (T)(rc + vals[q]);
        if (UP) {
            if (act) F[pos * k + j] = out;
        } else {
            int v = perm[pos];
            if (v >= 0 && act) {
                xout[(long long)v * k + j] = out;
                if (rdot) dacc += (double)rdot[(long long)v * k + j] * (double)out;
                double ao = fabs((double)out);
                mx = ao > mx ? ao : mx;
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
                for (int w = 0; w < kThreads / 64; w++) m2 = s_max[w] > m2 ? s_max[w] : m2;
                if (m2 > 0.0) atomicMax(absmax, (unsigned long long)__double_as_longlong(m2));
            }
        }
    }
}

// ------------------------------------------------------------ scoring
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_score(long long m, int k, const int *__restrict__ src,
                                                    const int *__restrict__ dst, const T *__restrict__ wT,
                                                    const uint8_t *__restrict__ mask, const T *__restrict__ H,
                                                    T *__restrict__ heat, double *__restrict__ part,
                                                    unsigned long long *__restrict__ hmax) {
    constexpr int G = kThreads / KP;
    constexpr int EPB = G * kEdgesPerGroup;
    __shared__ double s_num[G][KP];
    __shared__ double s_den[G][KP];
    __shared__ double s_max[kThreads / 64];
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    double num = 0.0, den = 0.0, hm = 0.0;
    long long e0 = (long long)blockIdx.x * EPB;
    for (int i = g; i < EPB; i += G) {
        long long e = e0 + i;
        if (e >= m) break;
        int p = src[e], q = dst[e];
        T w = wT[e];
        bool inP = mask[e] != 0;
        T d = act ? (T)(H[(long long)p * k + j] - H[(long long)q * k + j]) : (T)0;
        T sq = d * d;
#pragma unroll
        for (int off = KP / 2; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
        T h = w * sq;
        if (heat && j == 0) heat[e] = h;
        double cw = (double)w * (double)d * (double)d;
        num += cw;
        if (inP) den += cw;
        else hm = (double)h > hm ? (double)h : hm;
    }
    s_num[g][j] = num;
    s_den[g][j] = den;
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(hm, off, 64);
        hm = o > hm ? o : hm;
    }
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = hm;
    __syncthreads();
    if (g == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < G; q++) {
            a += s_num[q][j];
            b += s_den[q][j];
        }
        part[(long long)blockIdx.x * 2 * KP + j] = a;
        part[(long long)blockIdx.x * 2 * KP + KP + j] = b;
    }
    if (threadIdx.x == 0) {
        double m2 = 0.0;
        for (int w = 0; w < kThreads / 64; w++) m2 = s_max[w] > m2 ? s_max[w] : m2;
        if (m2 > 0.0) atomicMax(hmax, (unsigned long long)__double_as_longlong(m2));
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

// ------------------------------------------------------------ PCG pieces
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_axpy2(long long n, int k, const double *__restrict__ alpha,
                                                    const T *__restrict__ p, const T *__restrict__ q,
                                                    T *__restrict__ x, T *__restrict__ r, double *__restrict__ part) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    __shared__ double sh[G][KP];
    int g = threadIdx.x / KP, j = threadIdx.x % KP;
    double acc = 0.0;
    if (j < k) {
        T a = (T)alpha[j];
        long long r0 = (long long)blockIdx.x * RPB;
        for (int i = g; i < RPB; i += G) {
            long long v = r0 + i;
            if (v >= n) break;
            long long o = v * k + j;
            x[o] += a * p[o];
            T rn = r[o] - a * q[o];
            r[o] = rn;
            acc += (double)rn * (double)rn;
        }
    }
    sh[g][j] = acc;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int q2 = 0; q2 < G; q2++) t += sh[q2][j];
        part[(long long)blockIdx.x * KP + j] = t;
    }
}

template <typename T>
__global__ void k_xpby(long long nk, int k, const double *__restrict__ beta, const T *__restrict__ z,
                       T *__restrict__ p) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x) {
        int j = (int)(i % k);
        p[i] = z[i] + (T)beta[j] * p[i];
    }
}

template <typename T>
__global__ void k_copy(long long nk, const T *__restrict__ a, T *__restrict__ b) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// alpha_j = rz_j / (p_j' L_P p_j) for active vectors, 0 otherwise
__global__ void k_pcg_alpha(double *__restrict__ red, int *__restrict__ active, int k) {
    int j = threadIdx.x;
    if (j >= k) return;
    double pq = red[RED_PQ * kMaxK + j], rz = red[RED_RZ * kMaxK + j];
    double a = 0.0;
    if (active[j]) {
        if (pq > 0.0 && rz > 0.0) a = rz / pq;
        else active[j] = 0;
    }
    red[RED_ALPHA * kMaxK + j] = a;
}
// deactivate converged vectors; count the active ones
__global__ void k_pcg_check(double *__restrict__ red, int *__restrict__ active, int k, double tol2) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int j = threadIdx.x;
    if (j < k && active[j]) {
        double rr = red[RED_RR * kMaxK + j], rr0 = red[RED_RR0 * kMaxK + j];
        if (!(rr > tol2 * rr0)) active[j] = 0;
        else atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) active[kMaxK - 1] = cnt;
}
__global__ void k_pcg_beta(double *__restrict__ red, const int *__restrict__ active, int k) {
    int j = threadIdx.x;
    if (j >= k) return;
    double rzn = red[RED_RZN * kMaxK + j], rz = red[RED_RZ * kMaxK + j];
    double b = 0.0;
    if (active[j] && rz > 0.0) b = rzn / rz;
    red[RED_BETA * kMaxK + j] = b;
    red[RED_RZ * kMaxK + j] = rzn;
}
__global__ void k_pcg_start(const double *__restrict__ red_rn, double *__restrict__ red, int *__restrict__ active,
                            int k) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int j = threadIdx.x;
    if (j < kMaxK - 1) active[j] = 0;
    if (j < k) {
        double rr0 = red_rn[j];
        red[RED_RR0 * kMaxK + j] = rr0;
        active[j] = rr0 > 0.0 ? 1 : 0;
        if (rr0 > 0.0) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) active[kMaxK - 1] = cnt;
}

// r = b - L_P x in FP64 (difference form), grounded at root; r32 = r rounded to T
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_resid64(long long n, int k, const int *__restrict__ prow,
                                                      const int *__restrict__ pcol, const double *__restrict__ pval,
                                                      const T *__restrict__ b, const double *__restrict__ x,
                                                      T *__restrict__ r32, int root, double *__restrict__ part,
                                                      int nblk) {
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
__global__ void k_add_dx(long long nk, double *__restrict__ x64, const T *__restrict__ dx) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x)
        x64[i] += (double)dx[i];
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

inline int grid_nk(long long nk) { return (int)std::min<long long>(std::max<long long>(1, (nk + 255) / 256), 8192); }

}  // namespace

// ============================================================= host side

static int lap_blocks(const Dims &d) { return div_up(d.n, (kThreads / d.kp) * kRowsPerGroup); }
static int score_blocks(const Dims &d) { return div_up(d.m, (kThreads / d.kp) * kEdgesPerGroup); }
static int gauss_blocks(const Dims &d) {
    return (int)std::min<long long>(kGaussBlocksMax, div_up(d.n, kThreads / d.kp));
}

template <typename T>
void plan_vecs(Arena &a, const Dims &d, Vecs<T> &v) {
    long long n = d.n, m = d.m, nk = n * d.k;
    v.wT = a.take<T>(m);
    v.cval = a.take<T>(2 * m);
    v.pval = a.take<T>(2 * m);
    v.rpw = a.take<T>(d.Npad + 1);
    v.H = a.take<T>(nk);
    v.Y = a.take<T>(nk);
    v.F = a.take<T>((d.Npad + 1) * d.k);
    v.agg = a.take<T>(d.ntiles * d.kp);
    v.heat = a.take<T>(m);
    v.r = a.take<T>(nk);
    v.z = a.take<T>(nk);
    v.p = a.take<T>(nk);
    v.q = a.take<T>(nk);
    v.dx = a.take<T>(nk);
    v.x64 = a.take<double>(nk);
    v.r64 = nullptr;
    long long parts = std::max<long long>({(long long)lap_blocks(d) + 8, d.ntiles, 2ll * score_blocks(d),
                                           (long long)gauss_blocks(d)});
    v.part = a.take<double>(parts * d.kp + 64);
    v.red = a.take<double>(RED_SLOTS * kMaxK);
    v.active = a.take<int>(kMaxK);
    v.u64s = a.take<unsigned long long>(U_SLOTS);
}

template <typename T>
void start_vectors(const Dims &d, uint64_t seed, int pass, T *out, Vecs<T> &v, hipStream_t s) {
    int nb = gauss_blocks(d);
    double *mean = v.red + RED_MEAN * kMaxK;
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL(k_gauss_sum<KP>, dim3(nb), dim3(kThreads), 0, s, d.n, d.k, (unsigned long long)seed, pass,
                           v.part);
        hipLaunchKernelGGL(k_col_sum<KP>, dim3(1), dim3(kThreads), 0, s, v.part, nb, KP, 0, 1.0 / (double)d.n, mean);
        hipLaunchKernelGGL((k_gauss_write<T, KP>), dim3(nb), dim3(kThreads), 0, s, d.n, d.k, (unsigned long long)seed,
                           pass, mean, out);
    });
    GR_CHECK_LAUNCH();
}

template <typename T>
void lap_apply(const Dims &d, const int *rowptr, const int *col, const T *val, const T *x, T *y, int root,
               const unsigned long long *scale_from, double *dot_part, hipStream_t s) {
    int nb = lap_blocks(d);
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL((k_lap<T, KP>), dim3(xcd_grid(nb)), dim3(kThreads), 0, s, d.n, d.k, rowptr, col, val, x, y,
                           root, scale_from, dot_part, nb);
    });
    GR_CHECK_LAUNCH();
}

template <typename T>
void tree_solve(Topo &t, Vecs<T> &v, const Dims &d, const T *y, T *x, const T *rdot, double *dot_part,
                unsigned long long *absmax, hipStream_t s) {
    fill_i32(t.tickets, 2 * kMaxLevels, 0, s);
    if (dot_part) fill_f64(dot_part, (t.N / d.TN) * d.kp, 0.0, s);
    unsigned e_up = ++t.epoch;
    unsigned e_dn = ++t.epoch;
    KP_DISPATCH(d.kp, {
        for (int l = t.nlev - 1; l >= 0; l--) {
            long long lp0 = t.lvl_start[l];
            int nt = (int)((t.lvl_start[l + 1] - lp0) / d.TN);
            if (nt == 0) continue;
            hipLaunchKernelGGL((k_sweep<T, KP, true>), dim3(nt), dim3(kThreads), 0, s, lp0, nt, lp0 / d.TN, d.k, t.perm,
                               t.flags, t.ptop, t.lc_ptr, t.lc_pos, v.rpw, y, v.F, x, v.agg, t.hs, t.status, e_up,
                               t.tickets + 2 * l, t.devflags, (const T *)nullptr, (double *)nullptr,
                               (unsigned long long *)nullptr);
        }
        for (int l = 0; l < t.nlev; l++) {
            long long lp0 = t.lvl_start[l];
            int nt = (int)((t.lvl_start[l + 1] - lp0) / d.TN);
            if (nt == 0) continue;
            hipLaunchKernelGGL((k_sweep<T, KP, false>), dim3(nt), dim3(kThreads), 0, s, lp0, nt, lp0 / d.TN, d.k,
                               t.perm, t.flags, t.ptop, t.lc_ptr, t.lc_pos, v.rpw, y, v.F, x, v.agg, t.hs, t.status,
                               e_dn, t.tickets + 2 * l + 1, t.devflags, rdot, dot_part, absmax);
        }
    });
    GR_CHECK_LAUNCH();
}

template <typename T>
void absmax_of(const Dims &d, const T *x, unsigned long long *slot, hipStream_t s) {
    long long nk = d.n * d.k;
    hipLaunchKernelGGL(k_absmax<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, x, slot);
    GR_CHECK_LAUNCH();
}

template <typename T>
static void col_sum(const Dims &d, const double *part, int nblk, int stride, int offset, double *out, hipStream_t s) {
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL(k_col_sum<KP>, dim3(1), dim3(kThreads), 0, s, part, nblk, stride, offset, 1.0, out);
    });
    GR_CHECK_LAUNCH();
}

template <typename T>
SolveInfo pcg_solve(Topo &t, Vecs<T> &v, const Dims &d, const T *b, T *x, const grass_opts &o, hipStream_t s) {
    SolveInfo info;
    const long long nk = d.n * d.k;
    const int root = 0;
    const int nbl = lap_blocks(d);
    double *red = v.red;
    double *bn = red + RED_BN * kMaxK, *rn = red + RED_RN * kMaxK;
    // ||b|| per vector (grounded rows)
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL((k_norm2<T, KP>), dim3(nbl), dim3(kThreads), 0, s, d.n, d.k, b, root, v.part);
    });
    GR_CHECK_LAUNCH();
    col_sum<T>(d, v.part, nbl, d.kp, 0, bn, s);
    fill_f64(v.x64, nk, 0.0, s);
    std::vector<double> hb(2 * kMaxK);
    const double rtol = o.pcg_rtol > 0 ? o.pcg_rtol : 1e-6;
    const double itol = o.pcg_inner_rtol > 0 ? o.pcg_inner_rtol : 1e-3;
    const int max_outer = o.pcg_max_outer > 0 ? o.pcg_max_outer : 6;
    const int max_it = o.pcg_max_iters > 0 ? o.pcg_max_iters : 2000;
    for (int outer = 0;; outer++) {
        KP_DISPATCH(d.kp, {
            hipLaunchKernelGGL((k_resid64<T, KP>), dim3(xcd_grid(nbl)), dim3(kThreads), 0, s, d.n, d.k, t.prow, t.pcol,
                               t.pval64, b, v.x64, v.r, root, v.part, nbl);
        });
        GR_CHECK_LAUNCH();
        col_sum<T>(d, v.part, nbl, d.kp, 0, rn, s);
        GR_HIP(hipMemcpyAsync(hb.data(), bn, 2 * kMaxK * sizeof(double), hipMemcpyDeviceToHost, s));
        GR_HIP(hipStreamSynchronize(s));
        double worst = 0.0;
        for (int j = 0; j < d.k; j++) {
            double bj = std::sqrt(hb[j]), rj = std::sqrt(hb[kMaxK + j]);
            double rel = bj > 0 ? rj / bj : 0.0;
            worst = rel > worst ? rel : worst;
        }
        info.resid64 = worst;
        info.outer = outer;
        if (worst <= rtol || outer >= max_outer) break;
        // inner PCG on the residual: dx = L_P^+ r, r and dx updated in place
        fill_f64(red + RED_RZ * kMaxK, kMaxK, 0.0, s);
        hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(64), 0, s, rn, red, v.active, d.k);
        GR_CHECK_LAUNCH();
        fill_T(v.dx, nk, (T)0, s);
        tree_solve<T>(t, v, d, v.r, v.z, v.r, v.part, nullptr, s);
        col_sum<T>(d, v.part, (int)(t.N / d.TN), d.kp, 0, red + RED_RZ * kMaxK, s);
        hipLaunchKernelGGL(k_copy<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, v.z, v.p);
        GR_CHECK_LAUNCH();
        long long it = 0;
        for (; it < max_it;) {
            it++;
            lap_apply<T>(d, t.prow, t.pcol, v.pval, v.p, v.q, root, nullptr, v.part, s);
            col_sum<T>(d, v.part, nbl, d.kp, 0, red + RED_PQ * kMaxK, s);
            hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(64), 0, s, red, v.active, d.k);
            KP_DISPATCH(d.kp, {
                hipLaunchKernelGGL((k_axpy2<T, KP>), dim3(nbl), dim3(kThreads), 0, s, d.n, d.k,
                                   red + RED_ALPHA * kMaxK, v.p, v.q, v.dx, v.r, v.part);
            });
            GR_CHECK_LAUNCH();
            col_sum<T>(d, v.part, nbl, d.kp, 0, red + RED_RR * kMaxK, s);
            hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(64), 0, s, red, v.active, d.k, itol * itol);
            GR_CHECK_LAUNCH();
            if ((it & 7) == 0 || it == max_it) {
                if (read_i32(v.active + kMaxK - 1, s) == 0) break;
            }
            tree_solve<T>(t, v, d, v.r, v.z, v.r, v.part, nullptr, s);
            col_sum<T>(d, v.part, (int)(t.N / d.TN), d.kp, 0, red + RED_RZN * kMaxK, s);
            hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(64), 0, s, red, v.active, d.k);
            hipLaunchKernelGGL(k_xpby<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, d.k, red + RED_BETA * kMaxK,
                               v.z, v.p);
            GR_CHECK_LAUNCH();
        }
        info.iters += it;
        hipLaunchKernelGGL(k_add_dx<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, v.x64, v.dx);
        GR_CHECK_LAUNCH();
    }
    fill_u32(reinterpret_cast<unsigned *>(v.u64s + U_ABSMAX), 2, 0u, s);
    hipLaunchKernelGGL(k_x64_out<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, v.x64, x, v.u64s + U_ABSMAX);
    GR_CHECK_LAUNCH();
    return info;
}

template <typename T>
void score_edges(Topo &t, Vecs<T> &v, const Dims &d, const T *H, T *heat, hipStream_t s) {
    int nb = score_blocks(d);
    fill_u32(reinterpret_cast<unsigned *>(v.u64s + U_HMAX), 2, 0u, s);
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL((k_score<T, KP>), dim3(nb), dim3(kThreads), 0, s, d.m, d.k, t.src, t.dst, v.wT, t.mask, H,
                           heat, v.part, v.u64s + U_HMAX);
        GR_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_col_sum<KP>, dim3(1), dim3(kThreads), 0, s, v.part, nb, 2 * KP, 0, 1.0,
                           v.red + RED_NUM * kMaxK);
        hipLaunchKernelGGL(k_col_sum<KP>, dim3(1), dim3(kThreads), 0, s, v.part, nb, 2 * KP, KP, 1.0,
                           v.red + RED_DEN * kMaxK);
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
    template void lap_apply<T>(const Dims &, const int *, const int *, const T *, const T *, T *, int,           \
                               const unsigned long long *, double *, hipStream_t);                               \
    template void tree_solve<T>(Topo &, Vecs<T> &, const Dims &, const T *, T *, const T *, double *,            \
                                unsigned long long *, hipStream_t);                                              \
    template SolveInfo pcg_solve<T>(Topo &, Vecs<T> &, const Dims &, const T *, T *, const grass_opts &,         \
                                    hipStream_t);                                                                \
    template void score_edges<T>(Topo &, Vecs<T> &, const Dims &, const T *, T *, hipStream_t);                  \
    template PassScalars finish_estimates<T>(Topo &, Vecs<T> &, const Dims &, hipStream_t);                      \
    template void absmax_of<T>(const Dims &, const T *, unsigned long long *, hipStream_t);
INST(float)
INST(double)

}  // namespace grass
