// Laplacian products y = L x for k vectors at once (eq. 1), shared by the plain
// product kernel and the PCG product that also forms the block Gram matrices.
#pragma once
#include "kern.h"

namespace grass {

// 2^-e with e the exponent of the value stored (as FP64 bits) at slot: a power of
// two, so scaling by it is exact; 1 when there is no slot or no finite positive value
__device__ __forceinline__ double pow2_scale(const unsigned long long *slot) {
    if (!slot) return 1.0;
    double mx = __longlong_as_double((long long)*slot);
    if (!(mx > 0.0) || !(mx < INFINITY)) return 1.0;
    return ldexp(1.0, -ilogb(mx));
}

// Rows are taken over the padded first E entries of each row (rows longer than E
// finish from the CSR). The difference form y_v = sum_u w_vu (x_v - x_u) keeps
// FP32 accurate for smooth x.
// rows per lane group: 4 (C2: 2 -> 4 took the L_G product 118 -> 112 us); narrow
// blocks (k <= 2) fewer, so that a wave's staged rows stay within 512 entries
constexpr int lap_nit(int kp) { return kp >= 4 ? 4 : kp; }
template <int KP>
struct LapShape {
    static constexpr int NIT = lap_nit(KP);
};

// A tile of NT / KP lane groups x NIT rows from row r0 (NT threads per block): lane
// group g owns rows r0 + g*NIT .. r0 + g*NIT + NIT - 1, so each wave owns WR
// consecutive rows. Two dependent memory rounds:
//  - lap_load: the wave's padded rows (columns, weights, lengths) with coalesced
//    loads, one element per lane (a few loads per wave instead of one broadcast
//    load per entry and row);
//  - lap_fetch: the staged rows go to the wave's slice of LDS, every lane reads its
//    rows' columns there and issues its own values and all neighbour gathers at once;
// lap_rows then forms and stores y. A caller walking several tiles can overlap the
// next tile's first round with this tile's second.
template <typename T, int KP, int E>
struct LapTile {
    static constexpr int NIT = LapShape<KP>::NIT;
    static constexpr int WR = (KP < 64 ? 64 / KP : 1) * NIT;  // rows per wave
    static constexpr int NE = WR * E;                          // padded entries per wave
    static constexpr int CPL = (NE + 63) / 64;                 // staged entries per lane
    static constexpr int DPL = (WR + 63) / 64;                 // staged lengths per lane
    // LDS bytes of one wave's slice
    static constexpr int SLICE = NE * (int)sizeof(int) + NE * (int)sizeof(T) + WR * (int)sizeof(int);
    __device__ static long long row(long long r0, int g, int it) { return r0 + (long long)g * NIT + it; }
};
template <typename T, int KP, int E>
struct LapStage {  // one lane's share of its wave's padded rows, in flight
    int c[LapTile<T, KP, E>::CPL];
    T w[LapTile<T, KP, E>::CPL];
    int dg[LapTile<T, KP, E>::DPL];
};
template <typename T, int KP, int E>
struct LapFetch {
    static constexpr int NIT = LapShape<KP>::NIT;
    T xv[NIT], xn[NIT][E];
};

template <typename T, int KP, int E>
__device__ __forceinline__ void lap_load(long long r0, long long n, const int *__restrict__ ecol,
                                         const T *__restrict__ eval, const int *__restrict__ edeg,
                                         LapStage<T, KP, E> &S) {
    using L = LapTile<T, KP, E>;
    const int lane = threadIdx.x & 63;
    const long long w0 = r0 + (long long)(threadIdx.x >> 6) * L::WR;  // the wave's first row
    const long long lim = n * E;
    // the padded rows stream through once (each line is read whole by one wave):
    // non-temporal loads leave L2 to the vector rows that later tiles gather again
#pragma unroll
    for (int c = 0; c < L::CPL; c++) {
        const long long i = w0 * E + lane + 64 * c;
        const long long ii = i < lim ? i : 0;  // rows past n read row 0; lap_rows masks them
        S.c[c] = __builtin_nontemporal_load(&ecol[ii]);
        S.w[c] = __builtin_nontemporal_load(&eval[ii]);
    }
#pragma unroll
    for (int c = 0; c < L::DPL; c++) {
        const long long v = w0 + lane + 64 * c;
        S.dg[c] = __builtin_nontemporal_load(&edeg[v < n ? v : 0]);
    }
}

// the wave's slice of LDS: columns [NE], weights [NE], lengths [WR]
template <typename T, int KP, int E>
__device__ __forceinline__ char *lap_slice(char *lds) {
    return lds + (threadIdx.x >> 6) * LapTile<T, KP, E>::SLICE;
}

template <typename T, int KP, int E>
__device__ __forceinline__ void lap_fetch(long long r0, long long n, int k, const T *__restrict__ x,
                                          const LapStage<T, KP, E> &S, char *lds, LapFetch<T, KP, E> &F) {
    using L = LapTile<T, KP, E>;
    constexpr int G = 64 / (KP < 64 ? KP : 64);  // lane groups per wave
    (void)G;
    char *sl = lap_slice<T, KP, E>(lds);
    int *scol = reinterpret_cast<int *>(sl);
    T *sval = reinterpret_cast<T *>(sl + L::NE * sizeof(int));
    int *sdeg = reinterpret_cast<int *>(sl + L::NE * (sizeof(int) + sizeof(T)));
    const int lane = threadIdx.x & 63;
    // the previous tile's reads of this slice are done before it is overwritten
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < L::CPL; c++) {
        const int i = lane + 64 * c;
        if (i < L::NE) {
            scol[i] = S.c[c];
            sval[i] = S.w[c];
        }
    }
#pragma unroll
    for (int c = 0; c < L::DPL; c++) {
        const int i = lane + 64 * c;
        if (i < L::WR) sdeg[i] = S.dg[c];
    }
    // the wave's writes are seen by its later reads (one wave, in order)
    __builtin_amdgcn_wave_barrier();
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const int gw = (threadIdx.x & 63) / (KP < 64 ? KP : 64);  // lane group within the wave
    const bool act = j < k;
#pragma unroll
    for (int it = 0; it < L::NIT; it++) {
        const long long v = L::row(r0, g, it);
        const long long vv = v < n ? v : 0;
        F.xv[it] = x[act ? vv * k + j : 0];
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int cn = scol[(gw * L::NIT + it) * E + e];
            F.xn[it][e] = x[act ? (long long)cn * k + j : 0];
        }
    }
}

// Row `root` is grounded (y = 0); y is scaled by sc. xo / yo return this lane's x
// and y values (0 outside the matrix), for products that also reduce over rows.
// NTS: store y non-temporally (a product whose output is not read again soon).
template <typename T, int KP, int E, bool NTS = false>
__device__ __forceinline__ void lap_rows(long long r0, long long n, int k, const int *__restrict__ rowptr,
                                         const int *__restrict__ col, const T *__restrict__ val,
                                         const T *__restrict__ ltail, const T *__restrict__ x, T *__restrict__ y,
                                         int root, T sc, const LapFetch<T, KP, E> &F, char *lds,
                                         T (&xo)[LapShape<KP>::NIT], T (&yo)[LapShape<KP>::NIT]) {
    using L = LapTile<T, KP, E>;
    constexpr int NIT = LapShape<KP>::NIT;
    char *sl = lap_slice<T, KP, E>(lds);
    const T *sval = reinterpret_cast<const T *>(sl + L::NE * sizeof(int));
    const int *sdeg = reinterpret_cast<const int *>(sl + L::NE * (sizeof(int) + sizeof(T)));
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const int gw = (threadIdx.x & 63) / (KP < 64 ? KP : 64);
    const bool act = j < k;
#pragma unroll
    for (int it = 0; it < NIT; it++) {
        const long long v = L::row(r0, g, it);
        const int rl = gw * NIT + it;  // the row within the wave's slice
        const int dg = sdeg[rl];
        T acc = 0;
#pragma unroll
        for (int e = 0; e < E; e++) acc += sval[rl * E + e] * (F.xv[it] - F.xn[it][e]);
        if (dg < 0) {  // a long row: the rest was summed by lap_long
            acc += act ? ltail[(long long)(-dg - 1) * k + j] : (T)0;
        } else if (v < n && dg > E) {  // the rest of a row of at most kLongRow entries
            const int p0 = rowptr[v], p1 = rowptr[v + 1];
            for (int p = p0 + E; p < p1; p++) acc += val[p] * (F.xv[it] - x[(long long)col[p] * k + j]);
        }
        const bool live = act && v < n;
        acc *= sc;
        if (v == root) acc = 0;
        if (live) {
            if constexpr (NTS)
                __builtin_nontemporal_store(acc, &y[v * k + j]);
            else
                y[v * k + j] = acc;
        }
        xo[it] = live ? F.xv[it] : (T)0;
        yo[it] = live ? acc : (T)0;
    }
}

// One tile on its own: both rounds back to back
template <typename T, int KP, int E, bool NTS = false>
__device__ __forceinline__ void lap_tile(long long r0, long long n, int k, const int *__restrict__ rowptr,
                                         const int *__restrict__ col, const T *__restrict__ val,
                                         const T *__restrict__ ltail, const int *__restrict__ ecol,
                                         const T *__restrict__ eval, const int *__restrict__ edeg,
                                         const T *__restrict__ x, T *__restrict__ y, int root, T sc, char *lds,
                                         T (&xo)[LapShape<KP>::NIT], T (&yo)[LapShape<KP>::NIT]) {
    LapStage<T, KP, E> S;
    LapFetch<T, KP, E> F;
    lap_load<T, KP, E>(r0, n, ecol, eval, edeg, S);
    lap_fetch<T, KP, E>(r0, n, k, x, S, lds, F);
    lap_rows<T, KP, E, NTS>(r0, n, k, rowptr, col, val, ltail, x, y, root, sc, F, lds, xo, yo);
}

// ---------------------------------------------------------------------------
// Rows as 16-byte slices: for k a power of two of at least 16 / sizeof(T)
// values, a row of k values is read by k / W lanes with one 16-byte access each
// (W = 4 floats or 2 doubles), so a wave gathers 64 / (k / W) rows per load
// instruction instead of 64 / k. On the 100^3 mesh at k = 32 a six-neighbour
// gather took 83 us with one value per lane and 65 us with 16 bytes per lane.
template <typename T>
struct V16;
template <>
struct V16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int W = 4;
};
template <>
struct V16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int W = 2;
};

// y = L x over the padded rows with 16-byte lanes (see k_lap for the layout of the
// padded rows and the long-row tail). One row per group of KP / W lanes, RW rows
// per wave; the wave stages its rows' padded entries in LDS with coalesced
// non-temporal loads first. NTS: store y non-temporally.
template <typename T, int KP, int E, bool NTS>
__global__ __launch_bounds__(256) void k_lapv(long long n, const int *__restrict__ rowptr, const int *__restrict__ col,
                                               const T *__restrict__ val, const T *__restrict__ ltail,
                                               const int *__restrict__ ecol, const T *__restrict__ eval,
                                               const int *__restrict__ edeg, const T *__restrict__ x,
                                               T *__restrict__ y, int root,
                                               const unsigned long long *__restrict__ scale_from, int nblk) {
    using V = typename V16<T>::type;
    constexpr int W = V16<T>::W, LPR = KP / W, RW = 64 / LPR, NW = 256 / 64, RPB = NW * RW, NE = RW * E;
    constexpr int CPL = (NE + 63) / 64;
    static_assert(KP % W == 0 && LPR <= 64, "rows of whole 16-byte slices");
    __shared__ __align__(16) int s_col[NW][NE];
    __shared__ __align__(16) T s_val[NW][NE];
    __shared__ int s_deg[NW][RW];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= nblk) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long w0 = (long long)b * RPB + (long long)wv * RW;
    const long long lim = n * E;
#pragma unroll
    for (int c = 0; c < CPL; c++) {
        const int i = lane + 64 * c;
        if (i < NE) {
            const long long ii = w0 * E + i < lim ? w0 * E + i : 0;
            s_col[wv][i] = __builtin_nontemporal_load(&ecol[ii]);
            s_val[wv][i] = __builtin_nontemporal_load(&eval[ii]);
        }
    }
    if (lane < RW) s_deg[wv][lane] = __builtin_nontemporal_load(&edeg[w0 + lane < n ? w0 + lane : 0]);
    __builtin_amdgcn_wave_barrier();  // one wave: its LDS writes are seen by its later reads
    const int r = lane / LPR, c = lane % LPR;
    const long long v = w0 + r, vv = v < n ? v : 0;
    const V *xs = reinterpret_cast<const V *>(x);
    const V xv = xs[vv * LPR + c];
    V xn[E];
#pragma unroll
    for (int e = 0; e < E; e++) xn[e] = xs[(long long)s_col[wv][r * E + e] * LPR + c];
    V acc = (T)0;
#pragma unroll
    for (int e = 0; e < E; e++) acc += s_val[wv][r * E + e] * (xv - xn[e]);
    const int dg = s_deg[wv][r];
    if (dg < 0) {  // a long row: the rest was summed by lap_long
        acc += reinterpret_cast<const V *>(ltail)[(long long)(-dg - 1) * LPR + c];
    } else if (v < n && dg > E) {  // the rest of a row of at most kLongRow entries
        const int p0 = rowptr[v], p1 = rowptr[v + 1];
        for (int p = p0 + E; p < p1; p++) acc += val[p] * (xv - xs[(long long)col[p] * LPR + c]);
    }
    acc *= (T)pow2_scale(scale_from);
    if (v == root) acc = (T)0;
    if (v < n) {
        V *ys = reinterpret_cast<V *>(y) + v * LPR + c;
        if constexpr (NTS)
            __builtin_nontemporal_store(acc, ys);
        else
            *ys = acc;
    }
}
template <typename T, int KP>
constexpr bool lapv_ok() {
    return KP >= V16<T>::W;
}

// The entries past E of the long rows (ell list lrow), one workgroup per row: lane
// groups take every G-th entry, and the group sums are added in group order, so
// the result does not depend on timing. tail[li*k + j] feeds lap_rows.
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_lap_long(int k, int E, const int *__restrict__ rowptr,
                                                       const int *__restrict__ col, const T *__restrict__ val,
                                                       const int *__restrict__ lrow, const T *__restrict__ x,
                                                       T *__restrict__ tail, const int *__restrict__ gate = nullptr) {
    if (gate && *gate) return;
    constexpr int G = kThreads / KP, U = 4;
    __shared__ T s[G][KP];
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    const int v = lrow[blockIdx.x];
    const int p0 = rowptr[v] + E, p1 = rowptr[v + 1];
    const T xv = x[act ? (long long)v * k + j : 0];
    T acc = 0;
    for (int p = p0 + g; p < p1; p += G * U) {
        int c[U];
        T w[U], xn[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int q = p + u * G;
            c[u] = col[q < p1 ? q : p0];
            w[u] = val[q < p1 ? q : p0];
        }
#pragma unroll
        for (int u = 0; u < U; u++) xn[u] = x[act ? (long long)c[u] * k + j : 0];
#pragma unroll
        for (int u = 0; u < U; u++) acc += p + u * G < p1 ? w[u] * (xv - xn[u]) : (T)0;
    }
    s[g][j] = acc;
    __syncthreads();
    if (g == 0 && act) {
        T t = 0;
        for (int q = 0; q < G; q++) t += s[q][j];
        tail[(long long)blockIdx.x * k + j] = t;
    }
}

}  // namespace grass
