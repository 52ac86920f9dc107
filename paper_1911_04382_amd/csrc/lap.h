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
template <int E>
struct LapShape {
    static constexpr int NIT = E <= 4 ? 4 : 2;  // rows per lane group
};

// One tile of NT / KP lane groups x NIT rows from row r0 (NT threads per block): a lane group of KP
// lanes owns one row per step. Two dependent memory rounds: the neighbour lists
// (lap_load), then everything else at once (lap_fetch: own values, degrees,
// weights and neighbour rows); lap_rows forms and stores y. Each round issues all
// of a lane's loads together, and a caller walking several tiles can overlap the
// next tile's first round with this tile's second.
template <int E>
struct LapCols {
    int cn[LapShape<E>::NIT][E];
};
template <typename T, int E>
struct LapFetch {
    static constexpr int NIT = LapShape<E>::NIT;
    T xv[NIT], wn[NIT][E], xn[NIT][E];
    int dg[NIT];
};

template <int KP, int E, int NT = kThreads>
__device__ __forceinline__ void lap_load(long long r0, long long n, const int *__restrict__ ecol, LapCols<E> &L) {
    constexpr int G = NT / KP;
    const int g = threadIdx.x / KP;
#pragma unroll
    for (int it = 0; it < LapShape<E>::NIT; it++) {
        const long long v = r0 + g + it * G;
        const long long vv = v < n ? v : 0;  // rows past n read row 0; lap_rows masks them
#pragma unroll
        for (int e = 0; e < E; e++) L.cn[it][e] = ecol[vv * E + e];
    }
}

template <typename T, int KP, int E, int NT = kThreads>
__device__ __forceinline__ void lap_fetch(long long r0, long long n, int k, const T *__restrict__ eval,
                                          const int *__restrict__ edeg, const T *__restrict__ x,
                                          const LapCols<E> &L, LapFetch<T, E> &F) {
    constexpr int G = NT / KP;
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
#pragma unroll
    for (int it = 0; it < LapShape<E>::NIT; it++) {
        const long long v = r0 + g + it * G;
        const long long vv = v < n ? v : 0;
        F.xv[it] = x[act ? vv * k + j : 0];
        F.dg[it] = edeg[vv];
#pragma unroll
        for (int e = 0; e < E; e++) {
            F.wn[it][e] = eval[vv * E + e];
            F.xn[it][e] = x[act ? (long long)L.cn[it][e] * k + j : 0];
        }
    }
}

// Row `root` is grounded (y = 0); y is scaled by sc. xo / yo return this lane's x
// and y values (0 outside the matrix), for products that also reduce over rows.
template <typename T, int KP, int E, int NT = kThreads>
__device__ __forceinline__ void lap_rows(long long r0, long long n, int k, const int *__restrict__ rowptr,
                                         const int *__restrict__ col, const T *__restrict__ val,
                                         const T *__restrict__ ltail, const T *__restrict__ x, T *__restrict__ y,
                                         int root, T sc, const LapFetch<T, E> &F, T (&xo)[LapShape<E>::NIT],
                                         T (&yo)[LapShape<E>::NIT]) {
    constexpr int G = NT / KP;
    constexpr int NIT = LapShape<E>::NIT;
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
#pragma unroll
    for (int it = 0; it < NIT; it++) {
        const long long v = r0 + g + it * G;
        T acc = 0;
#pragma unroll
        for (int e = 0; e < E; e++) acc += F.wn[it][e] * (F.xv[it] - F.xn[it][e]);
        if (F.dg[it] < 0) {  // a long row: the rest was summed by lap_long
            acc += act ? ltail[(long long)(-F.dg[it] - 1) * k + j] : (T)0;
        } else if (v < n && F.dg[it] > E) {  // the rest of a row of at most kLongRow entries
            const int p0 = rowptr[v], p1 = rowptr[v + 1];
            for (int p = p0 + E; p < p1; p++) acc += val[p] * (F.xv[it] - x[(long long)col[p] * k + j]);
        }
        const bool live = act && v < n;
        acc *= sc;
        if (v == root) acc = 0;
        if (live) y[v * k + j] = acc;
        xo[it] = live ? F.xv[it] : (T)0;
        yo[it] = live ? acc : (T)0;
    }
}

// One tile on its own: the own values and weights join the first round (the
// second then holds only the neighbour rows)
template <typename T, int KP, int E>
__device__ __forceinline__ void lap_tile(long long r0, long long n, int k, const int *__restrict__ rowptr,
                                         const int *__restrict__ col, const T *__restrict__ val,
                                         const T *__restrict__ ltail, const int *__restrict__ ecol,
                                         const T *__restrict__ eval,
                                         const int *__restrict__ edeg, const T *__restrict__ x, T *__restrict__ y,
                                         int root, T sc, T (&xo)[LapShape<E>::NIT], T (&yo)[LapShape<E>::NIT]) {
    constexpr int G = kThreads / KP;
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    LapCols<E> L;
    LapFetch<T, E> F;
#pragma unroll
    for (int it = 0; it < LapShape<E>::NIT; it++) {
        const long long v = r0 + g + it * G;
        const long long vv = v < n ? v : 0;
        F.xv[it] = x[act ? vv * k + j : 0];
        F.dg[it] = edeg[vv];
#pragma unroll
        for (int e = 0; e < E; e++) {
            L.cn[it][e] = ecol[vv * E + e];
            F.wn[it][e] = eval[vv * E + e];
        }
    }
#pragma unroll
    for (int it = 0; it < LapShape<E>::NIT; it++)
#pragma unroll
        for (int e = 0; e < E; e++) F.xn[it][e] = x[act ? (long long)L.cn[it][e] * k + j : 0];
    lap_rows<T, KP, E>(r0, n, k, rowptr, col, val, ltail, x, y, root, sc, F, xo, yo);
}

// The entries past E of the long rows (ell list lrow), one workgroup per row: lane
// groups take every G-th entry, and the group sums are added in group order, so
// the result does not depend on timing. tail[li*k + j] feeds lap_rows.
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_lap_long(int k, int E, const int *__restrict__ rowptr,
                                                       const int *__restrict__ col, const T *__restrict__ val,
                                                       const int *__restrict__ lrow, const T *__restrict__ x,
                                                       T *__restrict__ tail) {
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
