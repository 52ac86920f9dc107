// Block preconditioned conjugate gradients for the L_P solves of the
// generalized power iteration (eq. 29) once P holds off-tree edges.
//
// The k right-hand sides of one step share one block Krylov space (O'Leary's
// block CG) with the grounded tree solve as preconditioner. Per iteration:
//   Q = L_P P, alpha = (P'Q)^-1 (P'R), X += P alpha, R -= Q alpha,
//   Z = L_T^+ R, beta = -(P'Q)^-1 (Q'Z), P = Z + P beta,
//   P <- P chol(P'P)^-1  (keeps the block well conditioned; a direction that
//                          becomes dependent is dropped).
// The k x k matrices are reduced in a fixed order and factorised in FP64 by one
// workgroup, so results are deterministic. Compared with k independent CG runs
// this needs several times fewer iterations: the block space captures the
// largest generalized eigenvalues of the tree-preconditioned system together.
#include "embed.h"
#include "kern.h"
#include "profiler.h"

namespace grass {

namespace {

template <int KP>
struct BShape {
    static constexpr int G = kThreads / KP;  // lane groups (one vector row each) per block
    static constexpr int RPT = G * 4;        // rows per tile
    static constexpr int CAP = RPT * 12 < 3072 ? RPT * 12 : 3072;  // staged CSR nonzeros per tile (fast path)
};

// persistent blocks: block b owns a contiguous range of row tiles; ranges are
// assigned XCD by XCD so that each XCD streams one contiguous part of the vectors
__device__ __forceinline__ void tile_range(long long ntile, int &t0, int &t1) {
    int b = xcd_block(blockIdx.x, gridDim.x);
    long long per = (ntile + gridDim.x - 1) / gridDim.x;
    long long a = (long long)b * per, e = a + per;
    if (a > ntile) a = ntile;
    if (e > ntile) e = ntile;
    t0 = (int)a;
    t1 = (int)e;
}

template <typename T>
struct Acc {
    using type = float;
};
template <>
struct Acc<double> {
    using type = double;
};

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Gram accumulator C += a'b over the rows a block holds (lane l of a wave: row
// l / KP of the wave, column l % KP). For FP32 with KP = 32 or 16 this is one MFMA
// per 2 (or 4) rows: in that lane layout the A operand of v_mfma_f32_32x32x2f32
// (lane l holds A[l % 32][l / 32]) is exactly a' and the B operand (lane l holds
// B[l / 32][l % 32]) is exactly b, so the instruction accumulates a'b. Other
// widths and FP64 keep per-lane column accumulators fed by shuffles.
// flush(): fixed-order FP64 sum over the block into out (KP x KP, row-major).
template <typename T, int KP, bool MF = (sizeof(T) == 4 && (KP == 32 || KP == 16))>
struct BlockGram {
    static constexpr int LDS = KP * KP;
    using A = typename Acc<T>::type;
    A acc[KP];
    __device__ void zero() {
#pragma unroll
        for (int i = 0; i < KP; i++) acc[i] = 0;
    }
    __device__ void add(T a, T b) {
        const A bb = (A)b;
#pragma unroll
        for (int q = 0; q < KP; q++) acc[q] += (A)__shfl(a, q, KP) * bb;
    }
    __device__ void flush(double *s, double *__restrict__ out) {
        constexpr int G = kThreads / KP;
        const int g = threadIdx.x / KP, j = threadIdx.x % KP;
        __syncthreads();
        for (int e = threadIdx.x; e < KP * KP; e += kThreads) s[e] = 0.0;
        __syncthreads();
        for (int gg = 0; gg < G; gg++) {
            if (g == gg)
                for (int i = 0; i < KP; i++) s[i * KP + j] += (double)acc[i];
            __syncthreads();
        }
        for (int e = threadIdx.x; e < KP * KP; e += kThreads) out[e] = s[e];
        __syncthreads();
    }
};
template <int KP>
__device__ void flush_waves(double *s, double *__restrict__ out) {
    __syncthreads();
    for (int e = threadIdx.x; e < KP * KP; e += kThreads)
        out[e] = ((s[e] + s[KP * KP + e]) + s[2 * KP * KP + e]) + s[3 * KP * KP + e];
    __syncthreads();
}
template <typename T>
struct BlockGram<T, 32, true> {
    static constexpr int LDS = 4 * 32 * 32;
    floatx16 c;
    __device__ void zero() {
#pragma unroll
        for (int r = 0; r < 16; r++) c[r] = 0.f;
    }
    __device__ void add(float a, float b) { c = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
    // accumulator layout: lane l, register r -> C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
    __device__ void flush(double *s, double *__restrict__ out) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; r++)
            s[w * 1024 + (8 * (r / 4) + 4 * (lane / 32) + (r % 4)) * 32 + (lane % 32)] = (double)c[r];
        flush_waves<32>(s, out);
    }
};
template <typename T>
struct BlockGram<T, 16, true> {
    static constexpr int LDS = 4 * 16 * 16;
    floatx4 c;
    __device__ void zero() {
#pragma unroll
        for (int r = 0; r < 4; r++) c[r] = 0.f;
    }
    __device__ void add(float a, float b) { c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // accumulator layout: lane l, register r -> C[4 (l / 16) + r][l % 16]
    __device__ void flush(double *s, double *__restrict__ out) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; r++) s[w * 256 + (4 * (lane / 16) + r) * 16 + (lane % 16)] = (double)c[r];
        flush_waves<16>(s, out);
    }
};

// Q = L_P P (grounded at root) and the Gram partials P'Q, P'R of this block.
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_bspmm(long long n, int k, const int *__restrict__ prow,
                                                    const int *__restrict__ pcol, const T *__restrict__ pval,
                                                    const T *__restrict__ P, T *__restrict__ Q,
                                                    const T *__restrict__ R, int root, double *__restrict__ gpart) {
    constexpr int G = BShape<KP>::G, RPT = BShape<KP>::RPT, CAP = BShape<KP>::CAP;
    __shared__ int s_ptr[RPT + 1];
    __shared__ int s_col[CAP];
    __shared__ T s_val[CAP];
    __shared__ double s_w[BlockGram<T, KP>::LDS];
    const int tid = threadIdx.x, g = tid / KP, j = tid % KP;
    const bool act = j < k;
    BlockGram<T, KP> gpq, gpr;
    gpq.zero();
    gpr.zero();
    long long ntile = (n + RPT - 1) / RPT;
    int t0, t1;
    tile_range(ntile, t0, t1);
    for (int tile = t0; tile < t1; tile++) {
        long long r0 = (long long)tile * RPT;
        int nrows = (int)min((long long)RPT, n - r0);
        __syncthreads();
        for (int i = tid; i <= nrows; i += kThreads) s_ptr[i] = prow[r0 + i];
        __syncthreads();
        int base = s_ptr[0], nnz = s_ptr[nrows] - base;
        bool staged = nnz <= CAP;
        if (staged)
            for (int i = tid; i < nnz; i += kThreads) {
                s_col[i] = pcol[base + i];
                s_val[i] = pval[base + i];
            }
        __syncthreads();
        for (int it = 0; it < RPT / G; it++) {  // every lane runs every iteration (MFMA needs the whole wave)
            int i = g + it * G;
            bool row = i < nrows;
            long long v = r0 + i;
            T pv = (act && row) ? P[v * k + j] : (T)0;
            T rv = (act && row) ? R[v * k + j] : (T)0;
            T acc = 0;
            if (act && row) {
                int p = s_ptr[i] - base, pe = s_ptr[i + 1] - base;
                if (staged) {
                    for (; p + 1 < pe; p += 2) {
                        T x0 = P[(long long)s_col[p] * k + j], x1 = P[(long long)s_col[p + 1] * k + j];
                        acc += s_val[p] * (pv - x0);
                        acc += s_val[p + 1] * (pv - x1);
                    }
                    for (; p < pe; p++) acc += s_val[p] * (pv - P[(long long)s_col[p] * k + j]);
                } else {
                    for (; p < pe; p++) acc += pval[base + p] * (pv - P[(long long)pcol[base + p] * k + j]);
                }
                if (v == root) acc = 0;
                Q[v * k + j] = acc;
            }
            gpq.add(pv, acc);
            gpr.add(pv, rv);
        }
    }
    double *out = gpart + (long long)blockIdx.x * 2 * KP * KP;
    gpq.flush(s_w, out);
    gpr.flush(s_w, out + KP * KP);
}

// Gram partials of this block: A'B, and with NG = 4 also B'B, C'B and C'C.
template <typename T, int KP, int NG>
__global__ __launch_bounds__(kThreads) void k_bgram(long long n, int k, const T *__restrict__ Am,
                                                    const T *__restrict__ Bm, const T *__restrict__ Cm,
                                                    double *__restrict__ gpart) {
    constexpr int G = BShape<KP>::G, RPT = BShape<KP>::RPT;
    __shared__ double s_w[BlockGram<T, KP>::LDS];
    const int tid = threadIdx.x, g = tid / KP, j = tid % KP;
    const bool act = j < k;
    BlockGram<T, KP> g0, g1, g2, g3;
    g0.zero();
    g1.zero();
    g2.zero();
    g3.zero();
    long long ntile = (n + RPT - 1) / RPT;
    int t0, t1;
    tile_range(ntile, t0, t1);
    long long v0 = (long long)t0 * RPT, v1 = min(n, (long long)t1 * RPT);
    for (long long vb = v0; vb < v1; vb += G) {  // uniform trip count across the block
        long long v = vb + g;
        bool ok = act && v < v1;
        T av = ok ? Am[v * k + j] : (T)0;
        T bv = ok ? Bm[v * k + j] : (T)0;
        g0.add(av, bv);
        if (NG == 4) {
            T cv = ok ? Cm[v * k + j] : (T)0;
            g1.add(bv, bv);
            g2.add(cv, bv);
            g3.add(cv, cv);
        }
    }
    double *out = gpart + (long long)blockIdx.x * NG * KP * KP;
    g0.flush(s_w, out);
    if (NG == 4) {
        g1.flush(s_w, out + KP * KP);
        g2.flush(s_w, out + 2 * KP * KP);
        g3.flush(s_w, out + 3 * KP * KP);
    }
}

// X += P alpha; R -= Q alpha; per-block partial sums of R's squared columns.
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_bupdate(long long n, int k, const T *__restrict__ alpha,
                                                      const T *__restrict__ P, const T *__restrict__ Q,
                                                      T *__restrict__ X, T *__restrict__ R,
                                                      double *__restrict__ part) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    __shared__ double sh[G][KP];
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    T acol[KP];
#pragma unroll
    for (int i = 0; i < KP; i++) acol[i] = act ? alpha[i * KP + j] : (T)0;
    double rr = 0.0;
    long long r0 = (long long)blockIdx.x * RPB;
    for (int i = g; i < RPB; i += G) {
        long long v = r0 + i;
        if (v >= n) break;
        T pv = act ? P[v * k + j] : (T)0;
        T qv = act ? Q[v * k + j] : (T)0;
        T sp = 0, sq = 0;
#pragma unroll
        for (int q = 0; q < KP; q++) {
            sp += __shfl(pv, q, KP) * acol[q];
            sq += __shfl(qv, q, KP) * acol[q];
        }
        if (act) {
            long long o = v * k + j;
            X[o] += sp;
            T rn = R[o] - sq;
            R[o] = rn;
            rr += (double)rn * (double)rn;
        }
    }
    sh[g][j] = rr;
    __syncthreads();
    if (g == 0) {
        double t = 0.0;
        for (int q = 0; q < G; q++) t += sh[q][j];
        part[(long long)blockIdx.x * KP + j] = t;
    }
}

// ------------------------------------------------ MFMA row-block products (FP32)
// A wave owns one tile of MF<KP>::ROWS consecutive rows and computes
// D = C + A_tile M for a k x k matrix M with ROWS x KP x KP MFMAs. The A operand
// wants rows on lanes (lane l: A[l % ROWS][kidx]), the transpose of the storage
// layout, so the tile goes through LDS (padded rows: conflict-free column reads).
// The D layout holds, per register, two (32-wide) or four (16-wide) whole rows
// across the lanes, so C loads and D stores are coalesced row segments and the
// same registers feed the Gram MFMA directly.
template <int KP>
struct MF;
template <>
struct MF<32> {
    using acc_t = floatx16;
    static constexpr int ROWS = 32, NR = 16, NS = 16;
    __device__ static acc_t mfma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
    __device__ static int drow(int lane, int r) { return 8 * (r / 4) + 4 * (lane / 32) + (r % 4); }
    __device__ static int dcol(int lane) { return lane % 32; }
    __device__ static int arow(int lane) { return lane % 32; }
    __device__ static int kidx(int lane, int s) { return 2 * s + lane / 32; }
};
template <>
struct MF<16> {
    using acc_t = floatx4;
    static constexpr int ROWS = 16, NR = 4, NS = 4;
    __device__ static acc_t mfma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int drow(int lane, int r) { return 4 * (lane / 16) + r; }
    __device__ static int dcol(int lane) { return lane % 16; }
    __device__ static int arow(int lane) { return lane % 16; }
    __device__ static int kidx(int lane, int s) { return 4 * s + lane / 16; }
};

// B operand registers of a KP x KP row-major matrix M (lane l: M[kidx][l % KP])
template <int KP>
__device__ __forceinline__ void mf_load_b(const float *__restrict__ M, float (&b)[MF<KP>::NS]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s2 = 0; s2 < MF<KP>::NS; s2++) b[s2] = M[MF<KP>::kidx(lane, s2) * KP + MF<KP>::dcol(lane)];
}
// stage rows [v0, v0 + ROWS) of an n x k block into this wave's LDS tile (zeros outside)
template <int KP>
__device__ __forceinline__ void mf_stage(float *sA, const float *__restrict__ X, long long v0, long long n, int k) {
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < MF<KP>::ROWS * KP; e += 64) {
        int r = e / KP, c = e % KP;
        long long v = v0 + r;
        sA[r * (KP + 1) + c] = (v < n && c < k) ? X[v * k + c] : 0.f;
    }
}
template <int KP>
__device__ __forceinline__ typename MF<KP>::acc_t mf_matmul(typename MF<KP>::acc_t acc, const float *sA,
                                                            const float (&b)[MF<KP>::NS]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s2 = 0; s2 < MF<KP>::NS; s2++) acc = MF<KP>::mfma(sA[MF<KP>::arow(lane) * (KP + 1) + MF<KP>::kidx(lane, s2)], b[s2], acc);
    return acc;
}
// load / store a tile in the D layout
template <int KP>
__device__ __forceinline__ typename MF<KP>::acc_t mf_load_d(const float *__restrict__ X, long long v0, long long n, int k) {
    const int lane = threadIdx.x & 63, c = MF<KP>::dcol(lane);
    typename MF<KP>::acc_t a;
#pragma unroll
    for (int r = 0; r < MF<KP>::NR; r++) {
        long long v = v0 + MF<KP>::drow(lane, r);
        a[r] = (v < n && c < k) ? X[v * k + c] : 0.f;
    }
    return a;
}
template <int KP>
__device__ __forceinline__ void mf_store_d(float *__restrict__ X, const typename MF<KP>::acc_t &a, long long v0,
                                           long long n, int k) {
    const int lane = threadIdx.x & 63, c = MF<KP>::dcol(lane);
#pragma unroll
    for (int r = 0; r < MF<KP>::NR; r++) {
        long long v = v0 + MF<KP>::drow(lane, r);
        if (v < n && c < k) X[v * k + c] = a[r];
    }
}

// X += P alpha; R -= Q alpha (negalpha = -alpha); per-block partial sums of R's
// squared columns. One row tile per wave.
template <int KP>
__global__ __launch_bounds__(kThreads) void k_mf_bupdate(long long n, int k, const float *__restrict__ alpha,
                                                         const float *__restrict__ negalpha,
                                                         const float *__restrict__ P, const float *__restrict__ Q,
                                                         float *__restrict__ X, float *__restrict__ R,
                                                         double *__restrict__ part) {
    constexpr int ROWS = MF<KP>::ROWS;
    __shared__ float sA[4][ROWS * (KP + 1)];
    __shared__ double sn[4][KP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float ba[MF<KP>::NS], bn[MF<KP>::NS];
    mf_load_b<KP>(alpha, ba);
    mf_load_b<KP>(negalpha, bn);
    // every wave runs the same steps (rows past n are zeros and are not stored), so
    // block barriers order the LDS tile between its writers and readers
    const long long v0 = ((long long)blockIdx.x * 4 + w) * ROWS;
    double rr = 0.0;
    mf_stage<KP>(sA[w], P, v0, n, k);
    __syncthreads();
    auto dx = mf_matmul<KP>(mf_load_d<KP>(X, v0, n, k), sA[w], ba);
    mf_store_d<KP>(X, dx, v0, n, k);
    __syncthreads();
    mf_stage<KP>(sA[w], Q, v0, n, k);
    __syncthreads();
    auto dr = mf_matmul<KP>(mf_load_d<KP>(R, v0, n, k), sA[w], bn);
    mf_store_d<KP>(R, dr, v0, n, k);
#pragma unroll
    for (int r = 0; r < MF<KP>::NR; r++) rr += (double)dr[r] * (double)dr[r];
    // lanes holding the same column: combine in a fixed order
    if (KP == 32) {
        rr += __shfl_xor(rr, 32, 64);
    } else {
        rr += __shfl_xor(rr, 16, 64);
        rr += __shfl_xor(rr, 32, 64);
    }
    if (lane < KP) sn[w][lane] = rr;
    __syncthreads();
    if (threadIdx.x < KP)
        part[(long long)blockIdx.x * KP + threadIdx.x] =
            ((sn[0][threadIdx.x] + sn[1][threadIdx.x]) + sn[2][threadIdx.x]) + sn[3][threadIdx.x];
}

// P_new = Z + P beta (stored unnormalized) and the Gram partials of P_new.
template <int KP>
__global__ __launch_bounds__(kThreads) void k_mf_bpupdate(long long n, int k, const float *__restrict__ beta,
                                                          const float *__restrict__ Z, float *__restrict__ P,
                                                          double *__restrict__ gpart) {
    constexpr int ROWS = MF<KP>::ROWS;
    __shared__ float sA[4][ROWS * (KP + 1)];
    __shared__ double s_w[BlockGram<float, KP>::LDS];
    const int w = threadIdx.x >> 6;
    float bb[MF<KP>::NS];
    mf_load_b<KP>(beta, bb);
    BlockGram<float, KP> gram;
    gram.zero();
    long long ntile = (n + ROWS - 1) / ROWS;
    long long per = (ntile + (long long)gridDim.x * 4 - 1) / ((long long)gridDim.x * 4);
    int bx = xcd_block(blockIdx.x, gridDim.x);
    long long t0 = ((long long)bx * 4 + w) * per;
    for (long long it = 0; it < per; it++) {  // same trip count in every wave
        long long tile = t0 + it;
        long long v0 = tile < ntile ? tile * ROWS : n;  // past the end: zeros, nothing stored
        __syncthreads();
        mf_stage<KP>(sA[w], P, v0, n, k);
        __syncthreads();
        auto d = mf_matmul<KP>(mf_load_d<KP>(Z, v0, n, k), sA[w], bb);
        mf_store_d<KP>(P, d, v0, n, k);
#pragma unroll
        for (int r = 0; r < MF<KP>::NR; r++) gram.add(d[r], d[r]);
    }
    gram.flush(s_w, gpart + (long long)blockIdx.x * KP * KP);
}

// P = P rinv
template <int KP>
__global__ __launch_bounds__(kThreads) void k_mf_bnormalize(long long n, int k, const float *__restrict__ rinv,
                                                            float *__restrict__ P) {
    constexpr int ROWS = MF<KP>::ROWS;
    __shared__ float sA[4][ROWS * (KP + 1)];
    const int w = threadIdx.x >> 6;
    float b[MF<KP>::NS];
    mf_load_b<KP>(rinv, b);
    const long long v0 = ((long long)blockIdx.x * 4 + w) * ROWS;
    mf_stage<KP>(sA[w], P, v0, n, k);
    __syncthreads();
    typename MF<KP>::acc_t z;
#pragma unroll
    for (int r = 0; r < MF<KP>::NR; r++) z[r] = 0.f;
    auto d = mf_matmul<KP>(z, sA[w], b);
    mf_store_d<KP>(P, d, v0, n, k);
}

// generic: P_new = Z + P beta with its Gram partials (other widths / FP64)
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_bpupdate_g(long long n, int k, const T *__restrict__ beta,
                                                         const T *__restrict__ Z, T *__restrict__ P,
                                                         double *__restrict__ gpart) {
    constexpr int G = BShape<KP>::G, RPT = BShape<KP>::RPT;
    __shared__ double s_w[BlockGram<T, KP>::LDS];
    const int tid = threadIdx.x, g = tid / KP, j = tid % KP;
    const bool act = j < k;
    T bcol[KP];
#pragma unroll
    for (int i = 0; i < KP; i++) bcol[i] = act ? beta[i * KP + j] : (T)0;
    BlockGram<T, KP> gram;
    gram.zero();
    long long ntile = (n + RPT - 1) / RPT;
    int t0, t1;
    tile_range(ntile, t0, t1);
    long long v0 = (long long)t0 * RPT, v1 = min(n, (long long)t1 * RPT);
    for (long long vb = v0; vb < v1; vb += G) {
        long long v = vb + g;
        bool ok = act && v < v1;
        T pv = ok ? P[v * k + j] : (T)0;
        T sv = ok ? Z[v * k + j] : (T)0;
#pragma unroll
        for (int q = 0; q < KP; q++) sv += __shfl(pv, q, KP) * bcol[q];
        if (ok) P[v * k + j] = sv;
        gram.add(sv, sv);
    }
    gram.flush(s_w, gpart + (long long)blockIdx.x * KP * KP);
}

// fixed-order sum over the kPersist blocks of width-wide partials
__global__ void k_reduce_wide(const double *__restrict__ part, int nblk, int width, double *__restrict__ out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= width) return;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int b = 0;
    for (; b + 3 < nblk; b += 4) {
        a0 += part[(long long)b * width + e];
        a1 += part[(long long)(b + 1) * width + e];
        a2 += part[(long long)(b + 2) * width + e];
        a3 += part[(long long)(b + 3) * width + e];
    }
    for (; b < nblk; b++) a0 += part[(long long)b * width + e];
    out[e] = (a0 + a1) + (a2 + a3);
}

// ---------------------------------------------------------- small k x k algebra
// In-place Cholesky of the k x k SPD matrix A (row-major, leading dimension KP) in
// LDS: lower factor L in the lower triangle. A pivot below tol * max diagonal marks
// its direction dependent: dead[j] = 1, L column j = e_j (solves then give 0 there).
template <int KP>
__device__ void chol_lds(double *A, int k, int *dead) {
    __shared__ double s_tol;
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int i = 0; i < k; i++) mx = fmax(mx, A[i * KP + i]);
        s_tol = mx * 1e-13;
    }
    __syncthreads();
    for (int jj = 0; jj < k; jj++) {
        if (threadIdx.x == 0) {
            double d = A[jj * KP + jj];
            for (int p = 0; p < jj; p++) d -= A[jj * KP + p] * A[jj * KP + p];
            if (!(d > s_tol)) {
                dead[jj] = 1;
                A[jj * KP + jj] = 1.0;
                for (int p = 0; p < jj; p++) A[jj * KP + p] = 0.0;
            } else {
                dead[jj] = 0;
                A[jj * KP + jj] = sqrt(d);
            }
        }
        __syncthreads();
        int i = jj + 1 + threadIdx.x;
        if (i < k) {
            if (dead[jj]) {
                A[i * KP + jj] = 0.0;
            } else {
                double s = A[i * KP + jj];
                for (int p = 0; p < jj; p++) s -= A[i * KP + p] * A[jj * KP + p];
                A[i * KP + jj] = s / A[jj * KP + jj];
            }
        }
        __syncthreads();
    }
}
// Solve L L' X = B for the k columns of B (row-major, ld KP) in place; rows of
// dead directions are set to 0.
template <int KP>
__device__ void chol_solve_lds(const double *L, int k, const int *dead, double *B) {
    int c = threadIdx.x;
    if (c < k) {
        for (int i = 0; i < k; i++) {
            double s = B[i * KP + c];
            for (int p = 0; p < i; p++) s -= L[i * KP + p] * B[p * KP + c];
            B[i * KP + c] = dead[i] ? 0.0 : s / L[i * KP + i];
        }
        for (int i = k - 1; i >= 0; i--) {
            double s = B[i * KP + c];
            for (int p = i + 1; p < k; p++) s -= L[p * KP + i] * B[p * KP + c];
            B[i * KP + c] = dead[i] ? 0.0 : s / L[i * KP + i];
        }
    }
    __syncthreads();
}

// A = L L' (Cholesky in place) and Rinv = (L')^-1, upper triangular, in B; columns
// of dead directions are zero, so P Rinv has orthonormal live columns and zero
// columns for directions that P no longer spans.
template <int KP>
__device__ void chol_rinv(double *A, double *B, int k, int *dead) {
    chol_lds<KP>(A, k, dead);
    for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) B[e] = 0.0;
    __syncthreads();
    int c = threadIdx.x;
    if (c < k && !dead[c]) {
        // back substitution L' x = e_c; x_i = 0 for i > c
        for (int i = c; i >= 0; i--) {
            double s = i == c ? 1.0 : 0.0;
            for (int p = i + 1; p <= c; p++) s -= A[p * KP + i] * B[p * KP + c];
            B[i * KP + c] = dead[i] ? 0.0 : s / A[i * KP + i];
        }
    }
    __syncthreads();
}

enum : int { SM_ALPHA = 0, SM_BETA = 1, SM_NORM = 2 };
// small-matrix slots (KP*KP doubles each) in Vecs::small
enum : int { S_PQ = 0, S_PR = 1, S_QZ = 2, S_PP = 3, S_L = 4, S_DEAD = 5, S_SLOTS = 6 };

// op ALPHA: L = chol(P'Q), alpha = (P'Q)^-1 P'R  -> outT[0] = alpha, outT[1] = -alpha
// op BETA:  beta = -(P'Q)^-1 Q'Z (L from ALPHA)  -> outT[2]
// op NORM:  P'P = R'R, rinv = R^-1 (upper); dependent directions get a zero
//           column (they leave the search block)  -> outT[3]
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_bsmall(int op, int k, double *__restrict__ sm, T *__restrict__ outT) {
    __shared__ double A[KP * KP];
    __shared__ double B[KP * KP];
    __shared__ int dead[KP];
    constexpr int KK = KP * KP;
    double *gPQ = sm + S_PQ * KK, *gPR = sm + S_PR * KK, *gQZ = sm + S_QZ * KK, *gPP = sm + S_PP * KK;
    double *gL = sm + S_L * KK;
    int *gdead = reinterpret_cast<int *>(sm + S_DEAD * KK);
    const int tid = threadIdx.x;
    if (op == SM_ALPHA || op == SM_NORM) {
        const double *src = op == SM_ALPHA ? gPQ : gPP;
        for (int e = tid; e < KK; e += kThreads) {
            int r = e / KP, c = e % KP;
            // symmetrise; rows/columns >= k become the identity
            A[e] = (r < k && c < k) ? 0.5 * (src[r * KP + c] + src[c * KP + r]) : (r == c ? 1.0 : 0.0);
        }
        __syncthreads();
        if (op == SM_ALPHA) {
            chol_lds<KP>(A, k, dead);
            for (int e = tid; e < KK; e += kThreads) {
                gL[e] = A[e];
                int r = e / KP, c = e % KP;
                B[e] = (r < k && c < k) ? gPR[e] : 0.0;
            }
            if (tid < KP) gdead[tid] = tid < k ? dead[tid] : 1;
            __syncthreads();
            chol_solve_lds<KP>(A, k, dead, B);
            for (int e = tid; e < KK; e += kThreads) {
                outT[e] = (T)B[e];
                outT[KK + e] = (T)(-B[e]);
            }
        } else {
            chol_rinv<KP>(A, B, k, dead);
            for (int e = tid; e < KK; e += kThreads) outT[3 * KK + e] = (T)B[e];
        }
    } else {  // SM_BETA
        for (int e = tid; e < KK; e += kThreads) {
            A[e] = gL[e];
            int r = e / KP, c = e % KP;
            B[e] = (r < k && c < k) ? -gQZ[e] : 0.0;
        }
        if (tid < KP) dead[tid] = gdead[tid];
        __syncthreads();
        chol_solve_lds<KP>(A, k, dead, B);
        for (int e = tid; e < KK; e += kThreads) outT[2 * KK + e] = (T)B[e];
    }
}

// generic P = P rinv
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_bnormalize_g(long long n, int k, const T *__restrict__ rinv,
                                                           T *__restrict__ P) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    T col[KP];
#pragma unroll
    for (int i = 0; i < KP; i++) col[i] = act ? rinv[i * KP + j] : (T)0;
    long long r0 = (long long)blockIdx.x * RPB;
    for (int i = g; i < RPB; i += G) {
        long long v = r0 + i;
        if (v >= n) break;
        T pv = act ? P[v * k + j] : (T)0;
        T sv = 0;
#pragma unroll
        for (int q = 0; q < KP; q++) sv += __shfl(pv, q, KP) * col[q];
        if (act) P[v * k + j] = sv;
    }
}

// convergence: count vectors with ||r_j||^2 > tol2 * ||r0_j||^2
__global__ void k_bcheck(const double *__restrict__ rr, const double *__restrict__ rr0, int k, double tol2,
                         int *__restrict__ out) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int j = threadIdx.x;
    if (j < k && rr[j] > tol2 * rr0[j]) atomicAdd(&cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0) *out = cnt;
}

__global__ void k_unpad(const double *__restrict__ in, int kp, int k, double *__restrict__ out) {
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) out[e] = in[(e / k) * kp + (e % k)];
}

template <typename T>
__global__ void k_copy_vec(long long nk, const T *__restrict__ a, T *__restrict__ b) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x)
        b[i] = a[i];
}

}  // namespace

template <typename T, int KP>
struct UseMF {
    static constexpr bool value = sizeof(T) == 4 && (KP == 16 || KP == 32);
};

// one dispatch per k-width: the MFMA kernels for FP32 with k in 9..32, else generic
template <typename T, int KP>
static void update_xr(const Dims &d, Vecs<T> &v, hipStream_t s) {
    const int KPP = KP * KP;
    if constexpr (UseMF<T, KP>::value) {
        int nb = (int)((d.n + 4 * MF<KP>::ROWS - 1) / (4 * MF<KP>::ROWS));
        hipLaunchKernelGGL((k_mf_bupdate<KP>), dim3(nb), dim3(kThreads), 0, s, d.n, d.k, v.smallT, v.smallT + KPP,
                           v.p, v.q, v.dx, v.r, v.part);
    } else {
        hipLaunchKernelGGL((k_bupdate<T, KP>), dim3(vec_blocks(d)), dim3(kThreads), 0, s, d.n, d.k, v.smallT, v.p,
                           v.q, v.dx, v.r, v.part);
    }
}
template <typename T, int KP>
static int update_xr_blocks(const Dims &d) {
    if constexpr (UseMF<T, KP>::value) return (int)((d.n + 4 * MF<KP>::ROWS - 1) / (4 * MF<KP>::ROWS));
    return vec_blocks(d);
}
template <typename T, int KP>
static void update_p(const Dims &d, Vecs<T> &v, int ngb, hipStream_t s) {
    const int KPP = KP * KP;
    if constexpr (UseMF<T, KP>::value)
        hipLaunchKernelGGL((k_mf_bpupdate<KP>), dim3(ngb), dim3(kThreads), 0, s, d.n, d.k, v.smallT + 2 * KPP, v.z,
                           v.p, v.gpart);
    else
        hipLaunchKernelGGL((k_bpupdate_g<T, KP>), dim3(ngb), dim3(kThreads), 0, s, d.n, d.k, v.smallT + 2 * KPP, v.z,
                           v.p, v.gpart);
}
template <typename T, int KP>
static void normalize_p(const Dims &d, Vecs<T> &v, hipStream_t s) {
    const int KPP = KP * KP;
    if constexpr (UseMF<T, KP>::value) {
        int nb = (int)((d.n + 4 * MF<KP>::ROWS - 1) / (4 * MF<KP>::ROWS));
        hipLaunchKernelGGL((k_mf_bnormalize<KP>), dim3(nb), dim3(kThreads), 0, s, d.n, d.k, v.smallT + 3 * KPP, v.p);
    } else {
        hipLaunchKernelGGL((k_bnormalize_g<T, KP>), dim3(vec_blocks(d)), dim3(kThreads), 0, s, d.n, d.k,
                           v.smallT + 3 * KPP, v.p);
    }
}

template <typename T>
long long block_pcg(Topo &t, Vecs<T> &v, const Dims &d, double itol, int max_it, hipStream_t s) {
    const long long nk = d.n * d.k;
    const int root = 0;
    const int KPP = d.kp * d.kp;
    const int ngb = gram_blocks(d.kp);
    double *sm = v.small;
    double *rr0 = v.red + RED_RN * kMaxK, *rr = v.red + RED_RR * kMaxK;
    int *cnt = v.active + kMaxK - 1;
    fill_T(v.dx, nk, (T)0, s);
    // P = Z R^-1 with Z = L_T^+ R and Z'Z = R'R
    tree_solve<T>(t, v, d, v.r, v.z, nullptr, nullptr, nullptr, s);
    hipLaunchKernelGGL(k_copy_vec<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, v.z, v.p);
    KP_DISPATCH(d.kp, {
        ProfScope ps(PK_PCG_VEC, 3.0 * nk * sizeof(T), s);
        hipLaunchKernelGGL((k_bgram<T, KP, 1>), dim3(ngb), dim3(kThreads), 0, s, d.n, d.k, v.p, v.p,
                           (const T *)nullptr, v.gpart);
        hipLaunchKernelGGL(k_reduce_wide, dim3(div_up(KPP, 256)), dim3(256), 0, s, v.gpart, ngb, KPP,
                           sm + S_PP * KPP);
        hipLaunchKernelGGL((k_bsmall<T, KP>), dim3(1), dim3(kThreads), 0, s, (int)SM_NORM, d.k, sm, v.smallT);
        normalize_p<T, KP>(d, v, s);
        GR_CHECK_LAUNCH();
    });
    long long it = 0;
    while (it < max_it) {
        it++;
        int nbu = 0;
        KP_DISPATCH(d.kp, {
            {
                ProfScope ps(PK_SPMM_P, 4.0 * (d.n + 1) + 8.0 * d.p_nnz + 3.0 * nk * sizeof(T), s);
                hipLaunchKernelGGL((k_bspmm<T, KP>), dim3(ngb), dim3(kThreads), 0, s, d.n, d.k, t.prow, t.pcol,
                                   v.pval, v.p, v.q, v.r, root, v.gpart);
            }
            hipLaunchKernelGGL(k_reduce_wide, dim3(div_up(2 * KPP, 256)), dim3(256), 0, s, v.gpart, ngb, 2 * KPP,
                               sm + S_PQ * KPP);
            hipLaunchKernelGGL((k_bsmall<T, KP>), dim3(1), dim3(kThreads), 0, s, (int)SM_ALPHA, d.k, sm, v.smallT);
            {
                ProfScope ps(PK_PCG_VEC, 6.0 * nk * sizeof(T), s);
                update_xr<T, KP>(d, v, s);
            }
            nbu = update_xr_blocks<T, KP>(d);
            GR_CHECK_LAUNCH();
        });
        col_sum<T>(d, v, v.part, nbu, d.kp, 0, rr, s);
        hipLaunchKernelGGL(k_bcheck, dim3(1), dim3(64), 0, s, rr, rr0, d.k, itol * itol, cnt);
        GR_CHECK_LAUNCH();
        if ((it & 3) == 0 || it == max_it) {
            if (read_i32(cnt, s) == 0) break;
        }
        tree_solve<T>(t, v, d, v.r, v.z, nullptr, nullptr, nullptr, s);
        KP_DISPATCH(d.kp, {
            {
                ProfScope ps(PK_PCG_VEC, 2.0 * nk * sizeof(T), s);
                hipLaunchKernelGGL((k_bgram<T, KP, 1>), dim3(ngb), dim3(kThreads), 0, s, d.n, d.k, v.q, v.z,
                                   (const T *)nullptr, v.gpart);
            }
            hipLaunchKernelGGL(k_reduce_wide, dim3(div_up(KPP, 256)), dim3(256), 0, s, v.gpart, ngb, KPP,
                               sm + S_QZ * KPP);
            hipLaunchKernelGGL((k_bsmall<T, KP>), dim3(1), dim3(kThreads), 0, s, (int)SM_BETA, d.k, sm, v.smallT);
            {
                ProfScope ps(PK_PCG_VEC, 3.0 * nk * sizeof(T), s);
                update_p<T, KP>(d, v, ngb, s);
            }
            hipLaunchKernelGGL(k_reduce_wide, dim3(div_up(KPP, 256)), dim3(256), 0, s, v.gpart, ngb, KPP,
                               sm + S_PP * KPP);
            hipLaunchKernelGGL((k_bsmall<T, KP>), dim3(1), dim3(kThreads), 0, s, (int)SM_NORM, d.k, sm, v.smallT);
            {
                ProfScope ps(PK_PCG_VEC, 2.0 * nk * sizeof(T), s);
                normalize_p<T, KP>(d, v, s);
            }
            GR_CHECK_LAUNCH();
        });
    }
    return it;
}

// Diagnostics: C = A'B (FP64, k x k, row-major ld k) for device n x k blocks,
// with the Gram kernel of the block PCG.
template <typename T>
void block_gram(const Dims &d, const T *A, const T *B, double *gpart, double *red, double *out, hipStream_t s) {
    const int KPP = d.kp * d.kp;
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL((k_bgram<T, KP, 1>), dim3(gram_blocks(d.kp)), dim3(kThreads), 0, s, d.n, d.k, A, B,
                           (const T *)nullptr, gpart);
        hipLaunchKernelGGL(k_reduce_wide, dim3(div_up(KPP, 256)), dim3(256), 0, s, gpart, gram_blocks(d.kp), KPP,
                           red);
        hipLaunchKernelGGL(k_unpad, dim3(1), dim3(256), 0, s, red, KP, d.k, out);
    });
    GR_CHECK_LAUNCH();
}
template void block_gram<float>(const Dims &, const float *, const float *, double *, double *, double *,
                                hipStream_t);
template void block_gram<double>(const Dims &, const double *, const double *, double *, double *, double *,
                                 hipStream_t);

template long long block_pcg<float>(Topo &, Vecs<float> &, const Dims &, double, int, hipStream_t);
template long long block_pcg<double>(Topo &, Vecs<double> &, const Dims &, double, int, hipStream_t);

}  // namespace grass
