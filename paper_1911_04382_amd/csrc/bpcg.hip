// Block preconditioned conjugate gradients for the L_P solves of the
// generalized power iteration (eq. 29) once P holds off-tree edges.
//
// The k right-hand sides of one step share one block Krylov space (O'Leary's
// block CG) with the grounded tree solve as preconditioner. Per iteration:
//   Q = L_P P, alpha = (P'Q)^-1 (P'R), X += P alpha, R -= Q alpha,
//   Z = L_T^+ R, beta = -(P'Q)^-1 (Q'Z), P = Z + P beta,
//   P <- P chol(P'P)^-1  (keeps the block well conditioned; a direction that
//                          becomes dependent is dropped).
// In FP32 each inner solve starts from an orthonormal basis of the FP64 residual
// (k_rhs_basis), and a phase that stalls turns on a stricter dependence test for the
// rest of its solve (kStallIters).
// X += P alpha is deferred to the pass that forms the next P (one read of P).
// The k x k matrices are reduced in a fixed order at the end of the kernel that
// produces them and factorised in FP64 by its last workgroup, so results are
// deterministic and each step costs one launch. Compared with k independent CG runs
// this needs several times fewer iterations: the block space captures the
// largest generalized eigenvalues of the tree-preconditioned system together.
#include "embed.h"
#include "kern.h"
#include "gram.h"
#include "lap.h"
#include "profiler.h"
#include "launch_sched.h"

#include <chrono>
#include <climits>
#include <cstddef>

namespace grass {

namespace {

template <int KP>
struct BShape {
    static constexpr int G = kThreads / KP;  // lane groups (one vector row each) per block
    static constexpr int RPT = G * 4;        // rows per tile
    static constexpr int CAP = RPT * 12 < 3072 ? RPT * 12 : 3072;  // staged CSR nonzeros per tile (fast path)
};

// FP32 block PCG: an inner phase longer than this has stalled, and the dependence
// threshold of the block normalisation (relative to the own diagonal entry) that the
// rest of that solve uses
constexpr long long kStallIters = 256;
constexpr double kOwnFp32 = 1e-6;

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


// ---------------------------------------------------------- small k x k algebra
// The k x k steps of the block PCG in FP64 by one workgroup (a separate launch, so
// that its registers do not lower the occupancy of the streaming kernels):
//   ALPHA (in = [G | P'R], G = P'Q): Gauss-Jordan on [G | P'R | I] gives
//          alpha = G^-1 P'R and G^-1 (kept for BETA)
//   BETA  (in = Q'Z):  beta = -G^-1 Q'Z (a plain product)
//   NORM  (in = P'P):  forward elimination on [P'P | I] gives P'P = L D L' and
//          L^-1, so rinv = L^-T D^-1/2 (upper triangular, (P rinv)'(P rinv) = I)
// G and P'P are symmetric positive semidefinite: they are symmetrised, the
// elimination needs no pivoting, and a pivot below 1e-13 times the largest
// diagonal entry marks its direction dependent. NORM also takes a pivot at or below
// `own` times its own diagonal entry as dependent (own = 0 turns that off): with
// own = 1e-6 in FP32, a direction whose part outside the span of the earlier ones
// is under 1e-3 of its length, ten times the rounding level of an FP32 Gram. Kept,
// such a direction is rounding noise scaled up to full length; it breaks the
// conjugacy of the next blocks and can stall the iteration. That step is skipped and the
// direction's row of alpha and G^-1 (its column of rinv) is zero: the solves
// return 0 there and the direction leaves the search block. Only the leading
// k x k block takes part; everything else is zero.
enum SmallOp : int { SM_ALPHA = 0, SM_BETA = 1, SM_NORM = 2 };
// ALPHA / NORM: the block holding the reduced Gram runs that small step itself
enum TailOp : int { TAIL_STORE = 0, TAIL_SAVE = 1, TAIL_CHECK = 2, TAIL_ALPHA = 3, TAIL_NORM = 4 };
// FP64 slots of Vecs::small, KP*KP doubles each: G^-1, reduced Gram input (two), and
// for the orthonormal right-hand sides r'r, R and R^-1
enum : int { S_GINV = 0, S_IN = 2, S_RC = 4, S_RF = 5, S_RS = 6, S_SLOTS = 7 };
// working-precision slots of Vecs::smallT (KP*KP each)
enum : int { T_ALPHA = 0, T_NEGALPHA = 1, T_BETA = 2, T_RINV = 3 };

template <typename T, int KP, int OP, int NT>
__device__ void small_op(int k, const double *in, double *__restrict__ ginv, T *__restrict__ outT,
                         double own = 0.0) {
    constexpr int KK = KP * KP;
    const int tid = threadIdx.x;
    if constexpr (OP == SM_BETA) {
        // Q'Z and G^-1 staged with coalesced loads (read in place for the widest
        // blocks, LDS-bound)
        constexpr bool STAGE = KP <= 32;
        __shared__ double s_in[STAGE ? 2 * KK : 1];
        if (STAGE) {
            for (int e = tid; e < 2 * KK; e += NT) s_in[e] = e < KK ? in[e] : ginv[e - KK];
            __syncthreads();
        }
        const double *qz = STAGE ? s_in : in, *gi = STAGE ? s_in + KK : ginv;
        for (int e = tid; e < KK; e += NT) {
            const int r = e / KP, c = e % KP;
            double acc = 0.0;
            if (r < k && c < k)
                for (int p = 0; p < k; p++) acc -= gi[r * KP + p] * qz[p * KP + c];
            outT[T_BETA * KK + e] = (T)acc;
        }
        return;
    }
    // Gauss-Jordan / forward elimination with the augmented matrix in registers:
    // thread (tr, tc) owns rows tr + RG a and columns tc + CG b. A step needs only
    // the pivot row and the pivot column, which their owners publish to LDS
    // (double-buffered, so one barrier per step).
    constexpr int W = OP == SM_ALPHA ? 3 * KP : 2 * KP;  // [G | RHS | I] or [G | I]
    constexpr int CG = 32, RG = NT / CG;
    constexpr int RPT = (KP + RG - 1) / RG, CPT = (W + CG - 1) / CG;
    __shared__ double s_prow[2][W];
    __shared__ double s_pcol[2][KP];
    __shared__ double s_piv[KP];
    __shared__ int s_dead[KP];
    __shared__ double s_dg;
    const int tr = tid / CG, tc = tid % CG;
    double m[RPT][CPT];
    {
        // every operand load first (clamped indices), then the selects
        double v1[RPT][CPT], v2[RPT][CPT];
#pragma unroll
        for (int a = 0; a < RPT; a++) {
#pragma unroll
            for (int b = 0; b < CPT; b++) {
                const int r = tr + RG * a < KP ? tr + RG * a : 0, c = tc + CG * b;
                const int i1 = c < KP ? r * KP + c : (OP == SM_ALPHA && c < 2 * KP ? KK + r * KP + (c - KP) : 0);
                const int i2 = c < KP ? c * KP + r : 0;
                v1[a][b] = in[i1];
                v2[a][b] = in[i2];
            }
        }
#pragma unroll
        for (int a = 0; a < RPT; a++) {
#pragma unroll
            for (int b = 0; b < CPT; b++) {
                const int r = tr + RG * a, c = tc + CG * b;
                double x;
                if (c < KP) x = c < k ? 0.5 * (v1[a][b] + v2[a][b]) : 0.0;
                else if (OP == SM_ALPHA && c < 2 * KP) x = c - KP < k ? v1[a][b] : 0.0;
                else x = (c - (W - KP)) == r ? 1.0 : 0.0;
                m[a][b] = (r < k && c < W) ? x : 0.0;
            }
        }
    }
    if (tid < 64) {  // largest diagonal entry, one wave
        double mx = 0.0;
        for (int i = tid; i < k; i += 64) mx = fmax(mx, in[i * KP + i]);
        for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
        if (tid == 0) s_dg = mx;
    }
    // owners publish row / column jj of the current matrix into buffer `buf`
    auto publish = [&](int jj, int buf) {
        if (tr == jj % RG) {
            const int aa = jj / RG;
#pragma unroll
            for (int b = 0; b < CPT; b++) {
                double v = 0.0;
#pragma unroll
                for (int a = 0; a < RPT; a++) v = a == aa ? m[a][b] : v;
                const int c = tc + CG * b;
                if (c < W) s_prow[buf][c] = v;
            }
        }
        if (tc == jj % CG) {
            const int bb = jj / CG;
#pragma unroll
            for (int a = 0; a < RPT; a++) {
                double v = 0.0;
#pragma unroll
                for (int b = 0; b < CPT; b++) v = b == bb ? m[a][b] : v;
                const int r = tr + RG * a;
                if (r < KP) s_pcol[buf][r] = v;
            }
        }
    };
    publish(0, 0);
    __syncthreads();
    const double tol = s_dg * 1e-13;
    for (int jj = 0; jj < k; jj++) {
        const int buf = jj & 1;
        const double d = s_pcol[buf][jj];
        double pr[CPT], pc[RPT];
#pragma unroll
        for (int b = 0; b < CPT; b++) pr[b] = s_prow[buf][tc + CG * b < W ? tc + CG * b : 0];
#pragma unroll
        for (int a = 0; a < RPT; a++) pc[a] = s_pcol[buf][tr + RG * a < KP ? tr + RG * a : 0];
        // uniform: every thread reads the same pivot and diagonal entry
        const bool ok = d > tol && (OP != SM_NORM || d > own * in[jj * KP + jj]);
        if (ok) {
            const double rp = 1.0 / d;
#pragma unroll
            for (int a = 0; a < RPT; a++) {
                const int r = tr + RG * a;
                const double f = pc[a] * rp;
#pragma unroll
                for (int b = 0; b < CPT; b++) {
                    if (OP == SM_ALPHA) m[a][b] = r == jj ? pr[b] * rp : m[a][b] - f * pr[b];
                    else if (r > jj) m[a][b] -= f * pr[b];
                }
            }
        }
        if (tid == 0) {
            s_piv[jj] = d;
            s_dead[jj] = ok ? 0 : 1;
        }
        if (jj + 1 < k) publish(jj + 1, buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < RPT; a++) {
#pragma unroll
        for (int b = 0; b < CPT; b++) {
            const int r = tr + RG * a, c = tc + CG * b;
            if (r >= KP || c < KP || c >= W) continue;
            if (OP == SM_ALPHA) {
                const int cc = c < 2 * KP ? c - KP : c - 2 * KP;
                const bool live = r < k && cc < k && !s_dead[r];
                const double x = live ? m[a][b] : 0.0;
                const int e = r * KP + cc;
                if (c < 2 * KP) {
                    outT[T_ALPHA * KK + e] = (T)x;
                    outT[T_NEGALPHA * KK + e] = (T)(-x);
                } else {
                    ginv[e] = x;
                }
            } else {
                // rinv[i][j] = (L^-1)[j][i] / sqrt(d_j); row j of L^-1 sits in columns KP..2KP
                const int j = r, i = c - KP;
                const double x = (i < k && j < k && !s_dead[j]) ? m[a][b] / sqrt(s_piv[j]) : 0.0;
                outT[T_RINV * KK + i * KP + j] = (T)x;
            }
        }
    }
}

template <typename T, int KP, int OP>
__global__ __launch_bounds__(kThreads) void k_small(int k, double *__restrict__ sm, T *__restrict__ outT,
                                                    const LoopCtl *__restrict__ loop) {
    small_op<T, KP, OP, kThreads>(k, sm + S_IN * KP * KP, sm + S_GINV * KP * KP, outT, loop ? loop->own : 0.0);
}

template <typename T>
struct Tail {
    double *part;       // level-0 partials (block b at part + b * width), then the level sums
    int *cnt;           // arrival counters, zero between launches
    double *vec;        // SAVE: the total (width doubles); STORE: k x k result (ld k); CHECK: norms
    const double *rr0;  // CHECK: squared norms of the right-hand sides
    int *count;         // CHECK: number of vectors not yet converged
    double tol2;
    int op;
    T *outT;            // ALPHA / NORM: the small-matrix outputs
    double *ginv;       // ALPHA: G^-1 for the later BETA step
    LoopCtl *loop;      // CHECK: counts the iteration and may end the inner phase;
                        // NORM: its dependence threshold `own`
    const int *gate;    // the kernel returns at once while *gate is set
};

// SAVE / STORE of the reduced total (tot in LDS, width doubles)
template <int KP>
__device__ void tail_finish(const double *tot, int width, int k, int op, double *vec) {
    if (op == TAIL_SAVE) {
        for (int e = threadIdx.x; e < width; e += blockDim.x) vec[e] = tot[e];
    } else {
        for (int e = threadIdx.x; e < k * k; e += blockDim.x) vec[e] = tot[(e / k) * KP + e % k];
    }
}
// CHECK: tot = squared residual norms. With loop control, the decisions of the host
// loop on the device: at every 4th iteration and at the cap the inner phase ends
// when every vector has converged, at the cap, or (FP32) after kStallIters
// iterations, which also switches on the dependence threshold for the rest of the
// solve.
template <typename T>
__device__ void tail_check(const Tail<T> &tl, int k, const double *tot) {
    __shared__ int c;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    int j = threadIdx.x;
    if (j < k) {
        tl.vec[j] = tot[j];
        if (tot[j] > tl.tol2 * tl.rr0[j]) atomicAdd(&c, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *tl.count = c;
        if (LoopCtl *L = tl.loop) {
            const int it = ++L->it;
            const bool last = it >= L->max_it;
            if (last || (it & 3) == 0) {
                const bool done = last || c == 0;
                const bool stall = !done && L->stall_ok && it - L->phase0 >= kStallIters;
                if (stall) {
                    L->own = kOwnFp32;
                    L->stall_ok = 0;
                }
                if (done || stall) L->gate = 1;
            }
        }
    }
}

// ------------------------------------------------------------------ kernels
// Gram partials A'B (and with NG = 2 also A'C) of this block; the last block to
// finish reduces them.
template <typename T, int KP, int NG, int NT>
__global__ __launch_bounds__(NT) void k_bgram(long long n, int k, const T *__restrict__ Am,
                                              const T *__restrict__ Bm, const T *__restrict__ Cm, Tail<T> tl) {
    constexpr int G = NT / KP, RPT = G * 4;
    __shared__ double s_w[2 * KP * KP];
    const int tid = threadIdx.x, g = tid / KP, j = tid % KP;
    const bool act = j < k;
    BlockGram<T, KP> g0, g1;
    g0.zero();
    g1.zero();
    long long ntile = (n + RPT - 1) / RPT;
    int t0, t1;
    tile_range(ntile, t0, t1);
    long long v0 = (long long)t0 * RPT, v1 = min(n, (long long)t1 * RPT);
    constexpr int U = sizeof(T) == 4 ? 8 : 4;  // rows per lane group in flight
    for (long long vb = v0; vb < v1; vb += (long long)G * U) {  // uniform trip count across the block
        T av[U], bv[U], cv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            long long v = vb + (long long)u * G + g;
            bool ok = act && v < v1;
            long long o = ok ? v * k + j : 0;
            av[u] = Am[o];
            bv[u] = Bm[o];
            av[u] = ok ? av[u] : (T)0;
            bv[u] = ok ? bv[u] : (T)0;
            if (NG == 2) {
                cv[u] = Cm[o];
                cv[u] = ok ? cv[u] : (T)0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            g0.add(av[u], bv[u]);
            if (NG == 2) g1.add(av[u], cv[u]);
        }
    }
    constexpr int KK = KP * KP;
    double *out = tl.part + (long long)blockIdx.x * NG * KK;
    g0.flush(s_w, out);
    if (NG == 2) g1.flush(s_w, out + KK);
    if (tail_reduce(tl.part, gridDim.x, NG * KK, tl.cnt, s_w)) tail_finish<KP>(s_w, NG * KK, k, tl.op, tl.vec);
}

// Workgroups of 1024 threads: at the kernel's occupancy (16 waves per CU) one per CU,
// so there are few k x k partials (a pair per CU) and the reduction at the end of
// the launch is two levels of two dependent rounds (256-thread workgroups made it
// three levels of eight).
constexpr int kLapGramThreads = 1024;

// Q = L_P P with the Gram matrices P'Q and P'R formed on the fly: a lane group
// holds one row of P and of Q (KP lanes), which is the operand layout of the FP32
// MFMA outer products, so each tile adds its rows to the two accumulators before
// the next tile. Blocks walk several tiles each; the last block reduces the FP64
// partials. One pass over P, Q and R instead of a product pass
// and a three-operand Gram pass.
template <int KP, int E>
__global__ __launch_bounds__(kLapGramThreads) void k_lap_gram(long long n, int k, const int *__restrict__ rowptr,
                                                       const int *__restrict__ col, const float *__restrict__ val,
                                                       const float *__restrict__ ltail,
                                                       const int *__restrict__ ecol, const float *__restrict__ eval,
                                                       const int *__restrict__ edeg, const float *__restrict__ P,
                                                       float *__restrict__ Q, int root, const float *__restrict__ R,
                                                       Tail<float> tl) {
    if (tl.gate && *tl.gate) return;
    constexpr int NT = kLapGramThreads, G = NT / KP, NIT = LapShape<KP>::NIT, RPB = G * NIT;
    constexpr int KK = KP * KP;
    using L = LapTile<float, KP, E>;
    __shared__ double s_w[2 * KK];
    __shared__ __align__(16) char lds[(NT / 64) * L::SLICE];
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    BlockGram<float, KP, true> gq, gr;
    gq.zero();
    gr.zero();
    // each XCD owns a contiguous eighth of the tiles, which its blocks sweep as one
    // front (block q takes tiles q, q + nq, ...), so neighbour rows a few thousand
    // rows back are still in that XCD's L2
    const long long ntile = (n + RPB - 1) / RPB;
    const int q = blockIdx.x >> 3, nq = gridDim.x >> 3;
    const long long per = (ntile + 7) / 8;
    const long long xs = std::min(ntile, (long long)(blockIdx.x & 7) * per), xe = std::min(ntile, xs + per);
    // software pipeline: the next tile's neighbour lists are loaded while this
    // tile's second round (issued first) is in flight
    LapStage<float, KP, E> cur, nxt;
    if (xs + q < xe) lap_load<float, KP, E>((xs + q) * RPB, n, ecol, eval, edeg, cur);
    for (long long t = xs + q; t < xe; t += nq) {
        const long long r0 = t * RPB;
        LapFetch<float, KP, E> F;
        float rv[NIT];
        lap_fetch<float, KP, E>(r0, n, k, P, cur, lds, F);
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const long long v = L::row(r0, g, it);
            // R streams through once here: a non-temporal load leaves L2 to the rows
            // of P that neighbouring tiles gather again (186 -> 183 us). Non-temporal
            // padded-row loads gained 1 us more but fetch each 128-byte line again for
            // every 8 rows; a non-temporal store of Q cost the R update its cache hits
            rv[it] = __builtin_nontemporal_load(&R[act && v < n ? v * k + j : 0]);
        }
        if (t + nq < xe) lap_load<float, KP, E>((t + nq) * RPB, n, ecol, eval, edeg, nxt);
        float xo[NIT], yo[NIT];
        lap_rows<float, KP, E>(r0, n, k, rowptr, col, val, ltail, P, Q, root, 1.f, F, lds, xo, yo);
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const bool ok = act && L::row(r0, g, it) < n;
            gq.add(xo[it], yo[it]);
            gr.add(xo[it], ok ? rv[it] : 0.f);
        }
        cur = nxt;
    }
    double *out = tl.part + (long long)blockIdx.x * 2 * KK;
    gq.flush(s_w, out);
    gr.flush(s_w, out + KK);
    if (tail_reduce(tl.part, gridDim.x, 2 * KK, tl.cnt, s_w)) {
        if (tl.op == TAIL_ALPHA)
            small_op<float, KP, SM_ALPHA, NT>(k, s_w, tl.ginv, tl.outT);
        else
            tail_finish<KP>(s_w, 2 * KK, k, tl.op, tl.vec);
    }
}

// generic R -= Q alpha; per-block squared column norms of R; the last block counts
// the vectors that have not converged.
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_rupdate(long long n, int k, const T *__restrict__ alpha,
                                                      const T *__restrict__ Q, T *__restrict__ R, Tail<T> tl) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    __shared__ double sh[G][KP];
    __shared__ double tot[KP];
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
        T qv = act ? Q[v * k + j] : (T)0;
        T sq = 0;
#pragma unroll
        for (int q = 0; q < KP; q++) sq += __shfl(qv, q, KP) * acol[q];
        if (act) {
            long long o = v * k + j;
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
        st_agent(&tl.part[(long long)blockIdx.x * KP + j], t);
    }
    if (tail_reduce(tl.part, gridDim.x, KP, tl.cnt, tot)) tail_check<T>(tl, k, tot);
}

// generic: X += P alpha, P_new = Z + P beta (one pass over P) with the Gram
// partials of P_new; the last block computes rinv.
template <typename T, int KP>
__global__ __launch_bounds__(kThreads) void k_pupdate(long long n, int k, const T *__restrict__ alpha,
                                                      const T *__restrict__ beta, const T *__restrict__ Z,
                                                      T *__restrict__ P, T *__restrict__ X, Tail<T> tl) {
    constexpr int G = BShape<KP>::G, RPT = BShape<KP>::RPT;
    __shared__ double s_w[2 * KP * KP];
    const int tid = threadIdx.x, g = tid / KP, j = tid % KP;
    const bool act = j < k;
    T bcol[KP], acol[KP];
#pragma unroll
    for (int i = 0; i < KP; i++) {
        bcol[i] = act ? beta[i * KP + j] : (T)0;
        acol[i] = act ? alpha[i * KP + j] : (T)0;
    }
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
        T xv = ok ? X[v * k + j] : (T)0;
#pragma unroll
        for (int q = 0; q < KP; q++) {
            T pq = __shfl(pv, q, KP);
            sv += pq * bcol[q];
            xv += pq * acol[q];
        }
        if (ok) {
            P[v * k + j] = sv;
            X[v * k + j] = xv;
        }
        gram.add(sv, sv);
    }
    constexpr int KK = KP * KP;
    gram.flush(s_w, tl.part + (long long)blockIdx.x * KK);
    if (tail_reduce(tl.part, gridDim.x, KK, tl.cnt, s_w)) tail_finish<KP>(s_w, KK, k, tl.op, tl.vec);
}

// generic Out = (ADD ? C : 0) + In M (Out may alias In or C)
template <typename T, int KP, bool ADD>
__global__ __launch_bounds__(kThreads) void k_rowmul(long long n, int k, const T *__restrict__ M, const T *In,
                                                     const T *C, T *Out) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const bool act = j < k;
    T col[KP];
#pragma unroll
    for (int i = 0; i < KP; i++) col[i] = act ? M[i * KP + j] : (T)0;
    long long r0 = (long long)blockIdx.x * RPB;
    for (int i = g; i < RPB; i += G) {
        long long v = r0 + i;
        if (v >= n) break;
        T pv = act ? In[v * k + j] : (T)0;
        T sv = (ADD && act) ? C[v * k + j] : (T)0;
#pragma unroll
        for (int q = 0; q < KP; q++) sv += __shfl(pv, q, KP) * col[q];
        if (act) Out[v * k + j] = sv;
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
// Rows [v0, v0 + ROWS) of an n x k block for this wave's LDS tile (zeros outside):
// mf_fetch issues the loads (unconditional: clamped address, then a select, all in
// flight together), mf_put writes the tile.
template <int KP>
struct MFTile {
    static constexpr int NE = MF<KP>::ROWS * KP / 64;
    float x[NE];
};
template <int KP>
__device__ __forceinline__ void mf_fetch(MFTile<KP> &t, const float *__restrict__ X, long long v0, long long n,
                                         int k) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < MFTile<KP>::NE; q++) {
        int e = lane + 64 * q, r = e / KP, c = e % KP;
        long long v = v0 + r;
        bool ok = v < n && c < k;
        float x = X[ok ? v * k + c : 0];
        t.x[q] = ok ? x : 0.f;
    }
}
template <int KP>
__device__ __forceinline__ void mf_put(float *sA, const MFTile<KP> &t) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < MFTile<KP>::NE; q++) {
        int e = lane + 64 * q, r = e / KP, c = e % KP;
        sA[r * (KP + 1) + c] = t.x[q];
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
// load / store a tile in the D layout (loads unconditional, as in mf_fetch)
template <int KP>
__device__ __forceinline__ typename MF<KP>::acc_t mf_load_d(const float *__restrict__ X, long long v0, long long n, int k) {
    const int lane = threadIdx.x & 63, c = MF<KP>::dcol(lane);
    typename MF<KP>::acc_t a;
#pragma unroll
    for (int r = 0; r < MF<KP>::NR; r++) {
        long long v = v0 + MF<KP>::drow(lane, r);
        bool ok = v < n && c < k;
        float x = X[ok ? v * k + c : 0];
        a[r] = ok ? x : 0.f;
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

// R -= Q alpha (negalpha = -alpha); per-block squared column norms of R; the last
// block counts the vectors that have not converged. One row tile per wave.
template <int KP>
__global__ __launch_bounds__(kThreads) void k_mf_rupdate(long long n, int k, const float *__restrict__ negalpha,
                                                         const float *__restrict__ Q, float *__restrict__ R,
                                                         Tail<float> tl) {
    if (tl.gate && *tl.gate) return;
    constexpr int ROWS = MF<KP>::ROWS;
    __shared__ float sA[4][ROWS * (KP + 1)];
    __shared__ double sn[4][KP];
    __shared__ double tot[KP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float bn[MF<KP>::NS];
    mf_load_b<KP>(negalpha, bn);
    // every wave runs the same steps (rows past n are zeros and are not stored)
    const long long v0 = ((long long)blockIdx.x * 4 + w) * ROWS;
    MFTile<KP> tq;
    mf_fetch<KP>(tq, Q, v0, n, k);
    auto cr = mf_load_d<KP>(R, v0, n, k);
    mf_put<KP>(sA[w], tq);
    __syncthreads();
    auto dr = mf_matmul<KP>(cr, sA[w], bn);
    mf_store_d<KP>(R, dr, v0, n, k);
    double rr = 0.0;
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
        st_agent(&tl.part[(long long)blockIdx.x * KP + threadIdx.x],
                 ((sn[0][threadIdx.x] + sn[1][threadIdx.x]) + sn[2][threadIdx.x]) + sn[3][threadIdx.x]);
    if (tail_reduce(tl.part, gridDim.x, KP, tl.cnt, tot)) tail_check<float>(tl, k, tot);
}

// X += P alpha and P_new = Z + P beta from one staged copy of P, the Gram partials
// of P_new; the last block computes rinv. Persistent: every wave takes the same
// number of row tiles.
template <int KP, int NT>
__global__ __launch_bounds__(NT) void k_mf_pupdate(long long n, int k, const float *__restrict__ alpha,
                                                   const float *__restrict__ beta, const float *__restrict__ Z,
                                                   float *__restrict__ P, float *__restrict__ X, Tail<float> tl) {
    if (tl.gate && *tl.gate) return;
    constexpr int ROWS = MF<KP>::ROWS;
    constexpr int NW = NT / 64;
    __shared__ float sA[NW][ROWS * (KP + 1)];
    __shared__ double s_w[2 * KP * KP];
    const int w = threadIdx.x >> 6;
    float bb[MF<KP>::NS], ba[MF<KP>::NS];
    mf_load_b<KP>(beta, bb);
    mf_load_b<KP>(alpha, ba);
    BlockGram<float, KP> gram;
    gram.zero();
    long long ntile = (n + ROWS - 1) / ROWS;
    long long per = (ntile + (long long)gridDim.x * NW - 1) / ((long long)gridDim.x * NW);
    int bx = xcd_block(blockIdx.x, gridDim.x);
    long long t0 = ((long long)bx * NW + w) * per;
    for (long long it = 0; it < per; it++) {  // same trip count in every wave
        long long tile = t0 + it;
        long long v0 = tile < ntile ? tile * ROWS : n;  // past the end: zeros, nothing stored
        MFTile<KP> tp;
        mf_fetch<KP>(tp, P, v0, n, k);
        auto cx = mf_load_d<KP>(X, v0, n, k);
        auto cz = mf_load_d<KP>(Z, v0, n, k);
        __syncthreads();  // the previous tile's reads of sA are done
        mf_put<KP>(sA[w], tp);
        __syncthreads();
        auto dx = mf_matmul<KP>(cx, sA[w], ba);
        mf_store_d<KP>(X, dx, v0, n, k);
        auto d = mf_matmul<KP>(cz, sA[w], bb);
        mf_store_d<KP>(P, d, v0, n, k);
#pragma unroll
        for (int r = 0; r < MF<KP>::NR; r++) gram.add(d[r], d[r]);
    }
    constexpr int KK = KP * KP;
    gram.flush(s_w, tl.part + (long long)blockIdx.x * KK);
    if (tail_reduce(tl.part, gridDim.x, KK, tl.cnt, s_w)) {
        if (tl.op == TAIL_NORM)
            small_op<float, KP, SM_NORM, NT>(k, s_w, tl.ginv, tl.outT, tl.loop ? tl.loop->own : 0.0);
        else
            tail_finish<KP>(s_w, KK, k, tl.op, tl.vec);
    }
}

// Out = (ADD ? C : 0) + In M, one row tile per wave (Out may alias In or C: each
// wave stages its rows of In before it stores them)
template <int KP, bool ADD>
__global__ __launch_bounds__(kThreads) void k_mf_rowmul(long long n, int k, const float *__restrict__ M,
                                                        const float *In, const float *C, float *Out,
                                                        const int *__restrict__ gate) {
    if (gate && *gate) return;
    constexpr int ROWS = MF<KP>::ROWS;
    __shared__ float sA[4][ROWS * (KP + 1)];
    const int w = threadIdx.x >> 6;
    float b[MF<KP>::NS];
    mf_load_b<KP>(M, b);
    const long long v0 = ((long long)blockIdx.x * 4 + w) * ROWS;
    MFTile<KP> ti;
    mf_fetch<KP>(ti, In, v0, n, k);
    typename MF<KP>::acc_t z;
    if (ADD) {
        z = mf_load_d<KP>(C, v0, n, k);
    } else {
#pragma unroll
        for (int r = 0; r < MF<KP>::NR; r++) z[r] = 0.f;
    }
    mf_put<KP>(sA[w], ti);
    __syncthreads();
    auto d = mf_matmul<KP>(z, sA[w], b);
    mf_store_d<KP>(Out, d, v0, n, k);
}

template <typename T>
__global__ void k_copy_vec(long long nk, const T *__restrict__ a, T *__restrict__ b) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// ------------------------------------------- orthonormal right-hand sides (FP32)
// The residual block of a later power step is dominated by the few largest
// generalized eigenvectors, so its k columns can agree to within FP32 rounding:
// the working-precision Gram of such a block cannot be factorised and the block
// PCG stalls. Each inner solve therefore starts from an orthonormal basis of the
// FP64 residual, r = Q R (Cholesky QR in FP64), solves L_P Y = Q in working
// precision and hands z = Y R back to the FP64 outer step. Block CG spans the same
// space for r and Q; only the rounding differs.
//
// Cholesky of C = r'r (k x k, ld k, symmetrised): R upper triangular (ld KP) with
// R'R = C on the kept directions, S = R^-1 on them (ld KP) and qn[j] = 1. A pivot
// at or below 1e-12 times its own diagonal entry (the column's part outside the
// span of the earlier ones is below 1e-6 of its length), or a zero column, drops
// direction j: row j of R, column j of S and qn[j] are 0, and column j of r is
// carried by the kept directions alone.
template <int KP>
__global__ __launch_bounds__(kThreads) void k_rhs_basis(int k, const double *__restrict__ C, double *__restrict__ R,
                                                        double *__restrict__ S, double *__restrict__ qn) {
    // a: the elimination in place; R ends in the upper triangle, S (upper triangular)
    // is kept transposed in the strict lower triangle and its diagonal in sd
    __shared__ double a[KP][KP + 1];
    __shared__ double sd[KP];
    __shared__ int live[KP];
    const int tid = threadIdx.x;
    for (int e = tid; e < KP * KP; e += kThreads) {
        const int i = e / KP, l = e % KP;
        a[i][l] = (i < k && l < k) ? 0.5 * (C[i * k + l] + C[l * k + i]) : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < k; j++) {
        const double dj = a[j][j];
        const bool ok = dj > 0.0 && dj > 1e-12 * C[j * k + j];  // uniform
        __syncthreads();  // every thread has read the pivot before row j is scaled
        if (ok) {
            const double rs = 1.0 / sqrt(dj);
            for (int l = j + tid; l < k; l += kThreads) a[j][l] *= rs;
        }
        if (tid == 0) live[j] = ok ? 1 : 0;
        __syncthreads();
        if (ok) {
            for (int e = tid; e < KP * KP; e += kThreads) {
                const int i = e / KP, l = e % KP;
                if (i > j && l > j && i < k && l < k) a[i][l] -= a[j][i] * a[j][l];
            }
        }
        __syncthreads();
    }
    // S: back substitution on the kept rows, one column per thread (column j of S is
    // row j of the lower triangle, written only by thread j)
    if (tid < k && live[tid]) {
        const int j = tid;
        for (int i = 0; i < j; i++) a[j][i] = 0.0;
        sd[j] = 1.0 / a[j][j];
        for (int i = j - 1; i >= 0; i--) {
            if (!live[i]) continue;
            double acc = a[i][j] * sd[j];
            for (int l = i + 1; l < j; l++) acc += a[i][l] * a[j][l];
            a[j][i] = -acc / a[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < KP * KP; e += kThreads) {
        const int i = e / KP, l = e % KP;
        const bool in = i < k && l < k && live[i] && live[l];
        R[e] = (i < k && l < k && live[i] && l >= i) ? a[i][l] : 0.0;
        S[e] = in && l > i ? a[l][i] : (in && l == i ? sd[i] : 0.0);
    }
    if (tid < kMaxK) qn[tid] = (tid < k && live[tid]) ? 1.0 : 0.0;
}

// out = in M for an upper-triangular k x k M (FP64, ld KP), row by row in FP64: a
// lane group stages its row in LDS (one coalesced load per value) and each lane
// sums its column from there
template <typename TI, typename TO, int KP>
__global__ __launch_bounds__(kThreads) void k_basis_map(long long n, int k, const TI *__restrict__ in,
                                                        const double *__restrict__ M, TO *__restrict__ out, int nblk) {
    constexpr int G = kThreads / KP;
    constexpr int RPB = G * kRowsPerGroup;
    static_assert(KP <= 64, "a lane group within one wave");
    __shared__ double sm[KP * KP];
    __shared__ double srow[G][KP];
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    if (bid >= nblk) return;  // whole block
    for (int e = threadIdx.x; e < KP * KP; e += kThreads) sm[e] = M[e];
    __syncthreads();
    const int g = threadIdx.x / KP, j = threadIdx.x % KP;
    const long long r0 = (long long)bid * RPB;
    for (int i = g; i < RPB; i += G) {  // the same trip count in every lane of a group
        const long long v = r0 + i;
        if (v >= n) break;
        srow[g][j] = j < k ? (double)in[v * k + j] : 0.0;
        __builtin_amdgcn_wave_barrier();  // the group's writes are seen by its reads (one wave)
        double acc = 0.0;
        for (int l = 0; l <= j; l++) acc += srow[g][l] * sm[l * KP + j];
        if (j < k) out[v * k + j] = (TO)acc;
        __builtin_amdgcn_wave_barrier();  // the group's reads are done before the next row
    }
}

}  // namespace

// Scratch of the tail reductions: level-0 partials and level sums (doubles) and
// arrival counters, for the widest launch of the block PCG.
// the product-and-Gram pass: at most this many blocks (a multiple of 8), so at most
// that many pairs of k x k partials
constexpr int kLapGramBlocks = 1024;
static long long tail_grid_max(const Dims &d) {
    long long mf_rows = d.kp == 16 ? 16 : 32;
    return std::max<long long>({(long long)gram_blocks(d.kp), (long long)kLapGramBlocks, (long long)vec_blocks(d),
                                div_up(d.n, 4 * mf_rows), d.ntiles});
}
long long bpcg_part_doubles(const Dims &d) {
    const long long KK = (long long)d.kp * d.kp;
    long long g = std::max<long long>({(long long)gram_blocks(d.kp), (long long)kLapGramBlocks, d.ntiles}),
              v = tail_grid_max(d);
    return std::max(tail_items(g) * 2 * KK, tail_items(v) * d.kp) + 64;
}
long long bpcg_counters(const Dims &d) { return tail_items(tail_grid_max(d)) + 64; }

// generic Gram passes: one workgroup per row tile up to gram_blocks (a multiple of
// 8, as the XCD mapping needs), so a small graph reduces few partials
template <int KP>
static int gram_grid(long long n) {
    return std::min(gram_blocks(KP), xcd_grid(div_up(n, (long long)BShape<KP>::RPT)));
}
// Gram launch shape: with MFMA one 1024-thread workgroup per CU (256 partials, two
// reduction levels), else 256-thread workgroups
constexpr int kMfGramBlocks = 256;
template <typename T, int KP, int NG>
static void launch_gram(const Dims &d, const T *A, const T *B, const T *C, const Tail<T> &tl, hipStream_t s) {
    if constexpr (UseMF<T, KP>::value)
        hipLaunchKernelGGL((k_bgram<T, KP, NG, 1024>), dim3(kMfGramBlocks), dim3(1024), 0, s, d.n, d.k, A, B, C, tl);
    else
        hipLaunchKernelGGL((k_bgram<T, KP, NG, kThreads>), dim3(gram_grid<KP>(d.n)), dim3(kThreads), 0, s, d.n, d.k, A,
                           B, C, tl);
}
// Q = L_P P, then P'Q and P'R: fused for FP32 blocks of 16 or 32 vectors, else a
// product pass and a Gram pass
// one resident wave of product blocks (each walks a range of tiles): more would
// leave a second, partial wave behind
template <int KP>
static int lap_gram_resident() {
    static const int resident = [] {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_lap_gram<KP, kEllP>, kLapGramThreads, 0) != hipSuccess)
            return kLapGramBlocks;
        return std::max(8, std::min(kLapGramBlocks, cus * per / 8 * 8));
    }();
    return resident;
}
template <typename T, int KP>
static void launch_lap_gram(Topo &t, Vecs<T> &v, const Dims &d, int root, const Tail<T> &tl, hipStream_t s) {
    if constexpr (UseMF<T, KP>::value) {
        constexpr long long RPB = (kLapGramThreads / KP) * LapShape<KP>::NIT;
        const int nb = (int)std::min<long long>(lap_gram_resident<KP>(), xcd_grid(div_up(d.n, RPB)));
        ProfScope ps(PK_SPMM_P, 4.0 * (d.n + 1) + (double)d.p_nnz * (4 + sizeof(T)) + 3.0 * d.n * d.k * sizeof(T), s);
        lap_long<T>(d, t.prow, t.pcol, v.pval, v.ep, v.p, s, tl.gate);
        hipLaunchKernelGGL((k_lap_gram<KP, kEllP>), dim3(nb), dim3(kLapGramThreads), 0, s, d.n, d.k, t.prow, t.pcol, v.pval,
                           v.ep.tail, v.ep.col, v.ep.val, v.ep.deg, v.p, v.q, root, v.r, tl);
    } else {
        lap_apply<T>(d, t.prow, t.pcol, v.pval, v.ep, v.p, v.q, root, nullptr, nullptr, s);
        ProfScope ps(PK_GRAM_PQR, 3.0 * d.n * d.k * sizeof(T), s);
        launch_gram<T, KP, 2>(d, v.p, v.q, v.r, tl, s);
    }
}
template <int KP>
static int mf_blocks(const Dims &d) {
    return div_up(d.n, 4 * MF<KP>::ROWS);
}

// tails that save the reduced Gram into the small-matrix input slot
template <typename T>
static Tail<T> save_tail(Vecs<T> &v, const Dims &d) {
    Tail<T> tl{};
    tl.part = v.gpart;
    tl.cnt = v.tcnt;
    tl.vec = v.small + (long long)S_IN * d.kp * d.kp;
    tl.op = TAIL_SAVE;
    return tl;
}
template <typename T, int KP, int OP>
static void launch_small(const Dims &d, Vecs<T> &v, hipStream_t s, const LoopCtl *loop = nullptr) {
    ProfScope ps(PK_SMALL, 0.0, s);
    hipLaunchKernelGGL((k_small<T, KP, OP>), dim3(1), dim3(kThreads), 0, s, d.k, v.small, v.smallT, loop);
}

// R -= Q alpha and the convergence count
template <typename T, int KP>
static void launch_rupdate(const Dims &d, Vecs<T> &v, Tail<T> tl, hipStream_t s) {
    const int KK = KP * KP;
    ProfScope ps(PK_RUPDATE, 3.0 * d.n * d.k * sizeof(T), s);
    if constexpr (UseMF<T, KP>::value) {
        hipLaunchKernelGGL((k_mf_rupdate<KP>), dim3(mf_blocks<KP>(d)), dim3(kThreads), 0, s, d.n, d.k,
                           v.smallT + T_NEGALPHA * KK, v.q, v.r, tl);
    } else {
        hipLaunchKernelGGL((k_rupdate<T, KP>), dim3(vec_blocks(d)), dim3(kThreads), 0, s, d.n, d.k,
                           v.smallT + T_ALPHA * KK, v.q, v.r, tl);
    }
}
// X += P alpha, P = Z + P beta and the Gram of the new P (with MFMA also rinv from
// it, in the block that completes the Gram)
template <typename T, int KP>
static void launch_pupdate(const Dims &d, Vecs<T> &v, hipStream_t s, const int *gate) {
    const int KK = KP * KP;
    ProfScope ps(PK_PUPDATE, 5.0 * d.n * d.k * sizeof(T), s);
    Tail<T> tl = save_tail(v, d);
    if constexpr (UseMF<T, KP>::value) {
        tl.op = TAIL_NORM;
        tl.outT = v.smallT;
        tl.loop = v.loop;
        tl.gate = gate;
    }
    if constexpr (UseMF<T, KP>::value)
        hipLaunchKernelGGL((k_mf_pupdate<KP, 512>), dim3(kMfGramBlocks), dim3(512), 0, s, d.n, d.k,
                           v.smallT + T_ALPHA * KK, v.smallT + T_BETA * KK, v.z, v.p, v.dx, tl);
    else
        hipLaunchKernelGGL((k_pupdate<T, KP>), dim3(gram_grid<KP>(d.n)), dim3(kThreads), 0, s, d.n, d.k,
                           v.smallT + T_ALPHA * KK, v.smallT + T_BETA * KK, v.z, v.p, v.dx, tl);
}
// Out = (ADD ? C : 0) + In M
template <typename T, int KP, bool ADD>
static void launch_rowmul(const Dims &d, const T *M, const T *In, const T *C, T *Out, hipStream_t s,
                          const int *gate = nullptr) {
    ProfScope ps(PK_ROWMUL, (ADD ? 3.0 : 2.0) * d.n * d.k * sizeof(T), s);
    if constexpr (UseMF<T, KP>::value)
        hipLaunchKernelGGL((k_mf_rowmul<KP, ADD>), dim3(mf_blocks<KP>(d)), dim3(kThreads), 0, s, d.n, d.k, M, In, C,
                           Out, gate);
    else
        hipLaunchKernelGGL((k_rowmul<T, KP, ADD>), dim3(vec_blocks(d)), dim3(kThreads), 0, s, d.n, d.k, M, In, C,
                           Out);
}

// v.r = Q = r64 S with r64 = Q R (Cholesky QR in FP64, R and S in v.small); the
// squared norms of Q's columns in red[RED_QN]
template <typename T>
static void rhs_basis(const Dims &d, Vecs<T> &v, hipStream_t s) {
    const long long KK = (long long)d.kp * d.kp;
    double *C = v.small + S_RC * KK, *R = v.small + S_RF * KK, *S = v.small + S_RS * KK;
    const int nbv = vec_blocks(d);
    ProfScope ps(PK_RESID64, (double)d.n * d.k * (16 + sizeof(T)), s);
    block_gram<double>(d, v.r64, v.r64, v.gpart, v.tcnt, C, s);
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL(k_rhs_basis<KP>, dim3(1), dim3(kThreads), 0, s, d.k, C, R, S, v.red + RED_QN * kMaxK);
        hipLaunchKernelGGL((k_basis_map<double, T, KP>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k, v.r64,
                           S, v.r, nbv);
    });
    GR_CHECK_LAUNCH();
}

// z64 = Y R for the inner solution Y = v.dx on the basis of rhs_basis
template <typename T>
static void basis_back(const Dims &d, Vecs<T> &v, hipStream_t s) {
    const long long KK = (long long)d.kp * d.kp;
    const int nbv = vec_blocks(d);
    ProfScope ps(PK_RESID64, (double)d.n * d.k * (8 + sizeof(T)), s);
    KP_DISPATCH(d.kp, {
        hipLaunchKernelGGL((k_basis_map<T, double, KP>), dim3(xcd_grid(nbv)), dim3(kThreads), 0, s, d.n, d.k, v.dx,
                           v.small + S_RF * KK, v.z64, nbv);
    });
    GR_CHECK_LAUNCH();
}

// device-side loop state of a solve, and the start of a new inner phase
__global__ void k_loop_init(LoopCtl *L, int max_it, int stall_ok) {
    L->gate = 0;
    L->it = 0;
    L->phase0 = 0;
    L->max_it = max_it;
    L->stall_ok = stall_ok;
    L->own = 0.0;
}
__global__ void k_loop_phase(LoopCtl *L) {
    L->phase0 = L->it;
    L->gate = 0;
}
// host copy of the loop state's gate and iteration count
static void read_loop(const LoopCtl *L, int out[2], hipStream_t s) {
    static_assert(offsetof(LoopCtl, it) == sizeof(int), "gate and it are read together");
    GR_HIP(hipMemcpyAsync(out, L, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    GR_HIP(hipStreamSynchronize(s));
}

template <typename T>
SolveInfo block_pcg(Topo &t, Vecs<T> &v, const Dims &d, const T *b, const PcgParams &pp, hipStream_t s,
                    const double *b64) {
    const long long nk = d.n * d.k;
    const int root = 0;
    const int KK = d.kp * d.kp;
    const Tail<T> tsave = save_tail(v, d);
    SolveInfo info;
    fill_i32(v.tcnt, bpcg_counters(d), 0, s);
    if (pp.single) {
        // r = b with x = 0 (b grounded by the caller); no FP64 residual
        hipLaunchKernelGGL(k_copy_vec<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, b, v.r);
        info.resid64 = -1.0;
    } else {
        // r = b - L_P x with x = 0; its norms are the reference of the first inner phase
        info.resid64 = true_residual<T>(t, v, d, b, s, b64);
        if (info.resid64 <= pp.rtol) return info;
    }
    // FP32 working precision: every inner solve runs on an orthonormal basis of the
    // FP64 residual (FP64 keeps the columns apart by itself), unless the caller
    // turns it off
    const bool basis = pp.basis && v.z64 != nullptr;
    constexpr bool fp32 = std::is_same<T, float>::value;
    // The loop's decisions are taken on the device (LoopCtl, in the check kernel's
    // tail): iteration count and cap, the end of an inner phase, and in FP32 the stall
    // rule: a phase that runs kStallIters iterations without every column converging
    // ends there (the FP64 step takes the partial solution) and the rest of the solve
    // normalises its blocks with the dependence threshold kOwnFp32.
    hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(1), 0, s, v.loop, (int)std::min<long long>(pp.max_it, INT_MAX),
                       fp32 && !pp.single ? 1 : 0);
    // a fresh search block: P = Z R^-1 with Z = L_T^+ R and Z'Z = R'R
    auto start_block = [&]() {
        if (basis) rhs_basis<T>(d, v, s);
        tree_solve<T>(t, v, d, v.r, v.z, nullptr, nullptr, nullptr, s);
        hipLaunchKernelGGL(k_copy_vec<T>, dim3(grid_nk(nk)), dim3(kThreads), 0, s, nk, v.z, v.p);
        KP_DISPATCH(d.kp, {
            {
                ProfScope ps(PK_BGRAM, 2.0 * nk * sizeof(T), s);
                launch_gram<T, KP, 1>(d, v.p, v.p, nullptr, tsave, s);
            }
            launch_small<T, KP, SM_NORM>(d, v, s, v.loop);
            launch_rowmul<T, KP, false>(d, v.smallT + T_RINV * KK, v.p, nullptr, v.p, s);
        });
        GR_CHECK_LAUNCH();
    };
    start_block();
    Tail<T> tcheck{};
    tcheck.part = v.gpart;
    tcheck.cnt = v.tcnt;
    tcheck.op = TAIL_CHECK;
    tcheck.vec = v.red + RED_RR * kMaxK;
    // squared norms of the inner solve's right-hand sides
    tcheck.rr0 = v.red + (basis ? RED_QN : RED_RN) * kMaxK;
    tcheck.count = v.active + kMaxK - 1;
    tcheck.tol2 = pp.itol * pp.itol;
    tcheck.loop = v.loop;
    // One iteration in two halves; the host loop looks between them. With a gate every
    // kernel returns at once while the inner phase has ended.
    //   first:  Q = L_P P, P'Q and P'R, alpha (with MFMA in the block that completes the
    //           Grams), R -= Q alpha and the check
    //   second: Z = L_T^+ R with Q'Z and beta (MFMA: formed by the down sweep's tiles),
    //           X += P alpha, P = Z + P beta with its Gram, P = P R^-1
    auto first_half = [&](const int *gate) {
        KP_DISPATCH(d.kp, {
            Tail<T> tc = tcheck;
            tc.gate = gate;
            if constexpr (UseMF<T, KP>::value) {
                Tail<T> ta = tsave;
                ta.op = TAIL_ALPHA;
                ta.outT = v.smallT;
                ta.ginv = v.small + (long long)S_GINV * KK;
                ta.gate = gate;
                launch_lap_gram<T, KP>(t, v, d, root, ta, s);
            } else {
                launch_lap_gram<T, KP>(t, v, d, root, tsave, s);
                launch_small<T, KP, SM_ALPHA>(d, v, s);
            }
            launch_rupdate<T, KP>(d, v, tc, s);
        });
        GR_CHECK_LAUNCH();
    };
    auto second_half = [&](const int *gate) {
        KP_DISPATCH(d.kp, {
            if constexpr (UseMF<T, KP>::value) {
                tree_solve<T>(t, v, d, v.r, v.z, nullptr, nullptr, nullptr, s, v.q, tsave.part, tsave.cnt, nullptr,
                              v.small + (long long)S_GINV * KK, v.smallT + T_BETA * KK, gate);
            } else {
                tree_solve<T>(t, v, d, v.r, v.z, nullptr, nullptr, nullptr, s);
                {
                    ProfScope ps(PK_BGRAM, 2.0 * nk * sizeof(T), s);
                    launch_gram<T, KP, 1>(d, v.q, v.z, nullptr, tsave, s);
                }
                launch_small<T, KP, SM_BETA>(d, v, s);
            }
            launch_pupdate<T, KP>(d, v, s, gate);
            if constexpr (!UseMF<T, KP>::value) launch_small<T, KP, SM_NORM>(d, v, s, v.loop);
            launch_rowmul<T, KP, false>(d, v.smallT + T_RINV * KK, v.p, nullptr, v.p, s, gate);
        });
        GR_CHECK_LAUNCH();
    };

    if (pp.single) {
        // one inner phase (an inexact L_P solve for a preconditioner): until every
        // vector's residual has fallen by itol, or max_it; X += P alpha completes it,
        // and there is no FP64 step
        long long it = 0;
        while (true) {
            it++;
            first_half(nullptr);
            if (it >= pp.max_it || (it & 3) == 0) {
                int lc[2];
                read_loop(v.loop, lc, s);
                if (lc[0]) break;
            }
            second_half(nullptr);
        }
        KP_DISPATCH(d.kp, { launch_rowmul<T, KP, true>(d, v.smallT + T_ALPHA * KK, v.p, v.dx, v.dx, s); });
        info.iters = it;
        info.outer = 1;
        return info;
    }

    // Concurrent paths (LaunchSched of the worker thread): chunks of four iterations
    // captured once per solve as a hipGraph and replayed `chunks` times between host
    // reads (the fused MFMA kernels only: FP32 at k = 16 or 32, and never while kernels
    // are timed). Replays past the end of a phase do nothing, so the results are those
    // of the kernel-by-kernel loop.
    LaunchSched *sc = g_sched;
    bool can_capture = sc != nullptr && sc->mode == 1 && fp32 && (d.kp == 16 || d.kp == 32) && s != nullptr &&
                       !(g_prof != nullptr && g_prof->on);
    struct GraphHold {
        hipGraphExec_t exec = nullptr;
        ~GraphHold() {
            if (exec) (void)hipGraphExecDestroy(exec);
        }
    } gh;
    auto capture = [&]() -> bool {
        const int *gate = &v.loop->gate;
        KP_DISPATCH(d.kp, {
            if constexpr (UseMF<T, KP>::value) (void)lap_gram_resident<KP>();  // host queries stay out of the capture
        });
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        hipGraph_t g = nullptr;
        try {
            for (int i = 0; i < 4; i++) {
                first_half(gate);
                second_half(gate);
            }
        } catch (...) {
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        if (hipStreamEndCapture(s, &g) != hipSuccess || g == nullptr) {
            (void)hipGetLastError();
            return false;
        }
        const hipError_t e = hipGraphInstantiate(&gh.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            gh.exec = nullptr;
            return false;
        }
        if (sc->stats) sc->stats->captures++;
        return true;
    };
    const int tkey = Tuner::key(d.n, d.kp);
    int cand = -1;  // tuner candidate of the current phase
    auto pick = [&]() -> int {
        cand = -1;
        if (!can_capture) return 0;
        if (sc->chunks > 0) return sc->chunks;
        if (!sc->tuner) return 4;
        cand = sc->tuner->pick(tkey);
        return kSchedCand[cand];
    };
    int chunks = pick();
    auto phase_t0 = std::chrono::steady_clock::now();
    long long phase_it0 = 0, reads = 0, replays = 0;
    long long prev_len = 0;  // length of the solve's previous inner phase (0: none yet)

    long long it = 0;
    bool fresh = true, checked = false;  // the next FCG step starts a recurrence; resid64 recomputed
    while (true) {
        bool end = false;
        if (chunks > 0 && can_capture && it + 4 <= pp.max_it) {
            if (!gh.exec && !capture()) {  // kernel by kernel for the rest of the solve
                can_capture = false;
                chunks = 0;
                cand = -1;  // this phase's timing says nothing about the tuner's candidate
                continue;
            }
            // up to `chunks` replays, but not past the end that the previous phase's
            // length predicts (then one at a time): replays after the end do nothing
            // but still take launch slots that other graphs' kernels could use
            long long want = chunks;
            if (prev_len > 0) want = std::max<long long>(1, std::min<long long>(chunks, (prev_len - (it - phase_it0)) / 4));
            const int nrep = (int)std::min<long long>(want, (pp.max_it - it) / 4);
            for (int i = 0; i < nrep; i++) GR_HIP(hipGraphLaunch(gh.exec, s));
            int lc[2];
            read_loop(v.loop, lc, s);
            replays += nrep;
            reads++;
            end = lc[0] != 0;
            it = lc[1];
        } else {
            it++;
            first_half(nullptr);
            if (it >= pp.max_it || (it & 3) == 0) {
                int lc[2];
                read_loop(v.loop, lc, s);
                reads++;
                end = lc[0] != 0;
            }
            if (!end) second_half(nullptr);
        }
        if (!end) continue;
        if (cand >= 0) {
            const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - phase_t0).count();
            sc->tuner->record(tkey, cand, sec / (double)std::max<long long>(1, it - phase_it0));
        }
        // every vector's recursive residual fell by itol since the inner solve started
        // (or the phase stalled): X += P alpha completes z ~ L_P^-1 r, which the FP64
        // flexible-CG step turns into its next direction; the inner solve then restarts
        // from the new FP64 residual
        KP_DISPATCH(d.kp, { launch_rowmul<T, KP, true>(d, v.smallT + T_ALPHA * KK, v.p, v.dx, v.dx, s); });
        if (basis) basis_back<T>(d, v, s);
        info.resid64 = fcg_outer_step<T>(t, v, d, fresh, s, basis ? v.z64 : nullptr);
        fresh = false;
        checked = false;
        if (info.resid64 <= pp.rtol) {
            // the recurrence's residual drifts from b - L_P x by rounding: check the
            // recomputed one, and if it misses the target go on from it with a fresh
            // recurrence (residual replacement)
            info.resid64 = true_residual<T>(t, v, d, b, s, b64);
            checked = fresh = true;
        }
        if (it >= pp.max_it || info.resid64 <= pp.rtol || info.outer + 1 >= pp.max_repl) break;
        info.outer++;
        hipLaunchKernelGGL(k_loop_phase, dim3(1), dim3(1), 0, s, v.loop);
        start_block();
        chunks = pick();
        prev_len = it - phase_it0;
        phase_t0 = std::chrono::steady_clock::now();
        phase_it0 = it;
    }
    info.outer++;
    info.iters = it;
    if (sc != nullptr && sc->stats != nullptr) {
        sc->stats->iterations += it;
        sc->stats->host_reads += reads;
        sc->stats->replays += replays;
    }
    // the reported residual is always the one recomputed from the solution
    if (!checked) info.resid64 = true_residual<T>(t, v, d, b, s, b64);
    return info;
}

// Diagnostics: C = A'B (FP64, k x k, row-major ld k) for device n x k blocks,
// with the Gram kernel of the block PCG; part and cnt as sized by
// bpcg_part_doubles / bpcg_counters.
template <typename T>
void block_gram(const Dims &d, const T *A, const T *B, double *part, int *cnt, double *out, hipStream_t s) {
    fill_i32(cnt, bpcg_counters(d), 0, s);
    Tail<T> tl{};
    tl.part = part;
    tl.cnt = cnt;
    tl.vec = out;
    tl.op = TAIL_STORE;
    KP_DISPATCH(d.kp, {
        launch_gram<T, KP, 1>(d, A, B, nullptr, tl, s);
    });
    GR_CHECK_LAUNCH();
}
template void block_gram<float>(const Dims &, const float *, const float *, double *, int *, double *, hipStream_t);
template void block_gram<double>(const Dims &, const double *, const double *, double *, int *, double *,
                                 hipStream_t);

template SolveInfo block_pcg<float>(Topo &, Vecs<float> &, const Dims &, const float *, const PcgParams &,
                                    hipStream_t, const double *);
template SolveInfo block_pcg<double>(Topo &, Vecs<double> &, const Dims &, const double *, const PcgParams &,
                                     hipStream_t, const double *);

}  // namespace grass
