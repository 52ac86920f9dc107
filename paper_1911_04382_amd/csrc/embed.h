// Embedding kernels (embed.hip): start vectors, Laplacian products, the
// level-scheduled tree solve, PCG on L_P with FP64 refinement, edge scoring.
#pragma once
#include "state.h"

namespace grass {

// reduction slots in Vecs::red (kMaxK doubles each)
enum : int {
    RED_NUM = 0, RED_DEN, RED_LMAX, RED_RR, RED_BN, RED_RN, RED_MEAN,
    // the FP64 flexible-CG outer iteration of the L_P solve (per column): z'A d_prev,
    // d'r, d'A d, the previous d'A d, its alpha and beta; squared norms of the inner
    // solve's orthonormal right-hand sides (1, or 0 for a dropped direction)
    RED_ZAD, RED_DR, RED_DAD, RED_DADP, RED_FA, RED_FB, RED_QN,
    RED_SLOTS = 16
};
// u64 slots in Vecs::u64s
enum : int { U_HMAX = 0, U_LMIN = 1, U_ABSMAX = 2, U_SLOTS = 8 };

template <typename T>
void plan_vecs(Arena &a, const Dims &d, Vecs<T> &v);

// h0 of eq. (28) into out (n x k, row stride k).
template <typename T>
void start_vectors(const Dims &d, uint64_t seed, int pass, T *out, Vecs<T> &v, hipStream_t s);

// y = L x over a CSR (difference form), optional grounding of `root`, optional
// scaling of y by the power of two that brings max|x| (u64 slot) to [1, 2), optional
// per-block partials of x.y.
template <typename T>
void lap_apply(const Dims &d, const int *rowptr, const int *col, const T *val, const Ell<T> &ell, const T *x, T *y,
               int root, const unsigned long long *scale_from, double *dot_part, hipStream_t s);
// The entries past E of the rows longer than kLongRow, one workgroup per row, into
// ell.tail (lap_apply calls it; callers of the product kernels directly must too).
// With gate: returns at once while *gate is set.
template <typename T>
void lap_long(const Dims &d, const int *rowptr, const int *col, const T *val, const Ell<T> &ell, const T *x,
              hipStream_t s, const int *gate = nullptr);

// Grounded tree solve x = L_T^+ y (x[root] = 0): up-sweep then down-sweep over the
// heavy-light levels. x may alias y. Optional fused outputs of the down-sweep:
// per-tile partials of rdot.x, max|x| (u64 slot bits of a double).
// With qz_q (FP32 at k = 16 or 32 only): the down sweep's tiles also form the Gram
// Q'x (qz_q n x k) from per-tile FP64 partials in qz_part (counters qz_cnt), and the
// last tile stores the k x k total (row-major, ld kp) at qz_out or, with beta_out,
// stores beta = -G^-1 Q'x there instead (G^-1 at beta_ginv, both k x k, ld kp).
// With gate: every kernel of the solve returns at once while *gate is set.
// y = L_G x64 (grounded nowhere) in FP64, scaled by the power of two from
// scale_from: the right-hand side of the next L_P solve, kept in FP64. The rows
// longer than kLongRow (lrow, nlong of them: the long rows of the L_G ELL) take a
// workgroup each.
void lap_apply_x64(Topo &t, const Dims &d, const double *x64, double *y, const unsigned long long *scale_from,
                   const int *lrow, int nlong, hipStream_t s);
template <typename T>
void tree_solve(Topo &t, Vecs<T> &v, const Dims &d, const T *y, T *x, const T *rdot, double *dot_part,
                unsigned long long *absmax, hipStream_t s, const T *qz_q = nullptr, double *qz_part = nullptr,
                int *qz_cnt = nullptr, double *qz_out = nullptr, const double *beta_ginv = nullptr,
                T *beta_out = nullptr, const int *gate = nullptr);

// L_P solve: block PCG in working precision with the tree preconditioner inside an
// FP64 flexible CG: whenever every vector's recursive residual has fallen by
// pcg_inner_rtol, the block PCG's solution becomes the next FP64 search direction
// and the block PCG restarts from the new FP64 residual (bpcg.hip).
// Ends when ||b - L_P x||_2 <= pcg_rtol ||b||_2 per vector (FP64). Returns the
// iterations, the FP64 relative residual and the number of restarts.
struct SolveInfo {
    long long iters = 0;
    double resid64 = 0.0;
    int outer = 0;
};
template <typename T>
// basis: in FP32, run each inner solve on an orthonormal basis of the FP64 residual
// (needed when the k right-hand sides can be nearly parallel, as in later power
// steps; a caller with independent right-hand sides and a fixed short iteration
// count may leave it off). single: an inexact solve for a preconditioner: one inner
// phase of the block PCG from x = 0 (until every vector's residual has fallen by
// max(pcg_inner_rtol, pcg_rtol), or pcg_max_iters) and x = its working-precision
// solution, with no FP64 outer step or residual (resid64 = -1: not computed).
SolveInfo pcg_solve(Topo &t, Vecs<T> &v, const Dims &d, const T *b, T *x, const grass_opts &o, hipStream_t s,
                    const double *b64 = nullptr, bool basis = true, bool single = false);

// r = b - L_P x64 in FP64 (v.r64, and v.r rounded to T), squared norms in
// red[RED_RN]; returns max_j ||r_j|| / ||b_j|| (b norms in red[RED_BN]).
template <typename T>
double true_residual(Topo &t, Vecs<T> &v, const Dims &d, const T *b, hipStream_t s, const double *b64 = nullptr);
// One FP64 flexible-CG step of the L_P solve with z = v.dx from the inner block PCG,
// or z = z64 when given (first: start the recurrence): x64, r64, v.r and the norms in
// red[RED_RN] are updated, v.dx is cleared; returns max_j ||r_j|| / ||b_j||.
template <typename T>
double fcg_outer_step(Topo &t, Vecs<T> &v, const Dims &d, bool first, hipStream_t s, const double *z64 = nullptr);

// Score every edge: heat (optional output), FP64 per-vector sums over E and over P,
// max heat over the edges not in P. Then reduce to lambda_max (host reads).
struct PassScalars {
    double lambda_max = 0, lambda_min = 0, heat_max = 0;
};
template <typename T>
void score_edges(Topo &t, Vecs<T> &v, const Dims &d, const T *H, T *heat, hipStream_t s,
                 const double *H64 = nullptr);
template <typename T>
PassScalars finish_estimates(Topo &t, Vecs<T> &v, const Dims &d, hipStream_t s);

// fixed-order column sums of per-block partials part[b * stride + offset + j]
template <typename T>
void col_sum(const Dims &d, Vecs<T> &v, const double *part, int nblk, int stride, int offset, double *out,
             hipStream_t s);

// Block PCG (block size k, tree preconditioner) with FP64 refinement restarts;
// x64 and dx hold zero and red[RED_BN] the squared norms of b on entry.
struct PcgParams {
    double rtol = 1e-6, itol = 1e-2;
    int max_it = 8000, max_repl = 50;
    bool basis = true;  // FP32: inner solves on an orthonormal basis of the FP64 residual
    bool single = false;  // one inner phase from x = 0 and x = its solution (no FP64 step);
                          // the squared norms of b must be in red[RED_RN]
};
template <typename T>
SolveInfo block_pcg(Topo &t, Vecs<T> &v, const Dims &d, const T *b, const PcgParams &pp, hipStream_t s,
                    const double *b64 = nullptr);

// Scratch of the block PCG's in-kernel reductions: doubles of Vecs::gpart and
// counters of Vecs::tcnt.
long long bpcg_part_doubles(const Dims &d);
long long bpcg_counters(const Dims &d);

// Diagnostics: C = A'B (k x k, FP64, row-major) with the block-PCG Gram kernel;
// part and cnt sized as above.
template <typename T>
void block_gram(const Dims &d, const T *A, const T *B, double *part, int *cnt, double *out, hipStream_t s);

// max|x| of an n x k block into the absmax slot
template <typename T>
void absmax_of(const Dims &d, const T *x, unsigned long long *slot, hipStream_t s);

// Sec. V-E: L_G x = b for k right-hand sides by flexible preconditioned CG (one
// recurrence per column, FP64 coefficients), the preconditioner being the exact tree
// solve (tree_only) or the L_P solve above. Grounded at the root like every solve.
template <typename T>
struct SddVecs {
    T *r = nullptr, *z0 = nullptr, *z1 = nullptr, *p = nullptr, *q = nullptr;  // n x k each
    double *gram = nullptr;  // [4 * kp * kp]
    double *sc = nullptr;    // [4 * kMaxK]: (unused), r'z, alpha, beta
};
template <typename T>
void plan_sdd(Arena &a, const Dims &d, SddVecs<T> &B);
struct SddInfo {
    int iters = 0;           // outer iterations
    long long inner = 0;     // inner block-PCG iterations over all preconditioner solves
    double resid = 0.0;      // max over columns of ||b - L_G x|| / ||b|| (working precision, recomputed)
    int restarts = 0;        // recurrences restarted from the recomputed residual
};
template <typename T>
SddInfo sdd_solve(Topo &t, Vecs<T> &v, const Dims &d, SddVecs<T> &B, const T *b, T *x, double rtol, int maxit,
                  bool tree_only, const grass_opts &o, hipStream_t s);

// Sec. V-F: `steps` inverse power iterations u <- (L_G^+ u - mean) / norm from the
// eq. (28) start vector (k = 1), each solve by sdd_solve to rtol; side = sign cut
// (1 where u >= 0). u: device [n] working precision; side: device [n].
template <typename T>
struct PartVecs {
    T *x = nullptr;           // [n] solve output
    double *part = nullptr;   // per-block sums
    double *stats = nullptr;  // [2]: sum, sum of squares
};
template <typename T>
void plan_part(Arena &a, const Dims &d, PartVecs<T> &P);
struct PartInfo {
    long long outer = 0, inner = 0;
    double resid = 0.0;
};
template <typename T>
PartInfo partition_run(Topo &t, Vecs<T> &v, const Dims &d, SddVecs<T> &B, PartVecs<T> &P, T *u, uint8_t *side,
                       int steps, double rtol, int maxit, bool tree_only, const grass_opts &o, hipStream_t s);

}  // namespace grass
