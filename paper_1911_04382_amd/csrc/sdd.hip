// The sparsifier as a preconditioner (Sec. V-E of the paper), and the spectral
// partitioner built on it (Sec. V-F). L_G x = b is solved by
// preconditioned CG with z = L_P^+ r, L_P being the spectrally similar subgraph
// that the densification loop produced (or the spanning tree alone). The inner
// solve is the block PCG of the power iterations, accurate to pcg_rtol, so the
// outer recurrence uses the flexible (Polak-Ribiere) coefficient
// beta = r'(z_new - z_old) / r_old'z_old, which equals the plain one for an exact
// preconditioner. Each column has its own recurrence; inner products are FP64
// Gram diagonals, coefficients are formed on the device.
#include <algorithm>
#include <cmath>
#include <vector>

#include "embed.h"
#include "kern.h"
#include "profiler.h"

namespace grass {
namespace {

enum : int { SC_RZ = 1, SC_ALPHA = 2, SC_BETA = 3 };
constexpr int kMaxRestarts = 5;  // restarts from the true residual per solve

// x += alpha p, r -= alpha q (alpha per column)
template <typename T>
__global__ void k_fcg_step(long long nk, int k, const double *__restrict__ alpha, const T *__restrict__ p,
                           const T *__restrict__ q, T *__restrict__ x, T *__restrict__ r) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x) {
        const T a = (T)alpha[i % k];
        x[i] += a * p[i];
        r[i] -= a * q[i];
    }
}
// p = z + beta p (beta per column)
template <typename T>
__global__ void k_fcg_dir(long long nk, int k, const double *__restrict__ beta, const T *__restrict__ z,
                          T *__restrict__ p) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x)
        p[i] = z[i] + (T)beta[i % k] * p[i];
}
// coefficients from Gram diagonals (k x k, row-major, ld k):
//   INIT  rz = diag(g0)                      (r'z of the first preconditioned residual)
//   ALPHA alpha = rz / diag(g0)              (g0 = P'Q)
//   BETA  beta = (diag(g0) - diag(g1)) / rz; rz = diag(g0)   (g0 = r'z_new, g1 = r'z_old)
enum : int { FC_INIT = 0, FC_ALPHA = 1, FC_BETA = 2 };
__global__ void k_fcg_coef(int k, int op, const double *__restrict__ g0, const double *__restrict__ g1,
                           double *__restrict__ sc) {
    const int j = threadIdx.x;
    if (j >= k) return;
    const double d0 = g0[j * k + j];
    double *rz = sc + SC_RZ * kMaxK;
    if (op == FC_INIT) {
        rz[j] = d0;
    } else if (op == FC_ALPHA) {
        sc[SC_ALPHA * kMaxK + j] = d0 > 0.0 ? rz[j] / d0 : 0.0;
    } else {
        const double d1 = g1[j * k + j];
        sc[SC_BETA * kMaxK + j] = rz[j] > 0.0 ? (d0 - d1) / rz[j] : 0.0;
        rz[j] = d0;
    }
}

// r = b - q
template <typename T>
__global__ void k_sub(long long nk, const T *__restrict__ b, const T *__restrict__ q, T *__restrict__ r) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += (long long)gridDim.x * blockDim.x)
        r[i] = b[i] - q[i];
}

template <typename T>
void zero_row(T *a, long long row, int k, hipStream_t s) {
    fill_u32(reinterpret_cast<unsigned *>(a + row * k), (long long)k * (sizeof(T) / 4), 0u, s);
}

// Sec. V-F: per-block FP64 sums of x and x^2 (one vector), then one workgroup adds
// the blocks in index order: stats = {sum x, sum x^2}
constexpr int kStatBlocks = 256;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vec_stats(long long n, const T *__restrict__ x,
                                                        double *__restrict__ part) {
    __shared__ double s1[kThreads], s2[kThreads];
    double a = 0.0, b = 0.0;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const double v = (double)x[i];
        a += v;
        b += v * v;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int h = kThreads / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}
__global__ void k_vec_stats_sum(int nb, const double *__restrict__ part, double *__restrict__ stats) {
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < nb; i++) {
            a += part[2 * i];
            b += part[2 * i + 1];
        }
        stats[0] = a;
        stats[1] = b;
    }
}
// u = (x - mean) / ||x - mean||, with ||x - mean||^2 = sum x^2 - n mean^2
template <typename T>
__global__ void k_center_scale(long long n, const T *__restrict__ x, const double *__restrict__ stats,
                               T *__restrict__ u) {
    const double mean = stats[0] / (double)n;
    const double nrm2 = stats[1] - (double)n * mean * mean;
    const double sc = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        u[i] = (T)(((double)x[i] - mean) * sc);
}
// the sign cut: side 1 where u >= 0
template <typename T>
__global__ void k_sign_cut(long long n, const T *__restrict__ u, uint8_t *__restrict__ side) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        side[i] = u[i] >= (T)0 ? 1 : 0;
}

template <typename T>
void center_scale(long long n, const T *x, T *u, double *part, double *stats, hipStream_t s) {
    hipLaunchKernelGGL(k_vec_stats<T>, dim3(kStatBlocks), dim3(kThreads), 0, s, n, x, part);
    hipLaunchKernelGGL(k_vec_stats_sum, dim3(1), dim3(64), 0, s, kStatBlocks, part, stats);
    hipLaunchKernelGGL(k_center_scale<T>, dim3(grid_nk(n)), dim3(kThreads), 0, s, n, x, stats, u);
    GR_CHECK_LAUNCH();
}

}  // namespace

template <typename T>
void plan_part(Arena &a, const Dims &d, PartVecs<T> &P) {
    P.x = a.take<T>(d.n);
    P.part = a.take<double>(2 * kStatBlocks);
    P.stats = a.take<double>(2);
}

template <typename T>
PartInfo partition_run(Topo &t, Vecs<T> &v, const Dims &d, SddVecs<T> &B, PartVecs<T> &P, T *u, uint8_t *side,
                       int steps, double rtol, int maxit, bool tree_only, const grass_opts &o, hipStream_t s) {
    PartInfo info;
    // u0: the Philox Gaussian start vector of eq. (28) (pass 0, mean removed), normalized
    start_vectors<T>(d, o.seed, 0, P.x, v, s);
    center_scale<T>(d.n, P.x, u, P.part, P.stats, s);
    for (int i = 0; i < steps; i++) {
        SddInfo si = sdd_solve<T>(t, v, d, B, u, P.x, rtol, maxit, tree_only, o, s);
        info.outer += si.iters;
        info.inner += si.inner;
        info.resid = std::max(info.resid, si.resid);
        center_scale<T>(d.n, P.x, u, P.part, P.stats, s);
    }
    hipLaunchKernelGGL(k_sign_cut<T>, dim3(grid_nk(d.n)), dim3(kThreads), 0, s, d.n, u, side);
    GR_CHECK_LAUNCH();
    return info;
}

template <typename T>
void plan_sdd(Arena &a, const Dims &d, SddVecs<T> &B) {
    const long long nk = d.n * d.k;
    B.r = a.take<T>(nk);
    B.z0 = a.take<T>(nk);
    B.z1 = a.take<T>(nk);
    B.p = a.take<T>(nk);
    B.q = a.take<T>(nk);
    B.gram = a.take<double>(4ll * d.kp * d.kp);
    B.sc = a.take<double>(4 * kMaxK);
}

template <typename T>
SddInfo sdd_solve(Topo &t, Vecs<T> &v, const Dims &d, SddVecs<T> &B, const T *b, T *x, double rtol, int maxit,
                  bool tree_only, const grass_opts &o, hipStream_t s) {
    const long long nk = d.n * d.k;
    const int k = d.k, KK = d.kp * d.kp;
    const int root = 0;
    const int g = grid_nk(nk);
    double *G0 = B.gram, *G1 = B.gram + KK;
    SddInfo info;
    std::vector<double> hg(KK);
    // host copy of a Gram diagonal (convergence test only)
    auto diag = [&](const double *gd, std::vector<double> &out) {
        GR_HIP(hipMemcpyAsync(hg.data(), gd, (size_t)k * k * sizeof(double), hipMemcpyDeviceToHost, s));
        GR_HIP(hipStreamSynchronize(s));
        out.resize(k);
        for (int j = 0; j < k; j++) out[j] = hg[j * k + j];
    };
    auto precond = [&](const T *r, T *z) {
        if (tree_only) {
            tree_solve<T>(t, v, d, r, z, nullptr, nullptr, nullptr, s);
        } else {
            // one inner block-PCG phase on the outer iteration's residuals: no
            // right-hand-side basis, no FP64 step
            SolveInfo si = pcg_solve<T>(t, v, d, r, z, o, s, nullptr, false, true);
            info.inner += si.iters;
        }
    };
    // r = b (grounded row cleared), x = 0
    GR_HIP(hipMemcpyAsync(B.r, b, nk * sizeof(T), hipMemcpyDeviceToDevice, s));
    zero_row(B.r, root, k, s);
    fill_u32(reinterpret_cast<unsigned *>(x), nk * (long long)(sizeof(T) / 4), 0u, s);
    std::vector<double> bn, rr;
    block_gram<T>(d, B.r, B.r, v.gpart, v.tcnt, G0, s);
    diag(G0, bn);
    bool any = false;
    for (int j = 0; j < k; j++) any = any || bn[j] > 0.0;
    if (!any) return info;
    T *z = B.z0, *zo = B.z1;
    // a fresh recurrence from the residual in B.r: z = M^-1 r, p = z, rz = r'z
    auto start = [&]() {
        precond(B.r, z);
        GR_HIP(hipMemcpyAsync(B.p, z, nk * sizeof(T), hipMemcpyDeviceToDevice, s));
        block_gram<T>(d, B.r, z, v.gpart, v.tcnt, G0, s);
        hipLaunchKernelGGL(k_fcg_coef, dim3(1), dim3(kMaxK), 0, s, k, (int)FC_INIT, G0, G0, B.sc);
        GR_CHECK_LAUNCH();
    };
    // r = b - L_G x recomputed (grounded row cleared); returns max_j ||r_j|| / ||b_j||
    auto true_resid = [&]() {
        lap_apply<T>(d, t.rowptr, t.col, v.cval, v.eg, x, B.q, root, nullptr, nullptr, s);
        hipLaunchKernelGGL(k_sub<T>, dim3(g), dim3(kThreads), 0, s, nk, b, B.q, B.r);
        GR_CHECK_LAUNCH();
        zero_row(B.r, root, k, s);
        block_gram<T>(d, B.r, B.r, v.gpart, v.tcnt, G0, s);
        diag(G0, rr);
        double worst = 0.0;
        for (int j = 0; j < k; j++)
            if (bn[j] > 0.0) worst = std::max(worst, std::sqrt(rr[j] / bn[j]));
        return worst;
    };
    start();
    for (int restarts = 0;; restarts++) {
        while (info.iters < maxit) {
            info.iters++;
            lap_apply<T>(d, t.rowptr, t.col, v.cval, v.eg, B.p, B.q, root, nullptr, nullptr, s);
            block_gram<T>(d, B.p, B.q, v.gpart, v.tcnt, G0, s);
            hipLaunchKernelGGL(k_fcg_coef, dim3(1), dim3(kMaxK), 0, s, k, (int)FC_ALPHA, G0, G0, B.sc);
            hipLaunchKernelGGL(k_fcg_step<T>, dim3(g), dim3(kThreads), 0, s, nk, k, B.sc + SC_ALPHA * kMaxK, B.p,
                               B.q, x, B.r);
            GR_CHECK_LAUNCH();
            block_gram<T>(d, B.r, B.r, v.gpart, v.tcnt, G0, s);
            diag(G0, rr);
            bool done = true;
            for (int j = 0; j < k; j++) done = done && rr[j] <= rtol * rtol * bn[j];
            if (done) break;
            std::swap(z, zo);
            precond(B.r, z);
            block_gram<T>(d, B.r, z, v.gpart, v.tcnt, G0, s);
            block_gram<T>(d, B.r, zo, v.gpart, v.tcnt, G1, s);
            hipLaunchKernelGGL(k_fcg_coef, dim3(1), dim3(kMaxK), 0, s, k, (int)FC_BETA, G0, G1, B.sc);
            hipLaunchKernelGGL(k_fcg_dir<T>, dim3(g), dim3(kThreads), 0, s, nk, k, B.sc + SC_BETA * kMaxK, z,
                               B.p);
            GR_CHECK_LAUNCH();
        }
        // the recursive residual drifts from the true one in working precision: check
        // the true one and, if it misses rtol, restart the recurrence from it
        info.resid = true_resid();
        if (info.resid <= rtol || info.iters >= maxit || restarts >= kMaxRestarts) break;
        info.restarts++;
        start();
    }
    return info;
}

#define INST(T)                                                                                                  \
    template void plan_sdd<T>(Arena &, const Dims &, SddVecs<T> &);                                              \
    template SddInfo sdd_solve<T>(Topo &, Vecs<T> &, const Dims &, SddVecs<T> &, const T *, T *, double, int, bool, \
                                  const grass_opts &, hipStream_t);                                             \
    template void plan_part<T>(Arena &, const Dims &, PartVecs<T> &);                                            \
    template PartInfo partition_run<T>(Topo &, Vecs<T> &, const Dims &, SddVecs<T> &, PartVecs<T> &, T *,         \
                                       uint8_t *, int, double, int, bool, const grass_opts &, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace grass
