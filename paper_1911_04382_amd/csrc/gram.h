// Deterministic block reductions shared by the block-PCG kernels and the tree
// sweeps: k x k Gram accumulators over row layouts (MFMA for FP32 at KP = 32 / 16)
// and the fixed-order reduction of per-item FP64 partials at the end of a kernel.
#pragma once
#include "kern.h"

namespace grass {

// FP32 blocks of 16 or 32 vectors take the MFMA Gram accumulators
template <typename T, int KP>
struct UseMF {
    static constexpr bool value = sizeof(T) == 4 && (KP == 16 || KP == 32);
};

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

// ------------------------------------------------------------ Gram accumulators
// C += a'b over the rows a block holds (lane l of a wave: row l / KP of the wave,
// column l % KP). For FP32 with KP = 32 or 16 this is one MFMA per 2 (or 4) rows:
// in that lane layout the A operand of v_mfma_f32_32x32x2f32 (lane l holds
// A[l % 32][l / 32]) is exactly a' and the B operand (lane l holds B[l / 32][l % 32])
// is exactly b, so the instruction accumulates a'b. Other widths and FP64 keep
// per-lane column accumulators fed by shuffles.
// flush(s, out): fixed-order FP64 sum over the block (through s, KP*KP doubles of
// LDS) stored to out with agent-scope stores (read by the tail reduction).
template <typename T, int KP, bool MF = (sizeof(T) == 4 && (KP == 32 || KP == 16))>
struct BlockGram {
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
        const int G = blockDim.x / KP;
        const int g = threadIdx.x / KP, j = threadIdx.x % KP;
        if constexpr (KP <= 8) {
            // narrow blocks have many lane groups (256 at k = 1): every group stores
            // its accumulators at once and each entry is summed over the groups in
            // group order, the order of the fold below, so the bits are the same
            __shared__ double s_all[kThreads * KP];
            if (blockDim.x <= kThreads) {
                __syncthreads();
                for (int i = 0; i < KP; i++) s_all[(g * KP + i) * KP + j] = (double)acc[i];
                __syncthreads();
                for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) {
                    double t = 0.0;
                    for (int q = 0; q < G; q++) t += s_all[q * KP * KP + e];
                    st_agent(&out[e], t);
                }
                __syncthreads();
                return;
            }
        }
        __syncthreads();
        for (int gg = 0; gg < G; gg++) {
            if (g == gg)
                for (int i = 0; i < KP; i++) s[i * KP + j] = (gg ? s[i * KP + j] : 0.0) + (double)acc[i];
            __syncthreads();
        }
        for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) st_agent(&out[e], s[e]);
        __syncthreads();
    }
};
// one wave's MFMA accumulator into s (wave order fixes the sum order)
template <int KP, typename F>
__device__ __forceinline__ void flush_mfma(double *s, double *__restrict__ out, F &&put) {
    const int w = threadIdx.x >> 6;
    __syncthreads();
    const int nw = blockDim.x / 64;
    for (int ww = 0; ww < nw; ww++) {
        if (w == ww) put(s, ww == 0);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) st_agent(&out[e], s[e]);
    __syncthreads();
}
template <typename T>
struct BlockGram<T, 32, true> {
    floatx16 c;
    __device__ void zero() {
#pragma unroll
        for (int r = 0; r < 16; r++) c[r] = 0.f;
    }
    __device__ void add(float a, float b) { c = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
    // accumulator layout: lane l, register r -> C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
    __device__ void flush(double *s, double *__restrict__ out) {
        flush_mfma<32>(s, out, [&](double *sh, bool first) {
            const int lane = threadIdx.x & 63;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                int e = (8 * (r / 4) + 4 * (lane / 32) + (r % 4)) * 32 + (lane % 32);
                sh[e] = (first ? 0.0 : sh[e]) + (double)c[r];
            }
        });
    }
};
template <typename T>
struct BlockGram<T, 16, true> {
    floatx4 c;
    __device__ void zero() {
#pragma unroll
        for (int r = 0; r < 4; r++) c[r] = 0.f;
    }
    __device__ void add(float a, float b) { c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // accumulator layout: lane l, register r -> C[4 (l / 16) + r][l % 16]
    __device__ void flush(double *s, double *__restrict__ out) {
        flush_mfma<16>(s, out, [&](double *sh, bool first) {
            const int lane = threadIdx.x & 63;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                int e = (4 * (lane / 16) + r) * 16 + (lane % 16);
                sh[e] = (first ? 0.0 : sh[e]) + (double)c[r];
            }
        });
    }
};

// ------------------------------------------------------------- tail reduction
// A kernel whose block b has stored `width` FP64 partials at part + b * width (with
// agent-scope stores) finishes its reduction itself: blocks are grouped kFan at a
// time, the last block of a group to arrive (integer arrival counter) sums the
// group's items in index order into the next level, and so on until one block
// holds the total. Sums are in a fixed order whatever the arrival order, so the
// result is deterministic. Counters are returned to zero by the block that
// consumes them, so consecutive launches (and graph replays) need no clearing.
constexpr int kFan = 16;

__host__ __device__ inline long long tail_items(long long nblk) {
    long long s = nblk;
    while (nblk > 1) {
        nblk = (nblk + kFan - 1) / kFan;
        s += nblk;
    }
    return s;
}

// true in exactly one block, which then holds the total in tot[0, width) (LDS)
__device__ inline bool tail_reduce(double *part, int nblk, int width, int *cnt, double *tot, int item = -1) {
    __shared__ int s_last;
    int idx = item >= 0 ? item : (int)blockIdx.x, nl = nblk;
    double *lvl = part;
    double *next = part + (long long)nblk * width;
    int *c = cnt;
    wait_mem();
    __syncthreads();
    if (nl == 1) {
        for (int e = threadIdx.x; e < width; e += blockDim.x) tot[e] = ld_agent(&part[e]);
        __syncthreads();
        return true;
    }
    while (true) {
        const int grp = idx / kFan, first = grp * kFan, gs = min(kFan, nl - first);
        const int ng = (nl + kFan - 1) / kFan;
        if (threadIdx.x == 0) {
            int old = atomicAdd(&c[grp], 1);
            s_last = old == gs - 1;
            if (old == gs - 1) atomicExch(&c[grp], 0);
        }
        __syncthreads();
        if (!s_last) return false;
        for (int e = threadIdx.x; e < width; e += blockDim.x) {
            double v[kFan];
#pragma unroll
            for (int i = 0; i < kFan; i++) {
                double x = ld_agent(&lvl[(long long)(first + (i < gs ? i : 0)) * width + e]);
                v[i] = i < gs ? x : 0.0;
            }
            double a = v[0];
#pragma unroll
            for (int i = 1; i < kFan; i++) a += v[i];
            if (ng == 1)
                tot[e] = a;
            else
                st_agent(&next[(long long)grp * width + e], a);
        }
        if (ng == 1) {
            __syncthreads();
            return true;
        }
        wait_mem();
        __syncthreads();
        idx = grp;
        lvl = next;
        next += (long long)ng * width;
        c += ng;
        nl = ng;
    }
}

}  // namespace grass
