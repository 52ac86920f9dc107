// Optional per-kernel-family timing with HIP events recorded on the launch stream.
#pragma once
#include "common.h"

namespace grass {

enum ProfKind : int {
    PK_SPMM_G = 0,  // y = L_G x (k_lap over the CSR of G)
    PK_SPMM_P,      // y = L_P x (k_lap over the CSR of P)
    PK_TREE_UP,     // tree solve, leaf-to-root sweep (k_sweep, up)
    PK_TREE_DOWN,   // tree solve, root-to-leaf sweep (k_sweep, down)
    PK_SCORE,       // edge scoring (k_score)
    PK_GRAM_PQR,    // block PCG: P'Q and P'R (Q = L_P P is PK_SPMM_P)
    PK_RUPDATE,     // block PCG: R -= Q alpha and the convergence count
    PK_BGRAM,       // block PCG: Q'Z (also P'P of the first block)
    PK_PUPDATE,     // block PCG: X += P alpha, P = Z + P beta and P'P
    PK_ROWMUL,      // block PCG: P = P R^-1 (and the last X += P alpha)
    PK_SMALL,       // block PCG: k x k FP64 steps (alpha, beta, R^-1), one wave
    PK_RESID64,     // FP64 outer iteration: residual, flexible-CG step, right-hand-side basis
    PK_START,       // start vectors
    PK_SELECT,      // candidate filter, sort and greedy
    PK_SPMM_G64,    // y = L_G x64 in FP64 (k_lap_x64): the right-hand side after an L_P solve
    PK_COUNT
};

struct Profiler {
    bool on = false;
    uint32_t mask = 0;  // bit i: time kernels of kind i
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double ms[PK_COUNT] = {};
    long long launches[PK_COUNT] = {};
    double bytes[PK_COUNT] = {};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        GR_HIP(hipEventCreate(&e));
        return e;
    }
    void reset() {
        for (int i = 0; i < PK_COUNT; i++) ms[i] = 0, launches[i] = 0, bytes[i] = 0;
    }
    // after the stream has been synchronized
    void resolve() {
        for (auto &r : recs) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                ms[r.kind] += t;
                launches[r.kind] += 1;
                bytes[r.kind] += r.bytes;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
    ~Profiler() {
        for (auto e : pool) (void)hipEventDestroy(e);
        for (auto &r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
    }
};

// The profiler of the calling context (set by the C-ABI layer for one call).
extern thread_local Profiler *g_prof;

struct ProfScope {
    Profiler *p = nullptr;
    hipStream_t s;
    int kind;
    double bytes;
    hipEvent_t a{};
    ProfScope(int kind_, double bytes_, hipStream_t s_) : s(s_), kind(kind_), bytes(bytes_) {
        if (g_prof && g_prof->on && ((g_prof->mask >> kind_) & 1u)) {
            p = g_prof;
            a = p->get();
            GR_HIP(hipEventRecord(a, s));
        }
    }
    ~ProfScope() {
        if (p) {
            hipEvent_t b = p->get();
            if (hipEventRecord(b, s) == hipSuccess) p->recs.push_back({kind, a, b, bytes});
        }
    }
};

}  // namespace grass
