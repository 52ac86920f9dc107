// Device-resident state of one graph: the CSR of L_G, the subgraph P, the rooted
// spanning tree and its heavy-light solve layout, the vectors of the power
// iterations and the PCG buffers. Every pointer lives in one Arena.
#pragma once
#include "common.h"

namespace grass {

constexpr int kMaxLevels = 64;   // light depth <= log2(n) < 32; margin
constexpr int kSolveThreads = 512;  // threads of a tree-sweep workgroup (one tile)
constexpr int kSolveNPR = 16;    // largest number of nodes per run in the tree-solve scans
constexpr int kMaxK = 64;

enum : uint8_t { SEG_TOP = 1, SEG_BOT = 2, SEG_LC = 4 };  // path top, path bottom, has light children

// Nodes per run of a tree-sweep tile: a run is the KP lanes of one vector row,
// a tile holds kSolveThreads / KP runs, so a tile covers at most 512 nodes.
constexpr int solve_npr(int kp) { return kp < kSolveNPR ? kp : kSolveNPR; }

// Sizes that fix the workspace plan.
struct Dims {
    long long n = 0, m = 0;
    int k = 1, kp = 1, prec = 32;
    int TN = 0;          // tree-solve tile, nodes
    long long Npad = 0;  // padded layout length bound
    long long ntiles = 0;
    long long p_nnz = 0;  // nonzeros of the CSR of L_P (off-diagonal), host copy
};

inline Dims make_dims(long long n, long long m, int k, int prec) {
    Dims d;
    d.n = n;
    d.m = m;
    d.k = k;
    d.kp = kpad(k);
    d.prec = prec;
    d.TN = solve_npr(d.kp) * kSolveThreads / d.kp;
    d.Npad = n + (long long)kMaxLevels * d.TN;
    d.ntiles = (d.Npad + d.TN - 1) / d.TN;
    return d;
}

// Graph topology (precision-independent part).
struct Topo {
    long long n = 0, m = 0;
    const int *src = nullptr, *dst = nullptr;
    const double *w = nullptr;
    int *rowptr = nullptr, *col = nullptr, *ceid = nullptr;  // CSR of G, rows sorted by neighbour
    double *degG = nullptr;
    unsigned *devflags = nullptr;  // device error bits
    int *scal_i = nullptr;         // small integer scratch (counters)
    // subgraph
    uint8_t *mask = nullptr;       // [m] 1 tree / 2 added / 0 off
    int *prow = nullptr, *pcol = nullptr;  // CSR of L_P
    double *pval64 = nullptr;      // FP64 weights of L_P (refinement residual)
    double *degP = nullptr;
    // rooted tree
    int *parent = nullptr, *heavy = nullptr, *head = nullptr, *off = nullptr, *ld = nullptr, *lp = nullptr;
    double *pw = nullptr;
    // layout
    long long N = 0;               // used layout length (tile aligned)
    int nlev = 0;
    std::vector<long long> lvl_start;  // host: [nlev+1] positions (tile aligned)
    int *perm = nullptr;           // [Npad] node or -1
    uint8_t *flags = nullptr;      // [Npad]
    int *ptop = nullptr;           // [Npad]
    int *lc_ptr = nullptr;         // [Npad+1]
    int *lc_pos = nullptr;         // [n]
    int *lc_owner = nullptr;       // [n] position of each entry's parent
    int *lcmax = nullptr;          // [1] most light children of one node (when more than 2)
    int max_lc = 0;                // host copy
    // tile scan state
    unsigned *done = nullptr;      // [ntiles] outputs written (epoch stamp)
    int *tickets = nullptr;        // [2*kMaxLevels]: sweep tickets
    unsigned *epoch_dev = nullptr; // [2]: current sweep epoch (device-side, advanced per solve)
    int *lvl_tile = nullptr;       // [kMaxLevels+1] first tile of each level (layout order), device
    int *dep_up_ptr = nullptr, *dep_up = nullptr;  // per-tile up-sweep dependencies (tiles of light children)
    int *dep_dn_ptr = nullptr, *dep_dn = nullptr;  // per-tile down-sweep dependencies (tiles of path parents)
    long long ntiles_used = 0;
    unsigned epoch = 0;
    // scratch for setup and selection
    ScanTmp scan;
    SortTmp sort;
    int *tmpA = nullptr, *tmpB = nullptr;  // [max(2m, n+1)] selection scratch
    unsigned long long *keys = nullptr;  // [max(m, n)] sort keys of the selection
    int *greedy_mark = nullptr, *greedy_owner = nullptr;  // [n]
    uint8_t *cand_acc = nullptr;   // [m]
};

// The first E entries of every CSR row of a Laplacian, row-major and padded with
// the row's own column and a zero weight (so padding adds w (x_v - x_v) = 0 and
// needs no branch); rows longer than E continue in the CSR. One SpMM row step then
// reads its neighbours without first reading the row pointers.
template <typename T>
struct Ell {
    int E = 0;
    int *col = nullptr;  // [n*E]
    T *val = nullptr;    // [n*E]
    int *deg = nullptr;  // [n] CSR row length, or -(1 + index in lrow) for a long row
    // rows longer than kLongRow: their entries past E are summed by a workgroup each
    // before the product (tail[li*k + j]), so one long row does not hold up a tile
    int cap = 0;           // capacity of lrow
    int nlong = 0;         // host copy of the count, set when the ELL is filled
    int *lcount = nullptr; // [1] device counter
    int *lrow = nullptr;   // [cap] row ids
    T *tail = nullptr;     // [cap*k]
};
constexpr int kEllG = 8;  // 7-point meshes and grids fit whole rows
constexpr int kEllP = 4;  // spanning tree plus a few edges
constexpr int kLongRow = 32;  // rows longer than this get a workgroup of their own

// Device-side control of the block PCG's inner loop (one per solve): the check
// kernel's tail counts the iteration and, where the host loop would look (every 4th
// iteration and the last), decides whether the inner phase ends (gate = 1). Kernels
// launched with a gate return at once while it is set, so a captured chunk of
// iterations replayed past the end does nothing.
struct LoopCtl {
    int gate;      // 1: the inner phase has ended
    int it;        // iterations so far in this solve
    int phase0;    // iterations before the current inner phase
    int max_it;    // iteration cap of the solve
    int stall_ok;  // a stall may still switch on the dependence threshold (FP32)
    int pad[3];
    double own;    // dependence threshold of the block normalisation (0: off)
};

// Precision-dependent buffers.
template <typename T>
struct Vecs {
    T *wT = nullptr;      // [m] edge weights
    T *cval = nullptr;    // [2m] CSR(G) weights
    T *pval = nullptr;    // [2m] CSR(P) weights
    Ell<T> eg, ep;        // padded first entries of the CSR rows of L_G and L_P
    T *rpw = nullptr;     // [Npad] 1/parent weight in layout order
    T *H = nullptr, *Y = nullptr;  // [n*kp]
    T *F = nullptr;       // [Npad*kp] subtree currents (layout order)
    unsigned long long *aggw = nullptr;  // [ntiles*kp*sizeof(T)/4] tagged tile aggregates of the sweeps
    T *heat = nullptr;    // [m] (internal heat when the caller gives none)
    // PCG
    T *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *dx = nullptr;  // [n*kp]
    // the FP64 outer iteration of the L_P solve: solution, residual, direction, A d, A z
    double *x64 = nullptr, *r64 = nullptr, *d64 = nullptr, *ad64 = nullptr, *w64 = nullptr;  // [n*k]
    double *b64 = nullptr;  // [n*k] FP64 right-hand side L_G x64 of a power step after an L_P solve
    double *z64 = nullptr;  // [n*k] inner-solve result mapped back from the orthonormal basis (FP32 only)
    // reductions
    double *part = nullptr;   // [ntiles*kp*2] per-block partials
    double *part2 = nullptr;  // [64*kp] first-stage column sums
    double *small = nullptr;  // k x k FP64 matrices of the block PCG
    T *smallT = nullptr;      // alpha, beta, R^-1 in working precision
    double *gpart = nullptr;  // block-PCG tail reductions: per-block partials and level sums
    int *tcnt = nullptr;      // their arrival counters (zero between launches)
    double *red = nullptr;    // [16*kMaxK] reduced vectors (num, den, rz, pq, rr, rr0, bnorm, ...)
    int *active = nullptr;    // [kMaxK] PCG column flags + count at [kMaxK-1]
    LoopCtl *loop = nullptr;  // inner-loop control of the block PCG
    unsigned long long *u64s = nullptr;  // [8]: heat max bits, lambda_min bits, absmax bits
};

}  // namespace grass
