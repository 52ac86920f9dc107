// Graph setup entry points (graph.hip).
#pragma once
#include "state.h"

namespace grass {

// Named temporaries of the setup phase (CSR build, Boruvka, tree orientation and
// heavy-light layout).
struct SetupTmp {
    int *n1[12] = {};                  // [n+1] each
    int *a1[10] = {};                  // [max(2m, n+1)] each
    unsigned long long *ku = nullptr;  // [max(m, n)]
    long long *lvl = nullptr;          // [2*(kMaxLevels+1)]
};

void plan_topo(Arena &a, const Dims &d, Topo &t, SetupTmp &st);
void validate_graph(Topo &t, hipStream_t s);
template <typename T>
void build_csr(Topo &t, Vecs<T> &v, SetupTmp &st, hipStream_t s);
void boruvka(Topo &t, SetupTmp &st, uint8_t *tree, hipStream_t s);
template <typename T>
void build_tree(Topo &t, Vecs<T> &v, const Dims &d, SetupTmp &st, hipStream_t s);
template <typename T>
void build_pcsr(Topo &t, Vecs<T> &v, hipStream_t s);
void count_mask(Topo &t, const uint8_t *mask, long long out[3], hipStream_t s);

}  // namespace grass
