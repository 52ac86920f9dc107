// Filtering and similarity check (select.hip).
#pragma once
#include "state.h"

namespace grass {

struct SelectOut {
    long long candidates = 0, accepted = 0, processed = 0;
};

// Greedy state (mark/owner arrays at INT_MAX) must be initialised once per graph.
void init_greedy_state(Topo &t, hipStream_t s);

// Candidates of eq. (58) (heat >= theta * heat_max off P, compared in FP64), ranked
// by heat descending then id ascending; greedy similarity check; accepted edges get
// mask value 2. scores (optional): heat / heat_max off P, 0 in P (written first).
template <typename T>
SelectOut select_edges(Topo &t, const Dims &d, const T *heat, double theta, double heat_max, int sim_hops,
                       long long budget, T *scores, hipStream_t s);
// max heat over the edges not in P (device reduction, exact)
template <typename T>
double heat_max_off(Topo &t, const T *heat, hipStream_t s);
template <typename T>
void normalized_scores(Topo &t, const T *heat, double heat_max, T *scores, hipStream_t s);

}  // namespace grass
