// Low-stretch spanning tree (lsst.hip).
#pragma once
#include "state.h"

namespace grass {

// Device bytes low_stretch_tree takes from its arena for n nodes and m edges.
size_t lsst_bytes(long long n, long long m);

// The spanning tree of the AKPW construction over binary weight classes with
// exponential start-time clustering (Sec. III-A suggests a low-stretch backbone):
// tree[e] = 1 for the tree edges, 0 otherwise (device [m]). t supplies n, m, src,
// dst, w (validated). Returns the number of rounds; throws GRASS_ERR_DISCONNECTED
// when no edge joins the clusters left.
int low_stretch_tree(Topo &t, Arena &a, uint64_t seed, int class_bits, uint8_t *tree, hipStream_t s);

}  // namespace grass
