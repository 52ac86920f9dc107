// Host-side pieces shared by the C-ABI entry points (api.hip) and the batch and
// serving drivers (serve.hip).
#pragma once
#include <string>

#include "common.h"
#include "profiler.h"
#include "launch_sched.h"

struct grass_ctx {
    int device = 0;
    void *static_ws = nullptr;  // this device's copy of the library's static scratch (grass_sparsify_static)
    std::string last_error;
    void *own_ws = nullptr;
    size_t own_bytes = 0;
    grass::Profiler prof;
    // launch schedule of the batch and server workers (grass_set_launch_mode), the
    // autotuner's choices per size class and the counters of grass_launch_stats_read
    int launch_mode = 1;
    int launch_chunks = 0;
    grass::Tuner tuner;
    grass::LaunchStats lstats;
};

namespace grass {

// Argument checks of grass_sparsify (throw Error).
void check_graph_args(const grass_graph *g);
void check_opts_args(const grass_opts &o);

// Workspace bytes of one sparsify call.
size_t sparsify_bytes(const grass_graph &g, const grass_opts &o);

// The whole method on one graph in the caller's workspace, on stream s (throws
// Error; returns GRASS_OK or GRASS_NOT_CONVERGED). Safe to call from several host
// threads at once with distinct workspaces and streams.
grass_status sparsify_run(grass_ctx *ctx, const grass_graph &g, const grass_opts &o, void *ws, size_t ws_bytes,
                          grass_result *res, hipStream_t s);

}  // namespace grass
