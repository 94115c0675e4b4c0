// HIP runtime objects of the SDMM solver: its two streams and four events, and the graphs
// one solve captures.  Host code only (no kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/purify.h"

namespace purify {

// The streams and events an SDMM solve runs on: the main stream (CG, branches i = 2 and 3),
// the stream of branch i = 1, the event that orders the solve after the caller's stream, and
// the fork/join events between the two streams.  Created once -- by a plan on its first solve,
// or by a server worker slot for all the solves it runs -- and reused by every later solve, so
// solves on several host threads create and destroy no runtime objects.  Released only after
// both streams have drained.
struct SolverStreams {
    hipStream_t cs = nullptr, cs2 = nullptr;
    hipEvent_t entry = nullptr, fork = nullptr, join = nullptr, hat = nullptr;
    bool ready = false;
};

// Create the streams and events on the current device (no-op if ready).
purify_status solver_streams_init(SolverStreams& ss);
// Drain both streams, then destroy every object (no-op if never created).
void solver_streams_release(SolverStreams& ss);

// Graph capture and instantiation, and graph destruction, take this process-wide lock: one
// thread at a time captures, instantiates or destroys a graph, whatever the other threads
// launch meanwhile.
std::mutex& graph_mutex();

// The graphs of one solve (the power-iteration step and the SDMM iteration).  The destructor
// drains the solver's streams before destroying the executable graphs, so no graph is
// destroyed while a launch of it may still run (also on error returns).
struct SolveGraphs {
    SolverStreams* ss = nullptr;
    hipGraph_t g[2] = {nullptr, nullptr};
    hipGraphExec_t x[2] = {nullptr, nullptr};
    explicit SolveGraphs(SolverStreams* s) : ss(s) {}
    SolveGraphs(const SolveGraphs&) = delete;
    SolveGraphs& operator=(const SolveGraphs&) = delete;
    ~SolveGraphs();
};

// End the capture begun on cs (caller holds graph_mutex) into graph slot k and instantiate it.
// On failure the capture is ended and the partial graph released.
purify_status end_capture(SolveGraphs& G, int k, hipStream_t cs);

}  // namespace purify
