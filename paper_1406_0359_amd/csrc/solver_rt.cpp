// HIP runtime objects of the SDMM solver (streams, events, captured graphs); see solver_rt.h.
#include "solver_rt.h"

#include "common.h"

namespace purify {

purify_status solver_streams_init(SolverStreams& ss) {
    if (ss.ready) return PURIFY_OK;
    SolverStreams t;
    hipError_t e = hipStreamCreateWithFlags(&t.cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&t.cs2, hipStreamNonBlocking);
    hipEvent_t* ev[4] = {&t.entry, &t.fork, &t.join, &t.hat};
    for (hipEvent_t* p : ev)
        if (e == hipSuccess) e = hipEventCreateWithFlags(p, hipEventDisableTiming);
    if (e != hipSuccess) {
        t.ready = true;   // release what was created
        solver_streams_release(t);
        set_error(std::string("solver streams: ") + hipGetErrorString(e));
        return PURIFY_E_DEVICE;
    }
    t.ready = true;
    ss = t;
    return PURIFY_OK;
}

void solver_streams_release(SolverStreams& ss) {
    if (!ss.ready) return;
    if (ss.cs) (void)hipStreamSynchronize(ss.cs);
    if (ss.cs2) (void)hipStreamSynchronize(ss.cs2);
    for (hipEvent_t e : {ss.entry, ss.fork, ss.join, ss.hat})
        if (e) (void)hipEventDestroy(e);
    if (ss.cs) (void)hipStreamDestroy(ss.cs);
    if (ss.cs2) (void)hipStreamDestroy(ss.cs2);
    ss = SolverStreams{};
}

std::mutex& graph_mutex() {
    static std::mutex mu;
    return mu;
}

SolveGraphs::~SolveGraphs() {
    if (!g[0] && !g[1] && !x[0] && !x[1]) return;
    if (ss && ss->cs) (void)hipStreamSynchronize(ss->cs);
    if (ss && ss->cs2) (void)hipStreamSynchronize(ss->cs2);
    std::lock_guard<std::mutex> lk(graph_mutex());
    for (int k = 0; k < 2; ++k) {
        if (x[k]) (void)hipGraphExecDestroy(x[k]);
        if (g[k]) (void)hipGraphDestroy(g[k]);
    }
}

purify_status end_capture(SolveGraphs& G, int k, hipStream_t cs) {
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        return PURIFY_E_DEVICE;
    }
    G.g[k] = g;
    PURIFY_HIP(hipGraphInstantiate(&G.x[k], g, nullptr, nullptr, 0));
    return PURIFY_OK;
}

}  // namespace purify
