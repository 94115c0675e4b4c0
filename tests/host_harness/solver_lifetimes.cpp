// Host-only harness for the solver's HIP object lifetimes.  The library's own host code --
// plan creation (plan.cpp), the SDMM driver and the C ABI (api.cpp), the solver streams and
// graphs (solver_rt.cpp) and the serving loop (server.cpp) -- runs unchanged on stand-ins for
// the HIP runtime defined here; the kernel launchers are no-op stubs generated from common.h
// (they only mark their stream busy).  Device memory is host memory.
//
// The stand-ins model what the runtime may still be doing: a stream is busy from any work
// enqueued on it until it is synchronised, a stream waits on the events it was told to wait
// on until then, and a graph launch runs until its stream is synchronised.  They report
// (and the run fails on) every use that is unsafe under that model:
//   - an event destroyed while a stream still waits on it;
//   - a stream destroyed with work pending;
//   - an executable graph destroyed while a launch of it may still run;
//   - any call on a destroyed stream, event or graph;
//   - two threads capturing or instantiating graphs at the same time.
//
// usage: solver_lifetimes <requests> <slots>; prints "done <k> requests, <b> bad, <u> misuses".
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_1406_0359_amd/csrc/common.h"

namespace {

struct SStream;
struct SEvent {
    bool alive = true;
};
struct SStream {
    bool alive = true;
    bool busy = false;
    std::set<SEvent*> waits;
};
struct SGraph {
    bool alive = true;
};
struct SExec {
    bool alive = true;
    SStream* launched_on = nullptr;
};

std::mutex g_mu;   // guards the model
std::set<void*> g_streams, g_events, g_graphs, g_execs;
SStream g_null_stream;
std::atomic<int> g_misuses{0};
std::atomic<int> g_building{0};   // threads between begin-capture and instantiate

void misuse(const std::string& what) {
    ++g_misuses;
    std::fprintf(stdout, "MISUSE: %s\n", what.c_str());
    std::fflush(stdout);
}

SStream* S(hipStream_t s, const char* call) {
    if (!s) return &g_null_stream;
    SStream* p = reinterpret_cast<SStream*>(s);
    if (!g_streams.count(p)) misuse(std::string(call) + " on an unknown stream");
    else if (!p->alive) misuse(std::string(call) + " on a destroyed stream");
    return p;
}
SEvent* E(hipEvent_t e, const char* call) {
    SEvent* p = reinterpret_cast<SEvent*>(e);
    if (!g_events.count(p)) misuse(std::string(call) + " on an unknown event");
    else if (!p->alive) misuse(std::string(call) + " on a destroyed event");
    return p;
}

void sync_stream(SStream* p) {
    p->busy = false;
    p->waits.clear();
}

}  // namespace

// ---- HIP runtime stand-ins -----------------------------------------------------------------
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "host stand-in"; }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    std::lock_guard<std::mutex> lk(g_mu);
    SStream* p = new SStream();
    g_streams.insert(p);
    *s = reinterpret_cast<hipStream_t>(p);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    SStream* p = S(s, "hipStreamDestroy");
    if (p->busy) misuse("stream destroyed with work pending");
    p->alive = false;   // kept, so a later use is caught
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    sync_stream(S(s, "hipStreamSynchronize"));
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
    std::lock_guard<std::mutex> lk(g_mu);
    SEvent* p = new SEvent();
    g_events.insert(p);
    *e = reinterpret_cast<hipEvent_t>(p);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(g_mu);
    SEvent* p = E(e, "hipEventDestroy");
    for (void* v : g_streams) {
        SStream* s = static_cast<SStream*>(v);
        if (s->alive && s->waits.count(p)) misuse("event destroyed while a stream waits on it");
    }
    if (g_null_stream.waits.count(p)) misuse("event destroyed while the null stream waits on it");
    p->alive = false;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    E(e, "hipEventRecord");
    S(s, "hipEventRecord")->busy = true;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    std::lock_guard<std::mutex> lk(g_mu);
    SEvent* pe = E(e, "hipStreamWaitEvent");
    SStream* ps = S(s, "hipStreamWaitEvent");
    ps->waits.insert(pe);
    ps->busy = true;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(g_mu);
    E(e, "hipEventSynchronize");
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_mu);
    E(a, "hipEventElapsedTime");
    E(b, "hipEventElapsedTime");
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* src, size_t b, hipMemcpyKind, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        S(s, "hipMemcpyAsync")->busy = true;
    }
    std::memcpy(d, src, b);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t b, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        S(s, "hipMemsetAsync")->busy = true;
    }
    std::memset(d, v, b);
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    if (g_building.fetch_add(1) != 0) misuse("two threads capture or instantiate graphs at once");
    std::lock_guard<std::mutex> lk(g_mu);
    S(s, "hipStreamBeginCapture");
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    std::lock_guard<std::mutex> lk(g_mu);
    S(s, "hipStreamEndCapture");
    SGraph* p = new SGraph();
    g_graphs.insert(p);
    *g = reinterpret_cast<hipGraph_t>(p);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        SGraph* pg = reinterpret_cast<SGraph*>(g);
        if (!g_graphs.count(pg) || !pg->alive) misuse("instantiate of an unknown or destroyed graph");
        SExec* p = new SExec();
        g_execs.insert(p);
        *x = reinterpret_cast<hipGraphExec_t>(p);
    }
    g_building.fetch_sub(1);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    SExec* p = reinterpret_cast<SExec*>(x);
    if (!g_execs.count(p) || !p->alive) misuse("launch of an unknown or destroyed graph");
    SStream* ps = S(s, "hipGraphLaunch");
    ps->busy = true;
    p->launched_on = ps;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    std::lock_guard<std::mutex> lk(g_mu);
    SExec* p = reinterpret_cast<SExec*>(x);
    if (!g_execs.count(p) || !p->alive) misuse("destroy of an unknown or destroyed graph exec");
    if (p->launched_on && p->launched_on->busy) misuse("graph exec destroyed while a launch of it may run");
    p->alive = false;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    std::lock_guard<std::mutex> lk(g_mu);
    SGraph* p = reinterpret_cast<SGraph*>(g);
    if (!g_graphs.count(p) || !p->alive) misuse("destroy of an unknown or destroyed graph");
    p->alive = false;
    return hipSuccess;
}

// Called by every generated kernel-launcher stub.
void harness_kernel(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    S(s, "kernel launch")->busy = true;
}

// ---- the requests ----------------------------------------------------------------------------
namespace {

std::vector<double> uv_draw(std::mt19937_64& g, int64_t M) {
    std::uniform_real_distribution<double> ang(-3.2, 3.2);
    std::vector<double> uv((size_t)2 * M);
    for (double& v : uv) v = ang(g);
    return uv;
}

purify_plan_desc desc_for(int n, int64_t M, const double* uv, int prec) {
    purify_plan_desc d{};
    d.n = n;
    d.oversample = 2;
    d.J = 6;
    d.M = M;
    d.uv = uv;
    d.dict_mask = PURIFY_DICT_SARA;
    d.levels = 4;
    d.precision = prec;
    return d;
}

purify_sdmm_params params_for(int i) {
    purify_sdmm_params p{};
    p.epsilon = 1;
    p.max_iter = 12;
    p.cg_iter = 1 + i % 3;
    p.halting = i % 2;
    p.check_every = 1 + (i % 4) * 3;
    p.nu_iter = 4;
    p.nu = i % 3 == 0 ? 0.0 : 2.0;   // 0: power iteration (captured graph)
    p.gamma = i % 5 == 0 ? 0.0 : 1e-3;
    p.flags = i % 7 == 3 ? PURIFY_SDMM_NO_GRAPH : 0;
    p.xi = 1e-4;
    p.slack = 1e-3;
    return p;
}

// Direct solves on one plan (the plan's own streams, created on its first solve): plain,
// eager, reweighted, then every stage timed; the plan is destroyed at the end (the caller
// runs this for one plan after another, as a timing script over several workloads does).
int direct_solves(int n, int64_t M, int precision, unsigned seed) {
    std::mt19937_64 g(seed);
    std::vector<double> uv = uv_draw(g, M);
    purify_plan_desc d = desc_for(n, M, uv.data(), precision);
    const size_t ws = purify_plan_workspace_bytes(&d);
    void* mem = aligned_alloc(256, (ws + 255) / 256 * 256);
    std::vector<unsigned char> y((size_t)M * 16, 0), x((size_t)n * n * 16, 0);
    std::vector<double> w((size_t)purify_plan_dict_size(&d), 1.0);
    purify_plan* plan = nullptr;
    int bad = 0;
    if (purify_plan_create(&d, mem, ws, nullptr, &plan) != PURIFY_OK) return 1;
    for (int i = 0; i < 4; ++i) {
        purify_sdmm_params p = params_for(i);
        purify_sdmm_info info{};
        if (purify_sdmm_solve(plan, y.data(), &p, x.data(), &info, nullptr) != PURIFY_OK) ++bad;
    }
    purify_sdmm_params p = params_for(1);
    purify_reweight_params rw{};
    rw.delta0 = 1.0;
    rw.decay = 0.5;
    rw.delta_min = 1e-3;
    rw.rel_var = 0.0;
    rw.reweights = 2;
    purify_sdmm_info info{};
    purify_reweight_info rinfo{};
    (void)purify_sdmm_reweighted(plan, y.data(), &p, &rw, w.data(), x.data(), &info, &rinfo, nullptr);
    for (int st = 0; st <= PURIFY_STAGE_TV_STEP; ++st) {
        double ms = 0;
        if (purify_time_stage(plan, st, 3, nullptr, &ms) != PURIFY_OK) ++bad;
    }
    for (int i = 4; i < 7; ++i) {   // short solves after the timings, as before the next plan
        purify_sdmm_params q = params_for(i);
        purify_sdmm_info qi{};
        if (purify_sdmm_solve(plan, y.data(), &q, x.data(), &qi, nullptr) != PURIFY_OK) ++bad;
    }
    purify_plan_destroy(plan);
    free(mem);
    return bad;
}

}  // namespace

int main(int argc, char** argv) {
    const int count = argc > 1 ? atoi(argv[1]) : 24, slots = argc > 2 ? atoi(argv[2]) : 8;
    int bad = direct_solves(64, 3000, PURIFY_FP64, 11);
    bad += direct_solves(128, 9000, PURIFY_FP32, 12);
    bad += direct_solves(64, 2500, PURIFY_FP64, 13);
    const size_t arena_bytes = (size_t)1 << 30;
    void* arena = aligned_alloc(256, arena_bytes);
    purify_server_desc sd{};
    sd.arena = arena;
    sd.arena_bytes = arena_bytes;
    sd.max_active = slots;
    purify_server* srv = nullptr;
    if (purify_server_create(&sd, &srv) != PURIFY_OK) {
        std::printf("create failed: %s\n", purify_last_error());
        return 1;
    }
    std::mt19937_64 g(7);
    const int sizes[4] = {64, 64, 128, 256};
    std::vector<int64_t> tickets;
    std::vector<int> ns, precs;
    for (int i = 0; i < count; ++i) {
        const int n = sizes[i % 4];
        std::uniform_real_distribution<double> ratio(0.2, 2.0);
        const int64_t M = (int64_t)(ratio(g) * n * n);
        std::vector<double> uv = uv_draw(g, M);
        const int prec = i % 3 == 0 ? PURIFY_FP64 : PURIFY_FP32;
        std::vector<unsigned char> y((size_t)M * (prec == PURIFY_FP64 ? 16 : 8), 0);
        purify_plan_desc d = desc_for(n, M, uv.data(), prec);
        purify_sdmm_params p = params_for(i);
        int64_t t = 0;
        if (purify_server_submit(srv, &d, y.data(), &p, &t) != PURIFY_OK) {
            std::printf("submit failed: %s\n", purify_last_error());
            return 1;
        }
        tickets.push_back(t);
        ns.push_back(n);
        precs.push_back(prec);
    }
    for (size_t i = 0; i < tickets.size(); ++i) {
        std::vector<unsigned char> x((size_t)ns[i] * ns[i] * (precs[i] == PURIFY_FP64 ? 16 : 8));
        purify_sdmm_info info{};
        const purify_status st = purify_server_wait(srv, tickets[i], x.data(), &info, nullptr);
        if (st != PURIFY_OK) {
            std::printf("request %zu: status %d (%s)\n", i, (int)st, purify_last_error());
            ++bad;
        }
    }
    purify_server_destroy(srv);
    free(arena);
    std::printf("done %zu requests, %d bad, %d misuses\n", tickets.size(), bad, g_misuses.load());
    return (bad != 0 || g_misuses.load() != 0) ? 1 : 0;
}
