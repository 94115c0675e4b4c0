// Host-only harness for the serving loop and plan creation.  The HIP runtime calls that
// server.cpp and plan.cpp make are replaced by host stand-ins (device memory is host memory,
// copies are memcpy, streams are dummies), the solve is replaced by a short sleep that writes
// a value derived from the request, and everything else -- descriptor checks, workspace
// layout, visibility binning on host threads, the first-fit arena, admission and the worker
// threads -- is the library's own code.  Built under ThreadSanitizer or AddressSanitizer it
// checks that concurrent requests share no unsynchronised host state and stay within their
// buffers.
//
// usage: server_plan_stub <requests> <slots>; prints "done <k> requests, <b> bad".
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_1406_0359_amd/csrc/common.h"

hipError_t hipMemcpyAsync(void* d, const void* s, size_t b, hipMemcpyKind, hipStream_t) {
    std::memcpy(d, s, b);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t b, hipStream_t) {
    std::memset(d, v, b);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = (hipStream_t) new int(0);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete (int*)s;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "host stand-in"; }
// the solver streams of a worker slot (solver_rt.cpp): events and graphs are dummies here
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
    *e = (hipEvent_t) new int(0);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete (int*)e;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
    *g = nullptr;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t, hipGraphNode_t*, char*, size_t) {
    *x = nullptr;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

namespace purify {
thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
}  // namespace purify
using namespace purify;

extern "C" {
const char* purify_last_error(void) { return purify::g_err.c_str(); }

size_t purify_plan_workspace_bytes(const purify_plan_desc* desc) {
    const DescCheck c = check_desc(desc);
    if (!c.ok) {
        set_error(c.why);
        return 0;
    }
    Plan P;
    return layout(P, desc, nullptr);
}

purify_status purify_plan_create(const purify_plan_desc* desc, void* ws, size_t bytes, void* stream,
                                 purify_plan** out) {
    *out = nullptr;
    const DescCheck c = check_desc(desc);
    if (!c.ok) {
        set_error(c.why);
        return PURIFY_E_INVALID;
    }
    purify_plan* h = new purify_plan();
    Plan& P = h->P;
    if (bytes < layout(P, desc, nullptr)) {
        delete h;
        return PURIFY_E_WORKSPACE;
    }
    layout(P, desc, (char*)ws);
    P.ws = (char*)ws;
    P.ws_bytes = bytes;
    const purify_status st = build_plan(P, desc, (hipStream_t)stream);
    if (st != PURIFY_OK) {
        delete h;
        return st;
    }
    *out = h;
    return PURIFY_OK;
}

void purify_plan_destroy(purify_plan* p) { delete p; }

// Stand-in solve: element j of x starts with the double M + j; info.nu = M.
purify_status purify_sdmm_solve(purify_plan* plan, const void*, const purify_sdmm_params*, void* x,
                                purify_sdmm_info* info, void*) {
    const Plan& P = plan->P;
    const size_t es = P.precision == PURIFY_FP64 ? 16 : 8;
    std::this_thread::sleep_for(std::chrono::microseconds(200 + P.M % 997));
    for (int64_t j = 0; j < P.N; ++j) {
        const double v = (double)(P.M + j);
        std::memcpy((char*)x + j * es, &v, sizeof v);
    }
    info->iterations = (int32_t)(P.M % 300);
    info->nu = (double)P.M;
    return PURIFY_OK;
}
}  // extern "C"

int main(int argc, char** argv) {
    const int count = argc > 1 ? atoi(argv[1]) : 24, slots = argc > 2 ? atoi(argv[2]) : 8;
    const size_t arena_bytes = (size_t)1 << 30;
    void* arena = aligned_alloc(256, arena_bytes);
    purify_server_desc sd{};
    sd.arena = arena;
    sd.arena_bytes = arena_bytes;
    sd.max_active = slots;
    purify_server* S = nullptr;
    if (purify_server_create(&sd, &S) != PURIFY_OK) {
        printf("create failed: %s\n", purify_last_error());
        return 1;
    }
    // Mixed sizes and precisions; M/N ~ U[0.2, 2]; uv uniform over a little more than one
    // period (the plan wraps it).
    std::mt19937_64 g(7);
    const int sizes[4] = {128, 128, 256, 512};
    std::vector<int64_t> tickets, Ms;
    std::vector<int> ns, precs;
    for (int i = 0; i < count; ++i) {
        const int n = sizes[i % 4];
        std::uniform_real_distribution<double> ratio(0.2, 2.0), ang(-3.2, 3.2);
        const int64_t M = (int64_t)(ratio(g) * n * n);
        std::vector<double> uv((size_t)2 * M);
        for (double& v : uv) v = ang(g);
        const int prec = i % 3 == 0 ? PURIFY_FP64 : PURIFY_FP32;
        std::vector<unsigned char> y((size_t)M * (prec == PURIFY_FP64 ? 16 : 8), 1);
        purify_plan_desc d{};
        d.n = n;
        d.oversample = 2;
        d.J = 6;
        d.M = M;
        d.uv = uv.data();
        d.dict_mask = PURIFY_DICT_SARA;
        d.levels = 4;
        d.precision = prec;
        purify_sdmm_params p{};
        p.epsilon = 1;
        p.max_iter = 10;
        p.cg_iter = 2;
        p.check_every = 1;
        p.nu_iter = 5;
        int64_t t = 0;
        if (purify_server_submit(S, &d, y.data(), &p, &t) != PURIFY_OK) {
            printf("submit failed: %s\n", purify_last_error());
            return 1;
        }
        tickets.push_back(t);
        Ms.push_back(M);
        ns.push_back(n);
        precs.push_back(prec);
        if (i % 5 == 0) std::this_thread::sleep_for(std::chrono::microseconds(300));
    }
    int bad = 0;
    // Two threads wait on the first ticket at once: exactly one collects it, intact.
    purify_status st2[2];
    std::vector<unsigned char> x2[2];
    purify_sdmm_info info2[2];
    {
        const size_t es = precs[0] == PURIFY_FP64 ? 16 : 8;
        std::vector<std::thread> waiters;
        for (int k = 0; k < 2; ++k) {
            x2[k].assign((size_t)ns[0] * ns[0] * es, 0);
            info2[k] = purify_sdmm_info{};
            waiters.emplace_back([&, k] { st2[k] = purify_server_wait(S, tickets[0], x2[k].data(), &info2[k], nullptr); });
        }
        for (auto& w : waiters) w.join();
        const int got = st2[0] == PURIFY_OK ? 0 : 1;
        double v0 = 0;
        std::memcpy(&v0, x2[got].data(), sizeof v0);
        if (st2[got] != PURIFY_OK || st2[1 - got] != PURIFY_E_INVALID || info2[got].nu != (double)Ms[0] ||
            v0 != (double)Ms[0]) {
            printf("request 0: double wait gave %d and %d\n", (int)st2[0], (int)st2[1]);
            ++bad;
        }
    }
    for (size_t i = 1; i < tickets.size(); ++i) {
        const size_t es = precs[i] == PURIFY_FP64 ? 16 : 8;
        std::vector<unsigned char> x((size_t)ns[i] * ns[i] * es);
        purify_sdmm_info info{};
        double tm[3];
        if (purify_server_wait(S, tickets[i], x.data(), &info, tm) != PURIFY_OK) {
            printf("wait failed on request %zu: %s\n", i, purify_last_error());
            ++bad;
            continue;
        }
        double v0 = 0, vl = 0;
        std::memcpy(&v0, x.data(), sizeof v0);
        std::memcpy(&vl, x.data() + x.size() - es, sizeof vl);
        if (info.nu != (double)Ms[i] || v0 != (double)Ms[i] || vl != (double)(Ms[i] + ns[i] * ns[i] - 1)) {
            printf("request %zu: wrong result\n", i);
            ++bad;
        }
    }
    purify_server_destroy(S);
    free(arena);
    printf("done %zu requests, %d bad\n", tickets.size(), bad);
    return bad != 0;
}
