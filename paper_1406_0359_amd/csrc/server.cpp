// Serving form: a persistent request loop that runs imaging solves of mixed sizes and
// visibility counts concurrently on one GPU.
//
// Requests are admitted against an HBM budget: the caller hands the server one device arena
// and every admitted solve gets a contiguous block of it (plan workspace, visibilities,
// image) from a first-fit allocator; the block returns to the arena when the result has
// reached the host.  Each of `max_active` worker slots owns a stream and runs one solve at a
// time -- plan creation (host binning, upload), then the same graph-replayed SDMM iteration
// as purify_sdmm_solve, on solver streams and events the slot creates once for all its
// solves -- so the device executes the kernels of up to `max_active` solves at once while
// new requests wait for a free slot and enough arena memory.  A waiting request
// may be overtaken by a later one that fits, at most 2 * max_active times, after which it
// is admitted first.  Results are identical to solving the request alone: the kernels are
// deterministic and no state is shared between solves.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t ALIGN = 256;
size_t round_up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

// First-fit allocator over [0, bytes) with coalescing on release.
struct Arena {
    size_t bytes = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void reset(size_t b) {
        bytes = b;
        free_.clear();
        if (b) free_[0] = b;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, next = it->first + n;
            free_.erase(it);
            if (rest) free_[next] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    int64_t ticket = 0;
    purify_plan_desc desc{};
    std::vector<double> uv;
    std::vector<unsigned char> y;
    purify_sdmm_params prm{};
    size_t ws_bytes = 0, y_bytes = 0, x_bytes = 0, block = 0, off = 0;   // block: arena bytes at `off`
    int skipped = 0;
    int state = 0;   // 0 waiting, 1 running, 2 done
    purify_status status = PURIFY_OK;
    std::string error;
    std::vector<unsigned char> x;
    purify_sdmm_info info{};
    Clock::time_point t_submit, t_start, t_done;
};

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct purify_server {
    int device = 0;
    char* arena_base = nullptr;
    Arena arena;
    int max_active = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> waiting;
    std::map<int64_t, std::shared_ptr<Request>> requests;
    std::vector<std::thread> workers;
    bool stop = false;
    int64_t next_ticket = 1;
};

namespace {

// Admission, under the server lock: the oldest waiting request that fits in the arena,
// unless an older one has already been overtaken 2 * max_active times (then only it).
std::shared_ptr<Request> admit(purify_server* S) {
    for (size_t i = 0; i < S->waiting.size(); ++i) {
        const std::shared_ptr<Request>& r = S->waiting[i];
        size_t off = 0;
        if (S->arena.alloc(r->block, &off)) {
            std::shared_ptr<Request> got = r;
            for (size_t k = 0; k < i; ++k) ++S->waiting[k]->skipped;
            S->waiting.erase(S->waiting.begin() + (std::ptrdiff_t)i);
            got->off = off;
            got->state = 1;
            got->t_start = Clock::now();
            return got;
        }
        if (r->skipped >= 2 * S->max_active) break;
    }
    return nullptr;
}

void run_request(purify_server* S, Request& r, size_t off, hipStream_t st, purify::SolverStreams& slot) {
    char* blk = S->arena_base + off;
    void* ws = blk;
    void* ydev = blk + round_up(r.ws_bytes);
    void* xdev = (char*)ydev + round_up(r.y_bytes);
    r.x.assign(r.x_bytes, 0);
    purify_plan* plan = nullptr;
    hipError_t e = hipMemcpyAsync(ydev, r.y.data(), r.y_bytes, hipMemcpyHostToDevice, st);
    // the image starts at zero: a solve that stops before writing it (a zero or non-finite
    // operator norm) then returns zeros, not a previous request's memory
    if (e == hipSuccess) e = hipMemsetAsync(xdev, 0, r.x_bytes, st);
    if (e != hipSuccess) {
        r.status = PURIFY_E_DEVICE;
        r.error = std::string("visibility upload: ") + hipGetErrorString(e);
        return;
    }
    purify_plan_desc d = r.desc;
    d.uv = r.uv.data();
    r.status = purify_plan_create(&d, ws, r.ws_bytes, st, &plan);
    if (r.status == PURIFY_OK) {
        plan->P.ss = &slot;   // the slot's streams and events, created once for all its solves
        r.status = purify_sdmm_solve(plan, ydev, &r.prm, xdev, &r.info, st);
    }
    if (r.status != PURIFY_OK) r.error = purify_last_error();
    if (r.status == PURIFY_OK || r.status == PURIFY_E_NONFINITE) {
        e = hipMemcpyAsync(r.x.data(), xdev, r.x_bytes, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            r.status = PURIFY_E_DEVICE;
            r.error = std::string("result download: ") + hipGetErrorString(e);
        }
    } else {
        (void)hipStreamSynchronize(st);
    }
    purify_plan_destroy(plan);
}

void worker_main(purify_server* S) {
    (void)hipSetDevice(S->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    purify::SolverStreams slot;
    if (st && purify::solver_streams_init(slot) != PURIFY_OK) {
        (void)hipStreamDestroy(st);
        st = nullptr;
    }
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                r = admit(S);
                if (r || (S->stop && S->waiting.empty())) break;
                S->cv_work.wait(lk);
            }
        }
        if (!r) break;
        const size_t off = r->off;
        if (st) run_request(S, *r, off, st, slot);
        else {
            r->status = PURIFY_E_DEVICE;
            r->error = "worker stream creation failed";
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena.release(off, r->block);
            r->state = 2;
            r->t_done = Clock::now();
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
    purify::solver_streams_release(slot);
    if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
}

}  // namespace

extern "C" {

purify_status purify_server_create(const purify_server_desc* desc, purify_server** out) {
    if (!out || !desc) {
        purify::set_error("null argument");
        return PURIFY_E_INVALID;
    }
    *out = nullptr;
    if (!desc->arena || desc->arena_bytes < ALIGN || (reinterpret_cast<uintptr_t>(desc->arena) & (ALIGN - 1)) ||
        desc->max_active < 1 || desc->max_active > 64) {
        purify::set_error("server needs a 256-byte aligned arena and 1 <= max_active <= 64");
        return PURIFY_E_INVALID;
    }
    purify_server* S = new (std::nothrow) purify_server();
    if (!S) {
        purify::set_error("host allocation failed");
        return PURIFY_E_INVALID;
    }
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        purify::set_error("no current HIP device");
        return PURIFY_E_DEVICE;
    }
    S->arena_base = (char*)desc->arena;
    S->arena.reset(desc->arena_bytes / ALIGN * ALIGN);
    S->max_active = desc->max_active;
    try {
        for (int i = 0; i < S->max_active; ++i) S->workers.emplace_back(worker_main, S);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        for (auto& t : S->workers) t.join();
        delete S;
        purify::set_error("could not start worker threads");
        return PURIFY_E_INVALID;
    }
    *out = S;
    return PURIFY_OK;
}

purify_status purify_server_submit(purify_server* server, const purify_plan_desc* desc, const void* y,
                                   const purify_sdmm_params* params, int64_t* ticket) {
    if (!server || !desc || !y || !params || !ticket) {
        purify::set_error("null argument");
        return PURIFY_E_INVALID;
    }
    const size_t ws = purify_plan_workspace_bytes(desc);
    if (ws == 0) return PURIFY_E_INVALID;   // error string set by the descriptor check
    if (!desc->uv) {
        purify::set_error("null uv");
        return PURIFY_E_INVALID;
    }
    if (params->max_iter < 1 || params->cg_iter < 1 || !(params->epsilon >= 0) ||
        (params->nu <= 0 && params->nu_iter < 1) || params->history || params->weights || params->nblocks > 1) {
        purify::set_error("invalid SDMM parameters for a served solve (history, weights and blocks are not served)");
        return PURIFY_E_INVALID;
    }
    auto r = std::make_shared<Request>();
    const size_t es = desc->precision == PURIFY_FP64 ? 16 : 8;
    r->desc = *desc;
    r->uv.assign(desc->uv, desc->uv + 2 * desc->M);
    r->desc.uv = nullptr;
    r->y_bytes = (size_t)desc->M * es;
    r->x_bytes = (size_t)desc->n * desc->n * es;
    r->y.assign((const unsigned char*)y, (const unsigned char*)y + r->y_bytes);
    r->prm = *params;
    r->ws_bytes = ws;
    r->block = round_up(ws) + round_up(r->y_bytes) + round_up(r->x_bytes);
    {
        std::lock_guard<std::mutex> lk(server->mu);
        if (r->block > server->arena.bytes) {
            purify::set_error("request needs " + std::to_string(r->block) + " bytes, more than the arena");
            return PURIFY_E_WORKSPACE;
        }
        if (server->stop) {
            purify::set_error("server is shutting down");
            return PURIFY_E_INVALID;
        }
        r->ticket = server->next_ticket++;
        r->t_submit = Clock::now();
        server->requests[r->ticket] = r;
        server->waiting.push_back(r);
        *ticket = r->ticket;
    }
    server->cv_work.notify_one();
    return PURIFY_OK;
}

int32_t purify_server_poll(purify_server* server, int64_t ticket) {
    if (!server) return -1;
    std::lock_guard<std::mutex> lk(server->mu);
    auto it = server->requests.find(ticket);
    return it == server->requests.end() ? -1 : it->second->state;
}

purify_status purify_server_wait(purify_server* server, int64_t ticket, void* x, purify_sdmm_info* info,
                                 double* timings) {
    if (!server) {
        purify::set_error("null server");
        return PURIFY_E_INVALID;
    }
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(server->mu);
        auto it = server->requests.find(ticket);
        if (it == server->requests.end()) {
            purify::set_error("unknown ticket (already collected?)");
            return PURIFY_E_INVALID;
        }
        r = it->second;
        server->cv_done.wait(lk, [&] { return r->state == 2; });
        // by key: another thread waiting on the same ticket may have collected it meanwhile
        if (server->requests.erase(ticket) == 0) {
            purify::set_error("ticket collected by another waiter");
            return PURIFY_E_INVALID;
        }
    }
    if (x && r->x.size() == r->x_bytes) std::memcpy(x, r->x.data(), r->x_bytes);
    if (info) *info = r->info;
    if (timings) {
        timings[0] = ms_between(r->t_submit, r->t_start);
        timings[1] = ms_between(r->t_start, r->t_done);
        timings[2] = ms_between(r->t_submit, r->t_done);
    }
    if (r->status != PURIFY_OK) purify::set_error(r->error);
    return r->status;
}

void purify_server_destroy(purify_server* server) {
    if (!server) return;
    {
        std::lock_guard<std::mutex> lk(server->mu);
        server->stop = true;
    }
    server->cv_work.notify_all();
    for (auto& t : server->workers) t.join();
    delete server;
}

}  // extern "C"
