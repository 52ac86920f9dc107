// Many graphs on one device: the batch driver (grass_sparsify_batch) and the
// serving loop (grass_server_*). Both run the per-graph method of Sec. IV-D
// unchanged; what they add is concurrency. Each host worker owns a HIP stream
// (default priority) and a slice of device memory, so several graphs' kernels
// are in flight together and the latency-bound phases of small graphs (single
// workgroup steps, host reads between passes) overlap with other graphs' work.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "driver.h"
#include "state.h"

namespace grass {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

const grass_opts &opts_of(const grass_opts *opts, int32_t opts_count, int i) {
    return opts[opts_count == 1 ? 0 : i];
}

// per-worker profiler merged into the context's when timing is on
void merge_profile(Profiler &into, Profiler &from, std::mutex &mu) {
    from.resolve();
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < PK_COUNT; i++) {
        into.ms[i] += from.ms[i];
        into.launches[i] += from.launches[i];
        into.bytes[i] += from.bytes[i];
    }
}

// First-fit allocator over one device arena (offsets; neighbours coalesce on free).
class ArenaAlloc {
  public:
    explicit ArenaAlloc(size_t cap) { free_[0] = cap; }
    static constexpr size_t npos = ~size_t(0);
    size_t alloc(size_t bytes) {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                size_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return off;
            }
        }
        return npos;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes);
        auto it = free_.emplace(off, bytes).first;
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

  private:
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    grass_graph g{};
    grass_opts o{};
    grass_result res{};
    size_t need = 0, off = 0;
    int state = GRASS_REQ_QUEUED;
    grass_status status = GRASS_OK;
    double t_submit = 0, t_start = 0, t_end = 0;
    int bypassed = 0;
    std::string err;
};

}  // namespace
}  // namespace grass

struct grass_server {
    grass_ctx *ctx = nullptr;
    int device = 0;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    grass::ArenaAlloc *alloc = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, grass::Request> reqs;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    bool stop = false;
    int64_t next_id = 0;
    int nworkers = 1;
    std::chrono::steady_clock::time_point t0;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    // Admission (mutex held): the first queued request, in arrival order, whose
    // workspace fits the arena; a head request passed over 2 x workers times
    // blocks everything behind it until it fits.
    grass::Request *pick() {
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            grass::Request &r = reqs[*it];
            if (it != queue.begin() && reqs[queue.front()].bypassed >= 2 * nworkers) break;
            size_t off = alloc->alloc(r.need);
            if (off == grass::ArenaAlloc::npos) continue;
            if (it != queue.begin()) reqs[queue.front()].bypassed++;
            r.off = off;
            queue.erase(it);
            return &r;
        }
        return nullptr;
    }

    void worker(int w) {
        (void)hipSetDevice(device);
        grass::g_prof = nullptr;
        grass::LaunchSched sched;
        sched.mode = ctx->launch_mode;
        sched.chunks = ctx->launch_chunks;
        sched.tuner = &ctx->tuner;
        sched.stats = &ctx->lstats;
        grass::g_sched = &sched;
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            grass::Request *r = nullptr;
            cv_work.wait(lk, [&] { return stop || (r = pick()) != nullptr; });
            if (!r) break;
            r->state = GRASS_REQ_RUNNING;
            r->t_start = now();
            lk.unlock();
            grass_status st;
            std::string err;
            try {
                st = grass::sparsify_run(ctx, r->g, r->o, arena + r->off, r->need, &r->res, streams[w]);
            } catch (const grass::Error &e) {
                st = e.code;
                err = e.what();
            } catch (const std::exception &e) {
                st = GRASS_ERR_DEVICE;
                err = e.what();
            }
            lk.lock();
            alloc->release(r->off, r->need);
            r->status = st;
            r->err = err;
            r->t_end = now();
            r->state = GRASS_REQ_DONE;
            cv_done.notify_all();
            cv_work.notify_all();
        }
        grass::g_sched = nullptr;
    }
};

using namespace grass;

extern "C" {

size_t grass_batch_workspace_bytes(int32_t count, const grass_graph *graphs, const grass_opts *opts,
                                   int32_t opts_count, int32_t workers) {
    if (count < 1 || !graphs || !opts || opts_count < 1 || workers < 1) return 0;
    size_t slot = 0;
    for (int i = 0; i < count; i++) {
        const grass_opts &o = opts_of(opts, opts_count, i);
        if (graphs[i].n < 2 || graphs[i].m < 1 || o.k < 1 || o.k > kMaxK) return 0;
        slot = std::max(slot, align_up(sparsify_bytes(graphs[i], o)));
    }
    return slot * (size_t)std::min(count, workers);
}

grass_status grass_sparsify_batch(grass_ctx *ctx, int32_t count, const grass_graph *graphs, const grass_opts *opts,
                                  int32_t opts_count, int32_t workers, void *workspace, size_t ws_bytes,
                                  grass_result *results, grass_status *statuses, void *stream) {
    if (!ctx) return GRASS_ERR_INVALID;
    try {
        require(count >= 1 && graphs && opts && results && statuses && workspace, GRASS_ERR_INVALID,
                "batch needs count >= 1, graphs, opts, results, statuses and a workspace");
        require(opts_count == 1 || opts_count == count, GRASS_ERR_INVALID, "opts_count must be 1 or count");
        require(workers >= 1, GRASS_ERR_INVALID, "workers must be >= 1");
        for (int i = 0; i < count; i++) {
            check_graph_args(&graphs[i]);
            check_opts_args(opts_of(opts, opts_count, i));
        }
        const int W = std::min(count, workers);
        size_t slot = 0;
        for (int i = 0; i < count; i++) slot = std::max(slot, align_up(sparsify_bytes(graphs[i], opts_of(opts, opts_count, i))));
        require(ws_bytes >= slot * (size_t)W, GRASS_ERR_OOM,
                "batch workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(slot * W));
        GR_HIP(hipSetDevice(ctx->device));
        // larger graphs first (they bound the batch's makespan)
        std::vector<int> order(count);
        for (int i = 0; i < count; i++) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return graphs[a].n + graphs[a].m > graphs[b].n + graphs[b].m;
        });
        hipStream_t caller = static_cast<hipStream_t>(stream);
        std::vector<hipStream_t> streams(W);
        std::vector<hipEvent_t> done(W);
        hipEvent_t fork;
        GR_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        GR_HIP(hipEventRecord(fork, caller));
        for (int w = 0; w < W; w++) {
            GR_HIP(hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking));
            GR_HIP(hipEventCreateWithFlags(&done[w], hipEventDisableTiming));
            GR_HIP(hipStreamWaitEvent(streams[w], fork, 0));
        }
        std::atomic<int> next{0};
        std::mutex mu;
        std::string first_err;
        const bool prof_on = ctx->prof.on;
        const uint32_t prof_mask = ctx->prof.mask;
        std::vector<std::thread> threads;
        for (int w = 0; w < W; w++) {
            threads.emplace_back([&, w] {
                (void)hipSetDevice(ctx->device);
                Profiler local;
                local.on = prof_on;
                local.mask = prof_mask;
                g_prof = prof_on ? &local : nullptr;
                LaunchSched sched;
                sched.mode = ctx->launch_mode;
                sched.chunks = ctx->launch_chunks;
                sched.tuner = &ctx->tuner;
                sched.stats = &ctx->lstats;
                g_sched = &sched;
                char *slice = static_cast<char *>(workspace) + slot * (size_t)w;
                for (int i; (i = next.fetch_add(1)) < count;) {
                    const int idx = order[i];
                    grass_status st;
                    try {
                        st = sparsify_run(ctx, graphs[idx], opts_of(opts, opts_count, idx), slice, slot,
                                          &results[idx], streams[w]);
                    } catch (const Error &e) {
                        st = e.code;
                        std::lock_guard<std::mutex> lk(mu);
                        if (first_err.empty()) first_err = "graph " + std::to_string(idx) + ": " + e.what();
                    } catch (const std::exception &e) {
                        st = GRASS_ERR_DEVICE;
                        std::lock_guard<std::mutex> lk(mu);
                        if (first_err.empty()) first_err = "graph " + std::to_string(idx) + ": " + e.what();
                    }
                    statuses[idx] = st;
                }
                if (prof_on) merge_profile(ctx->prof, local, mu);
                g_prof = nullptr;
                g_sched = nullptr;
            });
        }
        for (auto &th : threads) th.join();
        for (int w = 0; w < W; w++) {
            GR_HIP(hipEventRecord(done[w], streams[w]));
            GR_HIP(hipStreamWaitEvent(caller, done[w], 0));
        }
        GR_HIP(hipStreamSynchronize(caller));
        for (int w = 0; w < W; w++) {
            GR_HIP(hipEventDestroy(done[w]));
            GR_HIP(hipStreamDestroy(streams[w]));
        }
        GR_HIP(hipEventDestroy(fork));
        grass_status worst = GRASS_OK;
        for (int i = 0; i < count; i++) {
            if (statuses[i] < 0) {
                worst = statuses[i];
                break;
            }
            if (statuses[i] == GRASS_NOT_CONVERGED) worst = GRASS_NOT_CONVERGED;
        }
        ctx->last_error = first_err;
        return worst;
    } catch (const Error &e) {
        ctx->last_error = e.what();
        return e.code;
    } catch (const std::exception &e) {
        ctx->last_error = e.what();
        return GRASS_ERR_DEVICE;
    }
}

grass_status grass_server_create(grass_ctx *ctx, size_t arena_bytes, int32_t workers, grass_server **out) {
    if (!ctx || !out || arena_bytes < kAlign || workers < 1 || workers > 64) return GRASS_ERR_INVALID;
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return GRASS_ERR_DEVICE;
    auto *srv = new grass_server();
    srv->ctx = ctx;
    srv->device = ctx->device;
    srv->arena_bytes = arena_bytes / kAlign * kAlign;
    srv->nworkers = workers;
    if (hipMalloc(&srv->arena, srv->arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete srv;
        ctx->last_error = "server arena allocation of " + std::to_string(arena_bytes) + " bytes failed";
        return GRASS_ERR_OOM;
    }
    srv->alloc = new ArenaAlloc(srv->arena_bytes);
    srv->streams.resize(workers);
    for (int w = 0; w < workers; w++) {
        if (hipStreamCreateWithFlags(&srv->streams[w], hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            for (int q = 0; q < w; q++) (void)hipStreamDestroy(srv->streams[q]);
            (void)hipFree(srv->arena);
            delete srv->alloc;
            delete srv;
            return GRASS_ERR_DEVICE;
        }
    }
    srv->t0 = std::chrono::steady_clock::now();
    for (int w = 0; w < workers; w++) srv->workers.emplace_back([srv, w] { srv->worker(w); });
    *out = srv;
    return GRASS_OK;
}

grass_status grass_server_submit(grass_server *srv, const grass_graph *g, const grass_opts *opts,
                                 grass_result *res, int64_t *ticket) {
    if (!srv || !g || !opts || !res || !ticket) return GRASS_ERR_INVALID;
    try {
        check_graph_args(g);
        check_opts_args(*opts);
    } catch (const Error &e) {
        srv->ctx->last_error = e.what();
        return e.code;
    }
    size_t need = sparsify_bytes(*g, *opts);
    if (align_up(need) > srv->arena_bytes) {
        srv->ctx->last_error = "request needs " + std::to_string(need) + " bytes, more than the server arena";
        return GRASS_ERR_OOM;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    Request &r = srv->reqs[srv->next_id];
    r.id = srv->next_id++;
    r.g = *g;
    r.o = *opts;
    r.res = *res;
    r.need = need;
    r.t_submit = srv->now();
    srv->queue.push_back(r.id);
    *ticket = r.id;
    srv->cv_work.notify_one();
    return GRASS_OK;
}

grass_status grass_server_poll(grass_server *srv, int64_t ticket, grass_req_info *info) {
    if (!srv || !info) return GRASS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return GRASS_ERR_INVALID;
    const Request &r = it->second;
    info->state = r.state;
    info->status = r.status;
    info->t_submit = r.t_submit;
    info->t_start = r.t_start;
    info->t_end = r.t_end;
    info->footprint = r.need;
    return GRASS_OK;
}

grass_status grass_server_wait(grass_server *srv, int64_t ticket) {
    if (!srv) return GRASS_ERR_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (ticket >= 0) {
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) return GRASS_ERR_INVALID;
        Request &r = it->second;
        srv->cv_done.wait(lk, [&] { return r.state == GRASS_REQ_DONE || r.state == GRASS_REQ_CANCELLED; });
        return GRASS_OK;
    }
    srv->cv_done.wait(lk, [&] {
        for (auto &kv : srv->reqs)
            if (kv.second.state == GRASS_REQ_QUEUED || kv.second.state == GRASS_REQ_RUNNING) return false;
        return true;
    });
    return GRASS_OK;
}

grass_status grass_server_cancel(grass_server *srv, int64_t ticket) {
    if (!srv) return GRASS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second.state != GRASS_REQ_QUEUED) return GRASS_ERR_INVALID;
    srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), ticket));
    it->second.state = GRASS_REQ_CANCELLED;
    it->second.status = GRASS_ERR_CANCELLED;
    srv->cv_done.notify_all();
    return GRASS_OK;
}

const char *grass_server_error(grass_server *srv, int64_t ticket) {
    if (!srv) return "no server";
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    return it == srv->reqs.end() ? "no such request" : it->second.err.c_str();
}

void grass_server_destroy(grass_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (int64_t id : srv->queue) {
            srv->reqs[id].state = GRASS_REQ_CANCELLED;
            srv->reqs[id].status = GRASS_ERR_CANCELLED;
        }
        srv->queue.clear();
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    for (auto &th : srv->workers) th.join();
    (void)hipSetDevice(srv->device);
    for (auto s : srv->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    (void)hipFree(srv->arena);
    delete srv->alloc;
    delete srv;
}

}  // extern "C"
