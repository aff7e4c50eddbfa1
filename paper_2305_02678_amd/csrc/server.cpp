// Serving: continuous batching of decode requests over several resident materials.
//
// A worker thread owns the device work.  Requests enter an arrival queue (now, or at a
// replayed arrival time); the worker admits them in arrival order, cuts each into tiles of at
// most `max_tile` queries and runs tiles on a pool of HIP streams, so tiles of different
// requests and materials are on the device at the same time and a request that arrives while
// others run starts as soon as a stream and memory free up.  Every tile reserves its
// staging bytes (48 per query: uv, lod, wi, wo in, rgb out; 60 with the albedo outputs) from
// the HBM budget before it is
// launched and returns them when its completion event fires.  Tiles with device buffers whose
// materials share one matrix-core kernel (same shape and output width, precision, address mode
// and frame presence) are launched together, up to 8 in one grouped launch, taken in arrival order
// (the grouped launch across resident materials: one launch instead of one per tile); a request whose tiles cannot
// all be staged waits (admission by memory footprint).  Requests with host buffers are
// staged through a device arena carved from the budget; requests with device buffers only
// reserve their bytes.  The decode kernel depends only on the material and its precision,
// never on how requests are tiled or mixed, so each result is bitwise the same alone and in
// the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "nam_internal.h"

namespace nam {
hipError_t decode_launch(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                         const float* wi, const float* wo, float* rgb, hipStream_t s);
}

using Clock = std::chrono::steady_clock;

namespace {

constexpr size_t kBytesPerQuery = 48;   // 36 in + 12 out (RGB); the albedo head adds 12 out

// Staging bytes of one query of material m: 36 in plus 4 per decoder output.
inline size_t query_bytes(const nam_material* m) { return 36 + 4 * (size_t)m->shape.NO; }
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) for staging blocks.
class Arena {
public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
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
    uint64_t ticket = 0;
    int material = 0;
    int64_t n = 0;
    const float *uv = nullptr, *lod = nullptr, *wi = nullptr, *wo = nullptr;
    float* rgb = nullptr;
    bool host_io = false;
    Clock::time_point arrival;
    Clock::time_point completion;
    int64_t next = 0;        // first query not yet launched
    int64_t finished = 0;    // queries whose tiles completed
    int state = 0;           // 0 queued, 1 running, 2 done, 3 failed, 4 cancelled
    nam_status error = NAM_OK;
};

struct Tile {
    Request* r = nullptr;
    int64_t off = 0, cnt = 0;
    size_t bytes = 0;
    size_t arena_off = 0;
    bool staged = false;
    int stream = 0;
    hipEvent_t done = nullptr;
};

}  // namespace

struct nam_server {
    nam_ctx* ctx = nullptr;
    size_t budget = 0;
    int64_t max_tile = 0;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_busy;
    std::vector<hipEvent_t> events;               // one per stream
    std::vector<nam_material*> materials;
    void* arena_mem = nullptr;
    Arena* arena = nullptr;
    size_t reserved = 0;                          // bytes held by tiles on the device
    size_t peak_reserved = 0;
    int max_group = 8;                            // tiles per grouped launch (1: one per launch)
    int64_t launches = 0, tiles = 0;              // since the last reset
    int64_t peak_requests_on_device = 0;          // distinct requests with tiles on the device at once
    int64_t peak_launches_on_device = 0;          // launches on the device at once (streams busy)

    std::mutex mu;
    std::condition_variable cv;                   // wakes the worker
    std::condition_variable done_cv;              // wakes waiters
    std::multimap<Clock::time_point, Request*> arrivals;   // not yet arrived (replayed)
    std::deque<Request*> pending;                 // arrived, not fully launched, arrival order
    std::map<uint64_t, Request*> requests;        // every live request
    std::vector<Tile> inflight;
    uint64_t next_ticket = 1;
    bool stop = false;
    nam_status fatal = NAM_OK;

    // statistics since the last reset; replayed arrival times count from `epoch`
    Clock::time_point epoch;
    std::vector<double> latencies;
    int64_t done_queries = 0;
    bool have_first = false;
    Clock::time_point first_arrival, last_completion;

    std::thread worker;
};

namespace {

// After a launch: how many distinct requests and launches are on the device now.
void note_on_device(nam_server* s) {
    std::vector<const Request*> rs;
    for (const Tile& t : s->inflight)
        if (std::find(rs.begin(), rs.end(), t.r) == rs.end()) rs.push_back(t.r);
    int64_t busy = 0;
    for (int b : s->stream_busy) busy += b > 0 ? 1 : 0;
    s->peak_requests_on_device = std::max<int64_t>(s->peak_requests_on_device, (int64_t)rs.size());
    s->peak_launches_on_device = std::max<int64_t>(s->peak_launches_on_device, busy);
}

bool launch_tile(nam_server* s, Request* r, int si, int64_t cnt, Tile* t) {
    const nam_material* m = s->materials[r->material];
    const int NO = m->shape.NO;
    const size_t bytes = (size_t)cnt * query_bytes(m);
    if (s->reserved + bytes > s->budget) return false;
    t->r = r;
    t->off = r->next;
    t->cnt = cnt;
    t->bytes = bytes;
    t->stream = si;
    t->staged = r->host_io;
    if (r->host_io && !s->arena->alloc(bytes, &t->arena_off)) return false;
    hipStream_t st = s->streams[si];
    hipError_t e = hipSuccess;
    const int64_t o = t->off;
    if (r->host_io) {
        char* base = static_cast<char*>(s->arena_mem) + t->arena_off;
        float* uv = reinterpret_cast<float*>(base);
        float* lod = uv + 2 * cnt;
        float* wi = lod + cnt;
        float* wo = wi + 3 * cnt;
        float* rgb = wo + 3 * cnt;
        if (e == hipSuccess) e = hipMemcpyAsync(uv, r->uv + 2 * o, 8 * cnt, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(lod, r->lod + o, 4 * cnt, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(wi, r->wi + 3 * o, 12 * cnt, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(wo, r->wo + 3 * o, 12 * cnt, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = nam::decode_launch(m, cnt, uv, lod, nullptr, wi, wo, rgb, st);
        if (e == hipSuccess) e = hipMemcpyAsync(r->rgb + NO * o, rgb, 4 * NO * cnt, hipMemcpyDeviceToHost, st);
    } else {
        e = nam::decode_launch(m, cnt, r->uv + 2 * o, r->lod + o, nullptr, r->wi + 3 * o, r->wo + 3 * o, r->rgb + NO * o,
                                  st);
    }
    t->done = s->events[si];
    if (e == hipSuccess) e = hipEventRecord(t->done, st);
    if (e != hipSuccess) {
        if (r->host_io) s->arena->release(t->arena_off, bytes);
        r->state = 3;
        r->error = NAM_E_HIP;
        return false;
    }
    s->reserved += bytes;
    s->peak_reserved = std::max(s->peak_reserved, s->reserved);
    s->stream_busy[si] = 1;
    s->launches += 1;
    s->tiles += 1;
    r->next += cnt;
    r->state = 1;
    return true;
}

// Tiles from the front of the pending queue, in arrival order, whose buffers are on the device
// and whose materials share the front request's matrix-core kernel, as many as the budget and
// max_group allow, launched as one grouped kernel on stream si.  Returns the number of tiles
// launched (0: the first does not fit the budget).
int launch_group(nam_server* s, int si) {
    constexpr int kG = 8;
    const nam_material* m0 = s->materials[s->pending.front()->material];
    const nam_material* mats[kG];
    int64_t ns[kG];
    const float *uvs[kG], *lods[kG], *wis[kG], *wos[kG];
    float* rgbs[kG];
    Tile tiles[kG];
    int count = 0;
    size_t total = 0;
    const int limit = std::min(kG, s->max_group);
    for (size_t k = 0; k < s->pending.size() && count < limit; ++k) {
        Request* r = s->pending[k];
        if (r->state >= 2 || r->next >= r->n) continue;
        const nam_material* m = s->materials[r->material];
        if (r->host_io || !nam::mfma_same_kernel(m0, m)) break;
        int64_t next = r->next;
        for (int j = 0; j < count; ++j)
            if (tiles[j].r == r) next = std::max(next, tiles[j].off + tiles[j].cnt);
        bool full = false;
        while (next < r->n && count < limit) {
            const int64_t cnt = std::min<int64_t>(std::min<int64_t>(s->max_tile, (int64_t(1) << 30) - 1), r->n - next);
            const size_t bytes = (size_t)cnt * query_bytes(m);
            if (s->reserved + total + bytes > s->budget) {
                full = true;
                break;
            }
            Tile& t = tiles[count];
            t = Tile{};
            t.r = r;
            t.off = next;
            t.cnt = cnt;
            t.bytes = bytes;
            t.stream = si;
            mats[count] = m;
            ns[count] = cnt;
            uvs[count] = r->uv + 2 * next;
            lods[count] = r->lod + next;
            wis[count] = r->wi + 3 * next;
            wos[count] = r->wo + 3 * next;
            rgbs[count] = r->rgb + (int64_t)m->shape.NO * next;
            total += bytes;
            next += cnt;
            ++count;
        }
        if (full || next < r->n) break;          // later requests wait their turn
    }
    if (count == 0) return 0;
    hipStream_t st = s->streams[si];
    hipError_t e = nam::launch_decode_mfma_group(count, mats, ns, uvs, lods, wis, wos, rgbs, st);
    if (e == hipSuccess) e = hipEventRecord(s->events[si], st);
    if (e != hipSuccess) {
        for (int j = 0; j < count; ++j) {
            tiles[j].r->state = 3;
            tiles[j].r->error = NAM_E_HIP;
        }
        return -1;
    }
    for (int j = 0; j < count; ++j) {
        tiles[j].done = s->events[si];
        tiles[j].r->next = tiles[j].off + tiles[j].cnt;
        tiles[j].r->state = 1;
        s->inflight.push_back(tiles[j]);
    }
    s->reserved += total;
    s->peak_reserved = std::max(s->peak_reserved, s->reserved);
    s->stream_busy[si] = count;
    s->launches += 1;
    s->tiles += count;
    note_on_device(s);
    return count;
}

void finish_request(nam_server* s, Request* r, Clock::time_point now) {
    r->state = 2;
    r->completion = now;
    s->latencies.push_back(std::chrono::duration<double>(now - r->arrival).count());
    s->done_queries += r->n;
    if (!s->have_first || r->arrival < s->first_arrival) s->first_arrival = r->arrival;
    if (!s->have_first || now > s->last_completion) s->last_completion = now;
    s->have_first = true;
}

void worker_loop(nam_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        const Clock::time_point now = Clock::now();
        // arrivals whose time has come
        while (!s->arrivals.empty() && s->arrivals.begin()->first <= now) {
            s->pending.push_back(s->arrivals.begin()->second);
            s->arrivals.erase(s->arrivals.begin());
        }
        // retire completed tiles
        bool progressed = false;
        for (size_t i = 0; i < s->inflight.size();) {
            Tile& t = s->inflight[i];
            const hipError_t q = hipEventQuery(t.done);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            Request* r = t.r;
            if (q != hipSuccess) {
                r->state = 3;
                r->error = NAM_E_HIP;
            }
            if (t.staged) s->arena->release(t.arena_off, t.bytes);
            s->reserved -= t.bytes;
            s->stream_busy[t.stream] -= 1;
            r->finished += t.cnt;
            if (r->finished == r->n && r->state == 1) finish_request(s, r, Clock::now());
            if (r->state >= 2) s->done_cv.notify_all();
            s->inflight[i] = s->inflight.back();
            s->inflight.pop_back();
            progressed = true;
        }
        // launch tiles on free streams, oldest request first; a request blocked by the
        // budget blocks the ones behind it (arrival-order admission)
        for (int si = 0; si < (int)s->streams.size(); ++si) {
            if (s->stream_busy[si]) continue;
            while (!s->pending.empty() && (s->pending.front()->state >= 2 || s->pending.front()->next >= s->pending.front()->n))
                s->pending.pop_front();
            if (s->pending.empty()) break;
            Request* r = s->pending.front();
            if (!r->host_io && s->max_group > 1 && s->materials[r->material]->wprec != NAM_F32) {
                const int got = launch_group(s, si);
                if (got < 0) {
                    while (!s->pending.empty() && s->pending.front()->state == 3) s->pending.pop_front();
                    s->done_cv.notify_all();
                    progressed = true;
                    continue;
                }
                if (got == 0) break;   // waits for memory
                progressed = true;
                continue;
            }
            const int64_t cnt = std::min<int64_t>(s->max_tile, r->n - r->next);
            Tile t;
            if (!launch_tile(s, r, si, cnt, &t)) {
                if (r->state == 3) {
                    s->pending.pop_front();
                    s->done_cv.notify_all();
                    continue;
                }
                break;   // waits for memory
            }
            s->inflight.push_back(t);
            note_on_device(s);
            progressed = true;
            if (r->next >= r->n) s->pending.pop_front();
        }
        if (s->stop && s->inflight.empty() && s->pending.empty() && s->arrivals.empty()) break;
        if (!progressed) {
            // nothing changed: sleep until a submission, the next replayed arrival, or a
            // short poll interval for the events in flight
            auto until = Clock::now() + std::chrono::microseconds(s->inflight.empty() ? 2000 : 20);
            if (!s->arrivals.empty()) until = std::min(until, s->arrivals.begin()->first);
            if (s->inflight.empty()) s->cv.wait_until(lk, until);
            else {
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        }
    }
}

nam_status submit(nam_server* s, int material_id, int64_t n, const float* uv, const float* lod, const float* wi,
                  const float* wo, float* rgb, int host_io, double arrival_s, uint64_t* ticket) {
    if (!s || !ticket) return nam::set_error(NAM_E_INVALID_ARG, "NULL argument");
    if (n < 0) return nam::set_error(NAM_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!uv || !lod || !wi || !wo || !rgb)) return nam::set_error(NAM_E_INVALID_ARG, "query pointer is NULL");
    if (!(arrival_s == arrival_s)) return nam::set_error(NAM_E_INVALID_ARG, "arrival time is NaN");
    std::lock_guard<std::mutex> g(s->mu);
    if (material_id < 0 || material_id >= (int)s->materials.size())
        return nam::set_error(NAM_E_INVALID_ARG, "unknown material id");
    Request* r = new (std::nothrow) Request();
    if (!r) return nam::set_error(NAM_E_OOM, "host allocation failed");
    r->ticket = s->next_ticket++;
    r->material = material_id;
    r->n = n;
    r->uv = uv;
    r->lod = lod;
    r->wi = wi;
    r->wo = wo;
    r->rgb = rgb;
    r->host_io = host_io != 0;
    const Clock::time_point now = Clock::now();
    r->arrival = arrival_s < 0 ? now
                               : s->epoch + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s));
    s->requests[r->ticket] = r;
    *ticket = r->ticket;
    if (n == 0) {
        finish_request(s, r, r->arrival);
        return NAM_OK;
    }
    s->arrivals.emplace(r->arrival, r);     // released to the worker in arrival order
    s->cv.notify_one();
    return NAM_OK;
}

}  // namespace

using namespace nam;

extern "C" {

nam_status nam_server_create(nam_ctx* ctx, size_t hbm_budget_bytes, int n_streams, int64_t max_tile,
                             nam_server** out) {
    if (!ctx || !out) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (n_streams < 1 || n_streams > 16) return set_error(NAM_E_INVALID_ARG, "n_streams must be in [1, 16]");
    if (max_tile < 256) return set_error(NAM_E_INVALID_ARG, "max_tile must be >= 256 queries");
    if (hbm_budget_bytes < (size_t)max_tile * kBytesPerQuery)
        return set_error(NAM_E_BUDGET, "the budget must hold at least one tile of max_tile queries");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(NAM_E_HIP, "hipSetDevice failed");
    nam_server* s = new (std::nothrow) nam_server();
    if (!s) return set_error(NAM_E_OOM, "host allocation failed");
    s->ctx = ctx;
    s->budget = hbm_budget_bytes;
    s->max_tile = max_tile;
    hipError_t e = hipMalloc(&s->arena_mem, hbm_budget_bytes);
    if (e != hipSuccess) {
        delete s;
        return hip_error(e, "hipMalloc(serving arena)");
    }
    s->arena = new Arena(hbm_budget_bytes);
    for (int i = 0; i < n_streams; ++i) {
        hipStream_t st;
        hipEvent_t ev;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            for (auto x : s->events) (void)hipEventDestroy(x);
            (void)hipFree(s->arena_mem);
            delete s->arena;
            delete s;
            return set_error(NAM_E_HIP, "stream/event creation failed");
        }
        s->streams.push_back(st);
        s->events.push_back(ev);
        s->stream_busy.push_back(0);
    }
    s->epoch = Clock::now();
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return NAM_OK;
}

nam_status nam_server_add_material(nam_server* s, nam_material* m, int* material_id) {
    if (!s || !m || !material_id) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    if (m->ctx != s->ctx) return set_error(NAM_E_INVALID_ARG, "material belongs to another context");
    if (s->budget < (size_t)s->max_tile * query_bytes(m))
        return set_error(NAM_E_BUDGET, "the budget must hold one tile of max_tile queries of this material");
    std::lock_guard<std::mutex> g(s->mu);
    m->server_refs++;
    s->materials.push_back(m);
    *material_id = (int)s->materials.size() - 1;
    return NAM_OK;
}

nam_status nam_server_submit(nam_server* s, int material_id, int64_t n, const float* uv, const float* lod,
                             const float* wi, const float* wo, float* rgb, int host_io, double arrival_s,
                             uint64_t* ticket) {
    return submit(s, material_id, n, uv, lod, wi, wo, rgb, host_io, arrival_s, ticket);
}

nam_status nam_server_poll(nam_server* s, uint64_t ticket, int* done, double* latency_s) {
    if (!s || !done) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return set_error(NAM_E_INVALID_ARG, "unknown ticket");
    Request* r = it->second;
    *done = r->state >= 2 ? 1 : 0;
    if (latency_s) *latency_s = r->state == 2 ? std::chrono::duration<double>(r->completion - r->arrival).count() : -1.0;
    if (r->state == 3) return set_error(r->error, "request failed on the device");
    if (r->state == 4) return set_error(NAM_E_INVALID_ARG, "request was cancelled");
    return NAM_OK;
}

nam_status nam_server_cancel(nam_server* s, uint64_t ticket) {
    if (!s) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return set_error(NAM_E_INVALID_ARG, "unknown ticket");
    Request* r = it->second;
    if (r->state != 0 || r->next > 0) return set_error(NAM_E_BUSY, "request already started");
    for (auto a = s->arrivals.begin(); a != s->arrivals.end(); ++a)
        if (a->second == r) { s->arrivals.erase(a); break; }
    s->pending.erase(std::remove(s->pending.begin(), s->pending.end(), r), s->pending.end());
    r->state = 4;
    s->done_cv.notify_all();
    return NAM_OK;
}

nam_status nam_server_wait_all(nam_server* s) {
    if (!s) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.notify_one();
    s->done_cv.wait(lk, [s] {
        if (!s->arrivals.empty() || !s->pending.empty() || !s->inflight.empty()) return false;
        return true;
    });
    for (auto& kv : s->requests)
        if (kv.second->state == 3) return set_error(NAM_E_HIP, "a request failed on the device");
    return NAM_OK;
}

nam_status nam_server_stats(nam_server* s, nam_server_stats_t* out) {
    if (!s || !out) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof(*out));
    std::vector<double> l = s->latencies;
    out->completed = (int64_t)l.size();
    out->queries = s->done_queries;
    out->peak_reserved_bytes = s->peak_reserved;
    out->launches = s->launches;
    out->tiles = s->tiles;
    out->peak_requests_on_device = s->peak_requests_on_device;
    out->peak_launches_on_device = s->peak_launches_on_device;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        auto pct = [&](double p) {
            const double x = p * (double)(l.size() - 1);
            const size_t i = (size_t)x;
            const double f = x - (double)i;
            return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
        };
        out->p50_s = pct(0.50);
        out->p99_s = pct(0.99);
        double sum = 0;
        for (double v : l) sum += v;
        out->mean_s = sum / (double)l.size();
        out->max_s = l.back();
        const double span = std::chrono::duration<double>(s->last_completion - s->first_arrival).count();
        out->span_s = span;
        out->queries_per_s = span > 0 ? (double)s->done_queries / span : 0.0;
    }
    return NAM_OK;
}

nam_status nam_server_reset_stats(nam_server* s) {
    if (!s) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    s->latencies.clear();
    s->epoch = Clock::now();
    s->done_queries = 0;
    s->have_first = false;
    s->peak_reserved = s->reserved;
    s->launches = 0;
    s->tiles = 0;
    s->peak_requests_on_device = 0;
    s->peak_launches_on_device = 0;
    for (auto it = s->requests.begin(); it != s->requests.end();) {
        if (it->second->state >= 2) {
            delete it->second;
            it = s->requests.erase(it);
        } else {
            ++it;
        }
    }
    return NAM_OK;
}

nam_status nam_server_set_group(nam_server* s, int max_tiles) {
    if (!s) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    if (max_tiles < 1 || max_tiles > 8) return set_error(NAM_E_INVALID_ARG, "max_tiles must be 1 to 8");
    std::lock_guard<std::mutex> g(s->mu);
    s->max_group = max_tiles;
    return NAM_OK;
}

nam_status nam_server_destroy(nam_server* s) {
    if (!s) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_one();
    }
    s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto ev : s->events) (void)hipEventDestroy(ev);
    (void)hipFree(s->arena_mem);
    delete s->arena;
    for (auto m : s->materials) m->server_refs--;
    for (auto& kv : s->requests) delete kv.second;
    delete s;
    return NAM_OK;
}

}  // extern "C"
