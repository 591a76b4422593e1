// Serving runtime: continuous batching of timeslices on one GPU
// (include/trig_serve.h).  Admission logic lives in serve_core.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "serve_core.hpp"
#include "trig.h"
#include "trig_serve.h"

namespace {

using trig::serve::Admission;
using trig::serve::Arena;

constexpr size_t kAlign = 256;

size_t r256(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// Byte layout of one slice, identical in pinned staging and in HBM:
// offsets | x | y | status | n_accepted | counts | accept | ids [| workspace]
// Results come back in two copies: status to accept at once, then the first
// n_accepted ids once that number is on the host.
struct Layout {
    size_t off, x, y, status, n_acc, counts, accept, ids, ws, host_bytes, dev_bytes;
    Layout(int64_t n_events, int64_t n_hits, size_t ws_bytes) {
        size_t at = 0;
        off = at; at += r256(4 * (size_t)(3 * n_events + 1));
        x = at; at += r256(4 * (size_t)n_hits);
        y = at; at += r256(4 * (size_t)n_hits);
        status = at; at += r256(4);
        n_acc = at; at += r256(4);
        counts = at; at += r256(4 * (size_t)n_events);
        accept = at; at += r256((size_t)n_events);
        ids = at; at += r256(4 * (size_t)(n_events > 0 ? n_events : 1));
        host_bytes = at;
        ws = at; at += r256(ws_bytes);
        dev_bytes = at;
    }
};

enum class State { Queued, InFlight, Done, Polled };

// Host copies into pinned staging: large slices are split over a few threads
// (one host thread copies far below the PCIe rate).
struct CopySeg {
    char* dst;
    const char* src;
    size_t bytes;
};
constexpr size_t kCopyParallelMin = 8u << 20;  // below this, one memcpy per segment
constexpr size_t kStageChunk = 32u << 20;      // staging is published in chunks of this size
constexpr unsigned kCopyThreadsMax = 8;

void copy_segments(const CopySeg* seg, int n_seg) {
    size_t total = 0;
    for (int i = 0; i < n_seg; ++i) total += seg[i].bytes;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned nt = total < kCopyParallelMin ? 1u : std::min(kCopyThreadsMax, hw);
    // Thread q copies bytes [q*total/nt, (q+1)*total/nt) of the concatenation.
    auto part = [&](unsigned q) {
        const size_t lo = total * q / nt, hi = total * (q + 1) / nt;
        size_t base = 0;
        for (int i = 0; i < n_seg; ++i) {
            const size_t a = std::max(lo, base), b = std::min(hi, base + seg[i].bytes);
            if (a < b) std::memcpy(seg[i].dst + (a - base), seg[i].src + (a - base), b - a);
            base += seg[i].bytes;
        }
    };
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (unsigned q = 1; q < nt; ++q) th.emplace_back(part, q);
    part(0);
    for (auto& t : th) t.join();
}

struct Slice {
    uint64_t ticket = 0;
    int32_t n_events = 0, n_hits = 0;
    size_t pin_off = 0, dev_off = 0, ws_bytes = 0;
    size_t staged = 0;    // bytes of the input prefix (offsets | x | y) in pinned staging
    size_t issued = 0;    // bytes of it whose copy to the device is enqueued
    bool launched = false;  // selection and result copy enqueued
    bool ids_issued = false;  // copy of the accepted ids enqueued (after the first result copy)
    int stream = -1;
    State state = State::Queued;
    int32_t status = TRIG_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct trig_server {
    trig_server_config cfg;
    char* dev_base = nullptr;
    char* pin_base = nullptr;
    Arena pin_arena;
    Admission adm;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<uint64_t> stream_ticket;  // 0 = free
    std::map<uint64_t, Slice> slices;
    std::deque<uint64_t> done;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread dispatcher;
    bool stop = false;
    bool paused = false;  // admit nothing while set
    uint64_t next_ticket = 1;
    trig_server_stats stats{};
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    trig_server(const trig_server_config& c)
        : cfg(c), pin_arena(c.pinned_budget_bytes, kAlign), adm(c.hbm_budget_bytes, c.n_streams) {}

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    size_t workspace_for(int32_t n_events) const {
        trig_params p = cfg.params;
        p.flags |= TRIG_OUT_COMPACT;
        trig_events_csr ev{n_events, nullptr};
        return trig_workspace_bytes(&ev, &p);
    }

    // An admitted slice (mu held): takes stream si; its input is copied to the
    // device as far as it is staged, the rest by progress() as submit()
    // publishes it.
    void launch(Slice& s, int si) {
        s.stream = si;
        s.state = State::InFlight;
        s.t_admit = now();
        stream_ticket[si] = s.ticket;
        ++stats.in_flight;
        if (stats.in_flight > stats.max_in_flight) stats.max_in_flight = stats.in_flight;
        if (adm.arena().in_use() > stats.hbm_peak) stats.hbm_peak = adm.arena().in_use();
        progress(s);
    }

    // Enqueues the copy of newly staged input and, once all of it is on its
    // way, the selection, the result copy and the completion event (mu held).
    void progress(Slice& s) {
        if (s.launched) return;
        const Layout L(s.n_events, s.n_hits, s.ws_bytes);
        char* d = dev_base + s.dev_off;
        char* h = pin_base + s.pin_off;
        hipStream_t st = streams[s.stream];
        const size_t total = L.status;  // offsets | x | y
        int rc = TRIG_OK;
        if (s.staged > s.issued) {
            if (hipMemcpyAsync(d + s.issued, h + s.issued, s.staged - s.issued, hipMemcpyHostToDevice, st) !=
                hipSuccess)
                rc = TRIG_EHIP;
            s.issued = s.staged;
        }
        if (rc == TRIG_OK && s.issued < total) return;  // more to come
        s.launched = true;
        if (rc == TRIG_OK &&
            hipMemcpyAsync(d + L.status, h + L.status, 4, hipMemcpyHostToDevice, st) != hipSuccess)
            rc = TRIG_EHIP;
        if (rc == TRIG_OK) {
            trig_params p = cfg.params;
            p.flags |= TRIG_OUT_COMPACT;
            p.workspace = s.ws_bytes ? d + L.ws : nullptr;
            p.workspace_bytes = s.ws_bytes;
            p.out_accepted_ids = reinterpret_cast<int32_t*>(d + L.ids);
            p.out_n_accepted = reinterpret_cast<int32_t*>(d + L.n_acc);
            p.out_status = reinterpret_cast<uint32_t*>(d + L.status);
            trig_events_csr ev{s.n_events, reinterpret_cast<const int32_t*>(d + L.off)};
            trig_hits hits{s.n_hits, reinterpret_cast<const float*>(d + L.x), reinterpret_cast<const float*>(d + L.y)};
            rc = trig_select(&ev, &hits, &p, reinterpret_cast<int32_t*>(d + L.counts),
                             reinterpret_cast<uint8_t*>(d + L.accept), st);
        }
        if (rc == TRIG_OK &&
            hipMemcpyAsync(h + L.status, d + L.status, L.ids - L.status, hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = TRIG_EHIP;
        if (rc == TRIG_OK && hipEventRecord(events[s.stream], st) != hipSuccess) rc = TRIG_EHIP;
        s.status = rc;
    }

    // After the first result copy (mu held): enqueues the copy of the
    // n_accepted ids the host now holds; returns false if there are none.
    bool issue_ids(Slice& s) {
        s.ids_issued = true;
        const Layout L(s.n_events, s.n_hits, s.ws_bytes);
        char* h = pin_base + s.pin_off;
        int32_t n = 0;
        std::memcpy(&n, h + L.n_acc, 4);
        n = std::max(0, std::min(n, s.n_events));
        if (n == 0) return false;
        hipStream_t st = streams[s.stream];
        if (hipMemcpyAsync(h + L.ids, dev_base + s.dev_off + L.ids, 4 * (size_t)n, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipEventRecord(events[s.stream], st) != hipSuccess) {
            s.status = TRIG_EHIP;
            return false;
        }
        return true;
    }

    // Marks a slice finished (mu held): frees its device memory and stream.
    void finish(Slice& s) {
        // Also after a failed launch: nothing may still use the slice's memory.
        if (hipStreamSynchronize(streams[s.stream]) != hipSuccess && s.status == TRIG_OK) s.status = TRIG_EHIP;
        s.t_done = now();
        s.state = State::Done;
        adm.complete(s.dev_off);
        stream_ticket[s.stream] = 0;
        --stats.in_flight;
        ++stats.completed;
        stats.events_completed += (uint64_t)s.n_events;
        done.push_back(s.ticket);
    }

    void run() {
        (void)hipSetDevice(cfg.device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            // Admit queued slices while a stream is free and memory fits.
            if (!stop && !paused) {
                for (int si = 0; si < (int)streams.size(); ++si) {
                    if (stream_ticket[si]) continue;
                    uint64_t t;
                    size_t off;
                    if (!adm.admit_next(t, off)) break;
                    Slice& s = slices[t];
                    s.dev_off = off;
                    --stats.pending;
                    launch(s, si);
                }
            }
            // Retire finished slices (failed launches finish at once).
            bool any = false, busy = false;
            for (int si = 0; si < (int)streams.size(); ++si) {
                const uint64_t t = stream_ticket[si];
                if (!t) continue;
                Slice& s = slices[t];
                if (!s.launched) progress(s);
                if (!s.launched) {
                    busy = true;  // waiting for submit() to stage the rest
                    continue;
                }
                if (s.status != TRIG_OK || hipEventQuery(events[si]) == hipSuccess) {
                    if (s.status == TRIG_OK && !s.ids_issued && issue_ids(s)) {
                        busy = true;  // the ids are on their way
                        continue;
                    }
                    finish(s);
                    any = true;
                } else {
                    busy = true;
                }
            }
            if (any) {
                cv_done.notify_all();
                continue;  // freed memory and streams: try to admit again
            }
            if (stop && !busy) break;
            if (busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                cv_work.wait(lk);
            }
        }
    }
};

extern "C" {

int trig_server_create(const trig_server_config* cfg, trig_server** out) {
    if (!cfg || !out) return TRIG_EINVAL;
    *out = nullptr;
    if (cfg->hbm_budget_bytes < kAlign || cfg->pinned_budget_bytes < kAlign || cfg->n_streams < 1 ||
        cfg->n_streams > 64 || cfg->max_pending < 1 || cfg->reserved != 0)
        return TRIG_EINVAL;
    {
        // The selection parameters must be acceptable to trig_select.
        trig_params p = cfg->params;
        p.flags |= TRIG_OUT_COMPACT;
        if (int rc = trig_params_check(&p)) return rc;
    }
    if (hipSetDevice(cfg->device) != hipSuccess) return TRIG_EHIP;
    auto* s = new trig_server(*cfg);
    if (hipMalloc(&s->dev_base, cfg->hbm_budget_bytes) != hipSuccess ||
        hipHostMalloc(&s->pin_base, cfg->pinned_budget_bytes, hipHostMallocDefault) != hipSuccess) {
        if (s->dev_base) (void)hipFree(s->dev_base);
        delete s;
        return TRIG_EHIP;
    }
    // Touch the whole pinned arena once (in parallel): its first CPU writes
    // are an order of magnitude slower than later ones, and would otherwise
    // land on the first slices' latency.
    {
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const unsigned nt = std::min(kCopyThreadsMax, hw);
        const size_t total = cfg->pinned_budget_bytes;
        std::vector<std::thread> th;
        for (unsigned q = 0; q < nt; ++q)
            th.emplace_back([=] {
                const size_t lo = total * q / nt, hi = total * (q + 1) / nt;
                std::memset(s->pin_base + lo, 0, hi - lo);
            });
        for (auto& t : th) t.join();
    }
    s->streams.resize(cfg->n_streams);
    s->events.resize(cfg->n_streams);
    s->stream_ticket.assign(cfg->n_streams, 0);
    for (int i = 0; i < cfg->n_streams; ++i) {
        if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) != hipSuccess) {
            for (int k = 0; k <= i; ++k) {
                if (s->streams[k]) (void)hipStreamDestroy(s->streams[k]);
                if (s->events[k]) (void)hipEventDestroy(s->events[k]);
            }
            (void)hipFree(s->dev_base);
            (void)hipHostFree(s->pin_base);
            delete s;
            return TRIG_EHIP;
        }
    }
    s->dispatcher = std::thread([s] { s->run(); });
    *out = s;
    return TRIG_OK;
}

int trig_server_submit(trig_server* s, const int32_t* offsets, const float* x, const float* y, int32_t n_events,
                       int32_t n_hits, uint64_t* ticket) {
    if (!s || !ticket || n_events < 0 || n_hits < 0 || !offsets || (n_hits > 0 && (!x || !y))) return TRIG_EINVAL;
    const size_t ws = s->workspace_for(n_events);
    const Layout L(n_events, n_hits, ws);
    size_t pin_off;
    uint64_t t;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop || !s->adm.admissible(L.dev_bytes)) return TRIG_EINVAL;
        if (s->stats.pending >= s->cfg.max_pending) {
            ++s->stats.rejected_busy;
            return TRIG_EBUSY;
        }
        pin_off = s->pin_arena.alloc(L.host_bytes);
        if (pin_off == Arena::kFail) {
            ++s->stats.rejected_busy;
            return TRIG_EBUSY;
        }
        t = s->next_ticket++;
        Slice& sl = s->slices[t];
        sl.ticket = t;
        sl.n_events = n_events;
        sl.n_hits = n_hits;
        sl.pin_off = pin_off;
        sl.ws_bytes = ws;
        sl.state = State::Queued;
        sl.t_submit = s->now();
        ++s->stats.pending;
        // Queued before it is staged: it may be admitted (and its input start
        // moving to the device) while the copy below is still running.
        s->adm.enqueue(t, L.dev_bytes);
        ++s->stats.submitted;
    }
    s->cv_work.notify_one();
    char* h = s->pin_base + pin_off;
    std::memset(h + L.status, 0, 4);
    // Stage in layout order, publishing the staged prefix chunk by chunk.
    const CopySeg seg[3] = {{h + L.off, reinterpret_cast<const char*>(offsets), 4 * (size_t)(3 * n_events + 1)},
                            {h + L.x, reinterpret_cast<const char*>(x), n_hits ? 4 * (size_t)n_hits : 0},
                            {h + L.y, reinterpret_cast<const char*>(y), n_hits ? 4 * (size_t)n_hits : 0}};
    const size_t seg_end[3] = {L.x, L.y, L.status};  // the next segment's start (padding included)
    for (int k = 0; k < 3; ++k) {
        for (size_t done = 0; done < seg[k].bytes;) {
            const size_t piece = std::min(kStageChunk, seg[k].bytes - done);
            const CopySeg part{seg[k].dst + done, seg[k].src + done, piece};
            copy_segments(&part, 1);
            done += piece;
            const size_t prefix = done == seg[k].bytes ? seg_end[k] : (size_t)(seg[k].dst - h) + done;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->slices[t].staged = prefix;
            }
            s->cv_work.notify_one();
        }
        if (seg[k].bytes == 0) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->slices[t].staged = seg_end[k];
        }
    }
    s->cv_work.notify_one();
    *ticket = t;
    return TRIG_OK;
}

int trig_server_poll(trig_server* s, trig_slice_result* out, int32_t timeout_ms) {
    if (!s || !out) return TRIG_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return !s->done.empty(); };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        return TRIG_ETIMEOUT;
    const uint64_t t = s->done.front();
    s->done.pop_front();
    Slice& sl = s->slices[t];
    sl.state = State::Polled;
    const Layout L(sl.n_events, sl.n_hits, sl.ws_bytes);
    const char* h = s->pin_base + sl.pin_off;
    std::memset(out, 0, sizeof(*out));
    out->ticket = t;
    out->status = sl.status;
    out->n_events = sl.n_events;
    out->t_submit = sl.t_submit;
    out->t_admit = sl.t_admit;
    out->t_done = sl.t_done;
    if (sl.status == TRIG_OK) {
        out->counts = reinterpret_cast<const int32_t*>(h + L.counts);
        out->accept = reinterpret_cast<const uint8_t*>(h + L.accept);
        out->accepted_ids = reinterpret_cast<const int32_t*>(h + L.ids);
        std::memcpy(&out->n_accepted, h + L.n_acc, 4);
        std::memcpy(&out->event_status, h + L.status, 4);
    }
    return TRIG_OK;
}

int trig_server_release(trig_server* s, uint64_t ticket) {
    if (!s) return TRIG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->slices.find(ticket);
    if (it == s->slices.end() || it->second.state != State::Polled) return TRIG_EINVAL;
    s->pin_arena.release(it->second.pin_off);
    s->slices.erase(it);
    return TRIG_OK;
}

int trig_server_pause(trig_server* s, int32_t paused) {
    if (!s) return TRIG_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->paused = paused != 0;
    }
    s->cv_work.notify_all();
    return TRIG_OK;
}

int trig_server_stats_get(trig_server* s, trig_server_stats* out) {
    if (!s || !out) return TRIG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->hbm_in_use = s->adm.arena().in_use();
    return TRIG_OK;
}

double trig_server_now(trig_server* s) { return s ? s->now() : 0.0; }

int trig_server_destroy(trig_server* s) {
    if (!s) return TRIG_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    (void)hipSetDevice(s->cfg.device);
    for (size_t i = 0; i < s->streams.size(); ++i) {
        (void)hipStreamSynchronize(s->streams[i]);
        (void)hipStreamDestroy(s->streams[i]);
        (void)hipEventDestroy(s->events[i]);
    }
    (void)hipFree(s->dev_base);
    (void)hipHostFree(s->pin_base);
    delete s;
    return TRIG_OK;
}

}  // extern "C"
