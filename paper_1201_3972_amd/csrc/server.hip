// server.hip -- continuous-batching request loop (see include/irfilter.h):
// admission by device memory, resident per-stream slots, one batched launch per
// step on a compute stream, host -> device and device -> host copies on two
// copy streams of their own so the directions overlap.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <thread>
#include <vector>

#include "../../include/irfilter.h"
#include "arena.hpp"
#include "host_common.hpp"

namespace {

using irf::host::bytes_of;
using irf::host::Arena;
using irf::host::round_up;

constexpr int kMaxInflight = 8;

struct Slot {
    void *src = nullptr, *dst = nullptr;
    size_t pitch = 0;
    int width = 0, height = 0;
    irf_dtype dtype = IRF_U8;
    bool busy = false;
};

struct Item {
    irf_request r;
    void *dsrc = nullptr, *ddst = nullptr;
    size_t dpitch = 0;
    Slot *slot = nullptr;
    size_t a_off = 0, b_off = 0, bytes = 0;  // arena blocks (one-off frames)
};

struct Step {
    std::vector<Item> items;
    hipEvent_t in = nullptr, kernel = nullptr, done = nullptr;
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct irf_server {
    hipStream_t h2d = nullptr, compute = nullptr, d2h = nullptr;  // the two copy directions overlap
    unsigned char *arena_mem = nullptr;
    size_t arena_bytes = 0;
    Arena arena;
    std::map<int, std::vector<Slot>> streams;
    std::vector<irf_plan *> plans;
    int next_plan = 0;
    int max_frames = 0, max_tiles = 0, max_inflight = 0;
    std::deque<irf_request> future, pending;
    std::deque<Step> inflight;
    std::vector<hipEvent_t> events;  // idle events
    std::vector<std::pair<uint64_t, double>> completed;
    size_t completed_head = 0;
    std::vector<irf_frame> frames;  // staging for one step
    double last_arrival = 0.0;
    int steps = 0;
    std::chrono::steady_clock::time_point t0;
};

namespace {

irf_status take_event(irf_server *s, hipEvent_t *ev) {
    if (!s->events.empty()) {
        *ev = s->events.back();
        s->events.pop_back();
        return IRF_OK;
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming) == hipSuccess ? IRF_OK : IRF_ERR_HIP;
}

void free_server(irf_server *s) {
    if (!s) return;
    for (auto &st : s->inflight) {
        if (st.done) (void)hipEventSynchronize(st.done);
        for (hipEvent_t e : {st.in, st.kernel, st.done})
            if (e) s->events.push_back(e);
    }
    s->inflight.clear();
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (irf_plan *p : s->plans) ir_filter_plan_destroy(p);
    for (auto &kv : s->streams)
        for (Slot &sl : kv.second) {
            if (sl.src) (void)hipFree(sl.src);
            if (sl.dst) (void)hipFree(sl.dst);
        }
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    if (s->h2d) (void)hipStreamDestroy(s->h2d);
    if (s->compute) (void)hipStreamDestroy(s->compute);
    if (s->d2h) (void)hipStreamDestroy(s->d2h);
    delete s;
}

size_t frame_bytes(const irf_request &r) { return (size_t)r.width * r.height * bytes_of(r.dtype); }

// One frame between host and device: a single linear copy when both sides are
// contiguous, a 2-D copy otherwise.
hipError_t copy_frame(void *dst, size_t dpitch, const void *src, size_t spitch, size_t row, int rows,
                      hipMemcpyKind kind, hipStream_t st) {
    if (dpitch == row && spitch == row) return hipMemcpyAsync(dst, src, row * (size_t)rows, kind, st);
    return hipMemcpy2DAsync(dst, dpitch, src, spitch, row, rows, kind, st);
}

// Free resources of a finished step; its requests complete at time t.
void retire_step(irf_server *s, Step &st, double t) {
    for (Item &it : st.items) {
        s->completed.emplace_back(it.r.id, t - it.r.arrival);
        if (it.slot) {
            it.slot->busy = false;
        } else {
            s->arena.release(it.a_off, it.bytes);
            s->arena.release(it.b_off, it.bytes);
        }
    }
    for (hipEvent_t e : {st.in, st.kernel, st.done}) s->events.push_back(e);
}

int retire(irf_server *s, bool block) {
    int n = 0;
    while (!s->inflight.empty()) {
        Step &st = s->inflight.front();
        if (block) {
            if (hipEventSynchronize(st.done) != hipSuccess) return IRF_ERR_HIP;
        } else {
            const hipError_t q = hipEventQuery(st.done);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return IRF_ERR_HIP;
        }
        retire_step(s, st, seconds_since(s->t0));
        s->inflight.pop_front();
        ++n;
        block = false;
    }
    return n;
}

// Admit arrived requests that fit now, in arrival order (one that does not fit
// does not block later ones that do).
void admit(irf_server *s, std::vector<Item> &out) {
    std::deque<irf_request> keep;
    const irf_plan *plan = s->plans[s->next_plan];
    int tiles = 0;
    while (!s->pending.empty()) {
        irf_request r = s->pending.front();
        s->pending.pop_front();
        const int nt = ir_filter_plan_frame_tiles(plan, r.width, r.height);
        if ((int)out.size() >= s->max_frames || tiles + nt > s->max_tiles) {
            keep.push_back(r);
            continue;
        }
        Item it;
        it.r = r;
        if (r.stream_id >= 0) {
            auto f = s->streams.find(r.stream_id);
            Slot *free_slot = nullptr;
            if (f != s->streams.end())
                for (Slot &sl : f->second)
                    if (!sl.busy) {
                        free_slot = &sl;
                        break;
                    }
            if (!free_slot) {
                keep.push_back(r);  // the stream's earlier frames still hold its slots
                continue;
            }
            free_slot->busy = true;
            it.slot = free_slot;
            it.dsrc = free_slot->src;
            it.ddst = free_slot->dst;
            it.dpitch = free_slot->pitch;
        } else {
            it.bytes = frame_bytes(r);
            if (!s->arena.alloc(it.bytes, &it.a_off)) {
                keep.push_back(r);
                continue;
            }
            if (!s->arena.alloc(it.bytes, &it.b_off)) {
                s->arena.release(it.a_off, it.bytes);
                keep.push_back(r);
                continue;
            }
            it.dsrc = s->arena_mem + it.a_off;
            it.ddst = s->arena_mem + it.b_off;
            it.dpitch = (size_t)r.width * bytes_of(r.dtype);
        }
        tiles += nt;
        out.push_back(it);
    }
    s->pending.swap(keep);
}

// A step that could not be issued: wait for whatever of it reached the
// streams, give its events, stream slots and arena blocks back, and return its
// requests to the front of the pending queue in their order, so the server is
// left as it was before the step was admitted.
void abandon_step(irf_server *s, Step &st, std::vector<Item> &items) {
    (void)hipStreamSynchronize(s->h2d);
    (void)hipStreamSynchronize(s->compute);
    (void)hipStreamSynchronize(s->d2h);
    (void)hipGetLastError();
    for (hipEvent_t e : {st.in, st.kernel, st.done})
        if (e) s->events.push_back(e);
    for (auto it = items.rbegin(); it != items.rend(); ++it) {
        if (it->slot) {
            it->slot->busy = false;
        } else {
            s->arena.release(it->a_off, it->bytes);
            s->arena.release(it->b_off, it->bytes);
        }
        s->pending.push_front(it->r);
    }
    items.clear();
}

irf_status issue_step(irf_server *s, Step &st, const std::vector<Item> &items) {
    irf_status e;
    if ((e = take_event(s, &st.in)) || (e = take_event(s, &st.kernel)) || (e = take_event(s, &st.done))) return e;
    for (const Item &it : items) {
        const size_t row = (size_t)it.r.width * bytes_of(it.r.dtype);
        if (copy_frame(it.dsrc, it.dpitch, it.r.host_src, it.r.src_pitch, row, it.r.height, hipMemcpyHostToDevice,
                       s->h2d) != hipSuccess)
            return IRF_ERR_HIP;
    }
    if (hipEventRecord(st.in, s->h2d) != hipSuccess || hipStreamWaitEvent(s->compute, st.in, 0) != hipSuccess)
        return IRF_ERR_HIP;
    s->frames.clear();
    for (const Item &it : items)
        s->frames.push_back({it.dsrc, it.ddst, it.dpitch, it.dpitch, it.r.width, it.r.height, it.r.dtype,
                             it.r.window});
    irf_plan *plan = s->plans[s->next_plan];
    s->next_plan = (s->next_plan + 1) % (int)s->plans.size();
    if ((e = ir_filter_run_batch(plan, s->frames.data(), (int)s->frames.size(), nullptr, s->compute))) return e;
    if (hipEventRecord(st.kernel, s->compute) != hipSuccess || hipStreamWaitEvent(s->d2h, st.kernel, 0) != hipSuccess)
        return IRF_ERR_HIP;
    for (const Item &it : items) {
        const size_t row = (size_t)it.r.width * bytes_of(it.r.dtype);
        if (copy_frame(it.r.host_dst, it.r.dst_pitch, it.ddst, it.dpitch, row, it.r.height, hipMemcpyDeviceToHost,
                       s->d2h) != hipSuccess)
            return IRF_ERR_HIP;
    }
    if (hipEventRecord(st.done, s->d2h) != hipSuccess) return IRF_ERR_HIP;
    return IRF_OK;
}

irf_status issue(irf_server *s, std::vector<Item> &items) {
    Step st;
    const irf_status e = issue_step(s, st, items);
    if (e) {
        abandon_step(s, st, items);
        return e;
    }
    st.items.swap(items);
    s->inflight.push_back(std::move(st));
    ++s->steps;
    return IRF_OK;
}

}  // namespace

extern "C" {

irf_status ir_filter_server_create(irf_server **server, size_t arena_bytes, int max_batch_frames,
                                   int max_batch_tiles, int max_inflight, unsigned flags) {
    if (!server) return IRF_ERR_NULL;
    *server = nullptr;
    if (max_batch_frames < 1 || max_batch_tiles < 1 || max_inflight < 1 || max_inflight > kMaxInflight)
        return IRF_ERR_DIMS;
    irf_server *s = new (std::nothrow) irf_server();
    if (!s) return IRF_ERR_NOMEM;
    try {
        s->t0 = std::chrono::steady_clock::now();
        s->max_frames = max_batch_frames;
        s->max_tiles = max_batch_tiles;
        s->max_inflight = max_inflight;
        (void)hipGetLastError();
        if (hipStreamCreateWithFlags(&s->h2d, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&s->d2h, hipStreamNonBlocking) != hipSuccess) {
            free_server(s);
            return IRF_ERR_HIP;
        }
        s->arena_bytes = round_up(arena_bytes);
        if (s->arena_bytes && hipMalloc(&s->arena_mem, s->arena_bytes) != hipSuccess) {
            s->arena_mem = nullptr;
            free_server(s);
            (void)hipGetLastError();
            return IRF_ERR_NOMEM;
        }
        s->arena.reset(s->arena_bytes);
        for (int i = 0; i < max_inflight; ++i) {
            irf_plan *p = nullptr;
            const irf_status st = ir_filter_plan_create(&p, max_batch_frames, max_batch_tiles, flags);
            if (st) {
                free_server(s);
                return st;
            }
            s->plans.push_back(p);
        }
        *server = s;
        return IRF_OK;
    } catch (...) {
        free_server(s);
        return IRF_ERR_NOMEM;
    }
}

irf_status ir_filter_server_register_stream(irf_server *s, int stream_id, int width, int height,
                                            irf_dtype dtype, int depth) {
    if (!s) return IRF_ERR_NULL;
    irf_status st = irf::host::check_common(width, height, 1, dtype, 3);
    if (st) return st;
    if (stream_id < 0 || depth < 1 || depth > 16 || s->streams.count(stream_id)) return IRF_ERR_DIMS;
    try {
        std::vector<Slot> slots(depth);
        const size_t pitch = (size_t)width * bytes_of(dtype);
        for (Slot &sl : slots) {
            sl.width = width;
            sl.height = height;
            sl.dtype = dtype;
            sl.pitch = pitch;
            if (hipMalloc(&sl.src, pitch * height) != hipSuccess || hipMalloc(&sl.dst, pitch * height) != hipSuccess) {
                for (Slot &x : slots) {
                    if (x.src) (void)hipFree(x.src);
                    if (x.dst) (void)hipFree(x.dst);
                }
                (void)hipGetLastError();
                return IRF_ERR_NOMEM;
            }
        }
        s->streams[stream_id] = std::move(slots);
        return IRF_OK;
    } catch (...) {
        return IRF_ERR_NOMEM;
    }
}

irf_status ir_filter_server_submit(irf_server *s, const irf_request *reqs, int n) {
    if (!s || (!reqs && n > 0)) return IRF_ERR_NULL;
    if (n < 0) return IRF_ERR_DIMS;
    // validate everything before queueing anything
    double last = s->last_arrival;
    for (int i = 0; i < n; ++i) {
        const irf_request &r = reqs[i];
        if (!r.host_src || !r.host_dst) return IRF_ERR_NULL;
        irf_status st = irf::host::check_batch_frame(r.width, r.height, r.dtype, r.window);
        if (st) return st;
        const int b = bytes_of(r.dtype);
        if ((st = irf::host::check_layout(r.src_pitch, 0, r.width, r.height, 1, b))) return st;
        if ((st = irf::host::check_layout(r.dst_pitch, 0, r.width, r.height, 1, b))) return st;
        if (r.arrival < last) return IRF_ERR_DIMS;
        last = r.arrival;
        if (ir_filter_plan_frame_tiles(s->plans[0], r.width, r.height) > s->max_tiles) return IRF_ERR_CAPACITY;
        if (r.stream_id >= 0) {
            auto f = s->streams.find(r.stream_id);
            if (f == s->streams.end()) return IRF_ERR_DIMS;
            const Slot &sl = f->second[0];
            if (sl.width != r.width || sl.height != r.height || sl.dtype != r.dtype) return IRF_ERR_DIMS;
        } else if (2 * round_up(frame_bytes(r)) > s->arena_bytes) {
            return IRF_ERR_CAPACITY;
        }
    }
    try {
        for (int i = 0; i < n; ++i) s->future.push_back(reqs[i]);
    } catch (...) {
        return IRF_ERR_NOMEM;
    }
    s->last_arrival = last;
    return IRF_OK;
}

int ir_filter_server_poll(irf_server *s) {
    if (!s) return IRF_ERR_NULL;
    try {
        int r = retire(s, false);
        if (r < 0) return r;
        bool progressed = r > 0;
        const double now = seconds_since(s->t0);
        while (!s->future.empty() && s->future.front().arrival <= now) {
            s->pending.push_back(s->future.front());
            s->future.pop_front();
        }
        if ((int)s->inflight.size() < s->max_inflight && !s->pending.empty()) {
            std::vector<Item> items;
            admit(s, items);
            if (!items.empty()) {
                const irf_status st = issue(s, items);
                if (st) return st;
                progressed = true;
            }
        }
        return progressed ? 1 : 0;
    } catch (...) {
        return IRF_ERR_NOMEM;
    }
}

irf_status ir_filter_server_run(irf_server *s) {
    if (!s) return IRF_ERR_NULL;
    while (!s->future.empty() || !s->pending.empty() || !s->inflight.empty()) {
        const int p = ir_filter_server_poll(s);
        if (p < 0) return (irf_status)p;
        if (p > 0) continue;
        if ((int)s->inflight.size() >= s->max_inflight) {
            const int r = retire(s, true);  // wait for the oldest step
            if (r < 0) return (irf_status)r;
        } else if (!s->inflight.empty()) {
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else if (!s->pending.empty()) {
            return IRF_ERR_CAPACITY;  // an arrived request can never be admitted
        } else {
            const double wait = s->future.front().arrival - seconds_since(s->t0);
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 1e-3)));
        }
    }
    return IRF_OK;
}

int ir_filter_server_completed(irf_server *s, uint64_t *ids, double *latency_s, int max) {
    if (!s || max <= 0) return 0;
    int n = 0;
    while (n < max && s->completed_head < s->completed.size()) {
        const auto &c = s->completed[s->completed_head++];
        if (ids) ids[n] = c.first;
        if (latency_s) latency_s[n] = c.second;
        ++n;
    }
    if (s->completed_head == s->completed.size()) {
        s->completed.clear();
        s->completed_head = 0;
    }
    return n;
}

double ir_filter_server_now(const irf_server *s) { return s ? seconds_since(s->t0) : 0.0; }

int ir_filter_server_steps(const irf_server *s) { return s ? s->steps : 0; }

size_t ir_filter_server_arena_used(const irf_server *s) { return s ? s->arena.used() : 0; }

size_t ir_filter_server_resident_bytes(const irf_server *s) {
    if (!s) return 0;
    size_t n = s->arena_bytes;
    for (const auto &kv : s->streams)
        for (const Slot &sl : kv.second) n += 2 * sl.pitch * (size_t)sl.height;
    return n;
}

void ir_filter_server_destroy(irf_server *s) { free_server(s); }

}  // extern "C"
