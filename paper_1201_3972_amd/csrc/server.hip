// server.hip -- continuous-batching request loop (see include/irfilter.h):
// admission by device memory, resident per-stream slots, one batched launch per
// step on a compute stream, host -> device and device -> host copies on two
// copy streams of their own so the directions overlap.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <string.h>

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
    void *hsrc_dev = nullptr, *hdst_dev = nullptr;  // device views of the host buffers (null: none)
    Slot *slot = nullptr;
    size_t a_off = 0, b_off = 0, bytes = 0;  // arena blocks (one-off frames)
};

struct Step {
    std::vector<Item> items;
    hipEvent_t in = nullptr, kernel = nullptr, done = nullptr;
    int table = -1;  // the piece tables (in, out) this step's copy kernels read
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Frames move between pinned host memory and device memory by copy kernels, one
// launch per step and direction: a piece is a band of rows of one frame (about
// kPieceBytes), and each workgroup copies one piece.  The kernels read and
// write the host buffers through their device mappings, so a step costs two
// launches instead of one copy command per frame and direction.
struct CopyPiece {
    const uint8_t *src;
    uint8_t *dst;
    uint32_t spitch, dpitch;  // bytes between rows
    uint32_t rowbytes, rows;
};

constexpr size_t kPieceBytes = 128 << 10;
constexpr int kMaxPieces = 8192;  // per step and direction; further frames use copy commands
constexpr int kCopyThreads = 256;

__global__ __launch_bounds__(kCopyThreads) void copy_pieces_kernel(const CopyPiece *pieces) {
    const CopyPiece p = pieces[blockIdx.x];
    const bool vec = ((reinterpret_cast<uintptr_t>(p.src) | reinterpret_cast<uintptr_t>(p.dst) | p.spitch | p.dpitch |
                       p.rowbytes) & 15u) == 0;
    if (vec) {
        // four 16-byte units per thread in flight, then their stores
        const uint32_t upr = p.rowbytes >> 4, units = upr * p.rows;
        for (uint32_t u0 = threadIdx.x; u0 < units; u0 += 4 * kCopyThreads) {
            uint4 v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t u = u0 + (uint32_t)i * kCopyThreads;
                if (u < units) {
                    const uint32_t row = u / upr, col = u - row * upr;
                    v[i] = *reinterpret_cast<const uint4 *>(p.src + (size_t)row * p.spitch + 16u * col);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t u = u0 + (uint32_t)i * kCopyThreads;
                if (u < units) {
                    const uint32_t row = u / upr, col = u - row * upr;
                    *reinterpret_cast<uint4 *>(p.dst + (size_t)row * p.dpitch + 16u * col) = v[i];
                }
            }
        }
    } else {
        const uint32_t units = p.rowbytes * p.rows;
        for (uint32_t u = threadIdx.x; u < units; u += kCopyThreads) {
            const uint32_t row = u / p.rowbytes, col = u - row * p.rowbytes;
            p.dst[(size_t)row * p.dpitch + col] = p.src[(size_t)row * p.spitch + col];
        }
    }
}

// Split a frame copy into pieces (appended to `out` while it has room).
bool add_pieces(std::vector<CopyPiece> &out, const void *src, size_t spitch, void *dst, size_t dpitch,
                size_t rowbytes, int rows) {
    const int band = (int)std::max<size_t>(1, kPieceBytes / std::max<size_t>(rowbytes, 1));
    const int n = (rows + band - 1) / band;
    if ((int)out.size() + n > kMaxPieces) return false;
    for (int r0 = 0; r0 < rows; r0 += band) {
        const int nr = std::min(band, rows - r0);
        out.push_back({static_cast<const uint8_t *>(src) + (size_t)r0 * spitch,
                       static_cast<uint8_t *>(dst) + (size_t)r0 * dpitch, (uint32_t)spitch, (uint32_t)dpitch,
                       (uint32_t)rowbytes, (uint32_t)nr});
    }
    return true;
}

// The device address of a pinned host buffer, or null if it has none.
void *device_view(const void *host) {
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, const_cast<void *>(host), 0) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return d;
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
    // piece tables in pinned host memory: 2 per in-flight step (in, out), and
    // their device views; free table slots
    CopyPiece *tables = nullptr;
    CopyPiece *tables_dev = nullptr;
    std::vector<int> free_tables;
    std::vector<CopyPiece> pin, pout;  // pieces of the step being issued
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
    if (s->tables) (void)hipHostFree(s->tables);
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
    if (st.table >= 0) s->free_tables.push_back(st.table);
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
        it.hsrc_dev = device_view(r.host_src);
        it.hdst_dev = device_view(r.host_dst);
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
    if (st.table >= 0) s->free_tables.push_back(st.table);
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

// The copies of one step in one direction: pieces for every frame whose host
// buffer has a device view (one kernel launch), copy commands for the others.
irf_status copy_step(irf_server *s, const std::vector<Item> &items, bool to_device, CopyPiece *table,
                     const CopyPiece *table_dev, hipStream_t st) {
    std::vector<CopyPiece> &pieces = to_device ? s->pin : s->pout;
    pieces.clear();
    for (const Item &it : items) {
        const size_t row = (size_t)it.r.width * bytes_of(it.r.dtype);
        const void *hsrc = to_device ? it.r.host_src : it.ddst;
        void *hdst = to_device ? it.dsrc : it.r.host_dst;
        void *hview = to_device ? it.hsrc_dev : it.hdst_dev;
        const size_t spitch = to_device ? it.r.src_pitch : it.dpitch;
        const size_t dpitch = to_device ? it.dpitch : it.r.dst_pitch;
        const bool pieced = hview && spitch < ((size_t)1 << 32) && dpitch < ((size_t)1 << 32) &&
                            add_pieces(pieces, to_device ? hview : hsrc, spitch, to_device ? hdst : hview, dpitch,
                                       row, it.r.height);
        if (!pieced && copy_frame(hdst, dpitch, hsrc, spitch, row, it.r.height,
                                  to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost, st) != hipSuccess)
            return IRF_ERR_HIP;
    }
    if (!pieces.empty()) {
        memcpy(table, pieces.data(), sizeof(CopyPiece) * pieces.size());
        hipLaunchKernelGGL(copy_pieces_kernel, dim3((unsigned)pieces.size()), dim3(kCopyThreads), 0, st, table_dev);
        if (hipGetLastError() != hipSuccess) return IRF_ERR_HIP;
    }
    return IRF_OK;
}

irf_status issue_step(irf_server *s, Step &st, const std::vector<Item> &items) {
    irf_status e;
    if ((e = take_event(s, &st.in)) || (e = take_event(s, &st.kernel)) || (e = take_event(s, &st.done))) return e;
    if (s->free_tables.empty()) return IRF_ERR_HIP;  // cannot happen: one table pair per in-flight step
    st.table = s->free_tables.back();
    s->free_tables.pop_back();
    CopyPiece *tin = s->tables + (size_t)(2 * st.table) * kMaxPieces, *tout = tin + kMaxPieces;
    const CopyPiece *din = s->tables_dev + (size_t)(2 * st.table) * kMaxPieces, *dout = din + kMaxPieces;
    if ((e = copy_step(s, items, true, tin, din, s->h2d))) return e;
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
    if ((e = copy_step(s, items, false, tout, dout, s->d2h))) return e;
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
        const size_t tbytes = sizeof(CopyPiece) * (size_t)kMaxPieces * 2 * (size_t)max_inflight;
        if (hipHostMalloc(reinterpret_cast<void **>(&s->tables), tbytes, hipHostMallocCoherent) != hipSuccess ||
            !(s->tables_dev = static_cast<CopyPiece *>(device_view(s->tables)))) {
            if (s->tables) {
                (void)hipHostFree(s->tables);
                s->tables = nullptr;
            }
            free_server(s);
            (void)hipGetLastError();
            return IRF_ERR_NOMEM;
        }
        for (int i = max_inflight - 1; i >= 0; --i) s->free_tables.push_back(i);
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
