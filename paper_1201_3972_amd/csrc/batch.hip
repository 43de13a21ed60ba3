// batch.hip -- plans and batched launches over frames of uneven size, pixel
// type and window (see include/irfilter.h and batch_device.hpp).
#include <hip/hip_runtime.h>

#include <atomic>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "../../include/irfilter.h"
#include "batch_kernels.hpp"
#include "host_common.hpp"

using namespace irf;
using namespace irf::host;

namespace {

constexpr int kSets = 2;  // device table sets used alternately
constexpr size_t kQueueBytes = (kBatchClasses * sizeof(BatchQueue) + 255) / 256 * 256;  // queue records, padded

// Workgroup size of plans created from now on (0 = the default, 128 threads).
std::atomic<int> g_batch_threads{0};

int batch_threads_now() {
    const int t = g_batch_threads.load(std::memory_order_relaxed);
    return t == 0 ? kThreads : t;
}

int frame_tiles(int width, int height, int threads) {
    const int th = threads / kThreadsX * Geometry<3>::R;
    return ((width + kTileW - 1) / kTileW) * ((height + th - 1) / th);
}

int class_blocks_per_cu(int c, int threads) {
    switch (c) {
        case 0: return BatchClass<0>::blocks_per_cu(threads);
        case 1: return BatchClass<1>::blocks_per_cu(threads);
        case 2: return BatchClass<2>::blocks_per_cu(threads);
        case 3: return BatchClass<3>::blocks_per_cu(threads);
        case 4: return BatchClass<4>::blocks_per_cu(threads);
        case 5: return BatchClass<5>::blocks_per_cu(threads);
        case 6: return BatchClass<6>::blocks_per_cu(threads);
        case 7: return BatchClass<7>::blocks_per_cu(threads);
        case 8: return BatchClass<8>::blocks_per_cu(threads);
        default: return BatchClass<9>::blocks_per_cu(threads);
    }
}

void class_launch(int c, int threads, int grid, const FrameDesc *d, const uint32_t *map, BatchQueue *q,
                  hipStream_t s) {
    static_assert(kBatchClasses == 10, "one case per class");
    switch (c) {
        case 0: BatchClass<0>::launch(threads, grid, d, map, q, s); break;
        case 1: BatchClass<1>::launch(threads, grid, d, map, q, s); break;
        case 2: BatchClass<2>::launch(threads, grid, d, map, q, s); break;
        case 3: BatchClass<3>::launch(threads, grid, d, map, q, s); break;
        case 4: BatchClass<4>::launch(threads, grid, d, map, q, s); break;
        case 5: BatchClass<5>::launch(threads, grid, d, map, q, s); break;
        case 6: BatchClass<6>::launch(threads, grid, d, map, q, s); break;
        case 7: BatchClass<7>::launch(threads, grid, d, map, q, s); break;
        case 8: BatchClass<8>::launch(threads, grid, d, map, q, s); break;
        default: BatchClass<9>::launch(threads, grid, d, map, q, s); break;
    }
}

}  // namespace

// Device layout of one table set: [queues | descriptors | tile map].  The map
// holds every tile of a batch, class by class; queue c covers class c's part.
struct irf_plan {
    int max_frames = 0, max_tiles = 0;
    unsigned flags = 0;
    size_t desc_off = 0, map_off = 0, bytes = 0;
    int threads = kThreads;  // workgroup size of the batch kernels (tile height / 8 * 32)
    int grid[kBatchClasses] = {};
    int next_set = 0;
    hipStream_t capture = nullptr;  // graph capture stream (IRF_PLAN_GRAPH)
    struct Set {
        unsigned char *dev = nullptr;
        unsigned char *host = nullptr;  // pinned staging
        hipEvent_t copied = nullptr;    // staging may be rewritten
        hipEvent_t done = nullptr;      // device tables may be rewritten
        std::map<unsigned, hipGraphExec_t> graphs;  // by the set of classes a batch uses
        bool used = false;
    } set[kSets];
};

namespace {

// The kernels of the classes in `classes` (bit c = class c), one after the
// other; the arguments are fixed per table set, so a launch sequence can be
// captured in a graph once and replayed for every batch using those classes.
void launch_batch(const irf_plan *p, const irf_plan::Set &s, unsigned classes, hipStream_t stream) {
    BatchQueue *q = reinterpret_cast<BatchQueue *>(s.dev);
    const FrameDesc *d = reinterpret_cast<const FrameDesc *>(s.dev + p->desc_off);
    const uint32_t *map = reinterpret_cast<const uint32_t *>(s.dev + p->map_off);
    for (int c = 0; c < kBatchClasses; ++c)
        if (classes & (1u << c)) class_launch(c, p->threads, p->grid[c], d, map, q + c, stream);
}

// The graph of this set and class set, captured on first use.
irf_status set_graph(irf_plan *p, irf_plan::Set &s, unsigned classes, hipGraphExec_t *out) {
    auto it = s.graphs.find(classes);
    if (it != s.graphs.end()) {
        *out = it->second;
        return IRF_OK;
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    bool ok = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) launch_batch(p, s, classes, p->capture);
    ok = (hipStreamEndCapture(p->capture, &g) == hipSuccess) && ok;
    ok = ok && hipGraphInstantiate(&e, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        if (e) (void)hipGraphExecDestroy(e);
        (void)hipGetLastError();
        return IRF_ERR_HIP;
    }
    s.graphs[classes] = e;
    *out = e;
    return IRF_OK;
}

void free_plan(irf_plan *p) {
    if (!p) return;
    for (auto &s : p->set) {
        for (auto &kv : s.graphs) (void)hipGraphExecDestroy(kv.second);
        if (s.copied) (void)hipEventDestroy(s.copied);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.dev) (void)hipFree(s.dev);
        if (s.host) (void)hipHostFree(s.host);
    }
    if (p->capture) (void)hipStreamDestroy(p->capture);
    delete p;
}

// Every dst span must be disjoint from every other span (src or dst).
bool batch_aliases(const irf_frame *frames, int n) {
    struct Ev {
        uintptr_t lo, hi;
        bool dst;
    };
    std::vector<Ev> ev;
    ev.reserve(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const int b = bytes_of(frames[i].dtype);
        const Span s = span_of(frames[i].src, frames[i].src_pitch, 0, frames[i].width, frames[i].height, 1, b);
        const Span d = span_of(frames[i].dst, frames[i].dst_pitch, 0, frames[i].width, frames[i].height, 1, b);
        ev.push_back({s.lo, s.hi, false});
        ev.push_back({d.lo, d.hi, true});
    }
    std::sort(ev.begin(), ev.end(), [](const Ev &a, const Ev &b) { return a.lo < b.lo; });
    uintptr_t end_any = 0, end_dst = 0;
    for (const Ev &e : ev) {
        if (e.dst ? e.lo < end_any : e.lo < end_dst) return true;
        end_any = std::max(end_any, e.hi);
        if (e.dst) end_dst = std::max(end_dst, e.hi);
    }
    return false;
}

}  // namespace

extern "C" {

int ir_filter_frame_tiles(int width, int height) {
    if (width < 1 || height < 1 || width > IRF_MAX_DIM || height > IRF_MAX_DIM) return 0;
    return frame_tiles(width, height, batch_threads_now());
}

irf_status ir_filter_set_batch_threads(int threads) {
    if (threads != 0 && threads != 128 && threads != 256) return IRF_ERR_TUNING;
    g_batch_threads.store(threads, std::memory_order_relaxed);
    return IRF_OK;
}

int ir_filter_get_batch_threads(void) { return batch_threads_now(); }

int ir_filter_plan_frame_tiles(const irf_plan *plan, int width, int height) {
    if (!plan || width < 1 || height < 1 || width > IRF_MAX_DIM || height > IRF_MAX_DIM) return 0;
    return frame_tiles(width, height, plan->threads);
}

irf_status ir_filter_plan_create(irf_plan **plan, int max_frames, int max_tiles, unsigned flags) {
    if (!plan) return IRF_ERR_NULL;
    *plan = nullptr;
    if (max_frames < 1 || max_tiles < 1 || max_frames > (1 << 24) || max_tiles > (1 << 28))
        return IRF_ERR_DIMS;
    irf_plan *p = new (std::nothrow) irf_plan();
    if (!p) return IRF_ERR_NOMEM;
    try {
        p->max_frames = max_frames;
        p->max_tiles = max_tiles;
        p->flags = flags;
        p->desc_off = kQueueBytes;
        p->map_off = p->desc_off + sizeof(FrameDesc) * (size_t)max_frames;
        p->bytes = p->map_off + sizeof(uint32_t) * (size_t)max_tiles;
        (void)hipGetLastError();
        p->threads = batch_threads_now();
        for (int c = 0; c < kBatchClasses; ++c) p->grid[c] = class_blocks_per_cu(c, p->threads) * device_cus();
        for (auto &s : p->set) {
            if (hipMalloc(&s.dev, p->bytes) != hipSuccess) {
                free_plan(p);
                (void)hipGetLastError();
                return IRF_ERR_NOMEM;
            }
            if (hipHostMalloc(&s.host, p->bytes, hipHostMallocDefault) != hipSuccess) {
                free_plan(p);
                (void)hipGetLastError();
                return IRF_ERR_NOMEM;
            }
            if (hipEventCreateWithFlags(&s.copied, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
                free_plan(p);
                (void)hipGetLastError();
                return IRF_ERR_HIP;
            }
        }
        if (flags & IRF_PLAN_GRAPH) {
            // graphs are captured per set of classes on first use; the class of
            // windows 3..9, which video mixes use, is captured now
            hipGraphExec_t e = nullptr;
            if (hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess ||
                set_graph(p, p->set[0], 1u, &e) || set_graph(p, p->set[1], 1u, &e)) {
                free_plan(p);
                (void)hipGetLastError();
                return IRF_ERR_HIP;
            }
        }
        *plan = p;
        return IRF_OK;
    } catch (...) {
        free_plan(p);
        return IRF_ERR_NOMEM;
    }
}

irf_status ir_filter_run_batch(irf_plan *p, const irf_frame *frames, int n, uint64_t *counts,
                               hipStream_t stream) {
    try {
        if (!p || !frames) return IRF_ERR_NULL;
        if (n < 1) return IRF_ERR_DIMS;
        if (n > p->max_frames) return IRF_ERR_CAPACITY;
        long long tiles[kBatchClasses] = {};
        for (int i = 0; i < n; ++i) {
            const irf_frame &f = frames[i];
            if (!f.src || !f.dst) return IRF_ERR_NULL;
            irf_status st = check_batch_frame(f.width, f.height, f.dtype, f.window);
            if (st) return st;
            const int b = bytes_of(f.dtype);
            if ((st = check_layout(f.src_pitch, 0, f.width, f.height, 1, b))) return st;
            if ((st = check_layout(f.dst_pitch, 0, f.width, f.height, 1, b))) return st;
            tiles[batch_class(f.window)] += frame_tiles(f.width, f.height, p->threads);
        }
        long long all_tiles = 0;
        for (int c = 0; c < kBatchClasses; ++c) all_tiles += tiles[c];
        if (all_tiles > p->max_tiles) return IRF_ERR_CAPACITY;
        if (batch_aliases(frames, n)) return IRF_ERR_ALIAS;
        if (counts) {
            const Span cs = {reinterpret_cast<uintptr_t>(counts),
                             reinterpret_cast<uintptr_t>(counts) + sizeof(uint64_t) * (size_t)n};
            for (int i = 0; i < n; ++i) {
                const int b = bytes_of(frames[i].dtype);
                if (overlap(cs, span_of(frames[i].dst, frames[i].dst_pitch, 0, frames[i].width,
                                        frames[i].height, 1, b)) ||
                    overlap(cs, span_of(frames[i].src, frames[i].src_pitch, 0, frames[i].width,
                                        frames[i].height, 1, b)))
                    return IRF_ERR_ALIAS;
            }
        }

        (void)hipGetLastError();
        irf_plan::Set &s = p->set[p->next_set];
        p->next_set = (p->next_set + 1) % kSets;
        if (s.used && hipEventSynchronize(s.copied) != hipSuccess) return IRF_ERR_HIP;

        // host staging: queues, descriptors, tile map (one region per class)
        BatchQueue *q = reinterpret_cast<BatchQueue *>(s.host);
        FrameDesc *d = reinterpret_cast<FrameDesc *>(s.host + p->desc_off);
        uint32_t *map = reinterpret_cast<uint32_t *>(s.host + p->map_off);
        memset(q, 0, kQueueBytes);
        int begin[kBatchClasses] = {};  // class c's tiles fill map[base_c, base_c + tiles[c])
        unsigned base = 0;
        for (int c = 0; c < kBatchClasses; ++c) {
            q[c].total = (unsigned)tiles[c];
            q[c].base = base;
            base += (unsigned)tiles[c];
        }
        for (int i = 0; i < n; ++i) {
            const irf_frame &f = frames[i];
            const int b = bytes_of(f.dtype), c = batch_class(f.window), nt = frame_tiles(f.width, f.height, p->threads);
            FrameDesc &e = d[i];
            e.src = static_cast<const uint8_t *>(f.src);
            e.dst = static_cast<uint8_t *>(f.dst);
            e.src_pitch = f.src_pitch;
            e.dst_pitch = f.dst_pitch;
            e.count = counts ? reinterpret_cast<unsigned long long *>(counts + i) : nullptr;
            e.width = f.width;
            e.height = f.height;
            e.tiles_x = (f.width + kTileW - 1) / kTileW;
            e.tiles = nt;
            e.tile_begin = begin[c];
            e.kind = batch_kind(b, f.window);
            e.aligned = is16(f.src) && is16(f.dst) && is16(f.src_pitch) && is16(f.dst_pitch);
            e.pad = 0;
            uint32_t *m = map + q[c].base + begin[c];
            for (int t = 0; t < nt; ++t) m[t] = (uint32_t)i;
            begin[c] += nt;
        }

        // the kernels of this set's previous batch must be done with its tables
        if (s.used && hipStreamWaitEvent(stream, s.done, 0) != hipSuccess) return IRF_ERR_HIP;
        if (hipMemcpyAsync(s.dev, s.host, p->desc_off + sizeof(FrameDesc) * (size_t)n,
                           hipMemcpyHostToDevice, stream) != hipSuccess)
            return IRF_ERR_HIP;
        if (hipMemcpyAsync(s.dev + p->map_off, s.host + p->map_off, sizeof(uint32_t) * (size_t)all_tiles,
                           hipMemcpyHostToDevice, stream) != hipSuccess)
            return IRF_ERR_HIP;
        if (hipEventRecord(s.copied, stream) != hipSuccess) return IRF_ERR_HIP;
        s.used = true;
        if (counts) {
            hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                               reinterpret_cast<unsigned long long *>(counts), n);
        }
        unsigned classes = 0;
        for (int c = 0; c < kBatchClasses; ++c)
            if (tiles[c]) classes |= 1u << c;
        if (p->flags & IRF_PLAN_GRAPH) {
            hipGraphExec_t g = nullptr;
            irf_status st = set_graph(p, s, classes, &g);
            if (st) return st;
            if (hipGraphLaunch(g, stream) != hipSuccess) return IRF_ERR_HIP;
        } else {
            launch_batch(p, s, classes, stream);
        }
        if (hipEventRecord(s.done, stream) != hipSuccess) return IRF_ERR_HIP;
        if (hipGetLastError() != hipSuccess) return IRF_ERR_HIP;
        return IRF_OK;
    } catch (...) {
        return IRF_ERR_HIP;
    }
}

void ir_filter_plan_destroy(irf_plan *p) {
    if (!p) return;
    for (auto &s : p->set)
        if (s.used) (void)hipEventSynchronize(s.done);
    free_plan(p);
}

}  // extern "C"
