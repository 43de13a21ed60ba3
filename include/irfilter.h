/*
 * irfilter.h -- C ABI of the MI355X FNR impulse filter (libirfilter.so).
 *
 * The method is the Fast Noise Reduction (FNR) filter of Gupta, Beg and
 * Niranjan, "A Novel Approach to Fast Image Filtering Algorithm of Infrared
 * Images based on Intro Sort Algorithm":
 *   - S_xy is the k x k window around pixel (x, y), centre included; x is the
 *     column and y the row (Section 3.3);
 *   - a pixel is noisy when its grey level equals the minimum or the maximum of
 *     S_xy (Eq. 3a/3b, Step 2 of Section 3.3); ties count;
 *   - a noisy pixel is replaced by the median of S_xy, signal pixels keep their
 *     value (Section 3.4);
 *   - the whole frame may be filtered more than once (Section 4, Fig. 5-6).
 * Readings where the paper is silent: windows at the border repeat the edge
 * pixels (replicate); every pass reads an unchanged copy of its input; the
 * window side k is odd and the median is element (k*k-1)/2 of the sorted
 * window; 16-bit pixels are compared as full 16-bit values.
 *
 * Frames are single-channel, row-major, uint8 or uint16.  A "pitch" is the
 * byte distance between the starts of two rows (>= width * bytes per pixel,
 * < 2^24); a frame's span, (height - 1) * pitch + width * bytes per pixel, is
 * below 4 GiB (rows are addressed with 32-bit offsets inside a frame; frames
 * of a stack may lie anywhere).  Only the first width * bytes bytes of each
 * row are read or written.
 *
 * Memory and ownership: every frame, mask, scratch and counter pointer is a
 * DEVICE pointer owned by the caller (e.g. a torch CUDA tensor's data_ptr()).
 * The per-frame entry points allocate nothing.  Only an irf_plan owns device
 * memory (its descriptor table), released by ir_filter_plan_destroy.
 *
 * Execution: calls enqueue work on `stream` (NULL = the default stream) and
 * return without waiting.  The status reports argument validation, which runs
 * on the host before any HIP call, and launch errors.  No exception or abort
 * crosses this interface.  Calls on different streams may run concurrently.
 * Outputs must not overlap inputs (IRF_ERR_ALIAS): a tile's window reads would
 * race another tile's stores.
 *
 * Fast path: when every base address, pitch and frame stride is a multiple of
 * 16 bytes, interior tiles use 16-byte vector loads and stores; other layouts
 * are handled correctly with narrower accesses.
 */
#ifndef IRFILTER_H
#define IRFILTER_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { IRF_U8 = 1, IRF_U16 = 2 } irf_dtype;

typedef enum {
    IRF_OK = 0,
    IRF_ERR_NULL = -1,    /* a required pointer is NULL */
    IRF_ERR_DIMS = -2,    /* width/height outside 1..IRF_MAX_DIM, or frame count < 1 */
    IRF_ERR_PITCH = -3,   /* a pitch is smaller than one row or not below 2^24, a frame spans
                             4 GiB or more, or a stride is smaller than one frame */
    IRF_ERR_DTYPE = -4,   /* pixel type is not IRF_U8 or IRF_U16 */
    IRF_ERR_WINDOW = -5,  /* window is not odd or outside 3..IRF_MAX_WINDOW */
    IRF_ERR_PASSES = -6,  /* passes outside 1..IRF_MAX_PASSES, or scratch missing for passes >= 2 */
    IRF_ERR_ALIAS = -7,   /* an output overlaps an input or another output */
    IRF_ERR_HIP = -8,     /* a HIP call failed (the HIP error is cleared) */
    IRF_ERR_NOMEM = -9,   /* device or host allocation failed (plans only) */
    IRF_ERR_CAPACITY = -10, /* a batch exceeds the plan's capacity */
    IRF_ERR_TUNING = -11    /* no kernel for that workgroup size and selection algorithm */
} irf_status;

#define IRF_MAX_DIM 32768
/* The single-frame and stack entry points take windows up to 63x63, batch
 * plans and the server up to 31x31. */
#define IRF_MAX_WINDOW 63
#define IRF_MAX_BATCH_WINDOW 31
#define IRF_MAX_PASSES 16

/*
 * ir_filter_detect -- noise detection (Section 3.3, Eq. 3a/3b and Step 2).
 *   src, src_pitch       input frame (device, read only)
 *   mask, mask_pitch     output (device): mask[y*mask_pitch + x] = 1 if pixel (x, y)
 *                        equals its window's min or max, else 0; mask_pitch >= width
 *   width, height        1..IRF_MAX_DIM
 *   dtype, window        pixel type; odd window side 3..IRF_MAX_WINDOW
 *   flagged_count        nullable device uint64: set to the number of noisy pixels
 *                        (zeroed on the stream, then accumulated)
 */
irf_status ir_filter_detect(const void *src, size_t src_pitch, uint8_t *mask, size_t mask_pitch,
                            int width, int height, irf_dtype dtype, int window,
                            uint64_t *flagged_count, hipStream_t stream);

/*
 * ir_filter_detect_directional -- an opt-in detector that is NOT the paper's
 * (the method's detector is ir_filter_detect).  It reads the caption of
 * Fig. 1 (the central pixel against its two neighbours in the 3x3 window)
 * with Section 3's premise that signal grey levels vary monotonically along a
 * surface: pixel (x, y) is flagged when, on each of the four lines through it
 * in its 3x3 window (row, column, both diagonals), its grey level lies outside
 * the range of its two neighbours (ties count as inside; coordinates outside
 * the frame clamped to the edge, so border pixels are never flagged).  Unlike
 * the extreme test it keeps one-pixel lines.  The paper's figure is missing, so
 * the rule itself is a reading.  Compose with ir_filter_median(mask) to filter.
 *   src, src_pitch, mask, mask_pitch, width, height, dtype, flagged_count,
 *   stream: as for ir_filter_detect (there is no window argument)
 */
irf_status ir_filter_detect_directional(const void *src, size_t src_pitch, uint8_t *mask,
                                        size_t mask_pitch, int width, int height, irf_dtype dtype,
                                        uint64_t *flagged_count, hipStream_t stream);

/*
 * ir_filter_median -- median replacement (Section 3.4).
 *   mask (nullable)      where mask[y*mask_pitch + x] != 0 the pixel takes its window
 *                        median; other pixels are copied.  mask == NULL replaces
 *                        every pixel: the standard median filter of Section 2.
 *   dst, dst_pitch       output frame (device), same type and size as src
 */
irf_status ir_filter_median(const void *src, size_t src_pitch, const uint8_t *mask,
                            size_t mask_pitch, void *dst, size_t dst_pitch, int width, int height,
                            irf_dtype dtype, int window, hipStream_t stream);

/*
 * ir_filter_run -- the whole FNR filter, `passes` times (Sections 3.3-3.4, 4).
 *   Detection and median replacement are fused in one kernel per pass; pairs of
 *   passes may run as one fused launch instead (ir_filter_set_fusion,
 *   ir_filter_resolve_fusion), with the same results and per-pass counts.
 *   passes               1..IRF_MAX_PASSES; pass i reads the output of pass i-1
 *   scratch, scratch_pitch  device frame of the same size and type, required when
 *                        passes >= 2 (intermediate passes alternate between it and
 *                        dst so that the last one lands in dst); ignored otherwise
 *   flagged_count        nullable device array of `passes` uint64: noisy pixels found
 *                        by each pass (zeroed on the stream, then accumulated); it
 *                        must not overlap src, dst or scratch (IRF_ERR_ALIAS)
 */
irf_status ir_filter_run(const void *src, size_t src_pitch, void *dst, size_t dst_pitch, int width,
                         int height, irf_dtype dtype, int window, int passes, void *scratch,
                         size_t scratch_pitch, uint64_t *flagged_count, hipStream_t stream);

/*
 * ir_filter_run_noalloc -- ir_filter_run for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same results and counts, with the intermediate frame of
 * passes >= 2 taken from a 32 MiB device array the library holds on each GPU
 * (declared statically, looked up once per device; nothing is allocated or
 * freed per call).  Limit: for passes >= 2, height * round_up(width * bytes
 * per pixel, 256) must not exceed 32 MiB (IRF_ERR_CAPACITY otherwise, checked
 * before any HIP call), e.g. 4096 x 4096 u16.  All calls on one GPU share the
 * array: calls that overlap in time on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.  Other arguments as for
 * ir_filter_run.
 */
irf_status ir_filter_run_noalloc(const void *src, size_t src_pitch, void *dst, size_t dst_pitch, int width,
                                 int height, irf_dtype dtype, int window, int passes, uint64_t *flagged_count,
                                 hipStream_t stream);

/*
 * ir_filter_run_frames -- ir_filter_run over a stack of `nframes` frames of the
 * same size, one launch per pass (or per fused pair of passes, as for
 * ir_filter_run).  Frame i starts at src + i*src_stride (bytes),
 * dst + i*dst_stride, scratch + i*scratch_stride.  Frames are filtered
 * independently; flagged_count[p] (nullable, `passes` entries) receives the
 * noisy pixels of pass p summed over all frames.
 */
irf_status ir_filter_run_frames(const void *src, size_t src_pitch, size_t src_stride, void *dst,
                                size_t dst_pitch, size_t dst_stride, int width, int height,
                                int nframes, irf_dtype dtype, int window, int passes, void *scratch,
                                size_t scratch_pitch, size_t scratch_stride,
                                uint64_t *flagged_count, hipStream_t stream);

/*
 * Batches of uneven frames (one persistent launch over all their tiles).
 *
 * irf_frame describes one frame: device src/dst, pitches, size, pixel type and
 * window; frames of a batch are independent and may all differ.  Every frame
 * is filtered once with the FNR filter (same result as ir_filter_run with
 * passes = 1).  Frames with windows 3..9 share one persistent kernel, frames
 * with windows 11..15 a second, and each window above 15x15 has a kernel of
 * its own; a batch launches the kernels of the windows it holds, one after the
 * other on the same stream (a batch of windows 3..9 is one launch).  With
 * IRF_PLAN_GRAPH the launches are replayed from a graph captured per set of
 * kernels on its first use.
 */
typedef struct {
    const void *src;
    void *dst;
    size_t src_pitch, dst_pitch;
    int width, height;
    irf_dtype dtype;
    int window;
} irf_frame;

typedef struct irf_plan irf_plan;

#define IRF_PLAN_GRAPH 1u /* replay the batch kernels from a captured hipGraph */

/*
 * ir_filter_plan_create -- allocate a plan for batches of at most max_frames
 * frames holding at most max_tiles tiles in total (a frame of W x H has
 * ceil(W/128) * ceil(H/TH) tiles, TH = 32 or 64 rows for batch workgroups of
 * 128 or 256 threads: the batch tuning in force when the plan is created, see
 * ir_filter_set_batch_threads).  The plan owns two sets of device tables
 * (frame descriptors, tile map, work queues) with pinned host staging, used
 * alternately by consecutive batches; it is not thread-safe.  Returns
 * IRF_ERR_NOMEM or IRF_ERR_HIP on failure (*plan is then NULL).
 */
irf_status ir_filter_plan_create(irf_plan **plan, int max_frames, int max_tiles, unsigned flags);

/*
 * ir_filter_run_batch -- filter n frames (1 <= n <= max_frames) on `stream`.
 *   frames          host array of n descriptors (read before the call returns)
 *   flagged_counts  nullable device array of n uint64: noisy pixels per frame
 *                   (zeroed on the stream, then accumulated)
 * Validation covers every frame as in ir_filter_run, and no frame's dst may
 * overlap any frame's src or dst (IRF_ERR_ALIAS); a batch over the plan's
 * capacity returns IRF_ERR_CAPACITY.  May block the host until the batch
 * submitted two calls earlier on this plan has finished copying its tables.
 */
irf_status ir_filter_run_batch(irf_plan *plan, const irf_frame *frames, int n,
                               uint64_t *flagged_counts, hipStream_t stream);

/* Release a plan (waits for its outstanding work).  NULL is ignored. */
void ir_filter_plan_destroy(irf_plan *plan);

/* Tiles of one frame as counted against the max_tiles of a plan created under
 * the current batch tuning. */
int ir_filter_frame_tiles(int width, int height);

/* Tiles of one frame as counted against this plan's max_tiles (0 for a NULL
 * plan or a size outside 1..IRF_MAX_DIM). */
int ir_filter_plan_frame_tiles(const irf_plan *plan, int width, int height);

/*
 * Serving: a continuous-batching request loop over frames in pinned host
 * memory (the batched FNR filter of ir_filter_run_batch, one pass per frame).
 * Not part of the paper's method; it serves its filter to a stream of
 * requests.
 *
 * Each step admits arrived requests while device memory allows (frames of a
 * registered video stream use that stream's resident device slots, kept for
 * the server's lifetime; other frames take two blocks from a bounded device
 * arena, released when their result has reached the host), copies them host
 * -> device with ONE copy kernel on a copy stream (it reads the pinned host
 * buffers through their device mappings; a buffer without one is copied with
 * a copy command), filters them with ONE batched launch on a compute stream,
 * and copies the results back with one copy kernel on a second copy stream,
 * events ordering the three (the two copy directions overlap).  Up to
 * max_inflight steps are on the device at once, so copies of one step overlap
 * the kernels of another.  A request completes when
 * its device -> host copy has finished; its latency is completion time minus
 * its arrival time, both on the server's clock (seconds since creation).
 *
 * irf_request: one frame.  host_src / host_dst are pinned host buffers
 * (hipHostMalloc, torch pin_memory) owned by the caller, which must keep them
 * until the request completes; pitches are in bytes; stream_id is a
 * registered stream or -1; arrival is on the server's clock, and a request is
 * not admitted before it.  The server is not thread-safe.
 */
typedef struct irf_server irf_server;

typedef struct {
    uint64_t id;
    const void *host_src;
    void *host_dst;
    size_t src_pitch, dst_pitch;
    int width, height;
    irf_dtype dtype;
    int window;
    int stream_id;
    double arrival;
} irf_request;

/* arena_bytes: device memory for one-off frames (two blocks of W*H*b each,
 * rounded to 4 KiB); max_batch_frames / max_batch_tiles: limits of one step;
 * max_inflight: steps on the device at once (1..8); flags: IRF_PLAN_GRAPH. */
irf_status ir_filter_server_create(irf_server **server, size_t arena_bytes, int max_batch_frames,
                                   int max_batch_tiles, int max_inflight, unsigned flags);

/* Give a video stream `depth` resident device slots (input + output) of its
 * frame size and type; a frame of the stream takes any free slot, so up to
 * `depth` consecutive frames of it can be in flight. */
irf_status ir_filter_server_register_stream(irf_server *server, int stream_id, int width, int height,
                                            irf_dtype dtype, int depth);

/* Queue n requests (descriptors are copied).  They must come in
 * non-decreasing arrival order, also across calls (IRF_ERR_DIMS otherwise);
 * each is validated as in ir_filter_run_batch and must fit the arena or its
 * stream's slots (IRF_ERR_CAPACITY otherwise: it could never be admitted). */
irf_status ir_filter_server_submit(irf_server *server, const irf_request *requests, int n);

/* One engine iteration: retire finished steps, then issue a new one if there
 * is room and arrived work fits.  Returns 1 on progress, 0 if none, or a
 * negative irf_status. */
int ir_filter_server_poll(irf_server *server);

/* Serve until every submitted request has completed (sleeps briefly while
 * waiting for arrivals or completions). */
irf_status ir_filter_server_run(irf_server *server);

/* Move up to max completions (request id, latency in seconds) out of the
 * server, oldest first; returns how many were written. */
int ir_filter_server_completed(irf_server *server, uint64_t *ids, double *latency_s, int max);

/* Seconds since the server was created (its clock), its step count, the
 * arena bytes held by requests in flight, and all frame memory the server
 * holds on the device: the arena plus every registered stream's resident
 * slots (2 * depth frames each, allocated at registration, outside the
 * arena). */
double ir_filter_server_now(const irf_server *server);
int ir_filter_server_steps(const irf_server *server);
size_t ir_filter_server_arena_used(const irf_server *server);
size_t ir_filter_server_resident_bytes(const irf_server *server);

/* Waits for outstanding steps, then releases every device and host resource.
 * NULL is ignored. */
void ir_filter_server_destroy(irf_server *server);

/*
 * Tuning.  Not part of the method: these choices change the speed of a call,
 * never its result (every combination computes the same order statistic and
 * is tested bit-exact against the same oracle).  The table is process-wide;
 * set it before launching (a launch reads its entry once, but a change while
 * other host threads launch has no defined order with their launches).
 *
 * Single-size entry points (ir_filter_detect / _median / _run / _run_frames):
 * per pixel type and window, the workgroup size (128 threads on tiles of
 * 128x32 pixels, or 256 threads on 128x64) and the selection algorithm:
 *   IRF_SELECT_NETWORK  forgetful selection networks, two windows per lane
 *                       (windows up to 15x15)
 *   IRF_SELECT_BISECT   grey-level bisection, one window per lane (up to 15x15)
 *   IRF_SELECT_GROUP    grey-level bisection, one window per group of 4, 8,
 *                       16 or 32 lanes (above 15x15; above 31x31 the only
 *                       choice, with 128 threads)
 *   IRF_SELECT_HIST     two-pass radix select over a 256-bin LDS histogram,
 *                       one window per group of 16 lanes (17x17 to 31x31)
 * Untuned defaults: 256 threads for 5x5, 7x7 and 17x17 to 31x31, else 128;
 * networks up to 15x15, group bisection above.
 * ir_filter_set_tuning(dtype, window, 0, 0)
 * restores the default; an unavailable combination returns IRF_ERR_TUNING.
 * The autotuner of the Python package measures the choices and sets them.
 */
typedef enum { IRF_SELECT_NETWORK = 1, IRF_SELECT_BISECT = 2, IRF_SELECT_GROUP = 3, IRF_SELECT_HIST = 4 } irf_select;

irf_status ir_filter_get_tuning(irf_dtype dtype, int window, int *threads, int *select);
irf_status ir_filter_set_tuning(irf_dtype dtype, int window, int threads, int select);

/* Fusion of passes (ir_filter_run / ir_filter_run_frames with passes >= 2;
 * Section 4 applies the filter twice).  With fusion on, each pair of passes
 * runs as one launch: a tile gets pass 1 in LDS and pass 2 reads those results
 * there, so the intermediate frame never goes to memory; an odd last pass
 * runs on its own.  Results and per-pass counts equal those of separate
 * passes exactly.  Per pixel type and window:
 *   threads  0         every pass is its own launch
 *            256, 512  fused, workgroups of that size (blocks of 128x64 or
 *                      128x128 pixels, of which 120 x (64 or 128 - window + 1)
 *                      are output; the rest is recomputed by neighbours)
 *            -1        automatic, the default: separate passes.  Both kernels
 *                      are bound by ALU work per covered pixel; the fused
 *                      tiling never covers fewer pixels than two single passes,
 *                      and at equal coverage separate passes measured faster
 *                      at every window up to 9x9.  The autotuner sets a fused
 *                      size where it measures one faster.
 * Fused kernels exist for windows up to 9x9 (IRF_ERR_TUNING otherwise; -1
 * and 0 are accepted for every window).  The table is process-wide like the
 * one above. */
irf_status ir_filter_get_fusion(irf_dtype dtype, int window, int *threads);
irf_status ir_filter_set_fusion(irf_dtype dtype, int window, int threads);

/* The choice ir_filter_run makes for two or more passes over a width x height
 * frame of this type and window under the current settings: 0 (separate
 * passes) or the fused workgroup size. */
irf_status ir_filter_resolve_fusion(irf_dtype dtype, int window, int width, int height, int *threads);

/* Batch workgroup size for plans created from now on: 128 (tiles of 128x32,
 * the default) or 256 (128x64); 0 restores the default.  Other values return
 * IRF_ERR_TUNING. */
irf_status ir_filter_set_batch_threads(int threads);
int ir_filter_get_batch_threads(void);

/* Human-readable name of a status code (static string, never NULL). */
const char *ir_filter_status_string(irf_status status);

/* Library ABI version: (major << 16) | minor. */
int ir_filter_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IRFILTER_H */
