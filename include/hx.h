/*
 * hx.h -- C ABI of libhx.so, an MI355X (gfx950) implementation of the EDGE
 * edge-detection pipeline evaluated in "Hercules: A Compiler for Productive
 * Programming of Heterogeneous Systems" (Evaluation: the EDGE benchmark;
 * Use and Impact of Schedules: EDGE's max_gradient reduction tree).
 *
 * The pipeline is nested parallel loops plus one associative reduction, as
 * the paper's fork-join statement of a program has them ("Representing
 * Parallelism with Fork-Joins"):
 *   fork over [H, W]:  B = Gaussian blur of I          (k x k, clamped)
 *   fork over [H, W]:  L = 5-point Laplacian of B
 *   fork over [H, W]:  Z = 3x3 zero crossing of L (1 where signs differ)
 *   fork over [H, W]:  G = Sobel magnitude of B
 *   reduce  (monoid max over [H, W]):  M = max G
 *   fork over [H, W]:  mask = Z and G > thresh_frac * M   (uint8, 0 or 1)
 * Every stage reads its input at clamped coordinates.  The batched call
 * adds an outer fork over images whose factors differ per image.
 *
 * Conventions (all entry points):
 *  - Every call returns an hx_status and never throws.  On any validation
 *    failure nothing is enqueued and the call returns HX_E_INVALID (or
 *    HX_E_UNSUPPORTED); hx_last_error() then describes the problem.
 *  - Pointers named d_* or inside hx_image are DEVICE pointers on the
 *    pipeline's device; h_* are host pointers.  The caller owns them and
 *    must keep them alive until the enqueued work on `stream` completes.
 *  - Work is enqueued on `stream` (0 = the null stream) and the call
 *    returns without waiting.  Device-side failures (a kernel that could
 *    not launch) return HX_E_HIP; asynchronous faults surface at the next
 *    call or synchronisation.
 *  - The input is never written.  Every output element is written.
 *  - Pipelines and servers are not thread-safe unless stated (hx_serve_*
 *    are thread-safe).  hx_last_error() is thread-local.
 *  - Inputs must be finite fp32; masks are written as 0 or 1.
 */
#ifndef HX_H
#define HX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same opaque type as the HIP runtime's; a repeated identical typedef is
 * valid C11 and C++. */
typedef struct ihipStream_t* hipStream_t;

typedef enum {
    HX_OK = 0,
    HX_E_INVALID = 1,      /* bad argument; nothing enqueued            */
    HX_E_NOMEM = 2,        /* device or pinned host allocation failed   */
    HX_E_HIP = 3,          /* a HIP runtime call failed                 */
    HX_E_UNSUPPORTED = 4,  /* valid request the library does not support */
    HX_E_BUSY = 5,         /* server: request would never fit budget    */
    HX_E_PENDING = 6,      /* server: ticket not finished yet           */
    HX_E_NOT_FOUND = 7     /* server: unknown or already-collected id   */
} hx_status;

typedef struct hx_pipeline hx_pipeline;
typedef struct hx_server hx_server;

/* Pass structure of the fused (fusion_depth 4) pipeline.  The max must be
 * known before any mask bit can be written, so the work splits in two:
 *  STORE:      pass 1 computes every stage and stores one float per pixel
 *              (G^2 where Z = 1, else -1) plus the max; pass 2 thresholds.
 *  RECOMPUTE:  pass 1 computes blur and Sobel only, for the max; pass 2
 *              recomputes every stage and writes the mask directly.
 *  SPECULATE:  pass 0 computes G^2 on sampled row bands (8 rows at the
 *              top of every min(clamp(H/32, 128, 256), max(H/4, 8))
 *              rows) for a lower
 *              bound m <= max G^2 of each image; pass 1 computes every
 *              stage once, writes the mask against the threshold of m (a
 *              pixel it leaves at 0 is 0 under the true max too) and lists
 *              the pixels it set, with their G^2; pass 2 re-decides only
 *              those against the true max.  Exact for every input; fast
 *              when the listed pixels are few.  Runs 256-column sweep
 *              tiles of 16..256 rows (a multiple of 8). */
enum { HX_PASS_AUTO = 0, HX_PASS_STORE = 1, HX_PASS_RECOMPUTE = 2,
       HX_PASS_SPECULATE = 3 };

/* Shape of the max reduction (the paper's reduction_tree schedule and its
 * warp-primitive refinement, Use and Impact of Schedules):
 *  TREE:        per-lane max, wave64 shuffle tree, one atomic per wave.
 *  TWO_LEVEL:   the reduction_tree schedule: 4096 threads each fold a
 *               strided chunk of the stored G^2 plane from the identity,
 *               then one thread combines their 4096 partial maxima
 *               serially (a two-level tree without wave primitives).
 *  SEQUENTIAL:  one thread per image scans every G value (no tree).
 * TWO_LEVEL and SEQUENTIAL exist for the ablation; they need
 * fusion_depth 1. */
enum { HX_REDUCE_TREE = 0, HX_REDUCE_TWO_LEVEL = 1, HX_REDUCE_SEQUENTIAL = 2 };

/* A schedule: the knobs the autotuner searches (the role of the paper's
 * fork-tile / fork-chunk / fusion / fission schedules).
 *  fusion_depth 1: one kernel per stage (blur, Laplacian, zero crossing,
 *                  Sobel + max, threshold); tile_w x tile_h is the pixel
 *                  tile of one 256-thread workgroup, tile_w in {16,32,64},
 *                  tile_h in {16,32}.
 *  fusion_depth 2: [blur, Sobel + max] [Laplacian, zero crossing] [threshold]
 *  fusion_depth 3: [blur, Sobel + max, Laplacian] [zero crossing] [threshold]
 *  fusion_depth 4: all stencil stages in one pass (see pass_mode).
 *  For depth 2..4 the first kernel is a register sweep: each wave64 owns a
 *  strip of tile_w input columns (64, 128 or 256: 1, 2 or 4 per lane) and
 *  walks tile_h rows (a multiple of 8 in 8..256) down it. */
typedef struct {
    int32_t tile_w, tile_h, fusion_depth, pass_mode, reduce_mode;
} hx_schedule;

/* Which call forms a pipeline holds scratch for (hx_params.forms; 0 means
 * all of them).  Each form's scratch is allocated once, at creation, sized
 * by max_pixels and max_images; a call of a form the pipeline was created
 * without returns HX_E_UNSUPPORTED and enqueues nothing.
 *  IMAGE:        per-image calls at fusion depth 4 (STORE / RECOMPUTE):
 *                one max slot and a pass-1 code plane (4 B per pixel).
 *  STAGES:       fusion depths 1-3, the stage hook, the reduction variants:
 *                B, L, G^2 and Z planes (13 B per pixel) and the tree's
 *                partial maxima.
 *  BATCH:        batched calls (and per-image SPECULATE): per batch context
 *                the max slots, bounds, descriptor table and its pinned
 *                staging copy, and the listed-pixel store of SPECULATE
 *                (1.25 B per pixel).
 *  BATCH_STORE:  batched calls with the STORE pass structure: per batch
 *                context a pass-1 code plane (4 B per pixel).
 *  SRAD:         hx_srad: its second plane, c plane and partial sums
 *                (shared with the STAGES planes when both are present). */
enum { HX_FORM_IMAGE = 1, HX_FORM_STAGES = 2, HX_FORM_BATCH = 4,
       HX_FORM_BATCH_STORE = 8, HX_FORM_SRAD = 16, HX_FORM_ALL = 31 };

/* Pipeline parameters: the constants of the computation plus the "dynamic
 * constants" (Collections and Dynamic Constants) that size every scratch
 * buffer once, at creation (Global Code Motion: allocation is hoisted out
 * of every call).  Zero fields take defaults: ksize 5, sigma 1.0,
 * thresh_frac 0.1, schedule from the autotuner cache or the built-in
 * default, max_pixels 2^25, max_images 1024, forms HX_FORM_ALL,
 * batch_contexts 4. */
typedef struct {
    int32_t ksize;            /* odd, 1..15; fused kernels need 3, 5 or 7 */
    float sigma;              /* > 0                                       */
    float thresh_frac;        /* theta in tau = theta * M, in [0, 1]       */
    int32_t tile_w, tile_h, fusion_depth, pass_mode;  /* 0 = automatic    */
    int64_t max_pixels;       /* max sum of H*W over one call            */
    int64_t max_images;       /* max images in one batched call          */
    int32_t forms;            /* HX_FORM_* bits; 0 = HX_FORM_ALL          */
    int32_t batch_contexts;   /* batched calls in flight at once, 1..8    */
} hx_params;

/* One image: device pointers.  src is H rows of `width` fp32 values with a
 * row pitch of src_pitch elements (>= width); mask is H rows of `width`
 * bytes with a row pitch of mask_pitch bytes (>= width). */
typedef struct {
    const float* src;
    int64_t height, width, src_pitch;
    uint8_t* mask;
    int64_t mask_pitch;
} hx_image;

/* Create a pipeline on `device`.  Allocates ALL of its scratch, for the
 * forms in params->forms, sized by max_pixels and max_images (the sizes
 * per form are listed with HX_FORM_*; hx_pipeline_memory reports the
 * totals).  No later call on the pipeline allocates or frees device or
 * pinned host memory.  Per-image planes hold H * round_up(W, 4) <=
 * max_pixels + 3 * 65536 elements, so an image taller than 65536 rows and
 * narrower than 4 columns may not fit them (HX_E_UNSUPPORTED).
 * Returns HX_E_INVALID for bad parameters, HX_E_NOMEM / HX_E_HIP on
 * allocation or device errors.  *out is set only on HX_OK. */
hx_status hx_pipeline_create(const hx_params* params, int device,
                             hx_pipeline** out);

/* The pipeline's own memory: device bytes and pinned host bytes it holds
 * (all allocated by hx_pipeline_create), and the number of allocation
 * calls (device or pinned) it has made since creation -- constant after
 * hx_pipeline_create returns, which tests use to check that no call path
 * allocates.  Any pointer may be NULL. */
hx_status hx_pipeline_memory(const hx_pipeline* p, size_t* device_bytes,
                             size_t* pinned_bytes, uint64_t* allocations);

/* Wait for the pipeline's outstanding work, release its memory.  NULL is a
 * no-op. */
void hx_pipeline_destroy(hx_pipeline* p);

/* Wait until every call enqueued on this pipeline has finished (the whole
 * device is synchronised).  Returns HX_E_HIP if the device reported an
 * error. */
hx_status hx_pipeline_sync(hx_pipeline* p);

/* Timing mode, for benchmarks.  While enabled, batched calls launch their
 * kernels (reset, [pass 0,] pass 1, pass 2) directly instead of through the
 * graph and bracket each with HIP events on the call's stream.
 * hx_pipeline_last_timing waits for the last batched call and returns the
 * durations in milliseconds of its kernels in ms[0..3]: reset, pass 1,
 * pass 2, and pass 0 (SPECULATE only, 0 otherwise; it runs between the
 * reset and pass 1).  HX_E_INVALID if no batched call ran in timing mode. */
hx_status hx_pipeline_set_timing(hx_pipeline* p, int enable);
hx_status hx_pipeline_last_timing(hx_pipeline* p, float* ms);

/* The scheduling language.  A schedule is a list of transformations of the
 * EDGE fork-joins (labels blur, laplacian, zero_cross, sobel, max_gradient,
 * threshold; each initially its own kernel, max_gradient a sequential
 * reduction), in the manner of the Juno scheduling language (The Juno
 * Scheduling Language; the reduction_tree macro of Use and Impact of
 * Schedules), each statement ending with ';':
 *   fork-tile[rows, cols](labels);      fork-fuse(labels);
 *   fork-chunk[N](max_gradient);        fork-reshape(max_gradient);
 *   monoid-reassociate(max_gradient);   fork-fission(max_gradient);
 *   reduction_tree![N](max_gradient);   (the four steps above)
 *   warp-reduce(max_gradient);          (wave64 primitives + one atomic
 *                                        per wave)
 *   pass[store|recompute|speculate](threshold);
 * hx_schedule_compile applies them and lowers the result onto the kernels
 * that exist: HX_OK and *out set, HX_E_INVALID for text that does not
 * parse or a transformation that does not apply (e.g. fission of an
 * unchunked reduction), HX_E_UNSUPPORTED for a program no kernel
 * implements (e.g. fusing blur with laplacian only); hx_last_error says
 * which statement and why.  Tile values are checked later, by
 * hx_pipeline_set_schedule.  Needs no device.
 * hx_schedule_to_text writes the canonical text of a schedule (NUL-
 * terminated, at most len bytes; HX_E_INVALID if it does not fit). */
hx_status hx_schedule_compile(const char* text, hx_schedule* out);
hx_status hx_schedule_to_text(const hx_schedule* s, char* buf, size_t len);

/* Force a schedule for every later call (NULL restores automatic choice:
 * the autotuned schedule of the image's shape class if there is one, else
 * fusion depth 4, STORE, 256-column tiles of the tallest of 64, 32 or 16
 * rows that gives every SIMD a tile, and fusion depth 1 with 64 x 16
 * tiles for a blur size the sweeps do not cover).
 * HX_E_INVALID for knob values outside the sets documented above,
 * HX_E_UNSUPPORTED for a fused depth with ksize not in {3,5,7}. */
hx_status hx_pipeline_set_schedule(hx_pipeline* p, const hx_schedule* s);

/* The schedule a call on an H x W image would use right now. */
hx_status hx_pipeline_get_schedule(const hx_pipeline* p, int64_t height,
                                   int64_t width, hx_schedule* out);

/* One image, the per-image form: a handful of kernel launches on `stream`.
 * d_max (device, nullable) receives M = max G as one float.  Per-image
 * calls share one set of the pipeline's scratch: a call on a different
 * stream from the previous per-image call (hx_edge_detect,
 * hx_edge_detect_stages, hx_srad) first makes its stream wait for that
 * call's work, so calls on several streams are correct but do not
 * overlap.  (SPECULATE per-image calls use the batch contexts instead.) */
hx_status hx_edge_detect(hx_pipeline* p, const hx_image* img, float* d_max,
                         hipStream_t stream);

/* n images of any sizes in one launch sequence: [a reset of the per-image
 * max slots | SPECULATE's pass 0], then one kernel over the flattened list
 * of (image, tile) pass-1 items, then one over the pass-2 items.  No
 * workgroup waits on another; the kernel boundary makes each image's max
 * final before its mask is written.  A batch that a batch context already
 * ran (same descriptors, outputs and pass structure) replays its captured
 * HIP graph.  imgs is a HOST array of n descriptors (device pointers
 * inside); it is copied before the call returns.  d_max (device,
 * nullable) receives n floats.  Requires 1 <= n <= max_images and
 * sum H*W <= max_pixels.  Each image's result is bit-identical to
 * hx_edge_detect on it alone.  Batched calls use one of batch_contexts
 * scratch sets each, so calls on different streams overlap; a call whose
 * context is still in use waits (on the host) for it.  A batch with more
 * tiles than a context's descriptor table holds (only possible with many
 * images a few pixels wide or tall) runs as several launches in turn. */
hx_status hx_edge_detect_batched(hx_pipeline* p, const hx_image* imgs,
                                 int32_t n, float* d_max, hipStream_t stream);

/* For callers that cannot allocate -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation: hx_edge_detect in the
 * fused STORE form (one sweep writes a code per pixel and the max, a second
 * kernel thresholds), with its scratch -- the max slot and the pass-1 code
 * plane -- in one fixed device array of HX_STATIC_SCRATCH_BYTES instead of
 * the pipeline's buffers.  The call allocates and frees nothing (the
 * array's device address is looked up once per device, when a pipeline is
 * created on it).  Each GPU holds its own array for the life of the
 * process, and every call on that GPU shares it and leaves the last call's
 * contents there: calls that overlap on one GPU (on different streams, or
 * from different host threads) race and give undefined masks; calls on one
 * stream are ordered.  HX_E_INVALID if the image needs more than
 * HX_STATIC_MAX_ELEMS code elements (H * round_up(W, 4)) or fails the
 * argument checks of hx_edge_detect; HX_E_UNSUPPORTED for a ksize other
 * than 3, 5, 7.  The result is bit-identical to hx_edge_detect's. */
#define HX_STATIC_MAX_ELEMS ((size_t)8 << 20)
#define HX_STATIC_SCRATCH_BYTES (256 + 4 * HX_STATIC_MAX_ELEMS)
hx_status hx_edge_detect_static(hx_pipeline* p, const hx_image* img, float* d_max,
                                hipStream_t stream);

/* Test hook: the per-image pipeline at fusion depth 1 (or at the depth 1, 2
 * or 3 of a forced schedule) on one image, with every stage it keeps in
 * memory written out.  d_B, d_L, d_G: dense H*W floats (G is the
 * magnitude); d_Z: dense H*W bytes; d_max: one float (M); the mask goes to
 * img->mask.  Any of d_B, d_L, d_Z, d_G may be NULL; depth 2 keeps L on
 * chip and depth 3 keeps B on chip, so d_L (depth 2) / d_B (depth 3) must
 * be NULL there (HX_E_UNSUPPORTED otherwise). */
hx_status hx_edge_detect_stages(hx_pipeline* p, const hx_image* img,
                                float* d_B, float* d_L, uint8_t* d_Z,
                                float* d_G, float* d_max, hipStream_t stream);

/* Time every candidate schedule on a synthetic H x W image on this
 * pipeline's device (blocking; allocates and frees its own test image),
 * keep the fastest for that shape class, and append it to the JSON-lines
 * cache at cache_path (NULL = do not persist), after one {"trial": ...}
 * line per measured candidate (its schedule and best-of-three ms; the
 * loader skips those).  Later calls on images of the same shape class use
 * the chosen schedule unless a schedule is forced. */
hx_status hx_autotune(hx_pipeline* p, int64_t height, int64_t width,
                      const char* cache_path);

/* The batch autotuner: times the batched call on the caller's batch (imgs,
 * n: as hx_edge_detect_batched; their masks are written, with the same
 * bits as any schedule gives) under every candidate -- sweep tile heights
 * 16..160 rows x pass structures SPECULATE, RECOMPUTE and, when the
 * pipeline holds HX_FORM_BATCH_STORE, STORE -- and keeps the one with the
 * highest throughput for the batch's class (floor(log2) of its total
 * pixels and of n): the time per call with batch_contexts calls in flight
 * on as many streams of the tuner's own (median of three runs of
 * 12 calls per stream, after about 30 ms of warm-up calls; the time of
 * one call alone, median of five, is recorded beside it).  Later batched calls of that class use the choice
 * unless the pass structure is fixed or a schedule forced.  The calls in
 * flight all write the caller's masks, with the same bits, so on return
 * they hold the batch's result.  Blocking.  Appends one
 * {"batch_trial": ...} line per candidate and the chosen {"batch": ...}
 * line to cache_path (NULL = do not persist); *tile_h and *pass_mode
 * (nullable) receive the choice. */
hx_status hx_autotune_batch(hx_pipeline* p, const hx_image* imgs, int32_t n,
                            const char* cache_path, int32_t* tile_h, int32_t* pass_mode);

/* Load schedules from a cache written by hx_autotune or hx_autotune_batch
 * (entries for other ksize values are ignored). */
hx_status hx_autotune_load(hx_pipeline* p, const char* cache_path);

/* --------------------------------------------------------------- SRAD --
 * The second workload (Evaluation; Use and Impact of Schedules): niter
 * iterations of speckle reducing anisotropic diffusion on the fp32 image
 * d_J (device, height x width, row pitch `pitch` elements), in place.  Per
 * iteration, with the whole image as the region of interest and clamped
 * neighbours: q0^2 = var(J) / mean(J)^2 (sums in fp64 over a three-level
 * tree: lane, wave64 shuffles + the workgroup's waves, all workgroups'
 * pairs folded at the start of the next kernel); c = 1 / (1 + (q^2 -
 * q0^2) / (q0^2 (1 + q0^2))) clamped to [0, 1] (1 when q0^2 <= 0), q^2
 * from the pixel's four differences; J += lambda/4 (c dN + c_S dS + c dW
 * + c_E dE).  fused != 0 computes c in registers one row ahead of the
 * update (one kernel per iteration, 8 B/px of HBM traffic) instead of
 * writing and re-reading a c plane (two kernels, 20 B/px); both forms
 * give the same bits.  d_q0sqr (device, nullable)
 * receives the niter values of q0^2.  Inputs must be finite and > 0.
 * HX_E_INVALID for a NULL pipeline or image, a bad shape or pitch, more
 * than max_pixels pixels, niter < 0 or lambda outside [0, 4]; nothing is
 * enqueued then.  Scratch (a second plane, the c plane of the unfused
 * form, the partial sums) is owned by the pipeline. */
hx_status hx_srad(hx_pipeline* p, float* d_J, int64_t height, int64_t width,
                  int64_t pitch, int32_t niter, float lambda, int32_t fused,
                  double* d_q0sqr, hipStream_t stream);

/* ------------------------------------------------------------ serving --
 * A request loop with continuous batching.  Requests are admitted while
 * their device buffers fit in the HBM budget, copied to the device, and
 * every admitted request not yet launched joins the next batch; batches
 * run on `streams` round-robin compute streams so they overlap on the
 * device.  All hx_serve_* calls are thread-safe. */
typedef struct {
    size_t hbm_budget;     /* bytes of arena a request set may occupy     */
    int32_t streams;       /* concurrent compute streams (1..8)           */
    int32_t max_batch;     /* images per launched batch (<= max_images)   */
} hx_serve_params;

/* d_arena/arena_bytes: one caller-owned device allocation (e.g. a torch
 * uint8 tensor) that the server sub-allocates request buffers from.  The
 * pipeline's own scratch (hx_pipeline_memory) counts against the budget:
 * request buffers may occupy at most min(hbm_budget - pipeline device
 * bytes, arena_bytes); HX_E_INVALID if the budget does not exceed the
 * pipeline's scratch, HX_E_UNSUPPORTED if the pipeline lacks
 * HX_FORM_BATCH.  The server owns a scheduler thread and its streams; the
 * pipeline must outlive it and must not be used by anyone else meanwhile. */
hx_status hx_serve_create(hx_pipeline* p, const hx_serve_params* sp,
                          void* d_arena, size_t arena_bytes, hx_server** out);

/* Enqueue one request.  h_src: host fp32 image, h rows of w values, row
 * pitch `pitch` elements; it is copied (into the server's pinned pool)
 * before the call returns.  arrival_s: the request's scheduled arrival time
 * on the server's clock (hx_serve_now), used for latency.  Never blocks:
 * HX_E_PENDING if the pinned pool has no room right now (it fills with
 * finished requests until they are collected: poll, then submit again),
 * HX_E_BUSY if the request alone can never fit the budget. */
hx_status hx_serve_submit(hx_server* s, const float* h_src, int64_t h,
                          int64_t w, int64_t pitch, double arrival_s,
                          uint64_t* ticket);

/* Collect a finished request: copies its mask into h_mask (row pitch
 * mask_pitch bytes) and its latency (completion minus arrival, seconds)
 * into *latency_s (nullable).  HX_OK done (the ticket is then released),
 * HX_E_PENDING not yet, HX_E_NOT_FOUND unknown ticket, HX_E_HIP if the
 * server hit a device error. */
hx_status hx_serve_poll(hx_server* s, uint64_t ticket, uint8_t* h_mask,
                        int64_t mask_pitch, double* latency_s);

/* hx_serve_poll, also giving the request's service time (nullable): from
 * the launch of its batch (copy-in enqueued) until its mask is on the host,
 * i.e. the latency without the wait for admission and for a free stream. */
hx_status hx_serve_poll_timed(hx_server* s, uint64_t ticket, uint8_t* h_mask,
                              int64_t mask_pitch, double* latency_s,
                              double* service_s);

/* Zero-copy submission, for callers that produce the request image
 * themselves (a decoder, a camera ring): hx_serve_reserve takes room for
 * an h x w request in the server's pinned pool and returns it in *h_slot
 * (h rows of w fp32 values, row pitch w, 256-byte aligned); the caller
 * writes the image there and queues it with hx_serve_commit (arrival_s as
 * for submit), which copies nothing.  The slot is the caller's between the
 * two calls; hx_serve_cancel gives an uncommitted slot back.  Errors as for
 * submit (HX_E_PENDING: pool full, HX_E_BUSY: never fits); commit and
 * cancel return HX_E_NOT_FOUND for an unknown ticket and HX_E_INVALID for
 * one that is not a reserved slot. */
hx_status hx_serve_reserve(hx_server* s, int64_t h, int64_t w, float** h_slot,
                           uint64_t* ticket);
hx_status hx_serve_commit(hx_server* s, uint64_t ticket, double arrival_s);
hx_status hx_serve_cancel(hx_server* s, uint64_t ticket);

/* Zero-copy collection: once a request is done, *h_mask points at its mask
 * in the pinned pool (h rows of w bytes, row pitch w) and the latency and
 * service time are returned as by poll_timed (nullable); the mask stays
 * there, and the pool room held, until hx_serve_release.  HX_E_PENDING
 * while not done; errors otherwise as for poll.  (hx_serve_poll copies the
 * mask out and releases in one call.) */
hx_status hx_serve_view(hx_server* s, uint64_t ticket, const uint8_t** h_mask,
                        double* latency_s, double* service_s);
hx_status hx_serve_release(hx_server* s, uint64_t ticket);

/* Seconds on the server's monotonic clock. */
double hx_serve_now(const hx_server* s);

/* Counters since creation: requests completed, batches launched, pixels
 * processed, peak arena bytes in use.  Any pointer may be NULL. */
hx_status hx_serve_stats(const hx_server* s, uint64_t* completed,
                         uint64_t* batches, uint64_t* pixels,
                         uint64_t* peak_bytes);

/* Drain every admitted request, stop the scheduler, free the server. */
hx_status hx_serve_destroy(hx_server* s);

/* ------------------------------------------------------------ errors --- */
/* hx_status_str: the status's name.  hx_last_error: the text of the last
 * failure on the calling thread.  Diagnostics, read from the environment
 * once per process: HX_LOG=1 prints to stderr every failing call with its
 * text, pipeline and server creation (sizes, bytes), each batched call's
 * schedule (images, pixels, pass structure, tile height and its source,
 * context, groups) and the batch autotuner's trials; HX_LOG=2 adds each
 * per-image call's schedule, each batch's launch form (graph replay,
 * capture, direct) and each serving batch.  HX_TRACE=1 brackets API calls
 * and batch phases in roctx ranges (rocprofv3 --marker-trace). */
const char* hx_status_str(hx_status s);
const char* hx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HX_H */
