/*
 * recon.h -- C ABI of librecon: grayscale morphological reconstruction by
 * dilation and by erosion and the operations built on it (fill-holes, h-dome,
 * regional maxima), connected-component labelling with the area filter, and
 * the exact distance transform with the Pre-Watershed markers, on uint8 image
 * tiles, for AMD Instinct MI355X (gfx950).
 *
 * What is computed
 * ----------------
 * Morphological reconstruction (MR) is the operation the paper's nucleus
 * segmentation stage is built on: Table 1 (Sec. V-A), which lists where the
 * CPU and GPU versions of each segmentation and feature operation come from,
 * marks ReconToNuclei, FillHoles, Pre-Watershed and RBC detection as MR-based,
 * and the paragraph that follows it describes MR as an irregular
 * wave-propagation computation.  The reconstruction of a mask I
 * from a marker J is the fixed point of J <- min(dilate(J), I) started from
 * min(J, I), where dilate is the flat dilation over the 4- or 8-neighbourhood
 * (pixels outside the image do not exist).  The result is unique, so every
 * entry point below returns identical bytes for every tuning, batch
 * composition and arrival order.
 *
 * Fill-holes (the FillHoles operation of Table 1) is the reconstruction of the
 * complement: F = 255 - rho_{255-X}(m), with m = 255 - X on the one-pixel
 * image frame and 0 elsewhere; `conn` is the connectivity of that
 * reconstruction, i.e. of the background.
 *
 * The MR-based operations of Table 1 (ReconToNuclei, RBC detection,
 * Pre-Watershed) follow Vincent's grayscale reconstruction, which also defines
 * the dual and the derived transforms provided here:
 * * reconstruction by erosion rho^e_I(J): the fixed point of
 *   J <- max(erode(J), I) started from max(J, I) (erode: flat erosion over the
 *   same neighbourhood); computed as 255 - rho_{255-I}(255 - J);
 * * the h-dome D_h(I) = I - rho_I(max(I - h, 0)), 1 <= h <= 255;
 * * the regional maxima of I: 255 where D_1(I) > 0, else 0 (a plateau of
 *   value 0 is never one).
 *
 * BWLabel and AreaThreshold (Table 1) are provided too: the connected
 * components of the nonzero pixels (4- or 8-connectivity, pixels outside the
 * image absent), labelled 1..n in raster order of each component's first
 * pixel (0 on the background), and the filter keeping the components whose
 * pixel count lies in [min_area, max_area].
 *
 * Pre-Watershed (Table 1: reconstruction and a distance transformation) is
 * provided as the exact Euclidean distance transform -- dist2(p) = min over
 * the 0 pixels q of |p - q|^2, pixels outside the image not background,
 * 2^31 - 1 without any 0 pixel -- and the markers it feeds to the watershed:
 * the regional maxima of D8 = min(floor(sqrt(dist2)), 255).
 *
 * Conventions
 * -----------
 * * Images are single-channel uint8, row-major, `pitch` bytes between rows
 *   (pitch >= width).  `data` is a DEVICE pointer on the context's GPU.  The
 *   caller owns every image buffer; the library never allocates or frees
 *   them, and they must stay valid until the work on `stream` (or the
 *   ticket) has completed.
 * * Results are written in place: into the marker (recon_dilate,
 *   recon_erode) or the image (recon_fill_holes, recon_hdome,
 *   recon_regional_max, recon_area_threshold, recon_pre_watershed); labels
 *   and distances go into an int32 plane the caller passes (recon_label,
 *   recon_distance).  The marker and the mask must not overlap, nor an int32
 *   plane and its image.
 * * `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   device work is enqueued asynchronously on it; the call returns once the
 *   work is enqueued.
 * * Return values are recon_status codes; no exception crosses the ABI.
 *   Argument errors are detected synchronously, before anything is enqueued.
 *   Device errors are reported by the call that observes them (the next call,
 *   recon_poll or recon_wait).  recon_last_error() gives the message of the
 *   last failure on the calling thread.
 * * A context may be used from one host thread at a time, and its calls are
 *   ordered on the streams they name; calls on different streams that
 *   overlap in time share the context's workspace and must not be issued
 *   concurrently.
 * * Several contexts on one GPU may run launches at the same time (the
 *   serving lanes run up to three).  With four to eight contexts running
 *   4096 x 4096 reconstructions, labellings and distance transforms side by
 *   side, a few runs had a launch given up by its scheduler watchdog or
 *   results that differed, for a cause not found; a caller doing so should
 *   check every launch's outcome (recon_last_stats, recon_enqueue_status).
 */
#ifndef RECON_H
#define RECON_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RECON_OK = 0,
    RECON_EINVAL = -1,     /* bad argument (null pointer, conn, shape, pitch, overlap) */
    RECON_ENOMEM = -2,     /* device or host allocation failed */
    RECON_EDEVICE = -3,    /* HIP runtime or kernel error */
    RECON_EAGAIN = -4,     /* serving admission full: retry after polling */
    RECON_ETIMEDOUT = -5   /* recon_wait timed out; the work is still in flight */
} recon_status;

enum {
    RECON_OP_DILATE = 0,
    RECON_OP_FILL_HOLES = 1,
    RECON_OP_ERODE = 2,
    RECON_OP_HDOME = 3,
    RECON_OP_REGIONAL_MAX = 4
};

typedef struct recon_ctx recon_ctx;

/* One uint8 image: device pointer, shape, and row pitch in bytes. */
typedef struct {
    uint8_t *data;
    int32_t height;
    int32_t width;
    int64_t pitch;
} recon_image;

/* One unit of work for recon_batch / recon_submit.
 * op == RECON_OP_DILATE:       image = marker (in: J, out: rho_mask(J)), mask = I.
 * op == RECON_OP_FILL_HOLES:   image = X (in: X, out: filled), mask ignored.
 * op == RECON_OP_ERODE:        image = marker (in: J, out: rho^e_mask(J)), mask = I.
 * op == RECON_OP_HDOME:        image = I (in: I, out: D_h(I)), h = the height, mask ignored.
 * op == RECON_OP_REGIONAL_MAX: image = I (in: I, out: 0 / 255), mask ignored.
 * Fill-holes, h-dome and regional maxima hold their marker in a scratch plane
 * of the context (width rounded up to 4, times height bytes). */
typedef struct {
    int32_t op;
    int32_t conn;          /* 4 or 8 */
    recon_image image;
    recon_image mask;
    int32_t scan_rounds;   /* per-task tuning: directional pass rounds (0 = context default,
                              -1 = none, 1..8) */
    int32_t queue_capacity;/* per-task tuning: LDS queue entries, a power of two (0 = context
                              default; at most the context's queue_capacity) */
    int32_t h;             /* RECON_OP_HDOME: dome height 1..255; ignored by the others */
    int32_t block_rows;    /* per-task tuning: rows of the task's work blocks, 16, 32 or 64
                              (0 = the context's block_rows); honoured by recon_batch, while
                              the serving loop runs every request at the context's */
} recon_task;

/* Tuning and capacity knobs; zero fields take the defaults. */
typedef struct {
    int32_t block_rows;        /* rows per work block: 16, 32 or 64 (default 32) */
    int32_t queue_capacity;    /* LDS queue entries per workgroup: a power of two in 64..8192 */
    int32_t scan_rounds;       /* directional pass rounds on a block's first visit,
                                  1..8; 0 = default (3); -1 = none */
    int32_t wg_per_cu;         /* cap on resident workgroups per CU (0 = occupancy limit) */
    int64_t serve_mem_cap;     /* serving admission cap in device bytes (default 64 GiB) */
    int32_t serve_slots;       /* serving in-flight task slots (default 256) */
    int32_t stop_after_stage;  /* 0 = the persistent pipeline (default).  Test hooks that run
                                  the staged pipeline instead (dense pass, border seeding and
                                  revisits as separate kernels): 1 = stop after the dense
                                  per-block pass (each block reconstructed on its own);
                                  2 = also seed the border requests, but do not drain them;
                                  3 = run the staged pipeline to the end */
    int32_t timing;            /* 1: record HIP events between the kernels of each launch so
                                  that recon_last_stats reports per-kernel durations */
    int32_t drain_budget;      /* queue rounds a revisit drains before a round of sweeps takes
                                  over (1..4096; 0 = default 128) */
    int32_t binary_drain_budget; /* the same for blocks whose mask is binary (0 / 255 only),
                                  where a raise floods whole regions (1..4096; 0 = default 4) */
    int32_t test_fault;        /* test hook, 0 in production: 1 = every compare-and-swap that
                                  claims a block is made to fail, so that launches give up
                                  (their calls then report RECON_EDEVICE) */
    int32_t component_route;   /* The component route: a task whose mask takes at most two
                                  values, 0 and one c > 0 (a binary mask; fill-holes of a binary
                                  image), can be reconstructed through connected-component
                                  labelling: the result is then, on each component of the
                                  nonzero mask pixels, the largest min(marker, mask) over that
                                  component, and 0 elsewhere -- the same bytes, without the
                                  chains of block visits a long corridor causes.  0 (default):
                                  taken where it pays -- the foreground is thin (short runs:
                                  corridors, noise), or the launch has no grey task whose block
                                  visits the two-valued task's visits would overlap with.
                                  1: taken by every two-valued mask.  -1: never.  With 0 or 1
                                  each task holds an int32 label plane in the context's
                                  scratch area (4 bytes per pixel). */
    int32_t spill_capacity;    /* entries of each revisit wave's global spill queue, the level
                                  under its LDS queue: pushes that do not fit the LDS queue go
                                  there and are drained back when it runs empty; only when both
                                  are full does the block re-seed.  0 = default 8192 (64..65536;
                                  16 MiB per 1024 entries of the context's workspace), -1 = none */
    int32_t reserved[1];
} recon_config;

/* Per-call statistics of the last completed launch (for tests and tuning). */
typedef struct {
    int64_t dense_visits;      /* first visits of work blocks */
    int64_t revisits;          /* later visits triggered by neighbour changes */
    int64_t reruns;            /* in-place re-runs of a block re-requested while running */
    int64_t queue_overflows;   /* queue overflows, LDS queue and spill queue both full (each
                                  followed by a re-seed pass) */
    int64_t requests;          /* block revisits requested by border checks */
    int64_t aborted;           /* 1 if the scheduler watchdog stopped the launch */
    /* with recon_config.timing: durations in ms of the dense pass (K1), the border
       seeding (K2), the revisit drain (K3) and the whole launch (scheduler reset
       and marker preparation to result mapping); else 0.  A
       batch replayed from a captured graph is timed as a whole: the three
       kernel durations are then -1 */
    float dense_ms, seed_ms, drain_ms, total_ms;
    int64_t component_tasks;   /* tasks reconstructed by the component route (see recon_config) */
    float route_ms;            /* with recon_config.timing: duration in ms from the start of
                                  the launch to the end of the component route's kernels
                                  (scheduler reset and sampling, classification, labelling,
                                  maxima; they run beside the revisit drain), -1 for a
                                  replayed graph, 0 when the route is off */
    float reserved_f;
    int64_t queue_spills;      /* queue entries pushed to the global spill queues */
} recon_stats;

/* Create a context on HIP device `device`.  cfg may be NULL.  Runs a small
 * self-test kernel (with a 20 s deadline) and fails with RECON_EDEVICE if the
 * library's device code does not run on this device. */
int recon_create(recon_ctx **out, int device, const recon_config *cfg);
/* Destroy a context after all its work has completed. */
int recon_destroy(recon_ctx *ctx);

/* Reconstruction by dilation of `mask` from `marker`, in place on marker.
 * Shapes must match; conn is 4 or 8.  Enqueued on `stream`. */
int recon_dilate(recon_ctx *ctx, recon_image *marker, const recon_image *mask, int conn,
                 void *stream);

/* recon_dilate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same reconstruction, identical bytes, with the block scheduler's workspace
 * (counters, one state word per block, the visit ring) in a fixed device array
 * of the library (about 1.8 MB, held by every GPU the library runs on until
 * the process ends) instead of the context's allocations.  This call issues
 * no device or host allocation.  Limit: the image may have at most 8192
 * blocks of block_rows x 256 pixels (a 4096 x 4096 image at block_rows 16 or
 * more, 8192 x 8192 at 32 or more); larger images return RECON_EINVAL.  The
 * context must run the persistent pipeline (stop_after_stage 0).  The fixed
 * array is shared by every call on that GPU, from any context or thread, and
 * keeps the last call's contents (each call resets what it uses): calls whose
 * work overlaps in time on one GPU race and give wrong results, so order them
 * on one stream or synchronise between them.  recon_last_stats reports the
 * call's statistics until the next call on the device.  Enqueued on `stream`. */
int recon_dilate_noalloc(recon_ctx *ctx, recon_image *marker, const recon_image *mask, int conn,
                         void *stream);

/* Fill-holes of `img`, in place.  conn (4 or 8) is the background
 * connectivity.  Enqueued on `stream`. */
int recon_fill_holes(recon_ctx *ctx, recon_image *img, int conn, void *stream);

/* Reconstruction by erosion of `mask` from `marker`, in place on marker:
 * the fixed point of J <- max(erode(J), mask) from max(marker, mask).  Shapes
 * must match and the two must not overlap; conn is 4 or 8.  The marker is
 * complemented in place while the work runs (it holds 255 - J in between).
 * Enqueued on `stream`. */
int recon_erode(recon_ctx *ctx, recon_image *marker, const recon_image *mask, int conn,
                void *stream);

/* h-dome of `img`, in place: img <- img - rho_img(max(img - h, 0)), with h in
 * 1..255 (RECON_EINVAL otherwise).  conn is 4 or 8.  Enqueued on `stream`. */
int recon_hdome(recon_ctx *ctx, recon_image *img, int h, int conn, void *stream);

/* Regional maxima of `img`, in place: 255 where the 1-dome is positive (the
 * pixel belongs to a connected plateau with no higher neighbour, of value
 * > 0), else 0.  conn is 4 or 8.  Enqueued on `stream`. */
int recon_regional_max(recon_ctx *ctx, recon_image *img, int conn, void *stream);

/* Connected-component labelling (BWLabel) of `img` (nonzero = foreground):
 * labels[y * label_pitch + x] <- the label of pixel (y, x): 1..n in raster
 * order of each component's first pixel, 0 on the background.  `labels` is a
 * DEVICE int32 plane of height rows and label_pitch >= width elements per row,
 * owned by the caller and used as the union-find workspace while the work
 * runs; it must not overlap the image; height * label_pitch must stay below
 * 2^31.  conn (4 or 8) is the
 * foreground connectivity.  If `count` (a DEVICE int32) is not NULL it
 * receives n.  The image is not written.  Enqueued on `stream`. */
int recon_label(recon_ctx *ctx, const recon_image *img, int32_t *labels, int64_t label_pitch, int conn,
                int32_t *count, void *stream);

/* Area filter (AreaThreshold) of `img`, in place: 255 on the pixels of the
 * components (of the nonzero pixels, connectivity conn) whose pixel count lies
 * in [min_area, max_area] (inclusive; 0 <= min_area <= max_area), 0
 * elsewhere.  Uses a context scratch area of about 8 bytes per pixel.
 * Enqueued on `stream`. */
int recon_area_threshold(recon_ctx *ctx, recon_image *img, int conn, int64_t min_area, int64_t max_area,
                         void *stream);

/* Exact squared Euclidean distance transform of `img`: dist2[y * dist_pitch
 * + x] <- the squared distance from (y, x) to the nearest 0 pixel of the image
 * (0 on 0 pixels; 2^31 - 1 if the image has no 0 pixel).  `dist2` is a DEVICE
 * int32 plane (dist_pitch >= width elements per row) owned by the caller,
 * not overlapping the image; height and width at most 16384.  Enqueued on `stream`. */
int recon_distance(recon_ctx *ctx, const recon_image *img, int32_t *dist2, int64_t dist_pitch, void *stream);

/* Pre-Watershed markers of `img`, in place: 255 on the regional maxima
 * (connectivity conn) of D8 = min(floor(sqrt(dist2)), 255), 0 elsewhere
 * (background pixels never).  Height and width at most 16384; uses a context
 * scratch area of 4 bytes per pixel.  Enqueued on `stream`. */
int recon_pre_watershed(recon_ctx *ctx, recon_image *img, int conn, void *stream);

/* Run n tasks (any mix of ops, shapes and connectivities) in one persistent
 * launch sequence: up to 12 tasks are launched directly (their table in the
 * kernel arguments), larger batches replay a HIP graph captured once per block
 * shape (timed as a whole with timing = 1).  Tasks whose block_rows differ
 * run as one group per block height, each group's launch sequence on a stream
 * of its own forked from `stream` and joined back into it (the groups' kernels
 * run side by side; the call is timed as a whole, and recon_last_stats sums
 * the groups' counters).  The paper processes a dataset as a bag of independent
 * tile tasks (Sec. III-B: a stage instance is an (input chunk, stage) pair,
 * handed out on demand); here the bag is drained inside one launch, whose
 * waves pull blocks of any task as they free up, each task converging on its
 * own.  `tasks` is a host array read before the call returns; the images are
 * the caller's device buffers.  Enqueued on `stream`. */
int recon_batch(recon_ctx *ctx, const recon_task *tasks, int32_t n, void *stream);

/* Serving: a request loop in the manner of the paper's demand-driven
 * execution (Sec. III-B: workers ask for more work as they finish, with a
 * bounded number of instances in flight, the window size) and its overlap of
 * transfers with computation (Sec. IV-D).  recon_submit admits one task: on
 * success *ticket identifies it.  Admission counts the task's device bytes
 * (its images and scratch plane) and one slot against serve_mem_cap and
 * serve_slots; RECON_EAGAIN when either is reached (poll earlier tickets and
 * retry).  The task's images must stay valid until the ticket completes. */
int recon_submit(recon_ctx *ctx, const recon_task *task, uint64_t *ticket);
/* Non-blocking (Sec. III-B's completion notice): *done = 1 once the ticket's
 * result is in its image buffer; a completed ticket is forgotten after the
 * call that reports it. */
int recon_poll(recon_ctx *ctx, uint64_t ticket, int *done);
/* Block until the ticket completes or timeout_us elapses (< 0: no limit);
 * RECON_ETIMEDOUT leaves the ticket in flight. */
int recon_wait(recon_ctx *ctx, uint64_t ticket, int64_t timeout_us);
/* Stop the request loop after the admitted work has drained. */
int recon_serve_stop(recon_ctx *ctx);

/* Counters of the request loop since it started (all 0 before the first
 * recon_submit): launches made, requests launched, the most requests one
 * launch held, the most lanes running at once, and the tickets completed
 * before their launch ended (a reconstruction by dilation completes as soon
 * as its own last block visit has, Sec. III-B's per-instance completion
 * notice; the other operations map their result at the end of the launch). */
typedef struct {
    int64_t launches;
    int64_t requests;
    int64_t max_batch;
    int64_t max_busy_lanes;
    int64_t early_completions;
} recon_serve_counters;
int recon_serve_stats(recon_ctx *ctx, recon_serve_counters *out);

/* Statistics of the last completed recon_dilate / recon_fill_holes /
 * recon_erode / recon_hdome / recon_regional_max / recon_batch launch (synchronises with it).  Returns RECON_EDEVICE if that
 * launch was stopped by the scheduler watchdog (no block visit completed for
 * 8 s), in which case its results are incomplete. */
int recon_last_stats(recon_ctx *ctx, recon_stats *out);

/* Enqueue on `stream`, after the context's last launch (which must have been
 * enqueued on the same stream or be ordered before it), a write of that
 * launch's outcome into *host_flag: 0 if it converged, 1 if its scheduler
 * gave up (the case in which recon_last_stats returns RECON_EDEVICE).
 * Nothing waits: the caller reads the word once the stream has passed that
 * point (an event recorded after this call), and can meanwhile enqueue more
 * work on the context.  host_flag must be pinned, device-accessible host
 * memory (hipHostMalloc) of the caller's, at least 4 bytes; the word is
 * written once per call.  With no launch yet it receives 0.  For callers that
 * keep several operations in flight (the tile pipeline's GPU manager). */
int recon_enqueue_status(recon_ctx *ctx, uint32_t *host_flag, void *stream);

/* Kernel durations in ms of a recent launch of a context created with
 * timing = 1: `back` = 0 is the last launch sequence, 1 the one before, up to
 * 63.  dense_ms, seed_ms, drain_ms: the dense pass (K1), border seeding (K2)
 * and revisit drain (K3); total_ms: the whole launch, from the scheduler reset
 * and marker preparation to the result mapping; route_ms: from the start of
 * the launch to the end of the component route's kernels.  A replayed graph reports
 * only its total (the others are -1).  Waits (up to 60 s) for that launch to
 * complete.  RECON_EINVAL if the context does not time its launches or that
 * launch is no longer kept.  Lets a caller time many launches issued back to
 * back and read all their durations after one synchronisation. */
int recon_launch_times(recon_ctx *ctx, int back, float *dense_ms, float *seed_ms, float *drain_ms,
                       float *total_ms, float *route_ms);

/* ---- Co-scheduled tile pipeline (CPU cores + GPU)
 *
 * The paper's runtime maps the operations of each tile's analysis pipeline to
 * CPU cores and GPUs one operation instance (a tile, operation pair) at a
 * time, and its Performance Aware Task Scheduling (PATS, Sec. IV-B) orders the
 * ready instances by their estimated GPU-over-CPU speedup: an idle CPU core
 * takes the lowest, an idle GPU the highest; first-come-first-served (FCFS)
 * hands out the oldest.  With data locality (DL, Sec. IV-C) the GPU prefers
 * an instance whose inputs are in device memory already, unless another
 * instance's speedup exceeds its own by more than the transfers would cost:
 * the resident one is taken when S_resident >= S_other * (1 - transfer_impact
 * of the other's operation).  Without DL every GPU assignment uploads its
 * inputs and downloads its outputs.  A bounded number of tiles is in flight
 * (the demand-driven window, Sec. III-B); a finished tile frees its slot for
 * the next one.  Separate I/O threads download a finished tile's results and
 * copy the next tile's image in while the devices compute (the asynchronous
 * copies and prefetching of Sec. IV-D).  An optional limit keeps the CPU workers off the operations
 * whose estimated speedup exceeds it (on a GPU hundreds of times faster than
 * a core, such an instance taken by a core can outlast the whole GPU run).
 *
 * The pipeline of each tile, after the MR-based segmentation operations of
 * Table 1 (every operation's result is unique, so the bytes do not depend on
 * where each instance ran):
 *   RECON_PIPE_HDOME    A <- h-dome of the tile, D_h(I)            (ReconToNuclei)
 *   RECON_PIPE_FILL     A <- fill-holes of A                       (FillHoles)
 *   RECON_PIPE_AREA     A <- area filter of A, [area_min, area_max] (AreaThreshold)
 *   RECON_PIPE_MARKERS  B <- Pre-Watershed markers of A            (Pre-Watershed)
 *   RECON_PIPE_LABEL    L <- labels of A, and their count          (BWLabel)
 * with the dependencies HDOME -> FILL -> AREA -> {MARKERS, LABEL}.  The GPU
 * variants are this library's operations; the CPU variants are separate
 * single-core implementations of the same definitions. */
enum {
    RECON_PIPE_HDOME = 0,
    RECON_PIPE_FILL = 1,
    RECON_PIPE_AREA = 2,
    RECON_PIPE_MARKERS = 3,
    RECON_PIPE_LABEL = 4,
    RECON_PIPE_NOPS = 5
};
enum { RECON_SCHED_FCFS = 0, RECON_SCHED_PATS = 1 };

typedef struct {
    const uint8_t *image;   /* HOST: the grey tile, height x width, pitch bytes per row */
    int32_t height, width;  /* 1..16384 each */
    int64_t pitch;          /* >= width; also the row pitch of objects and markers */
    uint8_t *objects;       /* HOST out (or NULL): A after the area filter, 255 / 0 */
    uint8_t *markers;       /* HOST out (or NULL): B, the Pre-Watershed markers, 255 / 0 */
    int32_t *labels;        /* HOST out (or NULL): L, label_pitch elements per row */
    int64_t label_pitch;    /* >= width when labels is not NULL */
    int32_t *count;         /* HOST out (or NULL): the number of labelled components */
} recon_pipe_tile;

typedef struct {
    int32_t policy;         /* RECON_SCHED_FCFS or RECON_SCHED_PATS */
    int32_t cpu_workers;    /* host threads running CPU variants, one core each (0..256) */
    int32_t use_gpu;        /* 1: a GPU manager thread runs GPU variants through ctx */
    int32_t window;         /* tiles in flight at once, 1..1024 */
    int32_t data_locality;  /* 1: DL (the GPU keeps and prefers resident data) */
    int32_t conn;           /* 4 or 8, every operation */
    int32_t h;              /* dome height, 1..255 */
    float cpu_max_speedup;  /* > 0: a CPU worker leaves every instance whose estimated speedup
                               exceeds it to the GPU (0: no limit, the published PATS/FCFS) */
    int64_t area_min, area_max;   /* 0 <= area_min <= area_max */
    float speedup[RECON_PIPE_NOPS];          /* PATS: estimated GPU-over-CPU speedup per operation */
    float transfer_impact[RECON_PIPE_NOPS];  /* DL with PATS: share of an operation's GPU time
                                                spent on its transfers, 0..1 */
    int32_t io_threads;     /* threads that download finished tiles' results, copy them out and
                               copy the next tiles' images in (0: 2; at most 64) */
    int32_t cpu_guard;      /* 1: a CPU worker takes an instance only if its estimated CPU time
                               (speedup x gpu_ms) is at most the GPU's estimated remaining work
                               (gpu_ms summed over every instance not started yet); 0: off */
    float gpu_ms[RECON_PIPE_NOPS];           /* cpu_guard: estimated GPU time per operation */
    int32_t prefetch;       /* 1: a tile's image is uploaded when the tile is admitted, before its
                               first operation is queued (Sec. IV-D's prefetching); 0: on demand */
    int32_t trace_cap;      /* entries of `trace` (0: no trace) */
    struct recon_pipe_event *trace;  /* HOST out (or NULL): one entry per operation instance, in
                                        the order the devices took them (the first trace_cap) */
    int32_t gpu_inflight;   /* instances the GPU manager keeps enqueued on its stream at once, 1..4
                               (0: 1, the paper's one instance at a time).  With more, the next
                               instance is chosen and enqueued while the previous one runs, which
                               hides the host's round trip between them; the choice is then made
                               among the instances ready at that earlier moment */
    int32_t gpu_batch;      /* most ready instances of one reconstruction operation (h-dome or
                               fill-holes) the GPU manager runs in one recon_batch launch, 1..8
                               (0: 1).  With more, the instance the policy picks takes the other
                               ready instances of its operation along (oldest first): one tile's
                               reconstruction leaves most of the GPU idle, a batch fills it */
} recon_pipe_config;

/* One operation instance of a recon_pipeline_run, as it ran. */
typedef struct recon_pipe_event {
    int32_t tile;           /* index into the tiles array */
    int32_t op;             /* RECON_PIPE_* */
    int32_t device;         /* 0: the GPU; 1 + k: CPU worker k */
    int32_t reserved;
    double start_ms, end_ms;   /* from the start of the run: taken (inputs staged next), computed */
} recon_pipe_event;

typedef struct {
    double makespan_ms;                      /* first admission to the last tile's results */
    int64_t ops_cpu[RECON_PIPE_NOPS];        /* instances run by CPU workers, per operation */
    int64_t ops_gpu[RECON_PIPE_NOPS];        /* instances run by the GPU */
    double busy_cpu_ms[RECON_PIPE_NOPS];     /* summed compute time of those instances */
    double busy_gpu_ms[RECON_PIPE_NOPS];     /* (GPU: enqueue to completion, transfers excluded) */
    int64_t uploads, downloads;              /* plane transfers */
    int64_t upload_bytes, download_bytes;
    double transfer_ms;                      /* summed time of the transfers */
    double io_ms;                            /* summed time of tile completion and admission */
    int64_t trace_n;                         /* entries written to cfg->trace */
} recon_pipe_stats;

/* Run the pipeline on n host tiles and write each tile's outputs.  ctx may be
 * NULL when use_gpu is 0 (CPU cores only); with use_gpu = 1 the calling
 * thread's current device must be ctx's, and ctx must not be used by any
 * other thread until the call returns.  The call allocates, for `window`
 * tiles, pinned host planes and device planes of 6 bytes per pixel of the
 * largest tile, and frees them before it returns; it blocks until every tile
 * is done.  RECON_EINVAL for a bad configuration or tile (use_gpu without a
 * context, neither a GPU nor a CPU worker, a shape out of range); an operation
 * or transfer error stops the run and is returned (RECON_EDEVICE,
 * RECON_ETIMEDOUT after 60 s without progress of a GPU stream, RECON_ENOMEM).
 * `stats` (may be NULL) receives the run's counters; recon_pipeline_error()
 * describes a failure. */
int recon_pipeline_run(recon_ctx *ctx, const recon_pipe_tile *tiles, int32_t n,
                       const recon_pipe_config *cfg, recon_pipe_stats *stats);

/* Message of the calling thread's last failed recon_pipeline_run or
 * recon_pipeline_host_op ("" after a success). */
const char *recon_pipeline_error(void);

/* One pipeline operation's CPU variant on a HOST image, in place (what a CPU
 * worker of recon_pipeline_run executes, on the calling thread): op is a
 * RECON_PIPE_* value; cfg supplies conn, h and the area bounds; for
 * RECON_PIPE_LABEL the HOST labels plane (label_pitch >= width) receives the
 * labels, *count (if not NULL) their number, and the image is not written.
 * For calibrating speedup estimates and testing the CPU variants. */
int recon_pipeline_host_op(int op, recon_image *img, const recon_pipe_config *cfg, int32_t *labels,
                           int64_t label_pitch, int32_t *count);

/* Message describing the last failure on the calling thread ("" if none). */
const char *recon_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RECON_H */
