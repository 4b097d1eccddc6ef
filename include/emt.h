/*
 * emt.h -- C ABI of the MI355X 4pi emulsion track finder.
 *
 * What it computes (paper, Sec. 2, tracking paragraph and Fig. 4): for each
 * microscope view, given the 3D grains read from the tomographic focal
 * planes, every grain pair closer than a seed distance R (any direction,
 * full solid angle) is a seed; the grains within a radius r of the infinite
 * line through the seed pair are counted; seeds reaching n_min grains are
 * candidates; candidates are then taken best first (grain count descending,
 * then seed input indices ascending), each keeping only grains no earlier
 * track used, and kept as a track only if n_min grains remain. Each track is
 * returned with its grain list and a least-squares direction fit.
 *
 * Units: grain coordinates are int32 fixed point, 1 unit = 0.01 um. Within a
 * view the per-axis coordinate span (max - min) must not exceed 2^18 units
 * (2.62 mm) and a view holds fewer than 2^20 grains. All geometry decisions
 * are exact integer arithmetic, so track lists do not depend on the device
 * or on what else is in the batch.
 *
 * Threading: a context is not thread-safe; use one per host thread. Calls are
 * synchronous: when emt_track_views returns, results are on the host.
 */
#ifndef EMT_H
#define EMT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMT_ABI_VERSION 2u

/* Return codes. */
#define EMT_OK 0
#define EMT_EINVAL (-1)    /* null pointer, wrong abi_version, bad parameter   */
#define EMT_ERANGE (-2)    /* view span > 2^18 units, >= 2^20 grains, R or r
                              out of range                                    */
#define EMT_ENOMEM (-3)    /* host or device allocation failed, or a view's
                              working set exceeds the HBM budget              */
#define EMT_EDEVICE (-4)   /* HIP error; the context is poisoned: destroy it  */
#define EMT_EOVERFLOW (-5) /* internal capacity still short after retries     */

/* Flags for emt_config.flags. */
#define EMT_F_STATS 0x1u           /* time every stage with HIP events       */
#define EMT_F_FP64_FIT_ALWAYS 0x2u /* solve every fit in FP64                */
#define EMT_F_DEVICE_PTRS 0x4u     /* emt_view_in.xyz point to device memory */
#define EMT_F_CANDIDATES 0x8u      /* keep every candidate for
                                      emt_view_candidates                     */

/* Stage indices of emt_call_stats.ms. */
#define EMT_STAGE_STAGE 0   /* copy grains in                                */
#define EMT_STAGE_BIN 1     /* bounding box, cell histogram, scan, scatter   */
#define EMT_STAGE_SEED 2    /* seed pairs closer than R                      */
#define EMT_STAGE_COUNT 3   /* grains within r of every seed line           */
#define EMT_STAGE_MEMBERS 4 /* candidate member lists                       */
#define EMT_STAGE_MERGE 5   /* exclusive association rounds                 */
#define EMT_STAGE_FIT 6     /* track order, grain order, fit                */
#define EMT_STAGE_OUT 7     /* copy tracks out                              */
#define EMT_N_STAGES 8

/*
 * Configuration (emt_default_config fills the defaults).
 *   seed_dist   R in units (default 2500 = 25 um, paper Sec. 2); 1..4096.
 *   tol_radius  r in units (default 50 = 0.5 um); 0 <= r < R. Inclusive.
 *   min_grains  n_min (default 8); 2 <= n_min < 2^20. Applied to the count
 *               and again after exclusive association.
 *   cell        edge of a hash cell along x, y, z in units. All three 0:
 *               the library picks them per view from the view's grain
 *               density (a table written by the project's autotuner); else
 *               the given edges, with 250, 750, 500 for an axis left at 0.
 *               Cells only steer the work (paper Sec. 3 footnote), never the
 *               result; the library widens them if a view would need more
 *               than 4N + 4096 cells.
 *   device      HIP device ordinal.
 *   flags       EMT_F_* bits.
 *   hbm_budget  device bytes the context may hold (0 = 80 % of free memory).
 *   stream      hipStream_t to run on, or NULL for a library-owned stream.
 * Acceptance variants (defaults: off):
 *   cyl_ext     -1 (default): grains are counted along the infinite line
 *               through the seed. 0 .. 2^18: a finite cylinder, counting
 *               only grains whose projection on the line lies at most
 *               cyl_ext units beyond either seed grain, i.e. with
 *               t = (g_k - g_i).(g_j - g_i): -cyl_ext |d| <= t <=
 *               |d|^2 + cyl_ext |d| (exact).
 *   thr_slope   {num, den}: a seed needs n_min + ceil(num/den tan(theta))
 *               grains, theta the angle of the seed pair to the z axis
 *               (tan = sqrt(dx^2 + dy^2) / |dz|), in both threshold steps;
 *               after the paper's grain-count cut against track angle
 *               (Sec. 3, Fig. 8c). num 0 (default): the threshold is n_min.
 *               num 0..1024, den 1..1024.
 *   thr_max     cap of that threshold (0: none; else n_min..2^20-1); a seed
 *               with dz = 0 needs the cap (no cap: it is never a track).
 */
typedef struct {
    uint32_t abi_version;
    int32_t seed_dist;
    int32_t tol_radius;
    int32_t min_grains;
    int32_t cell[3];
    int32_t device;
    uint32_t flags;
    uint64_t hbm_budget;
    void *stream;
    int32_t cyl_ext;
    int32_t thr_slope[2];
    int32_t thr_max;
} emt_config;

/* One view in. xyz: n_grains x 3 int32 (x, y, z interleaved), owned by the
 * caller, read only during the call; a host pointer unless the context was
 * created with EMT_F_DEVICE_PTRS. n_grains may be 0. */
typedef struct {
    const int32_t *xyz;
    uint32_t n_grains;
    uint32_t reserved;
    uint64_t view_id;
} emt_view_in;

/* One track. seed: input indices (i < j) of the accepted seed pair.
 * grain_offset/n_grains: slice of emt_view_out.grains holding the track's
 * grains as input indices, ordered by (g_k - g_i).(g_j - g_i), then index.
 * axis: 0, 1, 2 for x, y, z, the axis of largest spread; slope: d(b)/d(axis)
 * and d(c)/d(axis) for the other two axes b < c; dir: unit direction with
 * dir.z > 0 (else dir.y > 0, else dir.x > 0); centroid in um; t_begin and
 * t_end: extent of the grains along dir about the centroid, um.
 * fit_fp64: 1 if the slopes were solved in FP64 (axis == z or RMS spread
 * along axis < 5 um or EMT_F_FP64_FIT_ALWAYS); degenerate: 1 if all grains
 * of the track coincide (no spread to fit: axis, slopes and dir are then
 * those of the seed direction g_j - g_i, slopes in FP64, fit_fp64 = 1). */
typedef struct {
    uint32_t seed[2];
    uint32_t grain_offset;
    uint32_t n_grains;
    uint32_t axis;
    uint32_t fit_fp64;
    uint32_t degenerate;
    float slope[2];
    float dir[3];
    float centroid[3];
    float t_begin;
    float t_end;
} emt_track;

typedef struct {
    uint64_t n_seeds;      /* pairs closer than R                   */
    uint32_t n_candidates; /* seeds reaching n_min                  */
    uint32_t n_tracks;
} emt_view_stats;

/* Results of one view, owned by the context and valid until the next call
 * on it or emt_destroy. */
typedef struct {
    uint64_t view_id;
    uint32_t n_tracks;
    uint32_t n_track_grains;
    const emt_track *tracks;
    const uint32_t *grains;
    emt_view_stats stats;
} emt_view_out;

/* Whole-call statistics of the last emt_track_views on a context. */
typedef struct {
    uint64_t n_seeds;
    uint64_t n_tests;      /* grains examined while counting             */
    uint64_t n_hits;       /* sum over seeds of the grain count          */
    uint32_t n_candidates;
    uint32_t n_tracks;
    uint32_t merge_rounds;
    uint32_t n_fp64_fits;
    uint32_t retries;      /* re-runs after a capacity overflow          */
    uint32_t n_views;
    float ms[EMT_N_STAGES]; /* device time per stage (EMT_F_STATS), else 0 */
    float ms_total;
} emt_call_stats;

/* Opaque context: device buffers, stream and events of one tracker. */
typedef struct emt_ctx emt_ctx;

/* Fill *cfg with defaults (abi_version set). */
void emt_default_config(emt_config *cfg);

/* Check a configuration and host-resident views without touching a device.
 * Returns EMT_OK, EMT_EINVAL or EMT_ERANGE. views may be NULL if
 * n_views == 0. Views are checked only when they are host pointers. */
int emt_validate(const emt_config *cfg, const emt_view_in *views,
                 uint32_t n_views);

/* Create a context on cfg->device. *out is set to NULL on failure. */
int emt_create(const emt_config *cfg, emt_ctx **out);

/* Track n_views views. n_views == 1 runs one view per launch sequence;
 * n_views > 1 runs all views through the same launches. out must hold
 * n_views entries. On error no output is valid. */
int emt_track_views(emt_ctx *ctx, const emt_view_in *views, uint32_t n_views,
                    emt_view_out *out);

/* Candidates of one view of the last successful emt_track_views on a
 * context created with EMT_F_CANDIDATES: every seed whose grain count
 * reached the threshold (paper Sec. 2, tracking paragraph; Fig. 4b), before
 * the exclusive association. *ijn receives n_cand triplets (i, j, n): the
 * input indices i < j of the seed pair and the number of grains within r of
 * its line, in the order the device listed them (not the priority order;
 * sort by (n descending, i, j) for that). Owned by the context, valid until
 * its next call or emt_destroy. Returns EMT_OK; EMT_EINVAL for a NULL
 * argument, a view index beyond the last call's views, or a context without
 * the flag. */
int emt_view_candidates(emt_ctx *ctx, uint32_t view, const uint32_t **ijn,
                        uint32_t *n_cand);

/* Statistics of the last successful emt_track_views. After emt_find_grains
 * or emt_filter_stack with EMT_F_STATS, every field is 0 except ms_total:
 * the device time of the recognition or filtering kernels. */
int emt_last_stats(emt_ctx *ctx, emt_call_stats *stats);

/* Release a context; NULL is ignored. */
void emt_destroy(emt_ctx *ctx);

/* Static text for a return code. */
const char *emt_strerror(int code);

/*
 * Grain recognition (paper, Sec. 2, grain recognition paragraph; Fig. 3c):
 * the step before tracking. On a filtered stack of nz frames of ny rows of
 * nx 8-bit pulse heights (x fastest), a pixel above the threshold defines a
 * grain if no pixel of its 3 x 3 x 3 neighbourhood inside the stack is
 * higher, or equal and earlier in frame, row, column order. The grain sits
 * at the pulse-height centre of mass of that neighbourhood, pixel k of an
 * axis being centred at k pitches: coordinates in 0.01 um units, rounded to
 * the nearest unit (halves up) from exact integer sums, i.e. exactly the
 * input of emt_track_views. Grains come out in frame, row, column order.
 *
 * geom: nx a multiple of 4 (4..65536), ny 1..65536, nz 1..4096, at most
 * 2^31 pixels; threshold 0..255; pitch_num, pitch_den 1..65536 (the
 * paper's 300 x 250 x 50 um view at 1280 x 1024 x 40 is 375/16, 3125/128,
 * 125/1).
 * stack: nx*ny*nz bytes, read during the call; xyz_out: room for max_out
 * grains of 3 int32 (x, y, z). Both are host pointers, or device pointers
 * (stack 16-byte and xyz_out 4-byte aligned, else EMT_EINVAL) if the
 * context was created with EMT_F_DEVICE_PTRS. *n_out receives the
 * number of grains found. Returns EMT_OK; EMT_EOVERFLOW if more than
 * max_out grains were found (the first max_out are written);
 * EMT_EINVAL/EMT_ERANGE for bad arguments; EMT_ENOMEM/EMT_EDEVICE.
 */
typedef struct {
    uint32_t nx, ny, nz;
    uint32_t threshold;
    uint32_t pitch_num[3];
    uint32_t pitch_den[3];
} emt_stack_geom;

int emt_find_grains(emt_ctx *ctx, const uint8_t *stack,
                    const emt_stack_geom *geom, int32_t *xyz_out,
                    uint32_t max_out, uint32_t *n_out);

/*
 * emt_find_grains without any allocation, for callers that cannot allocate
 * device or host memory during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc). Same computation,
 * arguments, results and return codes as emt_find_grains on a context
 * created with EMT_F_DEVICE_PTRS (stack and xyz_out are device pointers;
 * a context without the flag gives EMT_EINVAL). The working buffers
 * (per-tile counts, per-group sums, staging) live in one static device
 * array of EMT_NOALLOC_SCRATCH_BYTES per device, which the library holds
 * from emt_create until the process ends; a stack needing more (about one
 * byte per pixel: up to ~67 M pixels, e.g. 1280 x 1024 x 51 frames) gives
 * EMT_ERANGE before any work. Every call on one device shares that array:
 * calls that overlap on a device race and must not be made (one call at a
 * time per device, across all contexts and threads).
 */
#define EMT_NOALLOC_SCRATCH_BYTES (64u << 20)

int emt_find_grains_noalloc(emt_ctx *ctx, const uint8_t *stack,
                            const emt_stack_geom *geom, int32_t *xyz_out,
                            uint32_t max_out, uint32_t *n_out);

/*
 * Image filtering (paper, Sec. 2, image processing paragraph; Fig. 3a, 3b):
 * the step before grain recognition. The camera's pixels differ in gain, so
 * each camera pixel (x, y) has its own gain correction and threshold, used
 * in every frame, and the image is inverted so that grains (dark in the
 * bright-field image) become bright. Per pixel, on 8-bit pulse heights:
 * t = min(255, raw * gain / 256 rounded to nearest, halves up);
 * u = 255 - t; out = u - thr if u > thr, else 0.
 *
 * geom: nx, ny, nz as for emt_find_grains (its threshold and pitches are
 * not used). raw and out: nx*ny*nz bytes (x fastest, frames outermost);
 * gain: ny*nx uint16 in units of 1/256 (256 = unchanged); thr: ny*nx bytes.
 * All four are host pointers, or device pointers (each 16-byte aligned,
 * else EMT_EINVAL) if the context was created with EMT_F_DEVICE_PTRS. raw,
 * gain and thr are read during the call; out is written before it returns
 * and may be raw itself (in place; no other overlap). Returns EMT_OK,
 * EMT_EINVAL (NULL argument), EMT_ERANGE (geometry out of range),
 * EMT_ENOMEM, EMT_EDEVICE. With
 * EMT_F_STATS, emt_last_stats reports the kernel's device time in ms_total.
 */
int emt_filter_stack(emt_ctx *ctx, const uint8_t *raw,
                     const emt_stack_geom *geom, const uint16_t *gain,
                     const uint8_t *thr, uint8_t *out);

/*
 * Serving (paper, Sec. 3: the microscope delivers one view after another at
 * up to 5 Hz, and views are processed in parallel threads sharing the GPUs).
 * A server tracks views as they arrive. A worker thread runs n_pipes
 * pipelines, each a context with its own stream and device buffers; when a
 * pipeline is free it takes the views waiting, in arrival order, as many as
 * fit its share (1/n_pipes) of the HBM budget and at most max_batch_views,
 * as one batch. With n_pipes >= 2 a new batch starts while another is still
 * on the device. A view's tracks are identical to tracking it alone.
 *
 * cfg is as for emt_create; EMT_F_DEVICE_PTRS is rejected (EMT_EINVAL):
 * submissions are host arrays. Calls on one server may come from several
 * host threads.
 */
typedef struct emt_server emt_server;

/* One finished view. tracks/grains are as in emt_view_out, owned by the
 * server and valid until the next emt_server_poll on it or
 * emt_server_destroy. status: EMT_OK, or the error of its batch (EMT_ENOMEM
 * if the view alone exceeds a pipeline's share of the budget); on error no
 * tracks are returned. Times are milliseconds since emt_server_create:
 * submission, admission into a batch, and completion as seen by the
 * worker. */
typedef struct {
    uint64_t ticket;
    uint64_t view_id;
    int32_t status;
    uint32_t n_tracks;
    uint32_t n_track_grains;
    uint32_t batch_views; /* views in the batch this one ran in */
    const emt_track *tracks;
    const uint32_t *grains;
    emt_view_stats stats;
    double t_submit_ms;
    double t_admit_ms;
    double t_done_ms;
} emt_served;

typedef struct {
    uint64_t submitted;
    uint64_t completed;
    uint64_t batches;
    uint32_t max_batch_views_seen;
    uint32_t n_pipes;
    double busy_ms;    /* time with at least one batch on the device  */
    double overlap_ms; /* time with two or more batches on the device */
    double elapsed_ms; /* since emt_server_create                     */
} emt_server_stats;

/* Create a server: 1 <= n_pipes <= 8, max_batch_views >= 1; batches have
 * no grain limit. */
int emt_server_create(const emt_config *cfg, uint32_t n_pipes,
                      uint32_t max_batch_views, emt_server **out);

/* Limits of a server's batches. max_batch_grains > 0 also closes a batch
 * before the view that would take it past that many grains (a view larger
 * than the limit runs alone); 0 is no limit. Smaller batches finish sooner,
 * so a waiting view is admitted sooner, at some cost in throughput. */
typedef struct {
    uint32_t n_pipes;          /* 1..8 pipelines */
    uint32_t max_batch_views;  /* >= 1 */
    uint64_t max_batch_grains; /* 0: no limit */
} emt_server_limits;

/* Create a server with the given limits (as emt_server_create otherwise). */
int emt_server_create2(const emt_config *cfg, const emt_server_limits *lim,
                       emt_server **out);

/* Queue one view; its grains are copied before the call returns. *ticket
 * (may be NULL) receives a number that increases with every submission.
 * Returns EMT_EINVAL/EMT_ERANGE as emt_validate would, or the server's
 * sticky EMT_EDEVICE. */
int emt_server_submit(emt_server *srv, const emt_view_in *view,
                      uint64_t *ticket);

/* Collect up to max_out finished views, in completion order. wait_ms: 0
 * returns at once, > 0 waits up to that long for one, < 0 waits until one
 * is there. Returns EMT_OK or the sticky EMT_EDEVICE after a device error. */
int emt_server_poll(emt_server *srv, emt_served *out, uint32_t max_out,
                    uint32_t *n_out, int32_t wait_ms);

/* Counters since creation. */
int emt_server_get_stats(emt_server *srv, emt_server_stats *stats);

/* Stop admitting, wait for the batches on the device, release everything.
 * Views still waiting are dropped. NULL is ignored. */
void emt_server_destroy(emt_server *srv);

/*
 * Measured device rates, the denominators beside the specification's for
 * the roofline of each kernel: the counting test is 32-bit integer and FP32
 * lane work (paper Sec. 3: tracking is most of the time), binning and the
 * image steps stream HBM. Each rate is the fastest of five timed launches of
 * a kernel that does nothing else: chains of 24-bit integer multiply-adds,
 * chains of FP32 FMAs (one lane operation each, not packed), 128-bit LDS
 * reads, and a 1 GiB device-to-device copy (bytes read plus written).
 * Allocates 2 GiB of device memory for the call. Returns EMT_OK,
 * EMT_EINVAL (NULL out or no such device) or EMT_EDEVICE.
 */
typedef struct {
    double int_lane_ops;   /* 32-bit integer lane operations per second   */
    double fp32_lane_ops;  /* FP32 FMA lane operations per second         */
    double lds_bytes;      /* LDS bytes read per second, whole device     */
    double hbm_copy_bytes; /* HBM bytes read plus written per second      */
    uint32_t compute_units;
    uint32_t clock_khz;    /* peak engine clock the runtime reports       */
} emt_peaks;

int emt_measure_peaks(int32_t device, emt_peaks *out);

#ifdef __cplusplus
}
#endif
#endif
