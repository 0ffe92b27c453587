/*
 * cfar2d.h -- C ABI of libcfar2d.so: integral-image 2D cell-averaging CFAR
 * on AMD Instinct MI355X (gfx950).
 *
 * The operation is the detector of Rohman, Andra and Nishimoto, "Optimized 2D
 * CA-CFAR for Drone-Mounted Radar Signal Processing Using Integral Image
 * Algorithm" (arXiv 2012.11077), Sec. II.B:
 *
 *   map X in R^{M x N} (Sec. II.A): here `rows` range bins x `cols`
 *       slow-time-frequency bins, row-major, frequency contiguous, with a
 *       leading dimension `ld` >= cols (in elements);
 *   integral image (eq. 3): S(i,j) = sum of X over rows <= i, cols <= j;
 *   rectangle sum (eq. 4): four corners of S;
 *   training cells: the rectangle of half-widths (guard + train) around the
 *       cell under test (CUT) minus the guard rectangle of half-widths guard
 *       (Table I names these "Guard Cell" and "Background Cell"), both
 *       clipped to the map; N = number of training cells inside the map;
 *   threshold (eq. 2): T = alpha * A, A = (training sum) / N, with
 *       alpha = N (Pfa^(-1/N) - 1) (the exponent printed in eq. 2 has the
 *       opposite sign, which gives a negative alpha);
 *   decision (eq. 1): target (mask = 1) iff CUT > T; N = 0 gives mask = 0.
 *
 * Conventions for every entry point:
 *   - All map, mask, SAT and workspace pointers are DEVICE pointers owned by
 *     the caller, unless an argument says otherwise.  The library allocates
 *     and frees none of them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls enqueue work and return; the caller synchronises the stream
 *     before it reads the outputs.
 *   - Every argument is validated on the host before any device work; on
 *     error nothing is enqueued and nothing is written.  The return value is
 *     a cfar_status; cfar_last_error() describes the last failure of the
 *     calling thread.
 *   - Preconditions that are not checked on the device: X is finite and
 *     >= 0 (a square-law power map, which is what alpha assumes), and
 *     |X| <= 1e30.
 *   - Device faults surface as CFAR_EDEVICE from the next call that checks
 *     the HIP runtime.
 */
#ifndef CFAR2D_H
#define CFAR2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
typedef enum {
    CFAR_OK = 0,
    CFAR_EINVAL = -1,    /* an argument is invalid (nothing enqueued)          */
    CFAR_ENOSPC = -2,    /* sat_bytes or ws_bytes is too small                  */
    CFAR_EDEVICE = -3,   /* the HIP runtime reported an error                   */
    CFAR_EAGAIN = -4,    /* server queue full: submit again later               */
    CFAR_ESHUTDOWN = -5  /* server is shutting down / frame was never started   */
} cfar_status;

/* Storage type of the map. */
typedef enum { CFAR_F32 = 0, CFAR_F64 = 1 } cfar_dtype;

/* Precision forms.
 *   PLAIN: the integral image of eq. (3) is materialised in FP64 in device
 *          memory, then the eight-corner stencil of eq. (4) reads it back.  The
 *          image is built by work units of 64 rows x 256 columns (per-unit row
 *          and column totals, their exclusive scans across units, then each
 *          unit's own prefix sums plus those carries); the stencil takes the
 *          four corner rows of a cell's outer and guard windows from it, their
 *          per-column differences, and the column corners of those.  Any
 *          window size (guard_f + train_f above 247 takes a per-cell stencil).
 *   TILED: the integral image is never materialised.  The eight corners of
 *          eq. (4) are separable: each work unit (a strip of columns plus a
 *          halo of guard_f + train_f + 1 columns, times a chunk of rows)
 *          keeps FP64 running column sums over the outer and guard windows'
 *          rows (the row corners) and takes an FP64 row prefix of them across
 *          the strip (the column corners as differences).  The map stays in
 *          its storage type (FP32 or FP64); one pass over X.  Supports
 *          guard_f + train_f <= 247.
 *   DIRECT: no integral image: every cell sums its own training cells (the
 *          CA-CFAR route that Table I compares the integral image against),
 *          in FP64 from the map's storage type, then eqs. (1)-(2) as in the
 *          other forms.  Work per cell grows with the window area.  A
 *          workgroup stages a 4 x 64 output tile and its window halo in LDS,
 *          so it supports (4 + 2 hr) x (64 + 2 hf) x element size <= 65536
 *          bytes (hr = guard_r + train_r, hf = guard_f + train_f; e.g. every
 *          window of Table I, and hr = hf = 28 in FP64).  sat2d does not take
 *          this form.  Workspace: the threshold table only. */
typedef enum { CFAR_FORM_PLAIN = 0, CFAR_FORM_TILED = 1, CFAR_FORM_DIRECT = 2 } cfar_form;

/* CFAR window (Table I, eq. 2): half-widths per axis, in cells.  The outer
 * half-widths are guard + train.  train_r + train_f must be > 0; 0 < pfa < 1. */
typedef struct {
    int32_t guard_r, guard_f;  /* guard half-widths along rows (range) / cols (frequency) */
    int32_t train_r, train_f;  /* training half-widths beyond the guard                   */
    double pfa;                /* design probability of false alarm                       */
} cfar_window;

/* One map and its outputs. */
typedef struct {
    const void *x;        /* device: rows x cols map, leading dimension ld (elements)      */
    int32_t dtype;        /* cfar_dtype                                                     */
    int32_t reserved0;    /* must be 0                                                      */
    int64_t rows, cols, ld;
    cfar_window win;
    uint8_t *mask;        /* device: rows x cols, leading dimension ld_mask, 0/1 per cell   */
    int64_t ld_mask;      /* >= cols; also the leading dimension of the optional outputs    */
    double *train_sum;    /* device, optional (NULL = skip): training sum per cell          */
    double *threshold;    /* device, optional (NULL = skip): T per cell (+inf when N = 0)   */
} cfar_map;

/* ------------------------------------------------------------------------ */
/* Integral image (eq. 3)                                                    */
/* ------------------------------------------------------------------------ */

/* Bytes of the SAT output of sat2d for a rows x cols map.
 *   PLAIN: rows*cols FP64, row-major, leading dimension cols; entry (i,j) is
 *          S(i,j) of eq. (3) (the zero boundary S(-1,.) = S(.,-1) = 0 is implied).
 *   TILED: three regions, each starting at a 256-byte boundary:
 *          (a) FP32 tile-local sums, rows x cols row-major: entry (i,j) is the
 *              sum of X over rows 32*floor(i/32)..i and cols 32*floor(j/32)..j;
 *          (b) FP64 row lines, ceil(rows/32) x cols: line I, entry j is
 *              S(32*I - 1, j) (0 for I = 0);
 *          (c) FP64 column lines, ceil(cols/32) x rows: line J, entry i is
 *              S(i, 32*J - 1) (0 for J = 0).
 *          Then S(i,j) = rowline[I][j] + colline[J][i] - rowline[I][32*J-1]
 *          + local(i,j), with I = i/32, J = j/32 and the corner term 0 when J = 0.
 * Returns 0 when rows or cols < 1. */
size_t sat2d_bytes(int64_t rows, int64_t cols, int32_t form);

/* Bytes of device workspace sat2d needs (unit aggregates and carries). */
size_t sat2d_workspace_bytes(int64_t rows, int64_t cols, int32_t form);

/* Integral image of X (eq. 3) in the layout of `form` (see sat2d_bytes).
 * x: device map (dtype, rows, cols, ld).  sat_out: device, >= sat2d_bytes.
 * ws: device scratch, >= sat2d_workspace_bytes; its contents on entry do not
 * matter.  FP32 input is promoted to FP64 exactly before it is summed.
 * Errors: CFAR_EINVAL (rows/cols < 1, ld < cols, NULL pointer, unknown dtype
 * or form), CFAR_ENOSPC (sat_bytes or ws_bytes too small), CFAR_EDEVICE. */
int sat2d(const void *x, int32_t dtype, int64_t rows, int64_t cols, int64_t ld, int32_t form,
          void *sat_out, size_t sat_bytes, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* CA-CFAR (eqs. 1, 2, 4)                                                    */
/* ------------------------------------------------------------------------ */

/* Device workspace bytes for cfar2d / cfar2d_batched over `n` maps in `form`
 * (PLAIN: for every map its FP64 integral image, the carries and the
 * threshold table, plus the descriptors when n > 1; TILED: descriptors, work
 * counters and threshold tables; DIRECT: the largest map's threshold table).
 * Returns 0 when an argument is invalid (cfar_last_error() says which). */
size_t cfar_workspace_bytes(const cfar_map *maps, int32_t n, int32_t form);

/* CA-CFAR over one map.  m: host pointer to the descriptor (its x, mask and
 * optional outputs are device pointers).  ws: device, >= cfar_workspace_bytes
 * for this map; contents on entry do not matter; it must not be used by
 * another call until this call's work on `stream` has finished.
 * Errors: CFAR_EINVAL (see the conventions above: rows/cols < 1, ld or
 * ld_mask < cols, negative half-width, train_r + train_f == 0, pfa not in
 * (0,1), NULL x/mask, unknown dtype/form, reserved0 != 0, a window too
 * wide for the form), CFAR_ENOSPC, CFAR_EDEVICE. */
int cfar2d(const cfar_map *m, int32_t form, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): cfar2d in
 * the TILED form with its workspace (work counter and threshold table) in a
 * static device array of cfar2d_static_max_bytes() bytes that each GPU holds
 * until the process ends, instead of caller memory.  m as in cfar2d.  It
 * allocates nothing.  Every call on one GPU shares that GPU's array: calls
 * whose work overlaps on the device (different streams, or host threads)
 * race and must be ordered by the caller; the array keeps the last call's
 * contents, and the counter it needs zeroed is cleared by a kernel of the
 * call itself.  Results are those of cfar2d with CFAR_FORM_TILED.
 * Errors: as cfar2d; CFAR_ENOSPC when the window's threshold table does not
 * fit (more than (cfar2d_static_max_bytes() - 256) / 8 - 1 training cells). */
int cfar2d_static(const cfar_map *m, void *stream);
size_t cfar2d_static_max_bytes(void);

/* Batch flags. */
enum {
    CFAR_BATCH_GRAPH = 1  /* capture the launch sequence in a hipGraph and replay it when
                             the same batch layout (n, ws, per-map work) comes again */
};

/* CA-CFAR over `n` maps of any sizes, each with its own window and Pfa.
 * maps: host array of n descriptors.  TILED: one small kernel builds the
 * threshold tables, then one persistent launch per kernel class runs the work
 * units of all maps of that class (classes: k_cols 2 or 4 / 8, dtype, with or
 * without the optional outputs -- FP32 maps without optional outputs are one
 * launch); on a non-NULL stream, classes after the first run on the
 * library's own streams forked from and joined back into `stream`.  Each
 * map's tile plan depends only on that map's own size, window and dtype, so
 * every map's result is the same alone and in any batch.
 * PLAIN: the FP64 integral images of all maps, then their stencils, in five
 * launches on `stream` for the whole batch (threshold tables, unit totals,
 * carries, integral images, stencil), plus one per-cell stencil launch per
 * map wider than the strip stencil holds; flags other than 0 are accepted
 * and ignored.
 * DIRECT: one table + direct-sum stencil per map on `stream` (flags other
 * than 0 are accepted and ignored).
 * Errors as cfar2d; map k's problems are reported with its index. */
int cfar2d_batched(const cfar_map *maps, int32_t n, int32_t form, int32_t flags, void *ws,
                   size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Tile plans (TILED form) and the autotuned plan table                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t k_cols;        /* columns per lane: 2, 4 or 8 (a 64-lane wave covers 64*k_cols cols) */
    int32_t rows_per_unit; /* output rows per work unit, 1..4096                                  */
    int32_t ring_bytes;    /* LDS bytes per wave for the guard ring, 0..65536, or -1 for the
                            * library default (12 KiB): the rows r-g_r-1 .. r+g_r of the strip,
                            * when they fit, so a row step loads three rows instead of five.  A
                            * ring that needs more than a positive budget but at most 20 KiB is
                            * given its own size (batched: in a launch of its own); 0 = no ring.
                            * Results do not depend on it. */
} cfar_plan;

/* The plan the TILED form uses for map m (from the loaded table, else the
 * built-in cost model).  Depends only on m's dtype, rows, cols and window. */
int cfar_plan_for(const cfar_map *m, cfar_plan *out);

/* Load a plan table written by the autotuner (text; one rule per line:
 *   dtype cols_lo cols_hi rows_lo rows_hi hf_lo hf_hi hr_lo hr_hi k rows_per_unit [ring_bytes]
 * with dtype f32 | f64 | any, '#' starting a comment, first matching rule
 * winning; see paper_2012_11077_amd/autotune.py).  NULL or "" restores the
 * built-in model.
 * Not thread-safe with concurrent TILED calls. */
int cfar_plan_load(const char *path);

/* TILED CA-CFAR over one map with an explicit plan (the autotuner's probe). */
int cfar2d_with_plan(const cfar_map *m, const cfar_plan *plan, void *ws, size_t ws_bytes,
                     void *stream);

/* ------------------------------------------------------------------------ */
/* Streaming server: continuous batching of frames from many streams         */
/* ------------------------------------------------------------------------ */

typedef struct cfar_server cfar_server;

typedef struct {
    size_t device_budget_bytes; /* device memory the server may hold for frames in flight     */
    int32_t max_inflight_frames;/* frames admitted to the device at once                       */
    int32_t n_hip_streams;      /* HIP streams batches rotate over (1..16)                     */
    int32_t queue_depth;        /* submitted-but-not-admitted frames; more gives CFAR_EAGAIN   */
    int32_t max_batch_frames;   /* frames per launched batch (<= max_inflight_frames)          */
} cfar_server_opts;

typedef struct {
    uint64_t ticket, user_tag;
    int32_t status;             /* CFAR_OK, CFAR_EDEVICE or CFAR_ESHUTDOWN                     */
    int32_t reserved;
    int64_t t_submit_ns, t_start_ns, t_done_ns; /* CLOCK_MONOTONIC                             */
} cfar_completion;

typedef struct {
    uint64_t submitted, completed, failed, batches;
    size_t device_bytes_in_use, device_bytes_peak;
    int32_t inflight_frames, queued_frames;
} cfar_server_stats;

/* Page-locked host memory for frames and masks submitted with x_on_host = 1
 * (hipHostMalloc): copies from and to it run at full link speed and overlap
 * with other work.  *out is host memory of `bytes` bytes, freed with
 * cfar_host_free.  Errors: CFAR_EINVAL (bytes == 0 or out NULL),
 * CFAR_EDEVICE (allocation failed). */
int cfar_host_alloc(size_t bytes, void **out);
int cfar_host_free(void *p);

/* Create a server: allocates its device pool (device_budget_bytes, clamped
 * to the free device memory) and starts its scheduler thread. */
int cfar_server_create(const cfar_server_opts *opts, cfar_server **out);

/* Submit flags. */
enum {
    CFAR_SUBMIT_HOST = 1,        /* frame->x and frame->mask are host pointers               */
    CFAR_SUBMIT_PACKED_MASK = 2  /* with CFAR_SUBMIT_HOST: frame->mask receives the bit-packed
                                    mask (as cfar_mask_pack: rows x ld_mask uint32 words,
                                    ld_mask >= ceil(cols / 32)), an eighth of the bytes */
};

/* Submit one frame (TILED form, FP32 or FP64).  flags & CFAR_SUBMIT_HOST:
 * frame->x and frame->mask are HOST pointers (pinned memory gives overlap);
 * the server copies X in and the mask out (packed on the device first with
 * CFAR_SUBMIT_PACKED_MASK), and train_sum/threshold must be NULL.  Without
 * it all pointers are device pointers (flags 0; 1 is the former x_on_host =
 * 1); the server reads and writes them on its own HIP streams, which are not
 * ordered after the caller's: the work that produces a device frame must be
 * complete (synchronized) before cfar_submit, and its mask is ready when the
 * ticket completes.  Buffers must stay valid until the ticket completes.  Never blocks:
 * CFAR_EAGAIN when the queue is full, CFAR_EINVAL for a bad frame or flags or
 * one larger than the device budget, CFAR_ESHUTDOWN after destroy began. */
int cfar_submit(cfar_server *s, const cfar_map *frame, int32_t flags, uint64_t user_tag,
                uint64_t *ticket_out);

/* Collect up to `max` completions, waiting up to timeout_us (0 = do not
 * wait, < 0 = wait for at least one).  *n_out = number written.  A timeout
 * with nothing completed returns CFAR_OK with *n_out = 0. */
int cfar_poll(cfar_server *s, cfar_completion *out, int32_t max, int32_t timeout_us, int32_t *n_out);

/* Counters of the server (thread-safe snapshot). */
int cfar_server_stats_get(cfar_server *s, cfar_server_stats *out);

/* Stop accepting frames (later submits give CFAR_ESHUTDOWN) and wait until
 * nothing is in flight.  drain_queued = 1: frames still queued are run;
 * 0: they complete with status CFAR_ESHUTDOWN without touching the device.
 * Completions stay pollable afterwards.  Idempotent. */
int cfar_server_shutdown(cfar_server *s, int32_t drain_queued);

/* cfar_server_shutdown(s, 0) if not yet done, then stop the scheduler thread
 * and free the server, its streams and its device pool.  Completions not yet
 * polled are dropped. */
int cfar_server_destroy(cfar_server *s);

/* ------------------------------------------------------------------------ */
/* Building the map from a raw record (Sec. II.A)                            */
/* ------------------------------------------------------------------------ */

/* Parameters of the primary signal processing.  The paper names the steps
 * and the respiration band (0.3-0.8 Hz); the rest is not stated there. */
typedef struct {
    double fs_slow;     /* slow-time sample rate, traces per second, > 0        */
    double f_lo, f_hi;  /* band kept, Hz, 0 <= f_lo <= f_hi (inclusive)         */
    int32_t mean_len;   /* slow-time mean filter length, odd, 1..1023 (1: none) */
    int32_t out_dtype;  /* type of the map written: CFAR_F32 or CFAR_F64        */
} cfar_mapbuild_params;

/* The DFT bins the band keeps for n_traces traces: k = first_bin ..
 * first_bin + n_bins - 1 with first_bin = ceil(f_lo N / fs), last =
 * min(floor(f_hi N / fs), N / 2).  CFAR_EINVAL if the band holds none, or
 * n_traces is outside [1, 4000], or a parameter is out of range. */
int cfar_map_bins(int64_t n_traces, const cfar_mapbuild_params *params, int32_t *first_bin, int32_t *n_bins);

/* Device workspace bytes for cfar_map_build (0 if an argument is invalid). */
size_t cfar_map_build_workspace_bytes(int64_t n_traces, int64_t n_samples, const cfar_mapbuild_params *params);

/* The range x slow-time-frequency power map of a raw record (Sec. II.A):
 * raw: device, n_traces traces of n_samples fast-time samples, trace n at
 * raw + n * ld_raw (elements, raw_dtype CFAR_F32 or CFAR_F64).  Steps: per
 * trace, DC-shift removal and linear-trend subtraction (least-squares line
 * over the sample index); per range bin, the centred mean filter of
 * mean_len along slow time (averaging the samples inside the record at its
 * ends); normalisation by the record's largest filtered magnitude (one
 * scalar; an all-zero record gives a zero map); per range bin, the DFT over
 * slow time, kept for the band's bins, as power |F(k)|^2.  map_out: device,
 * n_samples rows (range bins) x n_bins columns (band bins, see
 * cfar_map_bins), leading dimension ld_map >= n_bins, params->out_dtype; it
 * is a map that cfar2d takes as is.  FP64 arithmetic throughout.  Errors:
 * CFAR_EINVAL, CFAR_ENOSPC, CFAR_EDEVICE. */
int cfar_map_build(const void *raw, int32_t raw_dtype, int64_t n_traces, int64_t n_samples, int64_t ld_raw,
                   const cfar_mapbuild_params *params, void *map_out, int64_t ld_map, void *ws, size_t ws_bytes,
                   void *stream);

/* ------------------------------------------------------------------------ */
/* Detection lists and bit-packed masks                                      */
/* ------------------------------------------------------------------------ */

/* One detection: a cell decided H1 (eq. 1: CUT > T). */
typedef struct {
    int32_t row, col;  /* the cell */
    double cut;        /* X(row, col) as FP64 */
    double threshold;  /* T of eq. (2) at the cell from the map's threshold
                          output, NaN when the map has none */
} cfar_detection;      /* 24 bytes */

/* Device workspace bytes for cfar_detections on map m (0 if m is invalid). */
size_t cfar_detections_workspace_bytes(const cfar_map *m);

/* The detections of map m -- the cells whose mask byte is nonzero, after
 * cfar2d / cfar2d_batched wrote m->mask on the same stream -- as records in
 * row-major order of the cells.  m: host descriptor (x, mask and the
 * optional threshold are read; win is not).  out: device array of
 * `capacity` records (may be NULL when capacity is 0); the first
 * min(count, capacity) records are written, the rest are not.  count:
 * device int64, receives the number of detections (which may exceed
 * capacity).  ws: device, >= cfar_detections_workspace_bytes(m), not used by
 * another call until this one's work on `stream` has finished.  Errors:
 * CFAR_EINVAL (invalid map fields, capacity < 0, out NULL with capacity > 0,
 * count or ws NULL), CFAR_ENOSPC, CFAR_EDEVICE. */
int cfar_detections(const cfar_map *m, cfar_detection *out, int64_t capacity, int64_t *count, void *ws,
                    size_t ws_bytes, void *stream);

/* Bit-packed copy of map m's mask: bit u of word w of row r is cell
 * (r, 32 w + u); bits past the last column are 0.  bits: device,
 * rows x ld_words uint32, ld_words >= ceil(cols / 32).  One eighth of the
 * mask's bytes to copy back.  Errors: CFAR_EINVAL, CFAR_EDEVICE. */
int cfar_mask_pack(const cfar_map *m, uint32_t *bits, int64_t ld_words, void *stream);

/* ------------------------------------------------------------------------ */
/* Kernel timing (benchmarks)                                                */
/* ------------------------------------------------------------------------ */

/* On the calling thread, on = 1 makes every following TILED launch
 * (cfar2d, cfar2d_with_plan, cfar2d_batched) record a pair of HIP events
 * on its stream right before and right after its persistent kernel; batches
 * are then launched without graph capture.  DIRECT launches record them
 * before the first map's stencil and after the last one's.  on = 0 turns
 * it off. */
int cfar_timing_enable(int32_t on);

/* Milliseconds between the two events of the calling thread's last timed
 * launch (waits for it to finish).  CFAR_EINVAL if there was none. */
int cfar_timing_read(double *kernel_ms);

/* Message describing the last failure on the calling thread ("" if none). */
const char *cfar_last_error(void);

/* Library version string. */
const char *cfar_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CFAR2D_H */
