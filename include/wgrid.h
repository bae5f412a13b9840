/*
 * wgrid.h -- C ABI of libwgrid: w-projection convolutional gridding with compression on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: D. Muscat, "High-Performance Image Synthesis for Radio Interferometry",
 * M.Sc. thesis 2013 (arXiv:1403.4209), chapter "The Malta-imager":
 *   - Convolution Function Generator (Algorithm convgen, eqs. choose, sat, sum)
 *     -> wg_ktable_sizes / wg_ktable_build
 *   - WImager preparation phase (PreProcessUVW, eqs. ci and conj, Algorithms index and
 *     compressindex, eqs. compress1 and conjugatetake, statistics logic, eq. normalizer)
 *     -> wg_compress
 *   - WImager gridding phase (eq. gridding) -> wg_grid
 *   - the whole WImager component, records to grid and normaliser -> wg_grid_records
 *   - the exact adjoint of eq. gridding (not in the thesis) -> wg_degrid
 *
 * Conventions shared by every call
 *   - Pointers are DEVICE pointers owned by the caller unless marked [host]. The library
 *     allocates nothing on the device and keeps no state between calls.
 *   - Calls check their arguments on the host and return an error before enqueuing any
 *     work; then they enqueue on `stream` (a hipStream_t; NULL = the null stream) and
 *     return without waiting, except wg_ktable_build, which waits for its own work.
 *   - A HIP error seen at launch is returned as WG_EHIP; an error of earlier asynchronous
 *     work may surface on a later call.
 *   - No C++ exception crosses this interface.
 *   - Records: nb baselines x nc channels x nt timesteps, record r = (b*nc + ch)*nt + t.
 *     uvw is float64 [nb][nt][3] in metres (input I-1), inv_lambda float64 [nc] in 1/m
 *     (I-2), vis complex64 [nb][nc][nt][P] as interleaved (re, im) float32 (I-5), weight
 *     float32 [nb][nc][nt][P] (I-3; NULL means 1), flag uint8 [nb][nc][nt][P] (I-4;
 *     nonzero = flagged; NULL means none), with P = g->n_pol polarisations per record
 *     (WImager inputs: flags, weights and visibilities per polarisation).
 *   - Grid: complex64 [P][n][n] interleaved, one plane per polarisation, row y follows v,
 *     column x follows u, cell (n/2, n/2) is u = v = 0 (gridding phase, Convolution Position
 *     sequence). Per-channel grids are [nc][P][n][n].
 *   - Off-grid, flagged or non-finite records are not errors: they are not griddable
 *     (gridding indicator g = 0) and are counted in wg_stats. A record with at least one
 *     unflagged polarisation is griddable; its flagged polarisations add 0.
 */
#ifndef WGRID_H
#define WGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *wg_stream_t; /* hipStream_t */

typedef enum wg_status {
    WG_OK = 0,
    WG_EINVAL = -1,        /* a pointer, size or geometry value is invalid              */
    WG_ECAPACITY = -3,     /* an output or workspace buffer is too small                 */
    WG_EHIP = -4,          /* the HIP runtime reported an error                          */
    WG_EUNSUPPORTED = -5   /* valid but outside what this build handles (sizes below)    */
} wg_status;

typedef enum wg_kdtype {
    WG_KF32 = 0,   /* complex samples as 2 x float32 (8 bytes)                          */
    WG_KBF16 = 1,  /* 2 x bfloat16 (4 bytes), round-to-nearest-even from the FP64 master */
    WG_KF16 = 2    /* 2 x float16 (4 bytes), round-to-nearest-even from the FP64 master  */
} wg_kdtype;

/* wg_geom.flags */
#define WG_COMPRESS 1u   /* merge consecutive records with the same key (eq. compression) */
#define WG_GRID_PER_CHANNEL 2u /* one grid per channel, as the thesis's imaging tool sets up one
                                  WImager instance per channel; without it every channel goes to
                                  one grid (the channel interleaving of its Data Set 0 runs)  */
#define WG_POL_CIRCULAR 8u     /* the records' products are RR, RL, LR, LL (or RR, LL) rather
                                  than XX, XY, YX, YY (or XX, YY); used by wg_finalise's Stokes
                                  conversion only                                              */
#define WG_PLAIN_SUMS 16u      /* wg_grid: plain FP32 sums per owned cell between commits, as the
                                  thesis's single-precision gridder; without it the sums are
                                  Kahan-compensated                                            */
#define WG_W_STACKING 4u       /* w-stacking (eq. stacking): one grid per w-plane, every record
                                  gridded with the w = 0 kernel (plane 0's support, slices and
                                  zeta) on the grid of its w-plane; the w-term is applied in the
                                  image plane by wg_finalise_stacked. Excludes
                                  WG_GRID_PER_CHANNEL.                                         */

/* Limits of this build. */
#define WG_MAX_SUPPORT 511   /* largest kernel support (odd)                            */
#define WG_MAX_PLANES 256    /* largest number of w-planes                              */
#define WG_MAX_FFT 2048      /* largest beta * m_img (oversampled table side)           */

/*
 * Imaging geometry (Convolution Function Generator "General points"; WImager outputs).
 *   n       grid side N, even, 2..32768 (the u = v = 0 cell is (n/2, n/2)).
 *   beta    oversampling factor (eq. local:o), a power of two in 2..32.
 *   n_w     number of w-planes, 1..WG_MAX_PLANES, planes at w_max*(k/(n_w-1))^2 (sqrt(w)
 *           spacing; |w| above w_max uses the last plane).
 *   s_lo, s_hi  odd supports, 1 <= s_lo <= s_hi <= WG_MAX_SUPPORT. Plane k gets
 *           S_k = min(s_hi, max(S_nat(k), s_lo + 2*floor(((s_hi-s_lo)*k + n_w-1)/(2(n_w-1)))))
 *           where S_nat is the support found from the 1e-3 threshold (pad/trim as in the
 *           generator's normal mode).
 *   m_img   image samples per side used to build the table (power of two, >= 16,
 *           beta*m_img <= WG_MAX_FFT, and (s_hi-1)/2*beta + beta/2 < beta*m_img/2).
 *   du      uv cell size in wavelengths (> 0); the image field of view is 1/du.
 *   w_max   largest |w| tabulated, wavelengths (>= 0).
 *   flags   WG_COMPRESS, WG_POL_CIRCULAR, WG_PLAIN_SUMS, and at most one of
 *           WG_GRID_PER_CHANNEL and WG_W_STACKING; or 0 (unknown bits or both grid modes:
 *           WG_EINVAL).
 *   n_pol   polarisations per record P: 1 (0 is read as 1), 2 (the parallel hands XX, YY or
 *           RR, LL) or 4 (XX, XY, YX, YY or RR, RL, LR, LL), in that order; others are
 *           WG_EINVAL.
 *           The flip of a record with w < 0 (eq. conj) conjugates each value; with P = 4 it
 *           also exchanges the cross hands with their weights and flags (the partner of a
 *           polarised record: V_pq(-u) = conj V_qp(u)).
 */
typedef struct wg_geom {
    int32_t n;
    int32_t beta;
    int32_t n_w;
    int32_t s_lo;
    int32_t s_hi;
    int32_t m_img;
    double du;
    double w_max;
    uint32_t flags;
    int32_t n_pol;
} wg_geom;

/*
 * Convolution-function table (outputs C-1, C-2, C-3 of the generator).
 *   support [n_w]      S_k (C-2, first element)
 *   offset  [n_w+1]    start of plane k in `data`, in complex elements (C-2, second)
 *   wbound  [n_w]      lower |w| edge of plane k (entry 0 unused): the nearest plane in
 *                      sqrt(w); wbound[j] = w_max*((j-1/2)/(n_w-1))^2
 *   zeta    [n_w*beta*beta]  sum of the real parts of each S_k x S_k matrix (eq. sum; the
 *                      repeated columns excluded), of the values as stored in `data`, in
 *                      FP64 (C-3)
 *   data               C-1: plane k holds beta*beta matrices of S_k rows, each row
 *                      S_k + 2P samples (P = 1 for WG_KF32, 3 for WG_KBF16 and WG_KF16),
 *                      row-major, matrix index (o_v + beta/2 - 1)*beta + (o_u + beta/2 - 1)
 *                      for oversample offsets o in (-beta/2, beta/2]; matrix element [i][j],
 *                      0 <= j < S_k, is the kernel at fine offsets ((i-H)*beta - o_v,
 *                      (j-H)*beta - o_u), H = (S_k-1)/2, normalised so the w=0 kernel's
 *                      centre is 1 (eq. choose with row = v, column = u), and sits at row
 *                      position P + j; positions 0..P-1 repeat columns S_k-P..S_k-1 and
 *                      positions P+S_k..P+S_k+P-1 repeat columns 0..P-1 (so that P + 1
 *                      neighbouring columns, one 16-byte load, read forwards or backwards,
 *                      are adjacent also where they wrap).
 *   data_cap           capacity of `data` in complex elements.
 *   dtype, n_w, beta   must match the geometry; s_max is written by wg_ktable_build.
 * All pointers are device memory owned by the caller.
 */
typedef struct wg_ktable {
    int32_t dtype;
    int32_t n_w;
    int32_t beta;
    int32_t s_max;
    int32_t *support;
    int64_t *offset;
    double *wbound;
    double *zeta;
    void *data;
    int64_t data_cap;
} wg_ktable;

/*
 * Runs produced by wg_compress (filtered sequences FS-1..FS-5 with the compression of
 * Algorithm compressindex folded in). Run q covers records start[q] .. start[q]+len[q]-1 of
 * one (baseline, channel) segment, all with pixel (x, y) relative to the grid centre,
 * w-plane `plane` and oversample offsets (ou, ov); gamma [capacity][P] is per polarisation
 * the sum over its records of weight * (1 - flag) * (vis, conjugated when w < 0), as float32
 * (re, im) (eqs. compress1, conjugatetake). Runs are in record order.
 * `plan` is a device work list the gridder reads (local chunks of equal support, grouped by
 * support); size it with wg_plan_elems. It also holds the work counters of wg_degrid and
 * (on grids of side 4096 and more) wg_grid, so two wg_degrid calls, or two wg_grid calls, on
 * the same runs must not overlap in time.
 * With WG_GRID_PER_CHANNEL, `grid` (one int16 per run: the channel of its records, i.e. the
 * grid it goes to) and `norm` (one double per channel: that channel's normaliser N of eq.
 * normalizer) are required and written by wg_compress. With WG_W_STACKING, `grid` is
 * required and holds the run's w-plane (its grid), `plane` is 0 (the kernel used) and `norm`
 * may be NULL (the one normaliser is in the statistics). With P > 1, `norm` is required
 * and holds the normaliser of each polarisation, [nc][P] with per-channel grids, else [P].
 * Otherwise both may be NULL. `work` is scratch that wg_degrid overwrites (P complex
 * floats per run). Every array has `capacity` entries (gamma and work 2P floats each);
 * capacity must be >= nb*nc*nt, so the run list can never overflow.
 */
typedef struct wg_runs {
    int64_t capacity;
    int32_t *start;
    int32_t *len;
    int32_t *x;
    int32_t *y;
    int16_t *plane;
    int8_t *ou;
    int8_t *ov;
    float *gamma;
    int32_t *plan;
    int64_t plan_elems;
    float *work;
    int16_t *grid;
    double *norm;
} wg_runs;

/*
 * Statistics of one wg_compress call (statistics logic and eq. normalizer), written on the
 * device: n_records; n_griddable = sum (g+c); n_runs = sum g (records gridded by the
 * gridder); n_compressed = sum c; upd_real = sum g*S^2 (grid-point updates executed);
 * upd_saved = sum c*S^2 (updates saved by compression); normaliser = N of eq. normalizer
 * (FP64; of the first polarisation, over all grids); n_items = number of local chunks in
 * the plan. Update counts are per polarisation (a run of support S updates S^2 cells of
 * each of the P grids).
 */
typedef struct wg_stats {
    int64_t n_records;
    int64_t n_griddable;
    int64_t n_runs;
    int64_t n_compressed;
    int64_t upd_real;
    int64_t upd_saved;
    double normaliser;
    int64_t n_items;
} wg_stats;

/* Human-readable name of a status code. Never NULL. */
const char *wg_status_str(int status);

/* Library ABI version (major*10000 + minor*100 + patch). */
int wg_version(void);

/*
 * Sizes for wg_ktable_build, from the geometry alone (Algorithm convgen).
 * [host] data_elems_max: complex elements `data` must hold for any table type (every plane
 *        at s_hi with the widest padding: n_w * beta^2 * s_hi * (s_hi + 6)).
 * [host] ws_bytes: device workspace the build needs.
 * Errors: WG_EINVAL (NULL pointer or invalid geometry), WG_EUNSUPPORTED (limits above).
 */
int wg_ktable_sizes(const wg_geom *g, int64_t *data_elems_max, size_t *ws_bytes);

/*
 * Build the table on the GPU (Algorithm convgen): evaluate the separable prolate
 * spheroidal taper (c = 3*pi) times the inverse w-screen exp(+2 pi i w (sqrt(1-l^2-m^2)-1))
 * on m_img x m_img image samples, zero-pad to beta*m_img, forward FFT, normalise by the w=0
 * plane's centre value, find each plane's natural support from the 1e-3 magnitude
 * threshold, apply the support law, trim, reorder into matrices, round to kt->dtype and
 * sum real parts into zeta. kt->dtype, n_w, beta and the device pointers are inputs; the
 * arrays behind them and kt->s_max are outputs. [host] support_out[n_w] and
 * offset_out[n_w+1] receive copies when non-NULL. Waits for its own work before returning.
 * Errors: WG_EINVAL, WG_EUNSUPPORTED, WG_ECAPACITY (ws_bytes or data_cap too small),
 * WG_EHIP.
 */
int wg_ktable_build(const wg_geom *g, wg_ktable *kt, void *ws, size_t ws_bytes,
                    int32_t *support_out, int64_t *offset_out, wg_stream_t stream);

/* int32 elements of wg_runs.plan for `capacity` records in `n_segments` = nb*nc segments. */
int64_t wg_plan_elems(int64_t capacity, int64_t n_segments);

/*
 * Preparation phase: per record the discrete choices (pixel, oversample offsets, w-plane,
 * take-conjugate, gridding indicator) in FP64 with the same rounding as the definitions:
 * x = fl(fl(u*inv_lambda) * beta/du), fine index t with t - 1/2 < x <= t + 1/2, pixel
 * X = floor((t + beta/2 - 1)/beta), o = t - beta*X, plane = #{j >= 1 : |w| >= wbound[j]},
 * flip when w(metres) < 0. A record is griddable when finite, unflagged and all its S x S
 * taps fall on the grid. With WG_COMPRESS, a griddable record whose griddable predecessor
 * in the same (baseline, channel) segment has the same (x, y, plane, ou, ov) joins that
 * run (eqs. compression and ci); otherwise it starts a new run. Writes runs, the plan and
 * *stats (device). Overwrites previous contents.
 * Errors: WG_EINVAL (NULL required pointer, sizes < 1, geometry/table mismatch),
 * WG_ECAPACITY (runs->capacity < nb*nc*nt or plan too small), WG_EUNSUPPORTED
 * (nb*nc*nt >= 2^31), WG_EHIP.
 */
int wg_compress(const wg_geom *g, const wg_ktable *kt, const double *uvw, const double *inv_lambda,
                const float *vis, const float *weight, const uint8_t *flag, int64_t nb, int32_t nc,
                int32_t nt, wg_runs *runs, wg_stats *stats, wg_stream_t stream);

/*
 * Gridding phase (eq. gridding): for every run and polarisation p, grid[p][row0+i][a+j] +=
 * gamma[p] * K[i][j] with
 * a = x + n/2 - H, row0 = y + n/2 - H, K the run's matrix. ACCUMULATES into `grid`
 * (complex64 [P][n][n], or [nc][P][n][n] with WG_GRID_PER_CHANNEL or [n_w][P][n][n]
 * with WG_W_STACKING, run q going to grid runs->grid[q]); the caller zeroes it first.
 * Accumulation is FP32: Kahan-compensated sums per owned cell between commits (plain sums
 * with g->flags & WG_PLAIN_SUMS, as in the thesis's single-precision gridder), and commits
 * with FP32 atomic adds, so the last bits depend on scheduling. `runs`, `stats` come from wg_compress with the same g and kt.
 * Errors: WG_EINVAL, WG_EUNSUPPORTED (kt->data_cap >= 2^28 elements: table byte offsets
 * are 32-bit), WG_EHIP.
 */
int wg_grid(const wg_geom *g, const wg_ktable *kt, const wg_runs *runs, const wg_stats *stats,
            float *grid, wg_stream_t stream);

/*
 * Workspace of wg_grid_records for nb x nc x nt records (WImager inputs I-1..I-5): the run
 * arrays of wg_runs with capacity nb*nc*nt (so the run list cannot overflow), the per-run
 * grid ids (per-channel grids or w-stacking), the normalisers ([nc][P] with per-channel
 * grids, else [P]) and the plan, each on a 256-byte boundary.
 *   ws == NULL: [host] *ws_bytes receives the size in bytes.
 *   ws != NULL: a device workspace of *ws_bytes bytes, 256-byte aligned; [host] *runs
 *           (when non-NULL) receives the wg_runs view of it that wg_grid_records uses, so the
 *           runs it leaves there can be passed to wg_degrid, wg_grid or wg_finalise
 *           (runs->norm). No device work is done.
 * Errors: WG_EINVAL (NULL ws_bytes, invalid geometry, sizes < 1, ws misaligned),
 * WG_ECAPACITY (*ws_bytes too small), WG_EUNSUPPORTED (nb*nc*nt >= 2^31).
 */
int wg_grid_records_ws(const wg_geom *g, int64_t nb, int32_t nc, int32_t nt, void *ws, size_t *ws_bytes,
                       wg_runs *runs);

/*
 * Records to grid in one call: the WImager component with the generator's table (inputs
 * I-1..I-5 and C-1..C-3; outputs O-1, the grid, and O-2, the normaliser of eq. normalizer).
 * The preparation phase of wg_compress (keys, compression of eqs. compression and ci with
 * g->flags & WG_COMPRESS, weighting of eqs. compress1 and conjugatetake; without
 * WG_COMPRESS every griddable record is its own run) followed by the gridding phase of
 * wg_grid (eq. gridding), with the same arguments, layouts and accumulation:
 *   grid   complex64 [P][n][n] (or [nc][P][n][n] / [n_w][P][n][n]), ACCUMULATES
 *   stats  device wg_stats of the batch (normaliser N of the first polarisation)
 *   ws     device workspace of at least wg_grid_records_ws's size, 256-byte aligned; the
 *          run list, plan and per-grid normalisers are left there (OVERWRITTEN each call)
 *   runs_out [host] optional: receives the wg_runs view of ws (as wg_grid_records_ws gives)
 * Enqueues on `stream` and returns without waiting. Two calls sharing a workspace must not
 * overlap in time.
 * Errors: those of wg_compress and wg_grid, all checked before any work is enqueued;
 * WG_ECAPACITY (ws_bytes too small), WG_EINVAL (ws NULL or misaligned).
 */
int wg_grid_records(const wg_geom *g, const wg_ktable *kt, const double *uvw, const double *inv_lambda,
                    const float *vis, const float *weight, const uint8_t *flag, int64_t nb, int32_t nc,
                    int32_t nt, float *grid, wg_stats *stats, void *ws, size_t ws_bytes, wg_runs *runs_out,
                    wg_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): wg_grid_records with its workspace in a fixed
 * array of WG_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on until the
 * process ends, instead of a workspace argument. Arguments, layouts, accumulation and
 * errors are those of wg_grid_records without ws and ws_bytes; it allocates nothing.
 *   runs_out [host] optional: the wg_runs view of the array on the current device, valid
 *            until the next call on that device (wg_degrid may use it in between).
 * The current device must be the one `stream` and the pointers belong to. Every call on a
 * GPU shares that GPU's array and leaves its contents there: calls that overlap in time on
 * one GPU (other streams or threads) race and give wrong results.
 * Errors: WG_ECAPACITY when the batch's workspace (wg_grid_records_ws) exceeds
 * WG_STATIC_SCRATCH_BYTES (about 1.5 million records with one polarisation, 0.7 million
 * with four); WG_EHIP when the array's device address cannot be had; otherwise those of
 * wg_grid_records.
 */
#define WG_STATIC_SCRATCH_BYTES (64u << 20)
int wg_grid_records_static(const wg_geom *g, const wg_ktable *kt, const double *uvw, const double *inv_lambda,
                           const float *vis, const float *weight, const uint8_t *flag, int64_t nb, int32_t nc,
                           int32_t nt, float *grid, wg_stats *stats, wg_runs *runs_out, wg_stream_t stream);

/*
 * Adjoint of wg_compress + wg_grid with respect to the visibilities: per run
 * d[p] = sum_ij conj(K[i][j]) * grid[p][row0+i][a+j] (grid complex64 [P][n][n], or
 * [nc][P][n][n] / [n_w][P][n][n] read at grid runs->grid[q] with WG_GRID_PER_CHANNEL /
 * WG_W_STACKING; FP32, pairwise/tree summation; partial sums of the waves sharing a run
 * are combined with FP32 atomic adds into runs->work, so the last
 * bits depend on scheduling); polarisation p of record r of the run gets weight_{r,p} *
 * (1 - flag_{r,p}) * (d[p], or conj(d[s]) when w_r(metres) < 0, s the slot its value went
 * to); records in no run get 0. OVERWRITES vis_out (complex64 [nb][nc][nt][P]) and
 * runs->work. uvw, weight, flag and the sizes must be those given to wg_compress.
 * Errors: WG_EINVAL (runs->work NULL among others), WG_ECAPACITY, WG_EUNSUPPORTED, WG_EHIP.
 */
int wg_degrid(const wg_geom *g, const wg_ktable *kt, const wg_runs *runs, const wg_stats *stats,
              const float *grid, const double *uvw, const float *weight, const uint8_t *flag, int64_t nb,
              int32_t nc, int32_t nt, float *vis_out, wg_stream_t stream);

/*
 * Image finaliser (Algorithm finalizer): inverse 2-D FFT of each polarised grid, each over
 * its normaliser N_p (eq. normalizer; read on the device, e.g. &stats->normaliser with P = 1,
 * or runs->norm (+ c*P for channel c of per-channel grids)), combined into Stokes images and
 * their real parts taken; then divided by the prolate taper psi_0(3 pi, 2 l du) normalised
 * to 1 at the centre (sec. convgriddingmath) and by sinc(pi l du / beta) sinc(pi m du /
 * beta) (eq. coversampled). Image pixel [q][p] holds (l, m) = ((p - n/2), (q - n/2)) /
 * (n du); the real part is taken because each record is gridded once, at its w >= 0
 * representative (eq. conj). Stokes images, by the feed relations XX = I + Q, XY = U + iV,
 * YX = U - iV, YY = I - Q (linear) or RR = I + V, RL = Q + iU, LR = Q - iU, LL = I - V
 * (WG_POL_CIRCULAR): P = 1 gives the one polarisation as I; P = 2 gives (I, Q), or (I, V)
 * for circular feeds; P = 4 gives (I, Q, U, V). A polarisation whose normaliser is 0 adds
 * 0. Pixels where the taper is zero (first row and column) are 0. FFTs in FP32.
 *   grid   complex64 [P][n][n] (device, read only)
 *   normaliser  P device doubles
 *   image  float32 [P][n][n] (device, OVERWRITTEN), the Stokes images in the order above
 *   ws     device workspace of wg_finalise_ws_bytes bytes (two n x n complex64 buffers,
 *          P n x n float32 accumulators, twiddles, corrections; the same size serves
 *          wg_finalise_stacked)
 * n must be a power of two, 16..8192 (one FP32 complex row in 64 KB of LDS).
 * Errors: WG_EINVAL, WG_ECAPACITY (ws too small), WG_EUNSUPPORTED (n), WG_EHIP.
 */
int wg_finalise_ws_bytes(const wg_geom *g, size_t *ws_bytes);
int wg_finalise(const wg_geom *g, const float *grid, const double *normaliser, float *image, void *ws,
                size_t ws_bytes, wg_stream_t stream);

/*
 * W-stacking image (eq. stacking): the w-plane grids of WG_W_STACKING are each inverse
 * transformed, multiplied in the image plane by the plane's w-term correction
 * exp(+2 pi i w_k (sqrt(1 - l^2 - m^2) - 1)) (0 where l^2 + m^2 > 1), w_k = w_max (k/(n_w-1))^2
 * the plane's w, and added; then, as in wg_finalise, the real part over the normaliser,
 * divided by the taper and sinc corrections. The correction is the image-plane factor that
 * the w-projection kernel of plane k carries (eq. C_W), so the stacked image equals the
 * w-projection image up to the truncation of the kernels to their supports.
 *   grids  complex64 [n_w][P][n][n] (device, read only), grid k holding w-plane k's records;
 *          with P > 1 each product is stacked and the Stokes images are formed as in
 *          wg_finalise (image [P][n][n], normaliser P doubles)
 *   normaliser, image, ws as for wg_finalise (ws of wg_finalise_ws_bytes bytes). The
 *   accumulation over planes is FP32, plane by plane in order.
 * Errors: as wg_finalise; WG_EINVAL also when g->flags lacks WG_W_STACKING.
 */
int wg_finalise_stacked(const wg_geom *g, const float *grids, const double *normaliser, float *image, void *ws,
                        size_t ws_bytes, wg_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* WGRID_H */
