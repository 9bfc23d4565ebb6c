/*
 * mgseg.h -- C ABI of libmgseg: FAS multigrid with the jump-aware Hybrid
 * Smoother 2 for the selective level-set segmentation models of
 * Roberts, Chen & Irion, "A Multigrid Algorithm with Non-Standard Smoother
 * for Two Selective Models in Variational Segmentation" (arXiv 1807.02137).
 *
 * Problem (Sec. 2.2): given an image z on the grid and a marker set S of
 * points on or near the object of interest, find the level-set function phi
 * whose positive set is the selected object, by solving the discrete
 * Euler-Lagrange equations of the Spencer-Chen model (eq. scel) or the
 * Rada-Chen model (eq. rcel, discretised in eq. rcabcd / abcdrc) with the FAS
 * V-cycle of the Algorithm-1 box driven by Hybrid Smoother 2 (Sec. 4.3;
 * "Algorithm 3" of Sec. 4).
 *
 * Conventions for every entry point:
 *  - All arrays are row-major, element (i, j) at ptr[i * pitch + j], with
 *    i the row (0..n-1) and j the column (0..m-1); pitches are in elements.
 *  - "_dev" pointers are device (HBM) pointers of the current HIP device;
 *    "_host" pointers are host memory.  The caller owns every pointer it
 *    passes in; the library copies what it needs before returning.
 *  - All work is enqueued on the stream given at setup.  Calls that return
 *    host values (vcycle, solve, get_stats, the debug getters) synchronise
 *    that stream before returning.
 *  - No entry point aborts or throws: each returns an mgseg_status.  On an
 *    argument error the context is left unchanged.
 *  - One host thread may use a context at a time; distinct contexts may be
 *    used concurrently on distinct streams.
 */
#ifndef MGSEG_H
#define MGSEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgseg_ctx mgseg_ctx;

typedef enum {
    MGSEG_OK = 0,
    MGSEG_E_ARG = 1,            /* invalid argument (null pointer, bad value)        */
    MGSEG_E_SHAPE = 2,          /* n, m not divisible by 2^(levels-1), or too small  */
    MGSEG_E_NOMEM = 3,          /* device allocation failed                          */
    MGSEG_E_HIP = 4,            /* a HIP runtime call failed                         */
    MGSEG_E_NONFINITE = 5,      /* a residual norm became NaN/Inf                    */
    MGSEG_E_NOT_CONVERGED = 6,  /* solve hit max_cycles; outputs are still valid     */
    MGSEG_E_STATE = 7,          /* call not valid in the context's current state     */
    MGSEG_E_SCRATCH = 8         /* image too large for mgseg_solve_noalloc's scratch */
} mgseg_status;

typedef enum { MGSEG_SPENCER_CHEN = 0, MGSEG_RADA_CHEN = 1 } mgseg_model;

/* Model and solver parameters.  Defaults (mgseg_params_default) follow the
 * paper where it fixes a value (Sec. 5: mu = 1/2, nu = 1, eps = 1, V-cycle)
 * and the project's stated readings elsewhere. */
typedef struct {
    uint32_t struct_size;   /* must be sizeof(mgseg_params)                          */
    int32_t model;          /* mgseg_model                                           */
    double mu;              /* curvature weight (eq. scfunc / rcfunc)                */
    double lambda1, lambda2;/* fitting weights, for intensities in [0, 1]            */
    double theta;           /* Spencer-Chen selection weight (eq. scfunc)            */
    double nu;              /* Rada-Chen area weight (eq. rcfunc)                    */
    double eps;             /* smoothed Heaviside width, in phi units (Sec. 2)       */
    double eps_tv_px;       /* |grad phi| regularisation, phi units per pixel        */
    double beta;            /* edge detector g(s) = 1/(1 + beta s), s per pixel      */
    double sigma_g;         /* pre-blur of z for the edge detector, pixels           */
    double sigma_d;         /* width of the marker distance function, domain units   */
    double Sigma;           /* jump threshold on the coefficient ratio (Sec. 5.2)    */
    double M;               /* bound |phi| <= M                                      */
    int32_t nu1, nu2;       /* pre/post smoothing: Hybrid-2 outer iterations         */
    int32_t levels;         /* grids including the finest; 0 = as many as fit        */
    int32_t coarse_iters;   /* most outer iterations on the coarsest grid            */
    int32_t mixed_precision;/* 1: FP32 cycles + FP64 finest defect correction        */
    int32_t scaled;         /* 1: each equation row divided by delta_eps(psi_ij)     */
    double coarse_rtol;     /* coarsest solve stops once an outer iteration moves no */
                            /* value by more than coarse_rtol times the largest      */
                            /* total change since that solve began                   */
    int32_t smoother;       /* 0: Hybrid Smoother 2 (Sec. 4.3, the paper's Algorithm */
                            /* 3); 1: GSLEX-I (Sec. 3.2), one point Gauss-Seidel     */
                            /* pass per outer iteration in the rows' four-class      */
                            /* order, the standard smoother of the paper's Algorithm */
                            /* 1; 2: Hybrid Smoother 1 (Sec. 4.2, Algorithm 2):      */
                            /* GSLINE-I on every column (four column classes), then  */
                            /* the collective update at every jump-set cell of the   */
                            /* cell and its neighbours except the one behind its     */
                            /* smallest coefficient (eight cell classes); needs      */
                            /* mixed_precision = 1 and columns of at most 1024       */
                            /* cells (n <= 1024); 3: GSLINE-I (Sec. 3.2, eq.         */
                            /* system), one line system per column per outer         */
                            /* iteration (four column classes; needs                 */
                            /* mixed_precision = 1 and n <= 1024); 4: NEWT-I (Sec.   */
                            /* 3.2, eq. newtrc), GSLEX-I's pass with the derivative  */
                            /* of the Rada-Chen area term on each diagonal (Spencer- */
                            /* Chen: the same as 1); 5 GSLEX-II, 6 GSLINE-II, 7      */
                            /* NEWT-II: the local variants, each pixel's (column's)  */
                            /* coefficients refreshed from the current iterate where */
                            /* they are used, rows (columns) in four classes;        */
                            /* Spencer-Chen only (NEWT-II is then GSLEX-II),         */
                            /* mixed_precision = 1, GSLINE-II columns of at most     */
                            /* 1024 cells (MGSEG_E_ARG otherwise); default 0         */
    int32_t run_max;        /* superpixels of Hybrid Smoother 2 (Sec. 4.3, Fig. 3):  */
                            /* 0 (default) solves every maximal run of starred cells */
                            /* on a line as one unit, as the paper does (lines       */
                            /* longer than 1024 cells cut runs at 1024 cells); k > 0 */
                            /* cuts longer runs into ceil(len / k) near-equal pieces */
                            /* (3: every unit in closed form); negative: MGSEG_E_ARG */
} mgseg_params;

typedef struct {
    double c1, c2;          /* region means (eq. c1c2)                               */
    double rel_res;         /* |r~_k| / |r~_0| on the finest grid: the projected     */
                            /* residual of the paper's equations (eq. abcdrc, every  */
                            /* row with its factor delta_eps(phi_ij)); mgseg_solve   */
                            /* stops on it                                           */
    double res;             /* |r~_k| (FP64)                                         */
    double res0;            /* |r~_0|                                                */
    double eta;             /* paper's relative change |phi_k - phi_k-1|/|phi_k-1|   */
    int32_t cycles;         /* V-cycles done since setup / last set_phi0             */
    int32_t levels;
    double frac_fg;         /* fraction of pixels with phi > 0                       */
    double energy;          /* the model's discrete energy at the finest phi with    */
                            /* the current c1, c2 (Sec. 2: the Spencer-Chen or       */
                            /* Rada-Chen functional; central differences, h^2 cells) */
    double frac_D;          /* fraction of finest cells in the jump set at the last  */
                            /* freeze (Sec. 4.3)                                     */
    double res_rows;        /* |r~_k| of the rows as the smoother holds them (each   */
    double res0_rows;       /* divided by delta_eps(phi_ij) when params.scaled), and */
    double rel_res_rows;    /* its |r~_0| and ratio                                  */
} mgseg_stats;

/* Fills *p with the defaults. */
void mgseg_params_default(mgseg_params *p);

/* Human-readable text for a status code (static storage). */
const char *mgseg_strerror(mgseg_status s);

/*
 * Sets up one image (Sec. 2.2, Sec. 5): edge detector g from the
 * pre-blurred image, marker distance function d, the curvature weight w
 * (g for Spencer-Chen, d g for Rada-Chen), the initial level set (signed
 * distance to the boundary of the marker polygon, Sec. 5), the polygon area
 * A1, the coarse-grid static maps (full-weighting restriction, Sec. 3.1),
 * the initial c1, c2 (eq. c1c2) and the initial residual norm.
 *   image_dev        : n x m float, values in [0, 1], row pitch `pitch`.
 *   markers_host     : k (row, col) pairs of floats in pixel coordinates;
 *                      the centre of cell (i, j) is (i + 0.5, j + 0.5);
 *                      every marker inside the image (0 <= row < n,
 *                      0 <= col < m), 1 <= k <= 64 (Rada-Chen: k >= 3,
 *                      for its polygon area A1).
 *   n, m             : at least 2.
 *   stream           : a hipStream_t (0 = default stream), passed as void*.
 * Memory: every device array of the context is a piece of one allocation
 * (about 230 B per finest-grid cell in the mixed mode, all levels), freed by
 * mgseg_destroy.
 * Errors: MGSEG_E_ARG (null pointers, k out of range, a marker outside the
 * image or not finite, pitch < m, bad struct_size),
 * MGSEG_E_SHAPE (n or m not divisible by 2^(levels-1), a side above 8192, or
 * lines longer than the device's LDS per workgroup allows), MGSEG_E_NOMEM.
 */
mgseg_status mgseg_setup(const float *image_dev, int n, int m, int pitch,
                         const float *markers_host, int k, const mgseg_params *p,
                         void *stream, mgseg_ctx **out);

/* Bytes of device memory that mgseg_solve_noalloc holds per device (static). */
#define MGSEG_NOALLOC_BYTES (32u << 20)

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc or hipFree: serving loops with fixed memory, harnesses that
 * forbid allocation): mgseg_setup + mgseg_solve + mgseg_get_phi for one image
 * in one call, with every device array of the solve placed in the library's
 * static scratch of MGSEG_NOALLOC_BYTES on the current device instead of an
 * allocated arena.  The V-cycles run as eager launches on `stream` (no HIP
 * graph).  The arguments are those of mgseg_setup (image, markers, params,
 * stream) and mgseg_solve (tol > 0, max_cycles >= 1, the cycle count and the
 * final relative residual, either output may be null), and the FP64 finest
 * phi goes to phi_dev (n x m doubles, row pitch phi_pitch >= m elements).
 * The scratch is about 230 B per finest cell over all grids in the mixed
 * mode, so images up to about 360 x 360 fit; a larger image returns
 * MGSEG_E_SCRATCH before any work is enqueued.  Other errors as mgseg_setup
 * and mgseg_solve (MGSEG_E_NOT_CONVERGED: phi_dev is still written).
 * The scratch is one array per device, shared by every call on that device
 * and cleared by each call: calls that overlap on one device (other host
 * threads, other streams) race and must be serialised by the caller.  Calls
 * on different devices are independent.
 */
mgseg_status mgseg_solve_noalloc(const float *image_dev, int n, int m, int pitch,
                                 const float *markers_host, int k, const mgseg_params *p,
                                 void *stream, double tol, int max_cycles,
                                 double *phi_dev, int phi_pitch, int *cycles_out,
                                 double *rel_res_out);

/* Replaces the finest phi (warm start), clamped to [-M, M]; recomputes c1,
 * c2 and the reference residual norm; resets the cycle counter. */
mgseg_status mgseg_set_phi0(mgseg_ctx *c, const float *phi_dev, int pitch);

/* Restores the marker-based initial level set of mgseg_setup (a copy kept
 * by the context), with c1, c2, the reference residual norm and the cycle
 * counter as after setup: the start of a fresh solve of the same image. */
mgseg_status mgseg_reset_phi0(mgseg_ctx *c);

/* One FAS V-cycle (Algorithm-1 box, gamma = 1) followed by the c1, c2
 * refresh (Sec. 5); returns |r~|/|r~_0| after the refresh. */
mgseg_status mgseg_vcycle(mgseg_ctx *c, double *rel_res_out);

/* V-cycles until |r~|/|r~_0| <= tol or max_cycles (then
 * MGSEG_E_NOT_CONVERGED with valid outputs). */
mgseg_status mgseg_solve(mgseg_ctx *c, double tol, int max_cycles, int *cycles_out,
                         double *rel_res_out);

/* AOS solver (additive operator splitting), the semi-implicit time stepper
 * of the timing comparison in Sec. 5 (Table 4) and an "exact" solver named
 * for the coarsest grid in Algorithm 1.  From the context's current finest
 * phi (FP64), each step freezes the coefficients of eq. abcdrc at phi^k,
 * solves one tridiagonal system per column (couplings A, B) and per row
 * (C, D) for y_l = (I - 2 tau A_l)^{-1} (phi^k - tau f), sets
 * phi^{k+1} = clamp((y_1 + y_2) / 2, -M, M), and refreshes c1, c2 (eq. c1c2).
 * tau: the step in units of h / mu (> 0).  Stops once the paper's relative
 * change |phi^{k+1} - phi^k| / |phi^k| falls below eta_tol (Sec. 5), or
 * after max_iters steps.  Outputs (each may be null): steps taken, the last
 * relative change, and the projected relative residual of the paper's rows
 * at the result (the stopping measure of mgseg_solve).  The next mgseg_vcycle
 * continues from the AOS result.  The first call allocates 48 bytes per
 * pixel of device memory, held until mgseg_destroy.  Errors: MGSEG_E_ARG
 * (null context, tau <= 0, eta_tol < 0, max_iters < 0), MGSEG_E_NOMEM,
 * MGSEG_E_HIP, MGSEG_E_NONFINITE;
 * MGSEG_E_NOT_CONVERGED when max_iters steps did not reach eta_tol (outputs
 * valid). */
mgseg_status mgseg_aos(mgseg_ctx *c, double tau, double eta_tol, int max_iters, int *iters_out,
                       double *eta_out, double *rel_res_out);

/* Local Fourier analysis of a smoother over the whole finest grid (Sec. 3.3,
 * Table 1): the coefficients of eq. abcdrc are frozen at the current finest
 * phi, and each pixel's smoothing rate is the largest amplification of the
 * frozen-coefficient smoother over the high frequencies
 * (a = 2 pi t / 128, t = -64 .. 64, max(|a1|, |a2|) > pi / 2).
 * smoother: 1 GSLEX-I (couplings B, D new), 3 GSLINE-I (column lines:
 * A, B, D new), 4 NEWT-I (GSLEX with the Rada-Chen Newton term on the
 * diagonal), 0 Hybrid Smoother 2 (at a jump-set pixel the sweep that lags
 * its smallest coupling, elsewhere GSLEX).  out5 (host): mu~_max and mu~_avg
 * over all pixels, the same two over the jump set, and the jump-set share.
 * mu_dev (optional, device, pitch mu_pitch >= m): each pixel's rate.  Needs
 * mixed_precision = 1 (MGSEG_E_STATE otherwise).  The first call allocates
 * 5 doubles per 256 pixels of device memory, held until mgseg_destroy.
 * Errors: MGSEG_E_ARG (null context or out5, another smoother, a short
 * pitch), MGSEG_E_STATE, MGSEG_E_NOMEM, MGSEG_E_HIP. */
mgseg_status mgseg_smoothing_rates(mgseg_ctx *c, int smoother, double *out5, float *mu_dev, int mu_pitch);

/* Launch schedule of a context.  Every schedule computes the same bits
 * (each kernel choice below evaluates the same arithmetic in the same
 * order); they differ only in speed.
 *   lds_side      grids below the finest with both sides at most lds_side
 *                 (and at most 64) run in one LDS-resident workgroup: the
 *                 coarsest solve, and the smoothing of grids of at most 32 x 32
 *                 (0: every grid through the global-memory kernels); default 64
 *   line_threads  0: each line of a sweep takes the smallest workgroup half
 *                 that holds it (default); 1: the next wider one (lines of at
 *                 most 512 cells)
 *   graph         1: each cycle is replayed from a captured HIP graph
 *                 (default); 0: launched eagerly
 *   split_long    lines longer than 512 cells: 1 (default) two launches
 *                 per sweep, the first three lines of every band of four,
 *                 then the fourth lines reading their final neighbours
 *                 (forward sweeps written in their own layout; on lines
 *                 longer than 1024 cells also the reverse sweeps, written
 *                 to a free plane in their own layout and then transposed
 *                 to the next sweep's); 0 one launch that recomputes the
 *                 next band's first line */
typedef struct {
    int32_t lds_side;
    int32_t line_threads;
    int32_t graph;
    int32_t split_long;
} mgseg_schedule;

mgseg_status mgseg_get_schedule(mgseg_ctx *c, mgseg_schedule *out);
/* MGSEG_E_ARG on a value out of range. */
mgseg_status mgseg_set_schedule(mgseg_ctx *c, const mgseg_schedule *s);

/* Autotuner: times trial_cycles V-cycles (after one untimed) of every
 * schedule of lds_side in {0, 16, 32, 64} x line_threads in {0, 1} x graph
 * in {0, 1} (x split_long in {0, 1} where a side exceeds 512 cells) from
 * the context's current state, keeps the fastest, and
 * restores the state (the solve continues where it stood; the cycle count
 * is unchanged).  Outputs (each may be null): the chosen schedule and its
 * milliseconds per cycle.  Errors: MGSEG_E_ARG (trial_cycles < 1),
 * MGSEG_E_HIP. */
mgseg_status mgseg_tune(mgseg_ctx *c, int trial_cycles, mgseg_schedule *best_out, double *ms_per_cycle_out);

/* Finest phi in FP64 (n x m, pitch in elements). */
mgseg_status mgseg_get_phi(mgseg_ctx *c, double *phi_dev, int pitch);

/* Segmentation mask: 1 where phi > 0, else 0 (Sec. 2.1). */
mgseg_status mgseg_get_mask(mgseg_ctx *c, uint8_t *mask_dev, int pitch);

mgseg_status mgseg_get_stats(mgseg_ctx *c, mgseg_stats *s);

/* Checkpoint of a solve: the FP64 finest phi with the cycle counter, the
 * residual norms and eta.  mgseg_get_state writes it to the host buffer
 * blob of *bytes bytes; with blob = NULL, or *bytes too small (then
 * MGSEG_E_ARG), it only sets *bytes to the size needed (a 64-byte header +
 * 8 n m).  mgseg_set_state restores it into a context set up from the same
 * image, markers and parameters (else MGSEG_E_SHAPE for another shape or
 * level count, MGSEG_E_ARG for a blob that is not a state): c1, c2 and the
 * residual are recomputed from phi, so the solve continues exactly as the
 * one the state was taken from. */
mgseg_status mgseg_get_state(mgseg_ctx *c, void *blob, size_t *bytes);
mgseg_status mgseg_set_state(mgseg_ctx *c, const void *blob, size_t bytes);

/* Releases every device buffer of the context (NULL is a no-op). */
void mgseg_destroy(mgseg_ctx *c);

/* ------------------------------------------------------------------------
 * Single steps, for tests and profiling.  They operate on one level of an
 * existing context; host buffers are n_l x m_l, dense (pitch m_l).
 * Fields: 0 z, 1 d, 2 w, 3 fit, 4 phi, 5 F, 6 lo, 7 hi, 8 g (level 0 only),
 *         9 phi64 (level 0, double), 10 labels (uint8, bit s = starred in
 *         sweep s of the current freeze).
 * ---------------------------------------------------------------------- */
mgseg_status mgseg_level_shape(mgseg_ctx *c, int level, int *n, int *m, double *h);
mgseg_status mgseg_debug_get(mgseg_ctx *c, int level, int field, void *host);
mgseg_status mgseg_debug_set(mgseg_ctx *c, int level, int field, const void *host);
/* scalars: out[0] c1, out[1] c2, out[2] A1, out[3] res0, out[4] h0 */
mgseg_status mgseg_debug_scalars(mgseg_ctx *c, double *out5);
mgseg_status mgseg_debug_set_c(mgseg_ctx *c, double c1, double c2);
/* op: 0 freeze (coefficients, labels and psi at the current phi),
 *     1..4 one sweep A..D of Hybrid Smoother 2 with the current freeze,
 *     5 `arg` outer iterations (freeze + 4 sweeps),
 *     6 the coarsest-grid solve (level must be the coarsest),
 *     7 the V-cycle from this level down (F of this level as set),
 *     8 residual r = F - N(phi), projected (result in field F of the next
 *       debug_get with field 11 = residual),
 *     9 c1, c2 refresh from the finest phi and fit maps of every level. */
mgseg_status mgseg_debug_op(mgseg_ctx *c, int level, int op, int arg);

/* ------------------------------------------------------------------------
 * Kernel timing with HIP events recorded on the context's stream around each
 * launch of one kernel class (kernel 0 = the finest-grid directional sweep
 * of Hybrid Smoother 2).  mgseg_profile(enable = 1) clears earlier records
 * and starts recording; enable = 0 stops.  mgseg_profile_read synchronises
 * the stream and returns the summed elapsed time, the number of timed
 * launches and the compulsory HBM bytes of one launch (cells x bytes per
 * cell read and written once).
 * ---------------------------------------------------------------------- */
mgseg_status mgseg_profile(mgseg_ctx *c, int kernel, int enable);
mgseg_status mgseg_profile_read(mgseg_ctx *c, int kernel, double *total_ms, int *count,
                                double *bytes_per_launch);

/* ------------------------------------------------------------------------
 * Batches of images of uneven size.  Each image is solved by its own
 * context exactly as by mgseg_setup / mgseg_solve (Algorithm-1 box with
 * Hybrid Smoother 2); the batch issues the images' V-cycles on `nstreams`
 * internal streams so that the latency-bound coarse grids of different
 * images overlap, waits once per round of cycles, and drops converged images
 * from later rounds.  Results are bit-identical to solving the images one by
 * one.
 *   images_dev[i], n[i], m[i], pitch[i], markers_host[i], k[i]: as in
 *     mgseg_setup for image i (count >= 1); p: shared parameters (levels = 0
 *     lets each image take as many grids as its size allows).
 *   stream: the caller's stream; setup work is enqueued on it, and
 *     mgseg_solve_batch makes the internal streams wait for it on entry and
 *     it wait for them on return.
 * Errors: as mgseg_setup, for the first image that fails (earlier contexts
 * are released).
 */
typedef struct mgseg_batch mgseg_batch;
mgseg_status mgseg_setup_batch(int count, const float *const *images_dev, const int *n, const int *m,
                               const int *pitch, const float *const *markers_host, const int *k,
                               const mgseg_params *p, void *stream, mgseg_batch **out);

/* Autotuner: one untimed round of cycles, then `trial_rounds` timed rounds of
 * one V-cycle on every image for each stream count in {1, 2, 4, 8} (at most
 * the image count); keeps the fastest.  The tuning cycles are real V-cycles
 * and count in the images' cycle totals.  Outputs (may be null): the chosen
 * stream count and its measured time per round in milliseconds.
 * The streams run side by side only on as many hardware queues as the HIP
 * runtime opens for the process (GPU_MAX_HW_QUEUES, read when the runtime
 * starts; 4 unless set): a caller that batches should set it to at least 8. */
mgseg_status mgseg_batch_tune(mgseg_batch *b, int trial_rounds, int *nstreams_out, double *ms_per_round_out);

/* Sets the stream count (1..8) without tuning. */
mgseg_status mgseg_batch_set_streams(mgseg_batch *b, int nstreams);

/* V-cycles on every image whose |r~|/|r~_0| is above tol, until all are at
 * tol or have done max_cycles cycles in total.  cycles_out[count] and
 * rel_out[count] (may be null) receive each image's totals.  Returns
 * MGSEG_E_NOT_CONVERGED (outputs valid) if any image stopped at max_cycles. */
mgseg_status mgseg_solve_batch(mgseg_batch *b, double tol, int max_cycles, int *cycles_out, double *rel_out);

/* The context of image `index` (owned by the batch; valid until
 * mgseg_destroy_batch): use it with mgseg_get_phi, mgseg_get_mask,
 * mgseg_get_stats. */
mgseg_status mgseg_batch_ctx(mgseg_batch *b, int index, mgseg_ctx **view);

/* Releases every context and stream of the batch (NULL is a no-op). */
void mgseg_destroy_batch(mgseg_batch *b);

/* ------------------------------------------------------------------------
 * Learned warm start.  A small convolutional encoder-decoder maps the
 * network input (image z, marker distance map d of Sec. 2.2, marker mask) to
 * an initial level set phi0 = M tanh(o); the V-cycle then finishes the solve
 * from it (mgseg_set_phi0), so the network only changes where the solve
 * starts, never its fixed point.  depth levels with widths base * 2^l; every
 * level's block is two 3x3 convolutions (zero padding) each followed by ReLU;
 * 2x2 average pooling down, nearest 2x up-sampling with the encoder's output
 * of the same level concatenated after it; 1x1 head.
 * Convolutions run as bf16 matrix-core products with FP32 accumulation;
 * FP32 master weights with Adam.  All tensors are device NCHW FP32 at the
 * boundary.
 */
typedef struct mgseg_net mgseg_net;

/* New network with He-normal weights from `seed` (deterministic).  Channel
 * counts are multiples of the 16-wide matrix-core tile.
 * Errors: MGSEG_E_ARG (base_channels not a multiple of 16 in 16..256, depth
 * not in 2..6, or base_channels * 2^(depth-1) above 512). */
mgseg_status mgseg_net_create(int base_channels, int depth, uint64_t seed, mgseg_net **out);

/* phi0_dev[B][H][W] = M tanh(net(in_dev[B][3][H][W])); keeps the activations
 * for mgseg_net_backward.  H, W multiples of 2^(depth-1) (else MGSEG_E_SHAPE). */
mgseg_status mgseg_net_forward(mgseg_net *n, const float *in_dev, int B, int H, int W, double M, float *phi0_dev,
                               void *stream);

/* Loss of the last forward against target_dev[B][H][W] and the gradients of
 * every parameter.  With tg = clip(target / M, -1, 1) and the object weight
 * w = pos_weight where tg > 0, 1 elsewhere (pos_weight > 0, else
 * MGSEG_E_ARG; it balances the small object class), the loss is the
 * weighted binary cross-entropy of (1 + tanh o) / 2 against (1 + tg) / 2,
 * mean(w (softplus(2 o) - o (1 + tg))): minimal at tanh o = tg, with
 * dloss/do = w (tanh o - tg) / N, which stays away from zero where the
 * output saturates on the wrong side.  *loss_host (may be null) after a
 * stream sync.  MGSEG_E_STATE without a preceding forward. */
mgseg_status mgseg_net_backward(mgseg_net *n, const float *target_dev, double M, double pos_weight, float *loss_host,
                                void *stream);

/* One Adam step (bias-corrected moments) with the gradients of the last
 * backward; 0 <= b1, b2 < 1, eps > 0, lr >= 0 (else MGSEG_E_ARG). */
mgseg_status mgseg_net_adam_step(mgseg_net *n, double lr, double b1, double b2, double eps, void *stream);

/* Parameters in a fixed order: the encoder's convolutions (two per level,
 * level 0 first), then the decoder's (two per level 0..depth-2), each weights
 * [OC][IC][3][3] then biases [OC]; head weights [base], head bias.  Count,
 * copy out (values and / or gradients; host buffers of `count` floats), copy
 * in (which also clears the Adam moments and step count). */
mgseg_status mgseg_net_param_count(mgseg_net *n, long long *count);
mgseg_status mgseg_net_get_params(mgseg_net *n, float *host, float *grad_host);
mgseg_status mgseg_net_set_params(mgseg_net *n, const float *host);
/* The Adam state in the same order: first moments m and second moments v
 * (host buffers of `count` floats; either may be null on _get, both are
 * required on _set) and the number of steps taken, which sets the bias
 * correction of the next step.  Restoring them after set_params resumes an
 * interrupted training run with the same updates it would have made.
 * _set: steps outside 0..2^31-1 or a null buffer give MGSEG_E_ARG. */
mgseg_status mgseg_net_get_adam(mgseg_net *n, float *m_host, float *v_host, long long *steps);
mgseg_status mgseg_net_set_adam(mgseg_net *n, const float *m_host, const float *v_host, long long steps);
void mgseg_net_destroy(mgseg_net *n);

/* Convolution timing.  While enabled, every k_conv launch (forward and data
 * gradient) is bracketed by HIP events on its stream and its algorithmic
 * flops (2 * 9 * input channels that carry data * output channels * pixels)
 * are added up; mgseg_net_profile(n, 1) also clears the record.  _read
 * synchronises the device and returns the summed launch time (ms), the launch
 * count and the flops (outputs may be null). */
mgseg_status mgseg_net_profile(mgseg_net *n, int enable);
mgseg_status mgseg_net_profile_read(mgseg_net *n, double *total_ms, int *launches, double *flops);

/* The network input of a context: out_dev[3][n][m] = (z, d, marker mask). */
mgseg_status mgseg_ctx_features(mgseg_ctx *c, float *out_dev);

/* Forward pass on the context's features, phi0 = scale M tanh(o)
 * (0 < scale <= 1, else MGSEG_E_ARG: a smaller amplitude leaves the
 * interfaces softer for the V-cycle to move); the result becomes the initial
 * level set (as mgseg_set_phi0) only if it is positive at the cell of every
 * marker: a selective segmentation contains its markers, and a network
 * output that leaves one out (the empty level set phi = -M is a stationary
 * point of the box-constrained problem) would lead the solve to another
 * fixed point.  Otherwise the marker-based phi0 is restored
 * (mgseg_reset_phi0), so the solve always starts from a valid guess.
 * *accepted_out (may be null): 1 if the network's phi0 was taken.  The first
 * call on a context allocates the features and the network output (4 n m
 * floats); they stay with the context until mgseg_destroy. */
mgseg_status mgseg_predict_phi0(mgseg_ctx *c, mgseg_net *n, double scale, int *accepted_out);

#ifdef __cplusplus
}
#endif
#endif /* MGSEG_H */
