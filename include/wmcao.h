/*
 * wmcao.h -- C ABI of the MI355X wavelet-domain MCAO tomography solver.
 *
 * The library solves the wavelet-domain MAP normal equations of multi-conjugate
 * adaptive optics atmospheric tomography (Helin & Yudytskiy, "Wavelet methods
 * in multi-conjugate adaptive optics", Sec. 5.1, eq. (19)):
 *
 *     (A~^T C^-1 A~ + alpha D) c = A~^T C^-1 s,    A~_m = Gamma_m P_m W^-1,
 *
 * with W a periodic orthonormal Daubechies-3 transform per layer, P_m the
 * natural- or laser-guide-star projection of the layered atmosphere (Sec. 2.1,
 * eq. (2) and its cone-effect variant), Gamma_m the Fried-geometry
 * Shack-Hartmann operator (eqs. (3)-(4)), C^-1 the block-diagonal noise
 * weight with tip/tilt removal for laser guide stars (Sec. 4.3, eqs. (16)-(18)),
 * D the diagonal wavelet prior (Sec. 3, eq. (13)), by conjugate gradients with
 * the modified Jacobi preconditioner and warm restart (Sec. 5.1).
 *
 * Conventions shared by every call
 * --------------------------------
 * Coefficients: per layer an N x N row-major array indexed [x][y] in Mallat
 *   layout (low-pass band top-left); layers concatenated in input order; frames
 *   contiguous with stride n_coeffs.
 * Layers (pixel fields): same layout as coefficients; pixel p of an N x N layer
 *   with spacing d sits at (p - N/2) d metres.
 * Slopes: per sensor in input order, the x-slopes of its active subapertures
 *   (row-major, x slow) then its y-slopes; low-order sensors give one slope pair
 *   per active k x k cell.  Frame stride n_slopes.  Slopes are phase
 *   differences across one subaperture, in radians.
 * Device buffers hold the plan's dtype (float for WMCAO_F32, double for
 *   WMCAO_F64) unless a parameter says otherwise.  They are owned by the caller.
 * Streams: every call enqueues on the given HIP stream (NULL = default stream)
 *   and does not synchronise the host, unless stated.
 * Errors: every int-returning call returns WMCAO_OK (0) or a negative
 *   WMCAO_ERR_* code; wmcao_last_error() gives a message for the calling
 *   thread.  Nothing is thrown or aborted across the ABI.
 * Threads: a plan is immutable after wmcao_plan except for its internal
 *   scratch, so at most one call may be in flight per plan at a time.
 */
#ifndef WMCAO_H
#define WMCAO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WMCAO_OK 0
#define WMCAO_ERR_INVALID_ARG (-1)   /* NULL pointer, bad count, bad option        */
#define WMCAO_ERR_SIZE (-2)          /* layer size not divisible by 2^levels, ... */
#define WMCAO_ERR_FOOTPRINT (-3)     /* a sensor node projects outside a layer    */
#define WMCAO_ERR_UNSUPPORTED (-4)   /* wavelet family/order or size not built    */
#define WMCAO_ERR_OOM (-5)           /* device or host allocation failed          */
#define WMCAO_ERR_HIP (-6)           /* a HIP runtime call failed                 */
#define WMCAO_ERR_BREAKDOWN (-7)     /* p^T A p <= 0 or non-finite in some frame  */

/* Per-frame status written by wmcao_solve into status_dev. */
#define WMCAO_FRAME_OK 0
#define WMCAO_FRAME_CONVERGED 1      /* residual became exactly zero; stopped      */
#define WMCAO_FRAME_BREAKDOWN (-7)   /* p^T A p <= 0 or non-finite; x kept          */

typedef struct wmcao_plan_s* wmcao_plan_t;

typedef enum { WMCAO_F32 = 0, WMCAO_F64 = 1 } wmcao_dtype;

/* Telescope pupil: an annulus (Sec. 5.1); obstruction_ratio is the inner
 * diameter over the outer one.  A subaperture is active iff its centre lies in
 * the closed annulus. */
typedef struct {
    double diameter_m;
    double obstruction_ratio;
} wmcao_pupil;

/* One turbulent layer phi_l at altitude h_l (Sec. 2.1): an n x n grid with the
 * given spacing; cn2_weight w_l scales the prior (c_rho = 0.023 w r0^-5/3). */
typedef struct {
    double altitude_m;
    double cn2_weight;
    double spacing_m;
    int n;
} wmcao_layer;

/* One guide star and its Fried-geometry Shack-Hartmann sensor (Sec. 2.1,
 * eqs. (3)-(5)).  Laser guide stars must come first (Sec. 2.1).
 *   theta_x, theta_y  direction in radians
 *   lgs_height_m      H of the cone projection (ignored for NGS)
 *   n_sub             subapertures across the pupil
 *   tt_aggregate      0: high-order sensor; k in 1..4: low-order k x k sensor
 *                     whose slopes average the fine slopes of each cell
 *   remove_tt         apply (I - T) (Sec. 4.3, eq. (17)); -1 = default (is_lgs)
 *   in_precond        counted in the Jacobi diagonal (Sec. 5.1); -1 = default
 *                     (n_sub > 2 and not tt_aggregate)
 *   sigma             noise standard deviation: C~ = sigma^2 I ...
 *   cinv_blocks       ... unless non-NULL: host array of 3 doubles (a, b, c) per
 *                     measurement (active subaperture or cell) giving the
 *                     symmetric 2x2 block [[a, b], [b, c]] of C~^-1 (eq. (16)).
 *                     Copied at plan time.
 *   kind              0: Fried Shack-Hartmann slopes.  1: the phase itself at
 *                     the pupil nodes that are corners of active subapertures
 *                     (one value per node, weight a of its block): the target
 *                     of the fitting step in one direction (Sec. 4.1, eq. (15)).
 *                     Natural-star geometry, no aggregation, no tip/tilt
 *                     removal. */
typedef struct {
    int is_lgs;
    double theta_x, theta_y;
    double lgs_height_m;
    int n_sub;
    int tt_aggregate;
    int remove_tt;
    int in_precond;
    double sigma;
    const double* cinv_blocks;
    int kind;
} wmcao_wfs;

/* Wavelet family: only Daubechies (family 0) of order 3 is built (Sec. 5.1). */
typedef struct {
    int family;
    int order;
} wmcao_wavelet;

/* Solver options.
 *   alpha                 weight of the prior (eq. (19))
 *   r0_m, L0_m            Fried parameter (at the phase wavelength) and outer
 *                         scale entering D (Sec. 3)
 *   dtype                 precision of the PCG vectors (x, b, r, p, A p, J) and
 *                         of the caller's buffers; inner products, step scalars
 *                         and the residual-replacement norms are always FP64
 *   max_batch             largest batch any call will pass (scratch is sized for it)
 *   resid_replace_every   R > 0: r <- b - A x every R iterations (0 = never)
 *   precond               0: plain CG, 1: modified Jacobi
 *   tile                  tile edge of the tiled wavelet kernels: 16, 32 or 64;
 *                         0 = library default
 *   lds_budget            bytes of LDS a whole-band wavelet kernel may use
 *                         (0 = library default): the levels whose low-pass
 *                         band exceeds it run as tiled launches, for all
 *                         layers as many as the largest layer needs
 *   streams               1: a solve runs on the caller's stream only; 2: a
 *                         solve (single-plan, or packed when every plan allows
 *                         it) whose half batch holds at least 2^20 coefficients
 *                         (6 or more E-ELT frames) runs its two halves
 *                         concurrently, the second on a
 *                         stream the plan owns (forked from and joined back to
 *                         the caller's stream with events, so stream order and
 *                         graph capture are unchanged; results are the same
 *                         bit for bit); 0 = library default (2).  A caller that
 *                         already overlaps several plans on streams of its own
 *                         should pass 1: streams beyond the device's hardware
 *                         queues can queue unrelated work behind each other
 *   op_precision          type of the operator stages of a WMCAO_F32 plan (the
 *                         wavelet tiles and low-pass scratch, the layer pixel
 *                         fields, the adjoint node fields and footprint images,
 *                         and their arithmetic): 32 or 64; 0 = library default:
 *                         64 for plans of fewer than 2^17 unknowns (their solves
 *                         are bound by launch latency, and their 10-step iterates
 *                         are sensitive enough to rounding that single-precision
 *                         operators move them by more than 1e-5), 32 otherwise.
 *                         WMCAO_F64 plans take 0 or 64.  The projection's node
 *                         fields, the slopes and the noise weighting are FP64 in
 *                         every plan.  Plans packed into one launch run in one
 *                         group per operator type (at most two types).
 *   op_fp64_stages        with 32-bit operator storage: the stages whose
 *                         arithmetic and LDS tiles are FP64, a mask of 1 (W^-1),
 *                         2 (P^T) and 4 (W, with the sum of the P^T images);
 *                         -1 = library default (4: the forward transform takes
 *                         small differences of the summed P^T image, the other
 *                         two stages run in FP32).
 *   proj_rows             sensor node rows per work item of the projection and
 *                         the noise weighting: 4 .. 48 (0 = 8; the weighting
 *                         takes at most 8)
 *   vec_chunk             vector elements per work item of the PCG updates:
 *                         1024, 2048, 4096 or 8192 (0 = 2048)
 *   adj_lds               LDS bytes one adjoint-projection work item may use
 *                         for its staged node rows and row pass, 8 KiB to
 *                         96 KiB (0 = 32 KiB); fewer footprint rows per item
 *                         when smaller
 * tile, lds_budget, streams and the last three change only how the work is
 * cut and in which order partial sums are formed; results agree to rounding. */
typedef struct {
    double alpha;
    double r0_m;
    double L0_m;
    wmcao_dtype dtype;
    int max_batch;
    int resid_replace_every;
    int precond;
    int tile;
    int lds_budget;
    int streams;
    int op_precision;
    int op_fp64_stages;
    int proj_rows;
    int vec_chunk;
    int adj_lds;
} wmcao_options;

/* Build a plan on the current HIP device: validates the geometry, builds the
 * projection and slope tables, the prior D and the Jacobi diagonal J (on the
 * device, synchronously), and allocates scratch for max_batch frames.
 * levels = 0 means no wavelet transform: the unknowns are the grid values
 * themselves and the regulariser is alpha times the identity (used for the
 * deformable-mirror grids of the fitting step, Sec. 4.1).
 * Errors: INVALID_ARG, SIZE (n % 2^levels != 0 or n/2^(levels-1) < 6),
 * FOOTPRINT, UNSUPPORTED (wavelet other than db3, n_sub too large), OOM, HIP.
 * On error *out is NULL. */
int wmcao_plan(const wmcao_pupil* pupil, const wmcao_layer* layers, int n_layers,
               const wmcao_wfs* wfs, int n_wfs, wmcao_wavelet wavelet, int levels,
               const wmcao_options* opts, wmcao_plan_t* out);

/* Sizes of one frame.  layer_offsets (n_layers+1 entries) and slope_offsets
 * (n_wfs+1 entries) may be NULL. */
int wmcao_sizes(wmcao_plan_t plan, int64_t* n_coeffs, int64_t* n_slopes,
                int64_t* layer_offsets, int64_t* slope_offsets);

/* W^-1 (Sec. 5.1): coefficients -> layer pixel fields, for batch frames. */
int wmcao_coeffs_to_layers(wmcao_plan_t plan, const void* coeffs, void* layers, int batch,
                           void* hip_stream);

/* W: layer pixel fields -> coefficients, for batch frames. */
int wmcao_layers_to_coeffs(wmcao_plan_t plan, const void* layers, void* coeffs, int batch,
                           void* hip_stream);

/* Forward model s = A phi (eq. (6)): raw slopes Gamma_m P_m phi of every
 * sensor from layer pixel fields (no noise weight, no tip/tilt removal). */
int wmcao_forward_layers(wmcao_plan_t plan, const void* layers, void* slopes, int batch,
                         void* hip_stream);

/* Right side b = A~^T C^-1 s of eq. (19) for batch frames of slopes. */
int wmcao_rhs(wmcao_plan_t plan, const void* slopes, void* b, int batch, void* hip_stream);

/* y = (A~^T C^-1 A~ + alpha D) x (the operator of Sec. 5.1) for batch frames.
 * x and y must not alias. */
int wmcao_apply_A(wmcao_plan_t plan, const void* x, void* y, int batch, void* hip_stream);

/* Copy the Jacobi diagonal J (n_coeffs doubles, Sec. 5.1) to device memory. */
int wmcao_precond_diag(wmcao_plan_t plan, double* j_dev, void* hip_stream);

/* PCG solve of eq. (19) for batch frames (Sec. 5.1): n_iter iterations, no
 * tolerance stop.  coeffs holds x0 on entry when warm_start != 0 (the previous
 * time step's reconstruction) and x on exit; with warm_start == 0 it is
 * overwritten.  resid_dev (optional, FP64 [batch][n_iter+1]) receives the
 * recursive residual norms |r_i|; status_dev (optional, int [batch]) the
 * per-frame WMCAO_FRAME_* status.  A frame that breaks down keeps its last
 * iterate and the other frames continue; the call itself still returns OK. */
int wmcao_solve(wmcao_plan_t plan, const void* slopes, void* coeffs, int batch, int n_iter,
                int warm_start, double* resid_dev, int* status_dev, void* hip_stream);

/* One PCG solve over frames of several plans (mixed telescope sizes and
 * dtypes of one kind): every stage of every plan's frames is packed into one
 * launch.  slopes[i], coeffs[i] and counts[i] belong to plans[i]; all plans
 * must share the dtype.  Same semantics per frame as wmcao_solve. */
int wmcao_solve_multi(const wmcao_plan_t* plans, const void* const* slopes, void* const* coeffs,
                      const int* counts, int n_plans, int n_iter, int warm_start,
                      void* hip_stream);

/* wmcao_solve_multi captured into a HIP graph and replayed.  The library keeps
 * up to 64 captures, keyed by every argument (plans, buffers,
 * counts, n_iter, warm_start, stream); a call with a known key replays without
 * re-recording.  Buffers must stay valid while the plans live; destroying a
 * plan drops the captures that use it.  hip_stream must not be the default
 * stream. */
int wmcao_solve_multi_graph(const wmcao_plan_t* plans, const void* const* slopes,
                            void* const* coeffs, const int* counts, int n_plans, int n_iter,
                            int warm_start, void* hip_stream);

/* One launch of a request loop that serves frames as they arrive, in three
 * steps on hip_stream (not the default stream), for a caller whose host time
 * per launch matters: one kernel copies frame i's slopes (slopes[i],
 * n_slopes values) and warm start (warm[i], n_coeffs values) into row i of
 * the staging buffers stage_slopes and stage_coeffs (the plan's dtype, at
 * least count rows each); the count frames are then solved as
 * wmcao_solve_multi_graph solves them with those buffers (warm start, n_iter
 * iterations, the capture kept and replayed for later calls with the same
 * buffers and count); one kernel then copies staging row out_rows[i] of the
 * solution to out_ptrs[i] (n_coeffs values) for i < n_out.  All pointers are
 * device pointers; the inputs must be complete when hip_stream reaches the
 * call.  The outputs are written after the solve, so an output may be one of
 * the call's inputs, but none may overlap the staging buffers.
 * count: 1 .. min(max_batch, 20); n_out: 0 .. 40.  Returns
 * WMCAO_ERR_INVALID_ARG for NULL pointers or counts and rows out of range,
 * otherwise as wmcao_solve_multi_graph. */
int wmcao_serve_launch(wmcao_plan_t plan, void* stage_slopes, void* stage_coeffs, int count,
                       const void* const* slopes, const void* const* warm, int n_out,
                       const int* out_rows, void* const* out_ptrs, int n_iter, void* hip_stream);

/* Capture the launches of wmcao_solve with these arguments into a HIP graph
 * owned by the plan, replacing any earlier capture, and replay it: later
 * wmcao_solve_graph calls with the same arguments replay without re-recording.
 * Buffers must stay valid while the plan lives. */
int wmcao_solve_graph(wmcao_plan_t plan, const void* slopes, void* coeffs, int batch, int n_iter,
                      int warm_start, double* resid_dev, int* status_dev, void* hip_stream);

/* wmcao_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, with every scratch buffer of the call (b, r, p, A p, the
 * operator's intermediates, slope sums, partial sums, per-frame scalars and,
 * if status_dev is NULL, the status) in one fixed device array of the
 * library, 32 MiB per GPU, held until the process ends.  The call allocates
 * nothing: no hipMalloc, no new schedule (it uses the first `batch` frames of
 * the max_batch schedule built with the plan) and no second stream (it runs
 * on hip_stream only).  Arguments and results are those of wmcao_solve, bit
 * for bit.  A batch whose scratch exceeds the array returns WMCAO_ERR_SIZE
 * before any launch (about 11 MB per E-ELT frame with FP32 vectors: 2 frames;
 * a few hundred KB per 8 m frame).  Every call on one GPU shares that GPU's
 * array and leaves its contents behind: calls that overlap on one GPU (other
 * streams, other threads, other plans) race, so callers serialise them. */
int wmcao_solve_noalloc(wmcao_plan_t plan, const void* slopes, void* coeffs, int batch,
                        int n_iter, int warm_start, double* resid_dev, int* status_dev,
                        void* hip_stream);

/* Kernel kinds for per-kernel timing. */
#define WMCAO_K_IDWT_COARSE 0   /* W^-1, low-pass block in LDS            */
#define WMCAO_K_IDWT_TILE 1     /* W^-1, one tiled level                  */
#define WMCAO_K_SENSOR 2        /* right side / forward model: C^-1, (I-T), Gamma^T of the slopes */
#define WMCAO_K_FDWT_TILE 3     /* W one tiled level (+ sum of the P^T footprint images at level 1) + alpha D, dot */
#define WMCAO_K_FDWT_COARSE 4   /* W coarse levels + alpha D, dot         */
#define WMCAO_K_INIT 5          /* r0, p0                                 */
#define WMCAO_K_UPDATE_R 6      /* r -= a q, <r, J^-1 r>                  */
#define WMCAO_K_UPDATE_P 7      /* x += a p, p = J^-1 r + beta p          */
#define WMCAO_K_REPLACE_R 8     /* r = b - A x                            */
#define WMCAO_K_PROJECT 9       /* P: layers -> sensor node fields        */
#define WMCAO_K_ADJOINT 10      /* P^T: node fields -> footprint images per sensor and layer */
#define WMCAO_K_WEIGHTS 11      /* operator apply: Gamma, C^-1, (I-T), Gamma^T per node band */
#define WMCAO_K_COUNT 12

/* Per-kernel timing of later wmcao_solve / wmcao_apply_A calls on this plan:
 * with enable != 0 every launch is bracketed by HIP events on the launch
 * stream (adds a little host overhead; not for graph capture).  enable == 0
 * stops recording; the accumulated times are kept until the next enable. */
int wmcao_profile_enable(wmcao_plan_t plan, int enable);

/* Accumulated device time (ms), launch count and algorithmic bytes (what the
 * launches must read and write, counted per frame from the plan's sizes; may be
 * NULL) of one kernel kind since the last enable.  Synchronises with the
 * recorded events. */
int wmcao_profile_read(wmcao_plan_t plan, int kind, double* total_ms, int* launches,
                       double* bytes);

/* out = a x + b y over n elements of the given dtype (out may alias x or y):
 * the vector step of the pseudo-open-loop control (Sec. 4.2, Alg. 4.1). */
int wmcao_axpby(wmcao_dtype dtype, int64_t n, double a, const void* x, double b, const void* y,
                void* out, void* hip_stream);

/* Free the plan and everything it owns (waits for the device). */
void wmcao_plan_destroy(wmcao_plan_t plan);

/* Static message for an error code. */
const char* wmcao_strerror(int code);

/* Message describing the last error on the calling thread ("" if none). */
const char* wmcao_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WMCAO_H */
