/*
 * fwh.h -- C ABI of the MI355X (gfx950) library for the wind-tunnel FW-H
 * far-field integral: permeable surface, Farassat 1A after the Garrick-triangle
 * change of frame and the angle-of-attack rotation, nondimensional (Sec. II C-D
 * of Zhang, Yu, Liu, Li, "An MPI-OpenMP mixing parallel open source FW-H code
 * for aeroacoustics calculation").
 *
 * What is computed.  For panels p (centre y_p, unit outward normal n_p, area
 * dS_p), observers o (position x_o) and source frames tau_n = tau0 + n*dtau,
 * n = 0..N-1, given density rho, velocity u (full values, nondimensional by the
 * mean flow) and the pressure pulsation p' (by rho0 U0^2) on every panel at
 * every frame (inputs listed at the end of Sec. II C):
 *   Q   = (-U0_i + rho u_i) n_i,  L_i = p' n_i + rho (u_i - U0_i) u_j n_j
 *                                               Eqs. (Qn_New_nd), (Li_New_nd), (U_0_nd)
 *   Qdot, Ldot_i: 2nd-order differences in source time, one-sided at the
 *   first and last frame (Sec. III B, "compute Noise");
 *   R, Rhat, M_R: Garrick distance and radiation direction with the AoA
 *   rotation, Eqs. (R_New)..(R2_New), surface Mach vector M = -M0 U0hat;
 *   delay R/c0 = M0 R (Eq. (tau2));
 *   observer window t_start = tau0 + max_p delay, t_end = tau_{N-1} + min_p
 *   delay (Eqs. (t_start), (t_end), per observer), observer samples
 *   t_k = t_start + k dtau, k < N_t = floor((t_end - t_start)/dtau + 1e-9) + 1;
 *   p'(o, k) = sum_p s_{p,o}(t_k - delay), with s the natural cubic spline
 *   (Sec. III B, "interp pressure signal") of the integrand of
 *   Eqs. (pT_WT_nd) + (pL_WT_nd).
 * In this frame every pair has a fixed delay, so the evaluation is a
 * fixed fractional-delay gather-sum over panels.
 *
 * Layouts (row-major, element counts):
 *   geometry (host):  y [P][3], normal [P][3], dS [P], x_obs [O][3]      (double)
 *   surface data (device, time-major, one frame after another as a solver
 *   writes them): rho [N][P], u [3][N][P], p' [N][P]       (FWH_F64 or FWH_F32)
 *   output (device):  p_out [O][n_t_max]; entries k >= N_t(o) are written 0.
 *                     double in FWH_MODE_F64, float otherwise.
 *   adjoint input:    grad_p [O][n_t_max], same type as p_out; entries
 *                     k >= N_t(o) are ignored.
 *   gradients:        g_rho [N][P], g_u [3][N][P], g_p [N][P], same type as
 *                     the surface data.
 *
 * Ownership.  Every device buffer belongs to the caller, including the
 * workspace whose size fwh_plan_create reports; the library never allocates
 * device memory.  The plan keeps host copies of the geometry and, after
 * fwh_setup, the device address of the workspace, which must stay valid and
 * untouched by the caller until fwh_destroy.
 *
 * Streams.  `stream` is a hipStream_t (0 = legacy default stream); all work is
 * enqueued on it.  fwh_setup synchronises `stream`: it reads two doubles per
 * observer back to size the observer window and, in the FP32/BF16 modes, the
 * per-tile window widths to size the gather's LDS staging.  fwh_forward and
 * fwh_adjoint do not synchronise.  Forward and adjoint calls on one plan share
 * workspace regions (coefficients and scratch), so the caller must order all
 * calls on one plan (one stream, or events between streams); plans with
 * different workspaces are independent.
 *
 * Errors.  Every call returns FWH_OK (0) or a negative code; fwh_last_error()
 * returns a message for the calling thread's most recent failure.  Nothing is
 * thrown across the ABI and nothing aborts.
 */
#ifndef FWH_H
#define FWH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWH_OK          0
#define FWH_EINVAL     -1   /* null pointer, bad enum, non-finite or non-positive geometry */
#define FWH_EDOMAIN    -2   /* Mach number outside (0, 1), dtau <= 0 */
#define FWH_EWINDOW    -3   /* some observer has t_end < t_start (record shorter than the delay spread) */
#define FWH_ESIZE      -4   /* P, O < 1, N < 4, or sizes beyond the supported range */
#define FWH_EWORKSPACE -5   /* workspace null, too small, or not 256-byte aligned */
#define FWH_EHIP       -6   /* a HIP runtime call or kernel launch failed */
#define FWH_ESTATE     -7   /* call out of order (e.g. forward before setup) */

/* data types of surface data and gradients */
#define FWH_F64  0
#define FWH_F32  1

/* arithmetic/storage modes */
#define FWH_MODE_F64   0   /* plain FP64 form: FP64 tables, coefficients and gather */
#define FWH_MODE_F32   1   /* FP32 gather with FP32 coefficient storage; FP64 geometry, delays and taps */
#define FWH_MODE_BF16  2   /* FP32 gather with BF16 (round-to-nearest-even) coefficient storage */

typedef struct {
    int64_t n_panels;        /* P >= 1 */
    int64_t n_obs;           /* O >= 1 */
    int64_t n_tau;           /* N >= 4 source frames */
    const double *y;         /* host [P][3] panel centres */
    const double *normal;    /* host [P][3] unit outward normals */
    const double *dS;        /* host [P] panel areas, > 0 */
    const double *x_obs;     /* host [O][3] observer positions */
    double mach;             /* M0 = U0/c0, 0 < M0 < 1 */
    double aoa_deg;          /* angle of attack (degrees) of the mean flow in the x1-x2 plane */
    double dtau;             /* source (and observer) time step, > 0 */
    double tau0;             /* time of frame 0 */
    int32_t mode;            /* FWH_MODE_* */
} fwh_setup_args;

typedef struct fwh_plan fwh_plan;

/* Validate the arguments, copy the geometry into a new plan and report the
 * device workspace size in bytes.  Host only: no HIP call.  Sec. II C lists the
 * inputs (coordinates, normals, areas; Mach number, AoA, time step), Sec. III A
 * the control parameters (Mach number, AoA, time step, number of observers,
 * number of frames).  On failure *out is NULL. */
int fwh_plan_create(const fwh_setup_args *args, fwh_plan **out, size_t *workspace_bytes);

/* Bind the caller-owned device workspace (>= workspace_bytes, 256-byte
 * aligned) and run the setup on `stream`: pair delays, per-observer window
 * (Eqs. (t_start), (t_end), via a device max/min reduction read back to the
 * host), then per-pair fractional-delay taps and integrand weights
 * (Eqs. (R_New)..(R2_New), (tau2), (pT_WT_nd), (pL_WT_nd)).  Synchronises
 * `stream`.  FWH_EWINDOW if a window is empty. */
int fwh_setup(fwh_plan *plan, void *workspace, size_t workspace_bytes, void *stream);

/* Launch choices of the FP32/BF16 forward gather, for tests and measurements
 * (the defaults pick by themselves).  gather: FWH_GATHER_AUTO (the first of
 * STREAM, LDS, MFMA, DIRECT that applies), FWH_GATHER_STREAM (whole coefficient
 * rows of each panel staged once, two waves per observer: at most 8 observers
 * and 32 x 61 samples per observer; for cases bound by HBM), FWH_GATHER_LDS
 * (coefficient windows of a 32-observer tile staged in LDS; needs one panel's
 * window over a tile to fit), FWH_GATHER_MFMA (channel combine on the matrix
 * cores for 32 observers x 16 samples at a time, then the taps; needs a tile's
 * delay-index spread below about 260 samples) or FWH_GATHER_DIRECT (direct
 * loads); STREAM, LDS and MFMA make fwh_setup fail with FWH_EINVAL when they do
 * not apply.
 * splits: number of panel ranges summed separately and then added in fixed
 * order (0: chosen by fwh_setup to fill whole rounds of resident workgroups;
 * else 1 .. min(256, ceil(P/128)), FWH_ESIZE beyond).  Every choice gives the
 * same sums up to FP32 rounding order.  Host only; takes effect at the next
 * fwh_setup, which must follow (until it does, forward and adjoint calls fail
 * with FWH_ESTATE).  FWH_EINVAL for an unknown variant, or for any choice but
 * (AUTO, 0) in FWH_MODE_F64. */
#define FWH_GATHER_AUTO    0
#define FWH_GATHER_LDS     1
#define FWH_GATHER_DIRECT  2
#define FWH_GATHER_MFMA    3
#define FWH_GATHER_STREAM  4
int fwh_plan_tune(fwh_plan *plan, int32_t gather, int32_t splits);
/* The gather kernel and panel-split count fwh_setup chose (FWH_GATHER_STREAM,
 * _LDS, _MFMA or _DIRECT; FWH_GATHER_AUTO and 1 in FWH_MODE_F64).  FWH_ESTATE before
 * fwh_setup.  Either pointer may be NULL. */
int fwh_plan_info(const fwh_plan *plan, int32_t *gather, int32_t *splits);

/* Observer window of a set-up plan (host values): t_start [O], n_t [O]
 * (samples per observer) and their maximum (row length of p_out).  Any
 * output pointer may be NULL. */
int fwh_obs_window(const fwh_plan *plan, double *t_start, int64_t *n_t, int64_t *n_t_max);

/* Forward: source terms, derivatives and spline coefficients (once per
 * panel, observer-independent), then the gather-sum over panels into
 * p_out [O][n_t_max] (Sec. III B-C: "compute Noise", "interp pressure signal",
 * surface integration).  in_dtype: FWH_F64 or FWH_F32 for rho, u, p'. */
int fwh_forward(fwh_plan *plan, int32_t in_dtype, const void *rho, const void *u, const void *p_prime,
                void *p_out, void *stream);

/* Adjoint of fwh_forward (not in the paper): given grad_p = dJ/dp'(o, k)
 * [O][n_t_max], write dJ/drho, dJ/du, dJ/dp' (time-major, in_dtype).  The
 * forward inputs are needed for the nonlinear source terms.  The transposed
 * gather is panel-major and uses no atomics, so results are deterministic. */
int fwh_adjoint(fwh_plan *plan, int32_t in_dtype, const void *rho, const void *u, const void *p_prime,
                const void *grad_p, void *g_rho, void *g_u, void *g_p, void *stream);

/* Per-stage timing (the analogue of the per-phase times of Table I): when
 * enabled, every stage launched on a plan is bracketed by a pair of HIP events
 * recorded on the call's stream.  fwh_profile_read waits for the recorded
 * events of one stage, returns their summed elapsed time (ms) and the number of
 * launches, and forgets them.  Stages: */
#define FWH_STAGE_SETUP       0   /* delays, window reduction, tables (device work only) */
#define FWH_STAGE_SOURCE      1   /* source terms, derivatives, spline coefficients */
#define FWH_STAGE_GATHER      2   /* forward gather-sum over panels */
#define FWH_STAGE_REDUCE      3   /* sum of panel-split partials (FP32/BF16 modes) */
#define FWH_STAGE_ADJ_GATHER  4   /* transposed gather */
#define FWH_STAGE_SOURCE_ADJ  5   /* transpose of the source stage and chain rule */
#define FWH_NUM_STAGES        6
int fwh_profile_enable(fwh_plan *plan, int enable);
int fwh_profile_read(fwh_plan *plan, int32_t stage, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------- batches
 * Many cases (surfaces, observer sets, record lengths, flows) of uneven size run
 * as one batch: forward and adjoint of all cases are each a fixed sequence of
 * batched launches (source stage of all cases, a persistent forward gather that
 * pulls longest-first work items of all cases from a queue, the split sums; then
 * the transposed gather and source-stage transpose of all cases), so a whole
 * forward + adjoint can be captured once in a HIP graph and replayed.  No call
 * below allocates, synchronises or copies from the host except fwh_batch_bind.
 * Not in the paper: its cases run one at a time (Sec. III B); the longest-first
 * ordering follows the paper's greedy Face partition (Sec. III A).
 *
 * Every case names a set-up plan (FWH_MODE_F32 or FWH_MODE_BF16, the same for
 * all cases) and its device buffers, with the layouts of fwh_forward/fwh_adjoint
 * (p_out and grad_p are float).  The plans and buffers must outlive the batch. */
typedef struct fwh_batch fwh_batch;
typedef struct {
    fwh_plan *plan;
    const void *rho, *u, *p_prime;   /* device surface data, in_dtype */
    void *p_out;                     /* device [O][n_t_max] float */
    const void *grad_p;              /* device [O][n_t_max] float (adjoint input) */
    void *g_rho, *g_u, *g_p;         /* device gradients, in_dtype */
} fwh_batch_case;

/* Host only: validate the cases and report the size of the batch's own device
 * workspace (descriptors, work list, queue counter). */
int fwh_batch_create(const fwh_batch_case *cases, int32_t n_cases, int32_t in_dtype, fwh_batch **out,
                     size_t *workspace_bytes);
/* Host only: tile granularity for the next fwh_batch_bind: target work per item
 * (panel-observer-samples; <= 0 keeps the default) and resident blocks per
 * compute unit of the persistent gather (1..4). */
int fwh_batch_tune(fwh_batch *batch, double item_units, int32_t blocks_per_cu);
/* Host only: tiles of one case for the next fwh_batch_bind: target work per
 * forward item (<= 0 keeps the batch's) and rows of 61 samples per block of
 * the matrix-core gather (2..4; 4 only when the batch uses the LDS-staged
 * gather).  Shorter blocks waste fewer rows past short windows and cost more
 * window overlap; the autotuner of the Python binding picks both per class of
 * case sizes. */
int fwh_batch_tune_case(fwh_batch *batch, int32_t case_index, double item_units, int32_t rows);
/* The forward gather the batch runs for all its cases: FWH_GATHER_LDS when
 * every case's windows fit it, unless every plan was tuned to FWH_GATHER_MFMA
 * (fwh_plan_tune); FWH_GATHER_MFMA when only it fits them all. */
int fwh_batch_gather(const fwh_batch *batch, int32_t *gather);
/* Build the work list and upload descriptors and list into the workspace
 * (>= workspace_bytes, 256-byte aligned) on `stream`; synchronises `stream`. */
int fwh_batch_bind(fwh_batch *batch, void *workspace, size_t workspace_bytes, void *stream);
/* Enqueue the batched forward (all p_out) / adjoint (all gradients) on `stream`. */
int fwh_batch_forward(fwh_batch *batch, void *stream);
int fwh_batch_adjoint(fwh_batch *batch, void *stream);
/* Number of work items of the persistent gather, total panel-observer-samples
 * and resident blocks of the persistent grid (any pointer may be NULL). */
int fwh_batch_info(const fwh_batch *batch, int64_t *n_items, int64_t *units, int64_t *grid);
void fwh_batch_destroy(fwh_batch *batch);

/* Release the plan (host memory only; the workspace stays the caller's). */
void fwh_destroy(fwh_plan *plan);

/* Post-processing of a forward result p_out ([O][n_t_max] as written by
 * fwh_forward on this plan, same type) for the comparisons of Sec. IV:
 *   rms [O] (float): sqrt of the mean of p'^2 over each observer's N_t samples
 *   (the RMS directivity of Sec. IV A-B);
 *   psd [O][seg_len/2 + 1] (float): one-sided Welch power spectral density of
 *   each observer's N_t samples (Sec. IV C): segments of seg_len samples with
 *   50 % overlap, periodic Hann window, averaged |DFT|^2 scaled to a density
 *   c_f / (n_seg f_s sum w^2) with f_s = 1/dtau and c_f = 2 except at f = 0
 *   and f_s/2, times span_ratio (the spanwise correction b_exp / b_m of
 *   Eq. (PSD_corr); 1 for none).  Frequency f_k = k / (seg_len dtau).
 * seg_len: power of two in [16, 4096], <= every N_t (FWH_ESIZE otherwise).
 * Device pointers, caller-owned; enqueued on `stream`, nothing allocated. */
int fwh_post(const fwh_plan *plan, const void *p_out, int64_t seg_len, double span_ratio, float *psd, float *rms,
             void *stream);

/* ------------------------------------------------------------------------
 * General motion (Sec. II B, Eqs. (pT), (pL), (tau)): a permeable surface in
 * prescribed motion, the medium and the observers at rest.  Nondimensional as
 * in Sec. II D with a reference speed: rho0 = 1, c0 = 1/mach (mach = reference
 * speed / c0), every speed in units of the reference speed.
 *
 * Device pointers (caller-owned, FP64, time-major; the kinematics must stay valid
 * until the last call on the plan):
 *   y, normal, vel [N][P][3]   panel centre, unit outward normal and velocity at
 *                              tau_n = tau0 + n dtau (rigid panels: dS constant)
 *   dS [P], x_obs [O][3]       panel areas (> 0), observer positions
 * and, per forward call, rho [N][P], u [3][N][P] (fluid velocity in the medium
 * frame), pp [N][P] (pressure pulsation p - p0).
 *
 * What is computed: per panel and frame Q_i = v_i + rho (u_i - v_i) and
 * L_i = p' n_i + rho u_i (u_j - v_j) n_j (Eqs. (Qn), (Li), P_ij = p' delta_ij),
 * M_i = mach v_i; second-order source-time differences (one-sided at the first
 * and last frame); the 19 observer-independent quantities of the integrand
 * (Qd.n + Q.nd, Q_n, L_i, Ld_i, L_M, M_i, Md_i, M^2, y_i) are each interpolated
 * in source time by a natural cubic spline.  For every observer sample
 * t_k = t_start + k dtau and panel, the retarded time solves tau + mach |x - Y(tau)|
 * = t_k on the splined trajectory Y (Eq. (tau)), and the integrand of
 * Eqs. (pT) + (pL) times dS / (4 pi) is evaluated there and summed over panels.
 * Window: t_start(o) = max_p [tau0 + mach |x_o - y_p(tau0)|],
 *         t_end(o) = min_p [tau_{N-1} + mach |x_o - y_p(tau_{N-1})|],
 *         N_t(o) = floor((t_end - t_start) / dtau + 1e-9) + 1.
 * The surface must move subsonically (mach |v| < 1); N_t < 2N then holds.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_panels, n_obs, n_tau;      /* P >= 1, O >= 1, N >= 4 */
    double mach, dtau, tau0;             /* 0 < mach < 1, dtau > 0, tau0 finite */
    const double *y, *normal, *vel;      /* device, [N][P][3] */
    const double *dS, *x_obs;            /* device, [P], [O][3] */
} fwh_gm_args;

typedef struct fwh_gm_plan fwh_gm_plan;

/* Host only: validates sizes and scalars (the device arrays are not read here)
 * and returns the workspace size in bytes (caller-owned, 256-byte aligned).
 * FWH_ESIZE / FWH_EDOMAIN / FWH_EINVAL on bad arguments. */
int fwh_gm_plan_create(const fwh_gm_args *args, fwh_gm_plan **out, size_t *workspace_bytes);

/* Binds the workspace, computes the observer window on the device (enqueued on
 * `stream`, then waits for the stream) and keeps t_start and N_t on the plan.
 * FWH_EWINDOW if some observer's window is empty, FWH_ESIZE if N_t >= 2N (the
 * surface moved supersonically). */
int fwh_gm_window(fwh_gm_plan *plan, void *workspace, size_t workspace_bytes, void *stream);

/* Host copies of the window (after fwh_gm_window): t_start [O], n_t [O] (may be
 * NULL), n_t_max. */
int fwh_gm_obs_window(const fwh_gm_plan *plan, double *t_start, int64_t *n_t, int64_t *n_t_max);

/* p_out [O][n_t_max] (FP64, device) = p'(x_o, t_start(o) + k dtau) for k < N_t(o),
 * 0 beyond.  Enqueued on `stream`; nothing allocated. */
int fwh_gm_forward(fwh_gm_plan *plan, const double *rho, const double *u, const double *pp, double *p_out,
                   void *stream);

/* Optional event timing of the two stages of fwh_gm_forward on its stream:
 * FWH_GM_STAGE_SOURCE (channels and spline coefficients) and
 * FWH_GM_STAGE_GATHER (retarded-time gather and the sum of panel ranges).
 * fwh_gm_profile_read waits for the recorded events, returns their total
 * milliseconds and count, and clears them. */
#define FWH_GM_STAGE_SOURCE 0
#define FWH_GM_STAGE_GATHER 1
#define FWH_GM_NUM_STAGES   2
int fwh_gm_profile_enable(fwh_gm_plan *plan, int enable);
int fwh_gm_profile_read(fwh_gm_plan *plan, int32_t stage, double *total_ms, int64_t *launches);

/* Frees the host side of the plan (the workspace is the caller's). */
void fwh_gm_destroy(fwh_gm_plan *plan);

/* ------------------------------------------------------------------------
 * Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * it): fwh_plan_create + fwh_setup + fwh_forward in one call, with the
 * workspace taken from a static device array of FWH_NOALLOC_BYTES that each
 * GPU the library runs on holds from the first such call until the process
 * ends.  Inputs as for fwh_forward (device, time-major, in_dtype); p_out is a
 * caller-owned device buffer of out_capacity elements (double in FWH_MODE_F64,
 * float otherwise) that receives [O][*n_t_max] as fwh_forward writes it
 * (O x N elements always suffice, since N_t <= N); *n_t_max (host) returns
 * the row length.  No hipMalloc, hipFree or other device allocation; the plan's
 * host copy of the geometry is allocated and freed inside the call.  Like
 * fwh_setup it synchronises `stream`.  FWH_ESIZE when the case needs a larger
 * workspace (the message names both sizes) or p_out is too small; the other
 * codes as for fwh_plan_create, fwh_setup and fwh_forward.  Every call on one
 * GPU uses that GPU's one array: calls that overlap on one GPU (other threads,
 * other streams) race and must be serialised by the caller.  Each call writes
 * every workspace region before reading it, so nothing needs clearing. */
#define FWH_NOALLOC_BYTES (64u << 20)
int fwh_forward_noalloc(const fwh_setup_args *args, int32_t in_dtype, const void *rho, const void *u,
                        const void *p_prime, void *p_out, int64_t out_capacity, int64_t *n_t_max, void *stream);

/* Message of the calling thread's last failure ("" if none). */
const char *fwh_last_error(void);

/* Library version string. */
const char *fwh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FWH_H */
