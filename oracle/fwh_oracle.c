/*
 * fwh_oracle.c -- plain, slow, FP64 CPU oracle of the wind-tunnel FW-H far-field
 * integral (permeable surface, Farassat 1A after the Garrick-triangle change of
 * frame and the angle-of-attack rotation, nondimensional form of Sec. II D).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU path.
 *
 * The oracle follows the paper literally and per (panel, observer) pair, in the
 * order of Sec. III B:
 *   "compute R"      -> pair geometry, Eqs. (R_New)..(R2_New), delay Eq. (tau2)
 *   "compute Noise"  -> source terms Eqs. (Qn_New_nd), (Li_New_nd) at every source
 *                       frame, 2nd-order derivatives in source time (one-sided at
 *                       the first and last frame, central elsewhere), integrand of
 *                       Eqs. (pT_WT_nd) + (pL_WT_nd)
 *   "compute t"      -> observer window Eqs. (t_start), (t_end)
 *   "interp"         -> cubic spline of each pair's source-time signal, evaluated
 *                       at the observer times
 *   surface sum      -> sum over panels.
 *
 * Readings where the paper is silent:
 *   - the surface Mach vector in the Garrick frame is M = -M0*U0hat (the surface
 *     moves against the mean flow), so M^2 = M0^2 and L_M = -M0 L.U0hat;
 *   - rho and u are full values, the pressure input is the pulsation p - p0;
 *   - the spline is the natural cubic spline (zero second derivative at both ends);
 *   - observer time step = source time step; N_t = floor((t_end-t_start)/dtau+1e-9)+1;
 *     the window uses per-observer max/min delays and a general tau0;
 *   - spline evaluation clamps the interval index to [0, N-2] and t to [0, 1].
 *
 * Layouts: inputs and gradients are PANEL-major here ([P][N] per variable); the
 * Python wrapper transposes from the time-major layout of the GPU interface.
 * Observer outputs are [O][nt_stride] with zero padding beyond N_t(o).
 *
 * Determinism: panels are summed in fixed blocks of ORC_BLOCK, block partial sums
 * are added in block order, so results do not depend on the thread count.
 *
 * A second section (orc_gm_*) is the general-motion form of Sec. II B: a surface
 * in prescribed motion, medium and observers at rest, Eqs. (pT), (pL) at the
 * retarded time of Eq. (tau); its readings are listed at the section head.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_BLOCK 256
#define ORC_PI 3.14159265358979323846

/* ---------------------------------------------------------------- geometry */

/* Pair geometry for one (observer x, panel y), Sec. II C:
 *   d = x - y; M1 = M0 cos(AoA), M2 = M0 sin(AoA)                       Eqs. (M1),(M2)
 *   R_* = sqrt((M1 d1 + M2 d2)^2 + beta^2 |d|^2)                        Eq. (R_s_New)
 *   R   = (-M1 d1 - M2 d2 + R_*) / beta^2                               Eq. (R_New)
 *   d1' = d1 cos + d2 sin, d2' = -d1 sin + d2 cos                       Eqs. (d1_prime),(d2_prime)
 *   R1' = (-M0 R_* + d1')/(beta^2 R), R2' = d2'/R, R3 = d3/R            Eqs. (R1_prime)..(R3_New)
 *   R1 = R1' cos - R2' sin, R2 = R1' sin + R2' cos                      Eqs. (R1_New),(R2_New)
 *   M_R = M . Rhat with M = -M0 (cos, sin, 0)                           Eq. (MR)
 *   delay = R / c0 = M0 R                                               Eq. (tau2), c0* = 1/M0
 */
static void pair_geometry(const double *x, const double *y, double M0, double aoa,
                          double *R_out, double *Rs_out, double Rhat[3], double *MR_out, double *D_out)
{
    const double ca = cos(aoa), sa = sin(aoa);
    const double M1 = M0 * ca, M2 = M0 * sa;
    const double beta2 = 1.0 - M0 * M0;
    const double d1 = x[0] - y[0], d2 = x[1] - y[1], d3 = x[2] - y[2];
    const double md = M1 * d1 + M2 * d2;
    const double Rs = sqrt(md * md + beta2 * (d1 * d1 + d2 * d2 + d3 * d3));
    const double R = (-M1 * d1 - M2 * d2 + Rs) / beta2;
    const double d1p = d1 * ca + d2 * sa;
    const double d2p = -d1 * sa + d2 * ca;
    const double R1p = (-M0 * Rs + d1p) / (beta2 * R);
    const double R2p = d2p / R;
    Rhat[0] = R1p * ca - R2p * sa;
    Rhat[1] = R1p * sa + R2p * ca;
    Rhat[2] = d3 / R;
    const double Mv[3] = {-M0 * ca, -M0 * sa, 0.0};
    *MR_out = Mv[0] * Rhat[0] + Mv[1] * Rhat[1] + Mv[2] * Rhat[2];
    *R_out = R;
    *Rs_out = Rs;
    *D_out = M0 * R;
}

void orc_pair_geometry(int64_t P, int64_t O, const double *y, const double *x_obs, double mach,
                       double aoa_deg, double *R, double *Rs, double *Rhat, double *MR, double *D)
{
    const double aoa = aoa_deg * (ORC_PI / 180.0);
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < O; ++o)
        for (int64_t p = 0; p < P; ++p) {
            const int64_t i = o * P + p;
            pair_geometry(x_obs + 3 * o, y + 3 * p, mach, aoa, R + i, Rs + i, Rhat + 3 * i, MR + i, D + i);
        }
}

/* ------------------------------------------------------------ source terms */

/* Eqs. (Qn_New_nd), (Li_New_nd), (U_0_nd) with P_ij = p' delta_ij (Eq. (Pij),
 * viscous stress dropped):
 *   Q   = (-U0_i + rho u_i) n_i
 *   L_i = p' n_i + rho (u_i - U0_i) u_j n_j
 * One panel, N frames, contiguous series. */
static void source_terms_panel(int64_t N, const double *rho, const double *u1, const double *u2,
                               const double *u3, const double *pp, const double *nrm, double aoa,
                               double *Q, double *L1, double *L2, double *L3)
{
    const double U0[3] = {cos(aoa), sin(aoa), 0.0};
    for (int64_t n = 0; n < N; ++n) {
        const double u[3] = {u1[n], u2[n], u3[n]};
        const double un = u[0] * nrm[0] + u[1] * nrm[1] + u[2] * nrm[2];
        const double U0n = U0[0] * nrm[0] + U0[1] * nrm[1] + U0[2] * nrm[2];
        Q[n] = -U0n + rho[n] * un;
        L1[n] = pp[n] * nrm[0] + rho[n] * (u[0] - U0[0]) * un;
        L2[n] = pp[n] * nrm[1] + rho[n] * (u[1] - U0[1]) * un;
        L3[n] = pp[n] * nrm[2] + rho[n] * (u[2] - U0[2]) * un;
    }
}

void orc_source_terms(int64_t N, int64_t P, const double *rho, const double *u, const double *pp,
                      const double *normal, double aoa_deg, double *Q, double *L)
{
    const double aoa = aoa_deg * (ORC_PI / 180.0);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p)
        source_terms_panel(N, rho + p * N, u + p * N, u + (P + p) * N, u + (2 * P + p) * N, pp + p * N,
                           normal + 3 * p, aoa, Q + p * N, L + p * N, L + (P + p) * N, L + (2 * P + p) * N);
}

/* ------------------------------------------------------ source derivatives */

/* Second-order derivative in source time (Sec. III B): one-sided three-point
 * formulas at the first and last frame, central difference elsewhere. N >= 3. */
void orc_fd(int64_t N, const double *f, double h, double *df)
{
    const double i2h = 1.0 / (2.0 * h);
    df[0] = (-3.0 * f[0] + 4.0 * f[1] - f[2]) * i2h;
    for (int64_t n = 1; n < N - 1; ++n) df[n] = (f[n + 1] - f[n - 1]) * i2h;
    df[N - 1] = (3.0 * f[N - 1] - 4.0 * f[N - 2] + f[N - 3]) * i2h;
}

/* --------------------------------------------------------- cubic spline */

/* Natural cubic spline through (tau_n, f_n), uniform spacing h: second
 * derivatives m with m_0 = m_{N-1} = 0 and, for n = 1..N-2,
 *   m_{n-1} + 4 m_n + m_{n+1} = 6 (f_{n+1} - 2 f_n + f_{n-1}) / h^2,
 * solved by the Thomas algorithm.  work: N doubles. */
void orc_spline_m(int64_t N, const double *f, double h, double *m, double *work)
{
    double *cp = work;
    m[0] = 0.0;
    m[N - 1] = 0.0;
    if (N < 3) return;
    const double s = 6.0 / (h * h);
    /* forward elimination on rows 1..N-2 (diagonal 4, off-diagonals 1) */
    double prev_c = 0.0, prev_d = 0.0;
    for (int64_t n = 1; n <= N - 2; ++n) {
        const double rhs = s * (f[n + 1] - 2.0 * f[n] + f[n - 1]);
        const double denom = 4.0 - (n > 1 ? prev_c : 0.0);
        const double c = 1.0 / denom;
        const double d = (rhs - (n > 1 ? prev_d : 0.0)) / denom;
        cp[n] = c;
        m[n] = d;
        prev_c = c;
        prev_d = d;
    }
    for (int64_t n = N - 3; n >= 1; --n) m[n] = m[n] - cp[n] * m[n + 1];
}

/* Spline value at tau (second-derivative form): interval j = floor((tau-tau0)/h)
 * clamped to [0, N-2], t = (tau - tau_j)/h clamped to [0, 1],
 *   s = (1-t) f_j + t f_{j+1} + h^2/6 [((1-t)^3 - (1-t)) m_j + (t^3 - t) m_{j+1}]. */
static void spline_locate(int64_t N, double tau0, double h, double tau, int64_t *j_out, double *t_out)
{
    const double x = (tau - tau0) / h;
    double jf = floor(x);
    if (jf < 0.0) jf = 0.0;
    if (jf > (double)(N - 2)) jf = (double)(N - 2);
    const int64_t j = (int64_t)jf;
    double t = x - (double)j;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    *j_out = j;
    *t_out = t;
}

double orc_spline_eval(int64_t N, const double *f, const double *m, double tau0, double h, double tau)
{
    int64_t j;
    double t;
    spline_locate(N, tau0, h, tau, &j, &t);
    const double u = 1.0 - t;
    return u * f[j] + t * f[j + 1] + (h * h / 6.0) * ((u * u * u - u) * m[j] + (t * t * t - t) * m[j + 1]);
}

/* ---------------------------------------------------------- observer window */

/* Eqs. (t_start), (t_end), per observer, with a general tau0:
 *   t_start = tau0 + max_p delay, t_end = tau_{N-1} + min_p delay,
 *   N_t = floor((t_end - t_start)/dtau + 1e-9) + 1.
 * Returns 0, or -1 if some observer has t_end < t_start (empty window). */
int orc_obs_window(int64_t P, int64_t O, const double *D, int64_t N, double tau0, double dtau,
                   double *t_start, int64_t *n_t)
{
    int status = 0;
    for (int64_t o = 0; o < O; ++o) {
        double dmax = -INFINITY, dmin = INFINITY;
        for (int64_t p = 0; p < P; ++p) {
            const double d = D[o * P + p];
            if (d > dmax) dmax = d;
            if (d < dmin) dmin = d;
        }
        const double ts = tau0 + dmax;
        const double te = tau0 + (double)(N - 1) * dtau + dmin;
        t_start[o] = ts;
        if (te < ts) {
            n_t[o] = 0;
            status = -1;
        } else {
            n_t[o] = (int64_t)floor((te - ts) / dtau + 1e-9) + 1;
        }
    }
    return status;
}

/* ------------------------------------------------------ per-pair signal */

typedef struct {
    double dS, M0, aoa, h, tau0;
    int64_t N;
} pair_ctx;

/* Integrand of Eqs. (pT_WT_nd) + (pL_WT_nd) for one pair at every source frame:
 *   f = dS/(4 pi) [ Qdot/(R(1-M_R)^2) + Q (M_R - M^2)/(M0 R^2 (1-M_R)^3)
 *                   + M0 Ldot_R/(R(1-M_R)^2) + (L_R - L_M)/(R^2(1-M_R)^2)
 *                   + L_R (M_R - M^2)/(R^2 (1-M_R)^3) ]
 * with L_R = L . Rhat (Eq. (LR)), L_M = L . M (Eq. (LM)), M^2 = M0^2. */
static void pair_integrand(const pair_ctx *c, const double *Q, const double *Qd, const double *const L[3],
                           const double *const Ld[3], double R, const double Rhat[3], double MR, double *f)
{
    const double M0 = c->M0;
    const double Mv[3] = {-M0 * cos(c->aoa), -M0 * sin(c->aoa), 0.0};
    const double M2 = M0 * M0;
    const double om = 1.0 - MR;
    const double w = c->dS / (4.0 * ORC_PI);
    for (int64_t n = 0; n < c->N; ++n) {
        const double LR = L[0][n] * Rhat[0] + L[1][n] * Rhat[1] + L[2][n] * Rhat[2];
        const double LdR = Ld[0][n] * Rhat[0] + Ld[1][n] * Rhat[1] + Ld[2][n] * Rhat[2];
        const double LM = L[0][n] * Mv[0] + L[1][n] * Mv[1] + L[2][n] * Mv[2];
        const double pT = Qd[n] / (R * om * om) + Q[n] * (MR - M2) / (M0 * R * R * om * om * om);
        const double pL = M0 * LdR / (R * om * om) + (LR - LM) / (R * R * om * om)
                          + LR * (MR - M2) / (R * R * om * om * om);
        f[n] = w * (pT + pL);
    }
}

/* Derivative of the integrand with respect to each source quantity at a frame:
 * coefficients of Qdot, Q, Ldot_i, L_i (the integrand is linear in them). */
static void pair_integrand_coeffs(const pair_ctx *c, double R, const double Rhat[3], double MR, double a[8])
{
    const double M0 = c->M0;
    const double Mv[3] = {-M0 * cos(c->aoa), -M0 * sin(c->aoa), 0.0};
    const double M2 = M0 * M0;
    const double om = 1.0 - MR;
    const double w = c->dS / (4.0 * ORC_PI);
    a[0] = w / (R * om * om);                                    /* Qdot   */
    a[1] = w * (MR - M2) / (M0 * R * R * om * om * om);          /* Q      */
    for (int i = 0; i < 3; ++i) {
        a[2 + i] = w * M0 * Rhat[i] / (R * om * om);             /* Ldot_i */
        a[5 + i] = w * ((Rhat[i] - Mv[i]) / (R * R * om * om)    /* L_i    */
                        + Rhat[i] * (MR - M2) / (R * R * om * om * om));
    }
}

/* --------------------------------------------------------------- forward */

typedef struct {
    int64_t P, O, N;
    const double *y, *normal, *dS, *x_obs;
    double mach, aoa_deg, dtau, tau0;
} orc_case;

static double *xmalloc(size_t n) { return (double *)malloc(n * sizeof(double)); }

/* Observer-time signal of one pair from its source series (Q, L_i), accumulated
 * into acc[0..nt-1]: derivative, integrand, spline, evaluation at
 * tau_k = t_start + k dtau - delay.  work: 12*N doubles. */
static void pair_accumulate(const pair_ctx *c, const double *Q, const double *const L[3], const double *x,
                            const double *y, double t_start, int64_t nt, double *acc, double *work)
{
    const int64_t N = c->N;
    double *Qd = work, *Ld0 = work + N, *Ld1 = work + 2 * N, *Ld2 = work + 3 * N;
    double *f = work + 4 * N, *m = work + 5 * N, *tmp = work + 6 * N;
    orc_fd(N, Q, c->h, Qd);
    orc_fd(N, L[0], c->h, Ld0);
    orc_fd(N, L[1], c->h, Ld1);
    orc_fd(N, L[2], c->h, Ld2);
    const double *Ld[3] = {Ld0, Ld1, Ld2};
    double R, Rs, Rhat[3], MR, D;
    pair_geometry(x, y, c->M0, c->aoa, &R, &Rs, Rhat, &MR, &D);
    pair_integrand(c, Q, Qd, L, Ld, R, Rhat, MR, f);
    orc_spline_m(N, f, c->h, m, tmp);
    for (int64_t k = 0; k < nt; ++k) {
        const double tau = t_start + (double)k * c->h - D;
        acc[k] += orc_spline_eval(N, f, m, c->tau0, c->h, tau);
    }
}

static int window_for_case(const orc_case *cs, double *t_start, int64_t *n_t)
{
    const double aoa = cs->aoa_deg * (ORC_PI / 180.0);
    double *D = xmalloc((size_t)cs->O * cs->P);
    for (int64_t o = 0; o < cs->O; ++o)
        for (int64_t p = 0; p < cs->P; ++p) {
            double R, Rs, Rhat[3], MR;
            pair_geometry(cs->x_obs + 3 * o, cs->y + 3 * p, cs->mach, aoa, &R, &Rs, Rhat, &MR, D + o * cs->P + p);
        }
    const int st = orc_obs_window(cs->P, cs->O, D, cs->N, cs->tau0, cs->dtau, t_start, n_t);
    free(D);
    return st;
}

/* Core forward: p'(o, k) = sum_p s_{p,o}(t_k), observers in obs_idx[0..n_sel-1]
 * (indices into the case's observers), source series given per panel either as
 * raw inputs (rho, u, p'; src_mode 0) or as source terms (Q, L; src_mode 1).
 * out: [n_sel][nt_stride], zero padded.  Returns 0, -1 (empty window), -2 (nt_stride
 * too small), -3 (bad sizes). */
static int forward_core(const orc_case *cs, int src_mode, const double *a0, const double *a1, const double *a2,
                        const int64_t *obs_idx, int64_t n_sel, double *out, int64_t nt_stride)
{
    const int64_t P = cs->P, N = cs->N, O = cs->O;
    if (P < 1 || cs->P < 1 || O < 1 || N < 4 || !(cs->mach > 0.0 && cs->mach < 1.0) || !(cs->dtau > 0.0))
        return -3;
    double *t_start = xmalloc((size_t)O);
    int64_t *n_t = (int64_t *)malloc((size_t)O * sizeof(int64_t));
    if (window_for_case(cs, t_start, n_t) != 0) { free(t_start); free(n_t); return -1; }
    for (int64_t s = 0; s < n_sel; ++s)
        if (n_t[obs_idx[s]] > nt_stride) { free(t_start); free(n_t); return -2; }
    const double aoa = cs->aoa_deg * (ORC_PI / 180.0);
    const int64_t nblk = (P + ORC_BLOCK - 1) / ORC_BLOCK;
    memset(out, 0, sizeof(double) * (size_t)n_sel * (size_t)nt_stride);
    for (int64_t s = 0; s < n_sel; ++s) {                      /* loop over observers */
        const int64_t o = obs_idx[s];
        const int64_t nt = n_t[o];
        double *part = (double *)calloc((size_t)nblk * (size_t)nt, sizeof(double));
#pragma omp parallel
        {
            double *work = xmalloc((size_t)16 * N);
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < nblk; ++b) {
                const int64_t p_end = (b + 1) * ORC_BLOCK < P ? (b + 1) * ORC_BLOCK : P;
                for (int64_t p = b * ORC_BLOCK; p < p_end; ++p) {
                    pair_ctx c = {cs->dS[p], cs->mach, aoa, cs->dtau, cs->tau0, N};
                    const double *Q;
                    const double *L[3];
                    double *src = work + 12 * N;
                    if (src_mode == 0) { /* recompute Q, L for this pair (Sec. III B: not stored) */
                        source_terms_panel(N, a0 + p * N, a1 + p * N, a1 + (P + p) * N, a1 + (2 * P + p) * N,
                                           a2 + p * N, cs->normal + 3 * p, aoa, src, src + N, src + 2 * N, src + 3 * N);
                        Q = src;
                        L[0] = src + N; L[1] = src + 2 * N; L[2] = src + 3 * N;
                    } else {
                        Q = a0 + p * N;
                        L[0] = a1 + p * N; L[1] = a1 + (P + p) * N; L[2] = a1 + (2 * P + p) * N;
                    }
                    pair_accumulate(&c, Q, L, cs->x_obs + 3 * o, cs->y + 3 * p, t_start[o], nt, part + b * nt, work);
                }
            }
            free(work);
        }
        for (int64_t b = 0; b < nblk; ++b)                     /* surface sum, fixed order */
            for (int64_t k = 0; k < nt; ++k) out[s * nt_stride + k] += part[b * nt + k];
        free(part);
    }
    free(t_start);
    free(n_t);
    return 0;
}

int orc_window(int64_t P, int64_t O, int64_t N, const double *y, const double *x_obs, double mach, double aoa_deg,
               double dtau, double tau0, double *t_start, int64_t *n_t)
{
    orc_case cs = {P, O, N, y, NULL, NULL, x_obs, mach, aoa_deg, dtau, tau0};
    return window_for_case(&cs, t_start, n_t);
}

int orc_forward(int64_t P, int64_t O, int64_t N, const double *y, const double *normal, const double *dS,
                const double *x_obs, double mach, double aoa_deg, double dtau, double tau0,
                const double *rho, const double *u, const double *pp,
                const int64_t *obs_idx, int64_t n_sel, double *out, int64_t nt_stride)
{
    orc_case cs = {P, O, N, y, normal, dS, x_obs, mach, aoa_deg, dtau, tau0};
    return forward_core(&cs, 0, rho, u, pp, obs_idx, n_sel, out, nt_stride);
}

int orc_forward_sources(int64_t P, int64_t O, int64_t N, const double *y, const double *normal, const double *dS,
                        const double *x_obs, double mach, double aoa_deg, double dtau, double tau0,
                        const double *Q, const double *L, const int64_t *obs_idx, int64_t n_sel, double *out,
                        int64_t nt_stride)
{
    orc_case cs = {P, O, N, y, normal, dS, x_obs, mach, aoa_deg, dtau, tau0};
    return forward_core(&cs, 1, Q, L, NULL, obs_idx, n_sel, out, nt_stride);
}

/* --------------------------------------------------------------- adjoint */

/* Transpose of the per-pair evaluation operator (spline of f, evaluated at the
 * nt observer times): fbar = E^T gbar.  E = E_f + E_m S, where E_f/E_m are the
 * evaluation weights on f and on the second derivatives m, and S maps f to m
 * (m = 6/h^2 T^{-1} Delta2 f on interior rows, T = tridiag(1,4,1) symmetric). */
static void spline_eval_transpose(int64_t N, double tau0, double h, double t_start, double D, int64_t nt,
                                  const double *gbar, double *fbar, double *work)
{
    double *mbar = work, *z = work + N, *cp = work + 2 * N;
    for (int64_t n = 0; n < N; ++n) { fbar[n] = 0.0; mbar[n] = 0.0; }
    const double h26 = h * h / 6.0;
    for (int64_t k = 0; k < nt; ++k) {
        const double tau = t_start + (double)k * h - D;
        int64_t j;
        double t;
        spline_locate(N, tau0, h, tau, &j, &t);
        const double u = 1.0 - t, g = gbar[k];
        fbar[j] += u * g;
        fbar[j + 1] += t * g;
        mbar[j] += h26 * (u * u * u - u) * g;
        mbar[j + 1] += h26 * (t * t * t - t) * g;
    }
    if (N < 3) return;
    /* z = T^{-1} mbar[1..N-2] (T symmetric: same Thomas solve as the forward) */
    double prev_c = 0.0, prev_d = 0.0;
    for (int64_t n = 1; n <= N - 2; ++n) {
        const double denom = 4.0 - (n > 1 ? prev_c : 0.0);
        const double c = 1.0 / denom;
        const double d = (mbar[n] - (n > 1 ? prev_d : 0.0)) / denom;
        cp[n] = c;
        z[n] = d;
        prev_c = c;
        prev_d = d;
    }
    for (int64_t n = N - 3; n >= 1; --n) z[n] = z[n] - cp[n] * z[n + 1];
    const double s = 6.0 / (h * h);
    for (int64_t n = 1; n <= N - 2; ++n) {   /* Delta2^T */
        fbar[n - 1] += s * z[n];
        fbar[n] -= 2.0 * s * z[n];
        fbar[n + 1] += s * z[n];
    }
}

/* Transpose of orc_fd: out += D^T v. */
static void fd_transpose_add(int64_t N, const double *v, double h, double *out)
{
    const double i2h = 1.0 / (2.0 * h);
    out[0] += -3.0 * v[0] * i2h;
    out[1] += 4.0 * v[0] * i2h;
    out[2] += -1.0 * v[0] * i2h;
    for (int64_t n = 1; n < N - 1; ++n) {
        out[n + 1] += v[n] * i2h;
        out[n - 1] -= v[n] * i2h;
    }
    out[N - 1] += 3.0 * v[N - 1] * i2h;
    out[N - 2] += -4.0 * v[N - 1] * i2h;
    out[N - 3] += 1.0 * v[N - 1] * i2h;
}

/* Gradient of J with dJ/dp'(o,k) = gbar[o][k] (k < N_t(o); padding ignored).
 * mode 0: raw inputs (rho, u, p') -> (g_rho, g_u, g_p), panel-major.
 * mode 1: source terms -> (Qbar, Lbar), panel-major (the linear part). */
/* Gradients of the panels pidx[0..np) (all P panels in order when pidx is NULL).
 * The window comes from every panel of the case; the data and the outputs are
 * those of the listed panels only ([np][N] per variable), since the gradient of
 * a panel depends on its own data and the observer windows alone. */
static int adjoint_core(const orc_case *cs, int mode, const double *rho, const double *u, const double *pp,
                        const double *gbar, int64_t nt_stride, const int64_t *pidx, int64_t np,
                        double *g0, double *g1, double *g2)
{
    const int64_t N = cs->N, O = cs->O;
    const int64_t P = pidx ? np : cs->P;  /* panels computed (data and output rows) */
    if (pidx)
        for (int64_t j = 0; j < np; ++j)
            if (pidx[j] < 0 || pidx[j] >= cs->P) return -3;
    if (P < 1 || cs->P < 1 || O < 1 || N < 4 || !(cs->mach > 0.0 && cs->mach < 1.0) || !(cs->dtau > 0.0))
        return -3;
    double *t_start = xmalloc((size_t)O);
    int64_t *n_t = (int64_t *)malloc((size_t)O * sizeof(int64_t));
    if (window_for_case(cs, t_start, n_t) != 0) { free(t_start); free(n_t); return -1; }
    for (int64_t o = 0; o < O; ++o)
        if (n_t[o] > nt_stride) { free(t_start); free(n_t); return -2; }
    const double aoa = cs->aoa_deg * (ORC_PI / 180.0);
    const double U0[3] = {cos(aoa), sin(aoa), 0.0};
#pragma omp parallel
    {
        double *work = xmalloc((size_t)16 * N);
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < P; ++p) {
            const int64_t pg = pidx ? pidx[p] : p;  /* panel of the case (geometry) */
            double *Sbar = work;               /* 8 channels: Qdot, Q, Ldot_1..3, L_1..3 */
            double *fbar = work + 8 * N;
            double *tmp = work + 9 * N;        /* 3N */
            double *srcbar = work + 12 * N;    /* Qbar, Lbar_1..3 */
            memset(Sbar, 0, sizeof(double) * 8 * (size_t)N);
            pair_ctx c = {cs->dS[pg], cs->mach, aoa, cs->dtau, cs->tau0, N};
            for (int64_t o = 0; o < O; ++o) {
                double R, Rs, Rhat[3], MR, D, a[8];
                pair_geometry(cs->x_obs + 3 * o, cs->y + 3 * pg, cs->mach, aoa, &R, &Rs, Rhat, &MR, &D);
                pair_integrand_coeffs(&c, R, Rhat, MR, a);
                spline_eval_transpose(N, cs->tau0, cs->dtau, t_start[o], D, n_t[o], gbar + o * nt_stride, fbar, tmp);
                for (int ch = 0; ch < 8; ++ch)
                    for (int64_t n = 0; n < N; ++n) Sbar[ch * N + n] += a[ch] * fbar[n];
            }
            /* source-term adjoints: Xbar = Sbar_X + D^T Sbar_Xdot */
            for (int64_t n = 0; n < N; ++n) {
                srcbar[n] = Sbar[1 * N + n];
                for (int i = 0; i < 3; ++i) srcbar[(1 + i) * N + n] = Sbar[(5 + i) * N + n];
            }
            fd_transpose_add(N, Sbar + 0 * N, cs->dtau, srcbar);
            for (int i = 0; i < 3; ++i) fd_transpose_add(N, Sbar + (2 + i) * N, cs->dtau, srcbar + (1 + i) * N);
            if (mode == 1) {
                for (int64_t n = 0; n < N; ++n) {
                    g0[p * N + n] = srcbar[n];
                    for (int i = 0; i < 3; ++i) g1[(i * P + p) * N + n] = srcbar[(1 + i) * N + n];
                }
                continue;
            }
            /* chain rule through Q = rho u.n - U0.n, L_i = p' n_i + rho (u_i - U0_i) u.n */
            const double *nr = cs->normal + 3 * pg;
            for (int64_t n = 0; n < N; ++n) {
                const double r = rho[p * N + n];
                const double uu[3] = {u[p * N + n], u[(P + p) * N + n], u[(2 * P + p) * N + n]};
                const double un = uu[0] * nr[0] + uu[1] * nr[1] + uu[2] * nr[2];
                const double Qb = srcbar[n];
                const double Lb[3] = {srcbar[N + n], srcbar[2 * N + n], srcbar[3 * N + n]};
                const double Lw = Lb[0] * (uu[0] - U0[0]) + Lb[1] * (uu[1] - U0[1]) + Lb[2] * (uu[2] - U0[2]);
                g0[p * N + n] = un * (Qb + Lw);
                for (int i = 0; i < 3; ++i) g1[(i * P + p) * N + n] = r * nr[i] * (Qb + Lw) + r * un * Lb[i];
                g2[p * N + n] = Lb[0] * nr[0] + Lb[1] * nr[1] + Lb[2] * nr[2];
            }
            (void)pp;
        }
        free(work);
    }
    free(t_start);
    free(n_t);
    return 0;
}

int orc_adjoint(int64_t P, int64_t O, int64_t N, const double *y, const double *normal, const double *dS,
                const double *x_obs, double mach, double aoa_deg, double dtau, double tau0,
                const double *rho, const double *u, const double *pp, const double *gbar, int64_t nt_stride,
                double *g_rho, double *g_u, double *g_p)
{
    orc_case cs = {P, O, N, y, normal, dS, x_obs, mach, aoa_deg, dtau, tau0};
    return adjoint_core(&cs, 0, rho, u, pp, gbar, nt_stride, NULL, 0, g_rho, g_u, g_p);
}

int orc_adjoint_panels(int64_t P, int64_t O, int64_t N, const double *y, const double *normal, const double *dS,
                       const double *x_obs, double mach, double aoa_deg, double dtau, double tau0,
                       const int64_t *pidx, int64_t np, const double *rho, const double *u, const double *pp,
                       const double *gbar, int64_t nt_stride, double *g_rho, double *g_u, double *g_p)
{
    if (!pidx || np < 1) return -3;
    orc_case cs = {P, O, N, y, normal, dS, x_obs, mach, aoa_deg, dtau, tau0};
    return adjoint_core(&cs, 0, rho, u, pp, gbar, nt_stride, pidx, np, g_rho, g_u, g_p);
}

int orc_adjoint_sources(int64_t P, int64_t O, int64_t N, const double *y, const double *normal, const double *dS,
                        const double *x_obs, double mach, double aoa_deg, double dtau, double tau0,
                        const double *gbar, int64_t nt_stride, double *Qbar, double *Lbar)
{
    orc_case cs = {P, O, N, y, normal, dS, x_obs, mach, aoa_deg, dtau, tau0};
    return adjoint_core(&cs, 1, NULL, NULL, NULL, gbar, nt_stride, NULL, 0, Qbar, Lbar, NULL);
}

/* ============================================ general motion (Sec. II B) */

/* The surface moves with prescribed kinematics sampled at the source frames
 * (panel positions y, unit normals n, velocities v); the medium and the observers
 * are at rest.  Nondimensional as in Sec. II D with the reference speed of the
 * mach argument: rho0 = 1, c0 = 1/M0, M_i = v_i / c0 = M0 v_i.
 *
 * Per panel and frame, Eqs. (Qn), (Li) with P_ij = p' delta_ij (Eq. (Pij)):
 *   Q_i = v_i + rho (u_i - v_i),   Q_n = Q_i n_i,
 *   L_i = p' n_i + rho u_i (u_j - v_j) n_j,   L_M = L_i M_i (Eq. (LM)),   M^2 = M_i M_i.
 * Source-time derivatives of Q_i, n_i, L_i, M_i by orc_fd (second order, one-sided
 * at the first and last frame).  The observer-independent quantities of the
 * integrand form 19 channels, each interpolated in source time by its own natural
 * cubic spline (orc_spline_m / orc_spline_eval):
 *   A = Qd_i n_i + Q_i nd_i,  Q_n,  L_1..3,  Ld_1..3,  L_M,  M_1..3,  Md_1..3,  M^2,  y_1..3.
 * Retarded time, Eq. (tau): tau + M0 |x - Y(tau)| = t with Y the splined
 * trajectory; the left side increases with tau for subsonic motion, so the root
 * is bracketed by [tau_0, tau_{N-1}] for every t in the observer window and found
 * by bisection.  At tau_ret: r = x - Y, rhat = r/|r|, M_r = M_i rhat_i,
 * Md_r = Md_i rhat_i, L_r = L_i rhat_i, Ld_r = Ld_i rhat_i (Eqs. (Mr), (Lr)), and the
 * integrand of Eqs. (pT) + (pL) times dS / (4 pi):
 *   A/(r (1-M_r)^2) + Q_n (r Md_r + c0 (M_r - M^2)) / (r^2 (1-M_r)^3)
 *   + Ld_r / (c0 r (1-M_r)^2) + (L_r - L_M) / (r^2 (1-M_r)^2)
 *   + L_r (r Md_r + c0 (M_r - M^2)) / (c0 r^2 (1-M_r)^3).
 * Observer window (the general form of Eqs. (t_start), (t_end)):
 *   t_start = max_p [tau_0 + M0 |x - y_p(tau_0)|],  t_end = min_p [tau_{N-1} + M0 |x - y_p(tau_{N-1})|],
 *   t_k = t_start + k dtau, N_t = floor((t_end - t_start)/dtau + 1e-9) + 1.
 *
 * Layouts (panel-major, contiguous series): y, n, v [3][P][N]; rho, p' [P][N];
 * u [3][P][N]. */
enum {
    GM_A, GM_QN, GM_L1, GM_L2, GM_L3, GM_LD1, GM_LD2, GM_LD3, GM_LM, GM_M1, GM_M2, GM_M3,
    GM_MD1, GM_MD2, GM_MD3, GM_MSQ, GM_Y1, GM_Y2, GM_Y3, GM_NCH
};

typedef struct {
    int64_t P, O, N;
    const double *y, *nrm, *vel, *dS, *x_obs;
    double mach, dtau, tau0;
} orc_gm_case;

/* Channels of panel p: ch[GM_NCH][N].  work: 9 N doubles. */
static void gm_channels_panel(const orc_gm_case *cs, const double *rho, const double *u, const double *pp,
                              int64_t p, double *ch, double *work)
{
    const int64_t N = cs->N, P = cs->P;
    const double M0 = cs->mach, h = cs->dtau;
    double *Q = work, *Qd = work + 3 * N, *nd = work + 6 * N;
    for (int64_t n = 0; n < N; ++n) {
        double v[3], nn[3], uu[3];
        for (int i = 0; i < 3; ++i) {
            v[i] = cs->vel[(i * P + p) * N + n];
            nn[i] = cs->nrm[(i * P + p) * N + n];
            uu[i] = u[(i * P + p) * N + n];
        }
        const double r = rho[p * N + n], pr = pp[p * N + n];
        const double urel_n = (uu[0] - v[0]) * nn[0] + (uu[1] - v[1]) * nn[1] + (uu[2] - v[2]) * nn[2];
        double qn = 0.0, lm = 0.0, msq = 0.0;
        for (int i = 0; i < 3; ++i) {
            Q[i * N + n] = v[i] + r * (uu[i] - v[i]);
            qn += Q[i * N + n] * nn[i];
            const double Li = pr * nn[i] + r * uu[i] * urel_n;
            const double Mi = M0 * v[i];
            ch[(GM_L1 + i) * N + n] = Li;
            ch[(GM_M1 + i) * N + n] = Mi;
            ch[(GM_Y1 + i) * N + n] = cs->y[(i * P + p) * N + n];
            lm += Li * Mi;
            msq += Mi * Mi;
        }
        ch[GM_QN * N + n] = qn;
        ch[GM_LM * N + n] = lm;
        ch[GM_MSQ * N + n] = msq;
    }
    for (int i = 0; i < 3; ++i) {
        orc_fd(N, Q + i * N, h, Qd + i * N);
        orc_fd(N, cs->nrm + (i * P + p) * N, h, nd + i * N);
        orc_fd(N, ch + (GM_L1 + i) * N, h, ch + (GM_LD1 + i) * N);
        orc_fd(N, ch + (GM_M1 + i) * N, h, ch + (GM_MD1 + i) * N);
    }
    for (int64_t n = 0; n < N; ++n) {
        double a = 0.0;
        for (int i = 0; i < 3; ++i)
            a += Qd[i * N + n] * cs->nrm[(i * P + p) * N + n] + Q[i * N + n] * nd[i * N + n];
        ch[GM_A * N + n] = a;
    }
}

static double gm_dist(const double *x, const double *y3) /* |x - y| */
{
    const double d0 = x[0] - y3[0], d1 = x[1] - y3[1], d2 = x[2] - y3[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

/* Retarded time of observer time t for one panel (channels ch, spline moments m). */
static double gm_retarded(const orc_gm_case *cs, const double *ch, const double *m, const double *x, double t)
{
    const int64_t N = cs->N;
    const double h = cs->dtau, tau0 = cs->tau0, M0 = cs->mach;
    double lo = tau0, hi = tau0 + (double)(N - 1) * h;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double Y[3];
        for (int i = 0; i < 3; ++i)
            Y[i] = orc_spline_eval(N, ch + (GM_Y1 + i) * N, m + (GM_Y1 + i) * N, tau0, h, mid);
        const double g = mid + M0 * gm_dist(x, Y) - t;
        if (g < 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Integrand of one pair at observer time t (dS / (4 pi) included). */
static double gm_integrand(const orc_gm_case *cs, const double *ch, const double *m, const double *x, double dS,
                           double t)
{
    const int64_t N = cs->N;
    const double h = cs->dtau, tau0 = cs->tau0, c0 = 1.0 / cs->mach;
    const double tau = gm_retarded(cs, ch, m, x, t);
    double q[GM_NCH];
    for (int c = 0; c < GM_NCH; ++c) q[c] = orc_spline_eval(N, ch + c * N, m + c * N, tau0, h, tau);
    double rv[3] = {x[0] - q[GM_Y1], x[1] - q[GM_Y2], x[2] - q[GM_Y3]};
    const double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    double Mr = 0.0, Mdr = 0.0, Lr = 0.0, Ldr = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double rh = rv[i] / r;
        Mr += q[GM_M1 + i] * rh;
        Mdr += q[GM_MD1 + i] * rh;
        Lr += q[GM_L1 + i] * rh;
        Ldr += q[GM_LD1 + i] * rh;
    }
    const double om = 1.0 - Mr;
    const double conv = r * Mdr + c0 * (Mr - q[GM_MSQ]);
    const double pT = q[GM_A] / (r * om * om) + q[GM_QN] * conv / (r * r * om * om * om);
    const double pL = Ldr / (c0 * r * om * om) + (Lr - q[GM_LM]) / (r * r * om * om)
                      + Lr * conv / (c0 * r * r * om * om * om);
    return (pT + pL) * dS / (4.0 * ORC_PI);
}

int orc_gm_window(int64_t P, int64_t O, int64_t N, const double *y, const double *x_obs, double mach, double dtau,
                  double tau0, double *t_start, int64_t *n_t)
{
    int st = 0;
    for (int64_t o = 0; o < O; ++o) {
        const double *x = x_obs + 3 * o;
        double ts = -INFINITY, te = INFINITY;
        for (int64_t p = 0; p < P; ++p) {
            double y0[3], y1[3];
            for (int i = 0; i < 3; ++i) {
                y0[i] = y[(i * P + p) * N];
                y1[i] = y[(i * P + p) * N + N - 1];
            }
            const double a0 = tau0 + mach * gm_dist(x, y0);
            const double a1 = tau0 + (double)(N - 1) * dtau + mach * gm_dist(x, y1);
            if (a0 > ts) ts = a0;
            if (a1 < te) te = a1;
        }
        t_start[o] = ts;
        if (te < ts) {
            n_t[o] = 0;
            st = -1;
        } else {
            n_t[o] = (int64_t)floor((te - ts) / dtau + 1e-9) + 1;
        }
    }
    return st;
}

/* p'(o, k) for the requested (observer, sample) pairs, or, with s_k == NULL, every
 * sample k < N_t of observers s_obs[0..n_s-1] into out[n_s][nt_stride] (zero
 * padded).  Returns 0, -1 (empty window), -2 (stride too small), -3 (bad sizes). */
static int gm_core(const orc_gm_case *cs, const double *rho, const double *u, const double *pp, const int64_t *s_obs,
                   const int64_t *s_k, int64_t n_s, double *out, int64_t nt_stride)
{
    const int64_t P = cs->P, N = cs->N, O = cs->O;
    if (P < 1 || O < 1 || N < 4 || !(cs->mach > 0.0 && cs->mach < 1.0) || !(cs->dtau > 0.0)) return -3;
    double *t_start = xmalloc((size_t)O);
    int64_t *n_t = (int64_t *)malloc((size_t)O * sizeof(int64_t));
    if (orc_gm_window(P, O, N, cs->y, cs->x_obs, cs->mach, cs->dtau, cs->tau0, t_start, n_t) != 0) {
        free(t_start); free(n_t); return -1;
    }
    int64_t n_out;
    if (s_k == NULL) {
        for (int64_t s = 0; s < n_s; ++s)
            if (n_t[s_obs[s]] > nt_stride) { free(t_start); free(n_t); return -2; }
        n_out = n_s * nt_stride;
    } else {
        n_out = n_s;
    }
    const int64_t nblk = (P + ORC_BLOCK - 1) / ORC_BLOCK;
    double *part = (double *)calloc((size_t)nblk * (size_t)n_out, sizeof(double));
#pragma omp parallel
    {
        double *ch = xmalloc((size_t)2 * GM_NCH * N + 10 * (size_t)N);
        double *m = ch + GM_NCH * N, *work = ch + 2 * GM_NCH * N;
#pragma omp for schedule(dynamic, 1)
        for (int64_t b = 0; b < nblk; ++b) {
            const int64_t p_end = (b + 1) * ORC_BLOCK < P ? (b + 1) * ORC_BLOCK : P;
            double *acc = part + b * n_out;
            for (int64_t p = b * ORC_BLOCK; p < p_end; ++p) {
                gm_channels_panel(cs, rho, u, pp, p, ch, work);
                for (int c = 0; c < GM_NCH; ++c) orc_spline_m(N, ch + c * N, cs->dtau, m + c * N, work);
                for (int64_t s = 0; s < n_s; ++s) {
                    const int64_t o = s_obs[s];
                    const double *x = cs->x_obs + 3 * o;
                    if (s_k == NULL) {
                        for (int64_t k = 0; k < n_t[o]; ++k)
                            acc[s * nt_stride + k] +=
                                gm_integrand(cs, ch, m, x, cs->dS[p], t_start[o] + (double)k * cs->dtau);
                    } else {
                        acc[s] += gm_integrand(cs, ch, m, x, cs->dS[p], t_start[o] + (double)s_k[s] * cs->dtau);
                    }
                }
            }
        }
        free(ch);
    }
    memset(out, 0, sizeof(double) * (size_t)n_out);
    for (int64_t b = 0; b < nblk; ++b)                     /* surface sum, fixed order */
        for (int64_t i = 0; i < n_out; ++i) out[i] += part[b * n_out + i];
    free(part);
    free(t_start);
    free(n_t);
    return 0;
}

int orc_gm_forward(int64_t P, int64_t O, int64_t N, const double *y, const double *nrm, const double *vel,
                   const double *dS, const double *x_obs, double mach, double dtau, double tau0, const double *rho,
                   const double *u, const double *pp, const int64_t *obs_idx, int64_t n_sel, double *out,
                   int64_t nt_stride)
{
    orc_gm_case cs = {P, O, N, y, nrm, vel, dS, x_obs, mach, dtau, tau0};
    return gm_core(&cs, rho, u, pp, obs_idx, NULL, n_sel, out, nt_stride);
}

int orc_gm_forward_samples(int64_t P, int64_t O, int64_t N, const double *y, const double *nrm, const double *vel,
                           const double *dS, const double *x_obs, double mach, double dtau, double tau0,
                           const double *rho, const double *u, const double *pp, const int64_t *s_obs,
                           const int64_t *s_k, int64_t n_s, double *out)
{
    orc_gm_case cs = {P, O, N, y, nrm, vel, dS, x_obs, mach, dtau, tau0};
    return gm_core(&cs, rho, u, pp, s_obs, s_k, n_s, out, 0);
}

/* Channels of every panel, [GM_NCH][P][N] (exposed for the tests). */
void orc_gm_channels(int64_t P, int64_t N, const double *y, const double *nrm, const double *vel, double mach,
                     double dtau, const double *rho, const double *u, const double *pp, double *out)
{
    orc_gm_case cs = {P, 1, N, y, nrm, vel, NULL, NULL, mach, dtau, 0.0};
#pragma omp parallel
    {
        double *ch = xmalloc((size_t)GM_NCH * N + 9 * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < P; ++p) {
            gm_channels_panel(&cs, rho, u, pp, p, ch, ch + GM_NCH * N);
            for (int c = 0; c < GM_NCH; ++c) memcpy(out + ((int64_t)c * P + p) * N, ch + c * N, sizeof(double) * N);
        }
        free(ch);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the following calls (results do not depend on it). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
