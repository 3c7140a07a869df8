// General-motion form (Sec. II B): a permeable surface in prescribed motion,
// medium and observers at rest, Eqs. (pT), (pL) at the retarded time of
// Eq. (tau).  FP64 throughout.  Nondimensional (Sec. II D) with rho0 = 1,
// c0 = 1/M0 and M_i = M0 v_i.
//
// Stages:
//  1. gm_channels_kernel, one thread per (frame n, panel p): Q_i, n_i, L_i, M_i
//     of Eqs. (Qn), (Li) (P_ij = p' delta_ij) at the frames of the second-order
//     source-time difference of frame n (central; one-sided three-point at the
//     first and last frame), recomputed from the inputs, giving the 19
//     observer-independent channels, channel-major per panel: coef[p][c][n + 1]
//     for c = [A, Q_n, L_1..3, Ld_1..3, L_M, M_1..3, Md_1..3, M^2, y_1..3] with
//     A = Qd_i n_i + Q_i nd_i.  A block computes 16 panels x 16 frames and writes
//     through an LDS transpose, so that both the time-major reads and the
//     time-contiguous writes are coalesced.
//  2. gm_prefilter_kernel, one thread per (panel, channel) row: the natural cubic
//     spline of each channel in source time as uniform cubic B-spline
//     coefficients c_{-1..N} (storage index n + 1), in place: c_0 = f_0,
//     c_{N-1} = f_{N-1}, c_{n-1} + 4 c_n + c_{n+1} = 6 f_n, c_{-1} = 2 c_0 - c_1,
//     c_N = 2 c_{N-1} - c_{N-2}; Thomas sweeps with the pivot table inv_beta.
//  3. gm_window_kernel, one block per observer: t_start = max_p [tau_0 +
//     M0 |x - y_p(tau_0)|], t_end = min_p [tau_{N-1} + M0 |x - y_p(tau_{N-1})|],
//     N_t = floor((t_end - t_start)/dtau + 1e-9) + 1 (-1 for an empty window).
//  4. gm_gather_kernel: a wave owns (observer, 64 consecutive samples, panel
//     range), a block four neighbouring observers at the same samples; per
//     panel each lane solves tau + M0 |x - Y(tau)| = t_k by Newton steps on the
//     splined trajectory (started from the linear extrapolation of its
//     solutions for the two previous panels; a step below 1e-6 dtau is accepted
//     without a further check, the iteration being quadratic, and the position
//     at tau_ret is the last evaluation advanced by that step; the next panel's
//     first taps are fetched after this panel's channel taps), evaluates the 16
//     integrand channels at tau_ret with the four B-spline taps, read from rows
//     the block copies once into LDS over its joint tap span (each lane loads
//     its own taps when the span is too wide), and adds the integrand of
//     Eqs. (pT) + (pL) times dS/(4 pi) in FP64.  Panel ranges (splits) are
//     summed by gm_reduce_kernel in fixed order.
#include <climits>

#include "fwh_internal.h"

namespace fwh {
namespace {

constexpr int kGmNewtonMax = 40;
constexpr double kPiD = 3.14159265358979323846;
// channel rows of coef[p][kGmRows][NS]
enum { GA, GQN, GL1, GL2, GL3, GLD1, GLD2, GLD3, GLM, GM1, GM2, GM3, GMD1, GMD2, GMD3, GMSQ, GY1, GY2, GY3 };

struct GmFrame {
    double Q[3], n[3], L[3], M[3], y[3];
};

// Frame quantities of panel p at frame m (time-major inputs).
__device__ __forceinline__ GmFrame gm_frame(const GmChanArgs &a, int64_t m, int64_t p) {
    const int64_t P = a.P, NP = a.N * a.P;
    const int64_t i1 = m * P + p, i3 = 3 * i1;
    GmFrame f;
    double v[3], u[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        f.y[i] = a.y[i3 + i];
        f.n[i] = a.normal[i3 + i];
        v[i] = a.vel[i3 + i];
        u[i] = a.u[i * NP + i1];
    }
    const double rho = a.rho[i1], pp = a.pp[i1];
    const double urel_n = (u[0] - v[0]) * f.n[0] + (u[1] - v[1]) * f.n[1] + (u[2] - v[2]) * f.n[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        f.Q[i] = v[i] + rho * (u[i] - v[i]);
        f.L[i] = pp * f.n[i] + rho * u[i] * urel_n;
        f.M[i] = a.mach * v[i];
    }
    return f;
}

constexpr int kGmTP = 16;  // panels per channel block
constexpr int kGmTF = 16;  // frames per channel block

// Block (bx, by): panels bx*16 .. +15 (thread & 15), frames by*16 .. +15 (thread >> 4).
__global__ __launch_bounds__(256) void gm_channels_kernel(GmChanArgs a) {
    __shared__ double tile[kGmRows][kGmTP][kGmTF + 1];
    const int64_t P = a.P, N = a.N;
    const int pl = threadIdx.x & 15, fl = threadIdx.x >> 4;
    const int64_t p = (int64_t)blockIdx.x * kGmTP + pl, n = (int64_t)blockIdx.y * kGmTF + fl;
    if (p < P && n < N) {
        // stencil frames and weights of the second-order difference at frame n
        int64_t f0, f1, f2;
        double w0, w1, w2;
        if (n == 0) {
            f0 = 0; f1 = 1; f2 = 2; w0 = -3.0; w1 = 4.0; w2 = -1.0;
        } else if (n == N - 1) {
            f0 = N - 3; f1 = N - 2; f2 = N - 1; w0 = 1.0; w1 = -4.0; w2 = 3.0;
        } else {
            f0 = n - 1; f1 = n; f2 = n + 1; w0 = -1.0; w1 = 0.0; w2 = 1.0;
        }
        const GmFrame F0 = gm_frame(a, f0, p), F1 = gm_frame(a, f1, p), F2 = gm_frame(a, f2, p);
        const GmFrame &C = n == 0 ? F0 : (n == N - 1 ? F2 : F1);  // the frame itself
        const double i2h = 1.0 / (2.0 * a.dtau);
        double Qd[3], nd[3];
        double A = 0.0, Qn = 0.0, LM = 0.0, Msq = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Qd[i] = (w0 * F0.Q[i] + w1 * F1.Q[i] + w2 * F2.Q[i]) * i2h;
            nd[i] = (w0 * F0.n[i] + w1 * F1.n[i] + w2 * F2.n[i]) * i2h;
            tile[GLD1 + i][pl][fl] = (w0 * F0.L[i] + w1 * F1.L[i] + w2 * F2.L[i]) * i2h;
            tile[GMD1 + i][pl][fl] = (w0 * F0.M[i] + w1 * F1.M[i] + w2 * F2.M[i]) * i2h;
            tile[GL1 + i][pl][fl] = C.L[i];
            tile[GM1 + i][pl][fl] = C.M[i];
            tile[GY1 + i][pl][fl] = C.y[i];
            A += Qd[i] * C.n[i] + C.Q[i] * nd[i];
            Qn += C.Q[i] * C.n[i];
            LM += C.L[i] * C.M[i];
            Msq += C.M[i] * C.M[i];
        }
        tile[GA][pl][fl] = A;
        tile[GQN][pl][fl] = Qn;
        tile[GLM][pl][fl] = LM;
        tile[GMSQ][pl][fl] = Msq;
    }
    __syncthreads();
    // write out with frames fastest: thread -> (panel t >> 4, frame t & 15)
    const int wp = threadIdx.x >> 4, wf = threadIdx.x & 15;
    const int64_t p2 = (int64_t)blockIdx.x * kGmTP + wp, n2 = (int64_t)blockIdx.y * kGmTF + wf;
    if (p2 < P && n2 < N) {
        double *dst = a.coef + p2 * kGmRows * a.NS + n2 + 1;
#pragma unroll
        for (int c = 0; c < kGmRows; ++c) dst[(int64_t)c * a.NS] = tile[c][wp][wf];
    }
}

// Natural cubic spline -> B-spline coefficients, in place, for each row
// coef[row * NS + s] (s = n + 1 holds f_n on entry, c_{s-1} on exit).  A block
// owns 256 rows (one per thread) and moves through time in chunks of 16
// positions staged in an LDS tile [256][17]: chunk loads and stores are
// coalesced (16 lanes per 128-byte row segment), the per-row recurrences read
// the tile conflict-free.
constexpr int kPfRows = 256;
constexpr int kPfT = 16;

__global__ __launch_bounds__(256) void gm_prefilter_kernel(double *coef, int64_t rows, int64_t N, int64_t NS,
                                                         const double *__restrict__ inv_beta) {
    __shared__ double tile[kPfRows][kPfT + 1];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kPfRows;
    const int64_t row = r0 + tid;
    const bool valid = row < rows;
    const double *fr = coef + (valid ? row : r0) * NS;
    const double f0 = fr[1], fN1 = fr[N];
    // chunk moves: all 16 loads of a thread are issued before the LDS stores
    auto move = [&](int64_t c0, int len, bool to_lds) {
        const int ss = tid & 15;
        if (to_lds) {
            double v[kPfRows / 16];
#pragma unroll
            for (int i = 0; i < kPfRows / 16; ++i) {
                const int64_t g = r0 + i * 16 + (tid >> 4);
                v[i] = (g < rows && ss < len) ? coef[g * NS + c0 + ss] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < kPfRows / 16; ++i) tile[i * 16 + (tid >> 4)][ss] = v[i];
        } else {
#pragma unroll
            for (int i = 0; i < kPfRows / 16; ++i) {
                const int rr = i * 16 + (tid >> 4);
                const int64_t g = r0 + rr;
                if (g < rows && ss < len) coef[g * NS + c0 + ss] = tile[rr][ss];
            }
        }
    };
    // forward sweep over rows n = 1 .. N-2 (storage n + 1 = 2 .. N-1): d_n = (rhs_n - d_{n-1}) / beta_n
    double d = 0.0;
    for (int64_t c0 = 2; c0 <= N - 1; c0 += kPfT) {
        const int len = (int)min<int64_t>(kPfT, N - c0);
        __syncthreads();
        move(c0, len, true);
        __syncthreads();
        if (valid) {
            for (int ss = 0; ss < len; ++ss) {
                const int64_t n = c0 + ss - 1;
                double rhs = 6.0 * tile[tid][ss];
                if (n == 1) rhs -= f0;
                if (n == N - 2) rhs -= fN1;
                const double ib = inv_beta[n < kGmPivots ? n : kGmPivots - 1];
                d = (rhs - (n > 1 ? d : 0.0)) * ib;
                tile[tid][ss] = d;
            }
        }
        __syncthreads();
        move(c0, len, false);
    }
    // back substitution from storage N - 1 down to 2: c_{N-2} = d_{N-2}, c_n = d_n - c_{n+1} / beta_n
    const int64_t nchunk = (N - 2 + kPfT - 1) / kPfT;
    double c_next = 0.0, c_top = 0.0;
    for (int64_t ci = nchunk - 1; ci >= 0; --ci) {
        const int64_t c0 = 2 + ci * kPfT;
        const int len = (int)min<int64_t>(kPfT, N - c0);
        __syncthreads();
        move(c0, len, true);
        __syncthreads();
        if (valid) {
            for (int ss = len - 1; ss >= 0; --ss) {
                const int64_t n = c0 + ss - 1;
                const double ib = inv_beta[n < kGmPivots ? n : kGmPivots - 1];
                const double dn = tile[tid][ss];
                const double cc = n == N - 2 ? dn : dn - c_next * ib;
                if (n == N - 2) c_top = cc;
                tile[tid][ss] = cc;
                c_next = cc;
            }
        }
        __syncthreads();
        move(c0, len, false);
    }
    // end coefficients (c_0 = f_0 and c_{N-1} = f_{N-1} are already in place); c_next = c_1
    if (valid) {
        double *f = coef + row * NS;
        f[0] = 2.0 * f0 - c_next;
        f[N + 1] = 2.0 * fN1 - c_top;
    }
}

__global__ __launch_bounds__(256) void gm_window_kernel(GmWinArgs a) {
    const int64_t o = blockIdx.x;
    const double x0 = a.x_obs[3 * o], x1 = a.x_obs[3 * o + 1], x2 = a.x_obs[3 * o + 2];
    const int64_t P = a.P, N = a.N;
    const double tlast = a.tau0 + (double)(N - 1) * a.dtau;
    double ts = -INFINITY, te = INFINITY;
    for (int64_t p = threadIdx.x; p < P; p += 256) {
        const double *y0 = a.y + 3 * p, *y1 = a.y + 3 * ((N - 1) * P + p);
        const double d00 = x0 - y0[0], d01 = x1 - y0[1], d02 = x2 - y0[2];
        const double d10 = x0 - y1[0], d11 = x1 - y1[1], d12 = x2 - y1[2];
        const double a0 = a.tau0 + a.mach * sqrt(d00 * d00 + d01 * d01 + d02 * d02);
        const double a1 = tlast + a.mach * sqrt(d10 * d10 + d11 * d11 + d12 * d12);
        ts = fmax(ts, a0);
        te = fmin(te, a1);
    }
    __shared__ double smax[256], smin[256];
    smax[threadIdx.x] = ts;
    smin[threadIdx.x] = te;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double t0 = smax[0], t1 = smin[0];
        a.t_start[o] = t0;
        a.n_t[o] = t1 < t0 ? -1 : (int32_t)(floor((t1 - t0) / a.dtau + 1e-9) + 1.0);
    }
}

// Uniform cubic B-spline weights of frac u for c_{j-1..j+2} and their derivatives.
__device__ __forceinline__ void bspline_w(double u, double w[4], double dw[4]) {
    const double v = 1.0 - u, u2 = u * u;
    w[0] = v * v * v * (1.0 / 6.0);
    w[1] = (3.0 * u2 * u - 6.0 * u2 + 4.0) * (1.0 / 6.0);
    w[2] = (-3.0 * u2 * u + 3.0 * u2 + 3.0 * u + 1.0) * (1.0 / 6.0);
    w[3] = u2 * u * (1.0 / 6.0);
    dw[0] = -0.5 * v * v;
    dw[1] = 1.5 * u2 - 2.0 * u;
    dw[2] = -1.5 * u2 + u + 0.5;
    dw[3] = 0.5 * u2;
}

// Interval j in [0, N-2] and frac u in [0, 1] of source time tau.
__device__ __forceinline__ int64_t gm_locate(double tau, double tau0, double dtau, int64_t N, double &u) {
    const double xs = (tau - tau0) / dtau;
    double jf = floor(xs);
    jf = fmin(fmax(jf, 0.0), (double)(N - 2));
    u = fmin(fmax(xs - jf, 0.0), 1.0);
    return (int64_t)jf;
}

typedef double gm_d2 __attribute__((ext_vector_type(2), aligned(8)));

// Value of a channel row at the taps of interval j (weights w): two 16-byte loads.
__device__ __forceinline__ double gm_tap(const double *row, int64_t j, const double w[4]) {
    const gm_d2 lo = *reinterpret_cast<const gm_d2 *>(row + j);
    const gm_d2 hi = *reinterpret_cast<const gm_d2 *>(row + j + 2);
    return w[0] * lo.x + w[1] * lo.y + w[2] * hi.x + w[3] * hi.y;
}

// The six 16-byte loads of the trajectory taps of interval j (rows y_1..3).
struct GmTraj {
    gm_d2 a0, b0, a1, b1, a2, b2;
    __device__ __forceinline__ void load(const double *ry0, const double *ry1, const double *ry2, int64_t j) {
        a0 = *reinterpret_cast<const gm_d2 *>(ry0 + j);
        b0 = *reinterpret_cast<const gm_d2 *>(ry0 + j + 2);
        a1 = *reinterpret_cast<const gm_d2 *>(ry1 + j);
        b1 = *reinterpret_cast<const gm_d2 *>(ry1 + j + 2);
        a2 = *reinterpret_cast<const gm_d2 *>(ry2 + j);
        b2 = *reinterpret_cast<const gm_d2 *>(ry2 + j + 2);
    }
};

// Rows GA .. GMSQ (the 16 channels of the integrand) are staged per block in LDS
// over the block's tap span: kGmSpanB positions per row, two buffers.
constexpr int kGmStaged = GMSQ + 1;
constexpr int kGmSpanB = 152;  // two buffers of 16 rows: 38 KB, four blocks per compute unit
typedef __attribute__((address_space(3))) void *gm_lds_ptr_t;

// Block = 4 waves = observers 4 og .. 4 og + 3 (wave wv: observer 4 og + wv), the same 64 samples
// k0 .. k0 + 63 and panel range; logical blocks run with the observer group fastest, regrouped per XCD.
__global__ __launch_bounds__(256) void gm_gather_kernel(GmGatherArgs a) {
    __shared__ double stage[2][kGmStaged][kGmSpanB];
    __shared__ int span_lo[4], span_hi[4];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nkb = a.nkb, O = a.O;
    const int64_t ngrp = (O + 3) / 4;
    const int64_t L = xcd_block(blockIdx.x, gridDim.x);
    const int64_t og = L % ngrp, rest = L / ngrp;
    const int64_t kb = rest % nkb, z = rest / nkb;
    // a wave past the last observer runs along (it meets every barrier) on observer O - 1 with
    // every lane outside the window, and writes nothing
    const bool obs_ok = og * 4 + wv < O;
    const int64_t o = obs_ok ? og * 4 + wv : O - 1;
    const int64_t k = kb * 64 + lane;
    const int64_t nt = obs_ok ? a.n_t[o] : 0;
    const bool active = k < nt;
    const bool wave_active = nt > kb * 64;
    // last lane of the wave inside the window
    const int last_active = __builtin_amdgcn_readfirstlane((int)max((int64_t)0, min((int64_t)63, nt - 1 - kb * 64)));
    const double x0 = a.x_obs[3 * o], x1 = a.x_obs[3 * o + 1], x2 = a.x_obs[3 * o + 2];
    const double t = a.t_start[o] + (double)k * a.dtau;
    const int64_t N = a.N, NS = a.NS;
    const double M0 = a.mach, c0 = 1.0 / M0, tau0 = a.tau0, dtau = a.dtau;
    const double tmax = tau0 + (double)(N - 1) * dtau;
    const double accept = 1e-6 * dtau;
    const int64_t pb = z * a.p_chunk;
    const int64_t pe = min(pb + a.p_chunk, a.P);
    double acc = 0.0;
    if (pb >= pe) {  // block-uniform
        if (obs_ok && k < a.nt_stride) a.part[(z * O + o) * a.nt_stride + k] = 0.0;
        return;
    }
    // first panel of the range: start from the emission time of frame 0's position
    double tau;
    {
        const double *cf = a.coef + pb * kGmRows * NS;
        const double d0 = x0 - cf[GY1 * NS + 1], d1 = x1 - cf[GY2 * NS + 1], d2 = x2 - cf[GY3 * NS + 1];
        tau = fmin(fmax(t - M0 * sqrt(d0 * d0 + d1 * d1 + d2 * d2), tau0), tmax);
    }
    // taps of the current panel at the current guess (loaded ahead: for the next panel they are
    // fetched after this panel's channel taps); the guess for the next panel extrapolates
    // the retarded times of the last two panels (neighbouring panels are visited in order)
    double tau_prev = 0.0;
    GmTraj tr;
    {
        double u;
        const int64_t j = gm_locate(tau, tau0, dtau, N, u);
        const double *cf = a.coef + pb * kGmRows * NS;
        tr.load(cf + GY1 * NS, cf + GY2 * NS, cf + GY3 * NS, j);
    }
    int buf = 0;
    for (int64_t p = pb; p < pe; ++p, buf ^= 1) {
        const double *cf = a.coef + p * kGmRows * NS;
        const double *ry0 = cf + GY1 * NS, *ry1 = cf + GY2 * NS, *ry2 = cf + GY3 * NS;
        // Newton on g(tau) = tau + M0 |x - Y(tau)| - t, g' = 1 - M0 rhat . Y'(tau); the first step
        // uses the preloaded taps.  Y and dY/dtau of the last evaluation are kept.
        double Y0, Y1, Y2, V0, V1, V2, taue;
        for (int it = 0; it < kGmNewtonMax; ++it) {
            double u;
            const int64_t j = gm_locate(tau, tau0, dtau, N, u);
            double w[4], dw[4];
            bspline_w(u, w, dw);
            if (it > 0) tr.load(ry0, ry1, ry2, j);
            Y0 = w[0] * tr.a0.x + w[1] * tr.a0.y + w[2] * tr.b0.x + w[3] * tr.b0.y;
            Y1 = w[0] * tr.a1.x + w[1] * tr.a1.y + w[2] * tr.b1.x + w[3] * tr.b1.y;
            Y2 = w[0] * tr.a2.x + w[1] * tr.a2.y + w[2] * tr.b2.x + w[3] * tr.b2.y;
            const double idt = 1.0 / dtau;
            V0 = (dw[0] * tr.a0.x + dw[1] * tr.a0.y + dw[2] * tr.b0.x + dw[3] * tr.b0.y) * idt;
            V1 = (dw[0] * tr.a1.x + dw[1] * tr.a1.y + dw[2] * tr.b1.x + dw[3] * tr.b1.y) * idt;
            V2 = (dw[0] * tr.a2.x + dw[1] * tr.a2.y + dw[2] * tr.b2.x + dw[3] * tr.b2.y) * idt;
            taue = tau;
            const double r0 = x0 - Y0, r1 = x1 - Y1, r2 = x2 - Y2;
            const double r = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
            const double g = tau + M0 * r - t;
            const double gd = 1.0 - M0 * (r0 * V0 + r1 * V1 + r2 * V2) / r;
            double step = active ? g / gd : 0.0;
            const double tn = fmin(fmax(tau - step, tau0), tmax);
            step = tau - tn;
            tau = tn;
            // quadratic convergence: after a step below 1e-6 dtau the error is far below rounding
            const bool done = !(fabs(step) > accept);
            if (__all(done)) break;
        }
        // position at tau_ret from the last evaluation by its first-order step (the step is below
        // 1e-6 dtau, the remainder O(step^2 |Y''|) is below rounding)
        const double dt_last = tau - taue;
        const double r0 = x0 - (Y0 + V0 * dt_last), r1 = x1 - (Y1 + V1 * dt_last), r2 = x2 - (Y2 + V2 * dt_last);
        double u;
        const int64_t j = gm_locate(tau, tau0, dtau, N, u);
        double w[4], dw[4];
        bspline_w(u, w, dw);
        // The active lanes' intervals do not decrease with the sample (subsonic motion), so a wave's
        // taps of one row span j(lane 0) .. j(last active lane) + 3, and the block's observers, a few
        // degrees apart, have overlapping spans.  When the block's span fits kGmSpanB positions, each
        // of the 16 integrand rows is copied once for the block into LDS by direct global -> LDS loads
        // (16 bytes, two positions, per lane; wave wv copies rows wv, wv + 4, ...) instead of every lane
        // loading its own four taps.  (A copy may read one position past the row end: the next row,
        // a trajectory row for the last one.)  The copies of the next panel go to the other buffer:
        // every wave has read this one before it reaches the next panel's first barrier.
        if (lane == 0) {
            span_lo[wv] = wave_active ? (int)j : INT_MAX;
            span_hi[wv] = wave_active ? __builtin_amdgcn_readlane((int)j, last_active) : INT_MIN;
        }
        __syncthreads();
        int lo = min(min(span_lo[0], span_lo[1]), min(span_lo[2], span_lo[3]));
        int hi = max(max(span_hi[0], span_hi[1]), max(span_hi[2], span_hi[3]));
        if (lo > hi) lo = hi = 0;  // no lane of the block is inside its window
        const int span = hi - lo + 4;
        double cv[kGmStaged];
        if (span <= kGmSpanB) {  // block-uniform
#pragma unroll
            for (int rr = 0; rr < kGmStaged / 4; ++rr) {
                const int c = wv + 4 * rr;
                const double *row = cf + c * NS + lo;
                if (2 * lane < span)
                    __builtin_amdgcn_global_load_lds((const void *)(row + 2 * lane), (gm_lds_ptr_t)&stage[buf][c][0], 16,
                                                     0, 0);
                if (2 * lane + 128 < span)
                    __builtin_amdgcn_global_load_lds((const void *)(row + 128 + 2 * lane),
                                                     (gm_lds_ptr_t)&stage[buf][c][128], 16, 0, 0);
            }
            __builtin_amdgcn_s_waitcnt(0);  // this wave's copies have landed ...
            __syncthreads();                // ... and every wave's
            const int sl = active ? (int)j - lo : 0;
#pragma unroll
            for (int c = 0; c < kGmStaged; ++c) {
                const double *q = &stage[buf][c][sl];
                cv[c] = w[0] * q[0] + w[1] * q[1] + w[2] * q[2] + w[3] * q[3];
            }
        } else {
#pragma unroll
            for (int c = 0; c < kGmStaged; ++c) cv[c] = gm_tap(cf + c * NS, j, w);
        }
        // next panel's guess and first Newton taps
        const double tau_next = p == pb ? tau : fmin(fmax(2.0 * tau - tau_prev, tau0), tmax);
        tau_prev = tau;
        if (p + 1 < pe) {
            double un;
            const int64_t jn = gm_locate(tau_next, tau0, dtau, N, un);
            const double *cn = cf + kGmRows * NS;
            tr.load(cn + GY1 * NS, cn + GY2 * NS, cn + GY3 * NS, jn);
        }
        const double r = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
        const double ir = 1.0 / r;
        const double h0 = r0 * ir, h1 = r1 * ir, h2 = r2 * ir;
        auto ch = [&](int c) { return cv[c]; };
        const double Mr = ch(GM1) * h0 + ch(GM2) * h1 + ch(GM3) * h2;
        const double Mdr = ch(GMD1) * h0 + ch(GMD2) * h1 + ch(GMD3) * h2;
        const double Lr = ch(GL1) * h0 + ch(GL2) * h1 + ch(GL3) * h2;
        const double Ldr = ch(GLD1) * h0 + ch(GLD2) * h1 + ch(GLD3) * h2;
        const double iom = 1.0 / (1.0 - Mr);
        const double conv = r * Mdr + c0 * (Mr - ch(GMSQ));
        // A/(r om^2) + Qn conv/(r^2 om^3) + Ld_r/(c0 r om^2) + (L_r - L_M)/(r^2 om^2) + L_r conv/(c0 r^2 om^3)
        const double F =
            ir * iom * iom * (ch(GA) + M0 * Ldr + ir * (Lr - ch(GLM)) + ir * iom * conv * (ch(GQN) + M0 * Lr));
        if (active) acc += F * a.dS[p];
        tau = tau_next;
    }
    if (obs_ok && k < a.nt_stride) a.part[(z * O + o) * a.nt_stride + k] = active ? acc * (1.0 / (4.0 * kPiD)) : 0.0;
}

__global__ __launch_bounds__(256) void gm_reduce_kernel(const double *__restrict__ part, int splits, int64_t n,
                                                      double *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * n + e];
    out[e] = s;
}

}  // namespace

hipError_t launch_gm_source(const GmChanArgs &a, const double *inv_beta, hipStream_t stream) {
    gm_channels_kernel<<<dim3((unsigned)((a.P + kGmTP - 1) / kGmTP), (unsigned)((a.N + kGmTF - 1) / kGmTF)), dim3(256), 0,
                         stream>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t rows = a.P * kGmRows;
    gm_prefilter_kernel<<<dim3((unsigned)((rows + kPfRows - 1) / kPfRows)), dim3(256), 0, stream>>>(a.coef, rows, a.N,
                                                                                                  a.NS, inv_beta);
    return hipGetLastError();
}

hipError_t launch_gm_window(const GmWinArgs &a, hipStream_t stream) {
    gm_window_kernel<<<dim3((unsigned)a.O), dim3(256), 0, stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_gm_gather(const GmGatherArgs &a, double *out, hipStream_t stream) {
    const int64_t blocks = (int64_t)a.splits * a.nkb * ((a.O + 3) / 4);
    gm_gather_kernel<<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = a.O * a.nt_stride;
    gm_reduce_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream>>>(a.part, a.splits, n, out);
    return hipGetLastError();
}

}  // namespace fwh
