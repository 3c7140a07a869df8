// Setup kernels: per-pair delay, per-observer delay extremes, and the per-pair
// tables of the fixed fractional-delay gather (gfx950).
//
// Geometry follows Sec. II C: Garrick distance with the AoA rotation,
// Eqs. (R_New), (R_s_New), (M1), (M2); radiation direction Eqs. (d1_prime)..(R2_New);
// surface Mach vector M = -M0 U0hat (the surface moves against the mean flow in
// the frame where the medium is at rest), M_R = M . Rhat; delay R/c0 = M0 R,
// Eq. (tau2) with c0 = 1/M0 (Sec. II D).  Everything here is FP64.
#include "fwh_internal.h"

namespace fwh {
namespace {

constexpr double kPi = 3.14159265358979323846;

// FP64 pair geometry, evaluated without contraction so that the delay is the
// correctly rounded result of each printed operation in order.
__device__ __forceinline__ void pair_geometry(const double *x, const double *y, const Flow &f, double &R, double Rh[3],
                                              double &MR) {
#pragma clang fp contract(off)
    const double M1 = f.M0 * f.ca, M2 = f.M0 * f.sa;
    const double d1 = x[0] - y[0], d2 = x[1] - y[1], d3 = x[2] - y[2];
    const double md = M1 * d1 + M2 * d2;
    const double Rs = sqrt(md * md + f.beta2 * (d1 * d1 + d2 * d2 + d3 * d3));
    R = (-M1 * d1 - M2 * d2 + Rs) / f.beta2;
    const double d1p = d1 * f.ca + d2 * f.sa;
    const double d2p = -d1 * f.sa + d2 * f.ca;
    const double R1p = (-f.M0 * Rs + d1p) / (f.beta2 * R);
    const double R2p = d2p / R;
    Rh[0] = R1p * f.ca - R2p * f.sa;
    Rh[1] = R1p * f.sa + R2p * f.ca;
    Rh[2] = d3 / R;
    MR = (-f.M0 * f.ca) * Rh[0] + (-f.M0 * f.sa) * Rh[1];
}

__global__ __launch_bounds__(256) void delay_kernel(const double *__restrict__ y, const double *__restrict__ x_obs,
                                                    int64_t P, int64_t O, Flow f, double *__restrict__ D) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * O) return;
    const int64_t o = i / P, p = i - o * P;
    double R, Rh[3], MR;
    pair_geometry(x_obs + 3 * o, y + 3 * p, f, R, Rh, MR);
    D[i] = f.M0 * R;
}

// Per observer: max and min delay over panels (the paper's per-observer R_max,
// R_min of Eqs. (t_start), (t_end)).
__global__ __launch_bounds__(256) void minmax_kernel(const double *__restrict__ D, int64_t P,
                                                     double *__restrict__ dmm) {
    const int64_t o = blockIdx.x;
    double mx = -HUGE_VAL, mn = HUGE_VAL;
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
        const double d = D[o * P + p];
        mx = fmax(mx, d);
        mn = fmin(mn, d);
    }
    __shared__ double smx[256], smn[256];
    smx[threadIdx.x] = mx;
    smn[threadIdx.x] = mn;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + s]);
            smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        dmm[2 * o] = smx[0];
        dmm[2 * o + 1] = smn[0];
    }
}

// Per pair: fractional delay index s0 = (t_start - delay - tau0)/dtau of observer
// sample k = 0 (sample k sits at s0 + k), its integer part n0 and the uniform
// cubic B-spline taps of frac = s0 - n0 acting on coefficients c[n0-1..n0+2];
// and the weights of the 8 source channels in the integrand of
// Eqs. (pT_WT_nd) + (pL_WT_nd), dS/(4 pi) included:
//   Qdot:   1/(R om^2)                 Q:   (M_R - M0^2)/(M0 R^2 om^3)
//   Ldot_i: M0 Rhat_i/(R om^2)         L_i: (Rhat_i - M_i)/(R^2 om^2) + Rhat_i (M_R - M0^2)/(R^2 om^3)
// with om = 1 - M_R (the L_M term is L . M, Eq. (LM)).  With rbf (BF16 mode)
// the weights are also stored split into bfloat16 high and low parts.
struct PairTab {
    double K[8], w[4];
    int32_t n0;
};

__device__ __forceinline__ PairTab pair_tables(const double *__restrict__ y, const double *__restrict__ dS,
                                               const double *__restrict__ x_obs, const double *__restrict__ t_start,
                                               const int32_t *__restrict__ nt, int64_t N, const Flow &f, int64_t o,
                                               int64_t p) {
    PairTab pt;
    double R, Rh[3], MR;
    pair_geometry(x_obs + 3 * o, y + 3 * p, f, R, Rh, MR);
    double D;
    {
#pragma clang fp contract(off)
        D = f.M0 * R;
    }
    double s0 = (t_start[o] - D - f.tau0) / f.dtau;
    if (!(s0 > 0.0)) s0 = 0.0;
    double nf = floor(s0);
    const double nmax = (double)(N - nt[o]);  // keeps n0 + N_t - 1 <= N - 1 (holds by construction)
    if (nf > nmax) nf = nmax;
    double t = s0 - nf;
    if (t > 1.0) t = 1.0;
    pt.n0 = (int32_t)nf;
    const double u = 1.0 - t;
    pt.w[0] = u * u * u / 6.0;
    pt.w[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    pt.w[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    pt.w[3] = t * t * t / 6.0;

    const double M0 = f.M0, M2 = f.M0 * f.M0;
    const double Mv[3] = {-M0 * f.ca, -M0 * f.sa, 0.0};
    const double om = 1.0 - MR, om2 = om * om, om3 = om2 * om;
    const double ws = dS[p] / (4.0 * kPi);
    pt.K[0] = ws / (R * om2);
    pt.K[1] = ws * (MR - M2) / (M0 * R * R * om3);
    for (int c = 0; c < 3; ++c) {
        pt.K[2 + c] = ws * M0 * Rh[c] / (R * om2);
        pt.K[5 + c] = ws * ((Rh[c] - Mv[c]) / (R * R * om2) + Rh[c] * (MR - M2) / (R * R * om3));
    }
    return pt;
}

// plain FP64 form: the tables as FP64 arrays [O][P]
__global__ __launch_bounds__(256) void tables_f64_kernel(const double *__restrict__ y, const double *__restrict__ dS,
                                                         const double *__restrict__ x_obs,
                                                         const double *__restrict__ t_start,
                                                         const int32_t *__restrict__ nt, int64_t P, int64_t O,
                                                         int64_t N, Flow f, double *__restrict__ K64,
                                                         double *__restrict__ W64, int32_t *__restrict__ N0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * O) return;
    const int64_t o = i / P, p = i - o * P;
    const PairTab pt = pair_tables(y, dS, x_obs, t_start, nt, N, f, o, p);
    for (int c = 0; c < 8; ++c) K64[i * 8 + c] = pt.K[c];
    for (int j = 0; j < 4; ++j) W64[i * 4 + j] = pt.w[j];
    N0[i] = pt.n0;
}

// FP32/BF16 forms: block = one observer tile (kObsTile observers) x kTabPanels panels; thread
// (observer slot j, panel q) computes the pair's tables, the block reduces n0 over the tile's
// observers per panel: tw[t][p] = (lo, hi) = (min n0, max n0), and wblk[block] = the widest window
// of the block's panels (blocks t * bpt .. t * bpt + bpt - 1 belong to tile t, bpt = ceil(P /
// kTabPanels)); then each thread writes its pair record [o][p] with n0 - lo in staged bytes (and,
// with rbf, the bfloat16 high/low split of the weights).
constexpr int kTabPanels = 256 / kObsTile;
__global__ __launch_bounds__(256) void tables_tile_kernel(const double *__restrict__ y, const double *__restrict__ dS,
                                                          const double *__restrict__ x_obs,
                                                          const double *__restrict__ t_start,
                                                          const int32_t *__restrict__ nt, int64_t P, int64_t O,
                                                          int64_t N, Flow f, int64_t bpt, PairRec *__restrict__ rec_op,
                                                          PairBf *__restrict__ rbf, int2 *__restrict__ tw,
                                                          int32_t *__restrict__ wblk) {
    const int64_t t = blockIdx.x / bpt;
    const int j = threadIdx.x / kTabPanels, q = threadIdx.x % kTabPanels;
    const int64_t o = t * kObsTile + j, p = (blockIdx.x - t * bpt) * kTabPanels + q;
    __shared__ int sn0[kObsTile][kTabPanels];
    __shared__ int slo[kTabPanels];
    __shared__ int sw[kTabPanels];
    const bool valid = o < O && p < P;
    PairTab pt;
    if (valid) pt = pair_tables(y, dS, x_obs, t_start, nt, N, f, o, p);
    sn0[j][q] = valid ? pt.n0 : 0;
    __syncthreads();
    if (threadIdx.x < kTabPanels) {
        const int64_t nobs = O - t * kObsTile < kObsTile ? O - t * kObsTile : kObsTile;
        int lo = INT_MAX, hi = INT_MIN;
        for (int jj = 0; jj < nobs; ++jj) {
            lo = sn0[jj][q] < lo ? sn0[jj][q] : lo;
            hi = sn0[jj][q] > hi ? sn0[jj][q] : hi;
        }
        int width = 0;
        if (p < P) {
            tw[t * P + p] = make_int2(lo, hi);
            width = hi - lo;
        }
        sw[q] = width;
        slo[q] = lo;
    }
    __syncthreads();
    if (valid) {
        PairRec r;
        for (int c = 0; c < 8; ++c) r.K[c] = (float)pt.K[c];
        for (int jj = 0; jj < 4; ++jj) r.w[jj] = (float)pt.w[jj];
        r.n0 = pt.n0;
        r.n0w = (pt.n0 - slo[q]) * (rbf ? 8 : 16);
        r.pad[0] = r.pad[1] = 0;
        const int64_t i = o * P + p;
        rec_op[i] = r;
        if (rbf) {
            // bfloat16 by round-to-nearest-even of the FP32 value (weights are finite)
            auto bf16 = [](double v) {
                const uint32_t b = __float_as_uint((float)v);
                return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
            };
            PairBf qb;
            for (int c = 0; c < 4; ++c) {
                uint32_t h[2], l[2];
                for (int e = 0; e < 2; ++e) {
                    h[e] = bf16(pt.K[2 * c + e]);
                    l[e] = bf16(pt.K[2 * c + e] - (double)__uint_as_float(h[e] << 16));
                }
                qb.hi[c] = h[0] | (h[1] << 16);
                qb.lo[c] = l[0] | (l[1] << 16);
            }
            rbf[i] = qb;
        }
    }
    if (threadIdx.x == 0) {
        int m = 0;
        for (int qq = 0; qq < kTabPanels; ++qq) m = sw[qq] > m ? sw[qq] : m;
        wblk[blockIdx.x] = m;
    }
}

}  // namespace

hipError_t launch_delay(const double *y, const double *x_obs, int64_t P, int64_t O, Flow f, double *D,
                        hipStream_t stream) {
    const int64_t n = P * O;
    delay_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream>>>(y, x_obs, P, O, f, D);
    return hipGetLastError();
}

hipError_t launch_minmax(const double *D, int64_t P, int64_t O, double *dmm, hipStream_t stream) {
    minmax_kernel<<<dim3((unsigned)O), dim3(256), 0, stream>>>(D, P, dmm);
    return hipGetLastError();
}

hipError_t launch_tables(int mode, const double *y, const double *dS, const double *x_obs, const double *t_start,
                         const int32_t *nt, int64_t P, int64_t O, int64_t N, Flow f, double *K64, double *W64,
                         int32_t *N0, PairRec *rec_op, PairBf *rbf, int2 *tw, int32_t *wblk, hipStream_t stream) {
    if (mode == 0) {
        const int64_t n = P * O;
        tables_f64_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream>>>(y, dS, x_obs, t_start, nt, P,
                                                                                        O, N, f, K64, W64, N0);
    } else {
        tables_tile_kernel<<<dim3((unsigned)tile_window_blocks(P, O)), dim3(256), 0, stream>>>(
            y, dS, x_obs, t_start, nt, P, O, N, f, (P + kTabPanels - 1) / kTabPanels, rec_op, rbf, tw, wblk);
    }
    return hipGetLastError();
}

}  // namespace fwh
