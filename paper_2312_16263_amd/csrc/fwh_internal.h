// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fwh {

constexpr int kChannels = 8;  // [Qdot, Q, Ldot_1, Ldot_2, Ldot_3, L_1, L_2, L_3]

// One (observer, panel) pair of the FP32 gather: integrand weights of the 8
// source channels (dS/(4 pi) included), the four cubic B-spline taps of the
// fixed fractional delay and the integer part of the delay index.  64 bytes, so
// a wave fetches a record with one scalar load.
struct alignas(64) PairRec {
    float K[8];
    float w[4];
    int32_t n0;
    int32_t pad[3];
};
static_assert(sizeof(PairRec) == 64, "PairRec must be 64 bytes");

// Geometry and flow constants passed by value to kernels.
struct Flow {
    double M0, ca, sa, beta2, dtau, tau0;
};

// Row stride (elements) of a panel's coefficient series: indices 0..N+1 hold
// the B-spline coefficients c_{-1}..c_N, the rest are zero padding so that
// gathers near the end of the record never leave the row.
inline int64_t coef_row_stride(int64_t N) { return ((N + 12 + 63) / 64) * 64; }

// Tuned gather geometry: a wave covers kGatherK consecutive observer samples
// (63 lanes x 4, the 64th lane only supplies the neighbour values for lane 62).
constexpr int kGatherLanesOut = 63;
constexpr int kGatherKT = 4;
constexpr int kGatherK = kGatherLanesOut * kGatherKT;  // 252
constexpr int kGatherObsPerBlock = 4;                   // one observer per wave
constexpr int kMaxPanelSplits = 16;

// Adjoint gather geometry: a wave covers 64 consecutive coefficient indices of one panel.
constexpr int kAdjPanelsPerBlock = 4;

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return the launch status.

hipError_t launch_delay(const double *y, const double *x_obs, int64_t P, int64_t O, Flow f, double *D,
                        hipStream_t stream);
hipError_t launch_minmax(const double *D, int64_t P, int64_t O, double *dmm, hipStream_t stream);
// mode 0: FP64 tables (K64 [O][P][8], W64 [O][P][4], N0 [O][P]); mode 1/2: PairRec [O][P] and [P][O].
hipError_t launch_tables(int mode, const double *y, const double *dS, const double *x_obs, const double *t_start,
                         const int32_t *nt, int64_t P, int64_t O, int64_t N, Flow f, double *K64, double *W64,
                         int32_t *N0, PairRec *rec_op, PairRec *rec_po, hipStream_t stream);

// Source terms + derivatives + natural-spline prefilter -> coefficients [8][P][NS].
// in_dtype 0 = double, 1 = float; coef_type 0 = double, 1 = float, 2 = bf16; scratch is
// [8][N][P] of double (coef_type 0) or float (otherwise).
hipError_t launch_source(int in_dtype, int coef_type, const void *rho, const void *u, const void *pp,
                         const double *normal, int64_t P, int64_t N, int64_t NS, Flow f, const double *cp,
                         void *scratch, void *coef, hipStream_t stream);

hipError_t launch_gather_f64(const double *K64, const double *W64, const int32_t *N0, const int32_t *nt,
                             const double *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max, double *out,
                             hipStream_t stream);
// coef_type 1 = float, 2 = bf16.  partial: [splits][O][nt_max] doubles.
hipError_t launch_gather_tuned(int coef_type, const PairRec *rec_op, const int32_t *nt, const void *coef, int64_t P,
                               int64_t O, int64_t NS, int64_t nt_max, int splits, double *partial,
                               hipStream_t stream);
// out[i] = sum over splits of partial[z][i], fixed order, rounded to float.
hipError_t launch_reduce_splits(const double *partial, int splits, int64_t total, float *out, hipStream_t stream);

hipError_t launch_adj_gather_f64(const double *K64, const double *W64, const int32_t *N0, const int32_t *nt,
                                 const double *gbar, int64_t P, int64_t O, int64_t NS, int64_t nt_max, double *cbar,
                                 hipStream_t stream);
hipError_t launch_adj_gather_tuned(const PairRec *rec_po, const int32_t *nt, const float *gbar, int64_t P, int64_t O,
                                   int64_t NS, int64_t nt_max, float *cbar, hipStream_t stream);

// Adjoint of the source stage: coefficient adjoints [8][P][NS] -> gradients (time-major, in_dtype).
// real_type 0 = double (cbar and scratch double), 1 = float.
hipError_t launch_source_adjoint(int real_type, int in_dtype, const void *cbar, const void *rho, const void *u,
                                 const double *normal, int64_t P, int64_t N, int64_t NS, Flow f, const double *cp,
                                 void *scratch, void *g_rho, void *g_u, void *g_p, hipStream_t stream);

}  // namespace fwh
