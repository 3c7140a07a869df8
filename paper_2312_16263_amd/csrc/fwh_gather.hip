// Gather kernels (gfx950): the surface sum of Sec. III C as a fixed
// fractional-delay gather, and its transpose for the adjoint.
//
// After the setup every (observer o, panel p) pair has a fixed delay index
// s0 = n0 + frac, fixed cubic B-spline taps w_0..w_3 (acting on spline
// coefficients c[n0+k-1 .. n0+k+2], storage indices n0+k .. n0+k+3) and fixed
// weights K_c of the 8 source channels, so
//   p'(o, k) = sum_p sum_jj w_jj(o,p) g_{o,p}(n0 + k + jj),
//   g_{o,p}(i) = sum_c K_c(o,p) coef_c(p, i).
// The tuned kernel combines the channels first (8 FMA per new index) and then
// applies the 4 taps (4 FMA per output): 12 FMA per (panel, observer, sample).
// No matrix cores: the contraction over channels has length 8 and each pair
// has its own shift, so the work is a shifted gather, not a dense GEMM.
#include "fwh_internal.h"

namespace fwh {
namespace {

// ---------------------------------------------------------- plain FP64 forms

// One thread per (observer, sample): loop over panels, interpolate each channel.
__global__ __launch_bounds__(256) void gather_f64_kernel(const double *__restrict__ K64,
                                                         const double *__restrict__ W64,
                                                         const int32_t *__restrict__ N0,
                                                         const int32_t *__restrict__ nt,
                                                         const double *__restrict__ coef, int64_t P, int64_t NS,
                                                         int64_t nt_max, int64_t kblocks, double *__restrict__ out) {
    const int64_t o = blockIdx.x / kblocks;
    const int64_t k = (blockIdx.x - o * kblocks) * blockDim.x + threadIdx.x;
    if (k >= nt_max) return;
    if (k >= nt[o]) {
        out[o * nt_max + k] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        const int64_t pr = o * P + p;
        const int64_t base = (int64_t)N0[pr] + k;
        double s = 0.0;
        for (int jj = 0; jj < 4; ++jj) {
            double g = 0.0;
            for (int c = 0; c < 8; ++c) g += K64[pr * 8 + c] * coef[((int64_t)c * P + p) * NS + base + jj];
            s += W64[pr * 4 + jj] * g;
        }
        acc += s;
    }
    out[o * nt_max + k] = acc;
}

// One thread per (panel, coefficient index i): loop over observers,
//   cbar_c(p, i) = sum_o K_c(o,p) sum_jj w_jj(o,p) gbar(o, i - n0(o,p) - jj),
// with gbar taken as zero outside 0 <= k < N_t(o).
__global__ __launch_bounds__(256) void adj_gather_f64_kernel(const double *__restrict__ K64,
                                                             const double *__restrict__ W64,
                                                             const int32_t *__restrict__ N0,
                                                             const int32_t *__restrict__ nt,
                                                             const double *__restrict__ gbar, int64_t P, int64_t O,
                                                             int64_t NS, int64_t nt_max, int64_t iblocks,
                                                             double *__restrict__ cbar) {
    const int64_t p = blockIdx.x / iblocks;
    const int64_t i = (blockIdx.x - p * iblocks) * blockDim.x + threadIdx.x;
    if (i >= NS) return;
    double acc[8];
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    for (int64_t o = 0; o < O; ++o) {
        const int64_t pr = o * P + p;
        const int64_t kb = i - (int64_t)N0[pr];
        const int64_t ntl = nt[o];
        double h = 0.0;
        for (int jj = 0; jj < 4; ++jj) {
            const int64_t k = kb - jj;
            if (k >= 0 && k < ntl) h += W64[pr * 4 + jj] * gbar[o * nt_max + k];
        }
        for (int c = 0; c < 8; ++c) acc[c] += K64[pr * 8 + c] * h;
    }
    for (int c = 0; c < 8; ++c) cbar[((int64_t)c * P + p) * NS + i] = acc[c];
}

// ---------------------------------------------------------------- tuned FP32

__device__ __forceinline__ float load_coef(const float *p) { return *p; }
__device__ __forceinline__ float load_coef(const uint16_t *p) { return __uint_as_float((uint32_t)(*p) << 16); }

// Value of lane l+1 (wavefront shift by one lane; lane 63 receives 0).
__device__ __forceinline__ float from_next_lane(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130 /* wave_shl:1 */, 0xF, 0xF, false));
}

constexpr int kChunk = 64;  // panels summed in FP32 before adding into the FP64 accumulator

// A wave owns one observer and 252 consecutive samples k0 + 4*lane + m (m = 0..3,
// lanes 0..62; lane 63 only computes the combined values its left neighbour
// needs).  Per panel the pair record is a uniform (scalar) load; each lane
// combines the 8 channels at its 4 coefficient indices, takes 3 more combined
// values from lane+1 by a wavefront shift and applies the taps.  Panels
// [z*p_chunk, (z+1)*p_chunk) go to partial[z][o][k].
template <typename TS>
__global__ __launch_bounds__(256) void gather_tuned_kernel(const PairRec *__restrict__ rec,
                                                           const int32_t *__restrict__ nt,
                                                           const TS *__restrict__ coef, int64_t P, int64_t O,
                                                           int64_t NS, int64_t nt_max, int64_t p_chunk,
                                                           double *__restrict__ partial) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t o = (int64_t)blockIdx.x * kGatherObsPerBlock + wv;
    if (o >= O) return;
    const int64_t k0 = (int64_t)blockIdx.y * kGatherK;
    const int64_t z = blockIdx.z;
    const int64_t pb = z * p_chunk;
    const int64_t pe = pb + p_chunk < P ? pb + p_chunk : P;
    const int64_t kl = k0 + kGatherKT * lane;
    const int64_t chs = P * NS;
    const PairRec *rr = rec + o * P;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    double accd[4] = {0.0, 0.0, 0.0, 0.0};
    int cnt = 0;
    for (int64_t p = pb; p < pe; ++p) {
        const PairRec r = rr[p];
        int64_t base = (int64_t)r.n0 + kl;
        if (base > NS - 4) base = NS - 4;  // only lanes whose samples are past N_t(o) reach the clamp
        const TS *cp = coef + p * NS + base;
        float g[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
#pragma unroll
            for (int i = 0; i < 4; ++i) g[i] = fmaf(r.K[c], load_coef(cp + c * chs + i), g[i]);
        }
        float G[7];
        G[0] = g[0];
        G[1] = g[1];
        G[2] = g[2];
        G[3] = g[3];
        G[4] = from_next_lane(g[0]);
        G[5] = from_next_lane(g[1]);
        G[6] = from_next_lane(g[2]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) acc[m] = fmaf(r.w[jj], G[m + jj], acc[m]);
        }
        if (++cnt == kChunk) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                accd[m] += (double)acc[m];
                acc[m] = 0.f;
            }
            cnt = 0;
        }
    }
    const int64_t ntl = nt[o];
    if (lane < kGatherLanesOut) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int64_t k = kl + m;
            if (k < nt_max) partial[(z * O + o) * nt_max + k] = (k < ntl) ? accd[m] + (double)acc[m] : 0.0;
        }
    }
}

// out[o][k] = sum_z partial[z][o][k] in fixed order.
__global__ __launch_bounds__(256) void reduce_splits_kernel(const double *__restrict__ partial, int splits,
                                                            int64_t total, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += partial[(int64_t)z * total + i];
    out[i] = (float)s;
}

// A wave owns one panel and 64 consecutive coefficient indices; loop over all
// observers with uniform record loads; chunks of observers summed in FP32,
// then into FP64.
__global__ __launch_bounds__(256) void adj_gather_tuned_kernel(const PairRec *__restrict__ rec_po,
                                                               const int32_t *__restrict__ nt,
                                                               const float *__restrict__ gbar, int64_t P, int64_t O,
                                                               int64_t NS, int64_t nt_max,
                                                               float *__restrict__ cbar) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t p = (int64_t)blockIdx.x * kAdjPanelsPerBlock + wv;
    if (p >= P) return;
    const int64_t i = (int64_t)blockIdx.y * 64 + lane;
    const PairRec *rr = rec_po + p * O;
    float acc[8];
    double accd[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        acc[c] = 0.f;
        accd[c] = 0.0;
    }
    int cnt = 0;
    for (int64_t o = 0; o < O; ++o) {
        const PairRec r = rr[o];
        const int64_t ntl = nt[o];
        const float *g = gbar + o * nt_max;
        const int64_t kb = i - r.n0;
        float h = 0.f;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int64_t k = kb - jj;
            const bool ok = k >= 0 && k < ntl;
            const float v = g[ok ? k : 0];
            h = fmaf(r.w[jj], ok ? v : 0.f, h);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = fmaf(r.K[c], h, acc[c]);
        if (++cnt == kChunk) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                accd[c] += (double)acc[c];
                acc[c] = 0.f;
            }
            cnt = 0;
        }
    }
    if (i < NS) {
#pragma unroll
        for (int c = 0; c < 8; ++c) cbar[((int64_t)c * P + p) * NS + i] = (float)(accd[c] + (double)acc[c]);
    }
}

}  // namespace

hipError_t launch_gather_f64(const double *K64, const double *W64, const int32_t *N0, const int32_t *nt,
                             const double *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max, double *out,
                             hipStream_t stream) {
    const int64_t kblocks = (nt_max + 255) / 256;
    gather_f64_kernel<<<dim3((unsigned)(kblocks * O)), dim3(256), 0, stream>>>(K64, W64, N0, nt, coef, P, NS, nt_max,
                                                                              kblocks, out);
    return hipGetLastError();
}

hipError_t launch_gather_tuned(int coef_type, const PairRec *rec_op, const int32_t *nt, const void *coef, int64_t P,
                               int64_t O, int64_t NS, int64_t nt_max, int splits, double *partial,
                               hipStream_t stream) {
    const int64_t p_chunk = (P + splits - 1) / splits;
    dim3 grid((unsigned)((O + kGatherObsPerBlock - 1) / kGatherObsPerBlock),
              (unsigned)((nt_max + kGatherK - 1) / kGatherK), (unsigned)splits);
    if (coef_type == 1)
        gather_tuned_kernel<float><<<grid, dim3(256), 0, stream>>>(rec_op, nt, (const float *)coef, P, O, NS, nt_max,
                                                                   p_chunk, partial);
    else
        gather_tuned_kernel<uint16_t><<<grid, dim3(256), 0, stream>>>(rec_op, nt, (const uint16_t *)coef, P, O, NS,
                                                                      nt_max, p_chunk, partial);
    return hipGetLastError();
}

hipError_t launch_reduce_splits(const double *partial, int splits, int64_t total, float *out, hipStream_t stream) {
    reduce_splits_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream>>>(partial, splits, total, out);
    return hipGetLastError();
}

hipError_t launch_adj_gather_f64(const double *K64, const double *W64, const int32_t *N0, const int32_t *nt,
                                 const double *gbar, int64_t P, int64_t O, int64_t NS, int64_t nt_max, double *cbar,
                                 hipStream_t stream) {
    const int64_t iblocks = (NS + 255) / 256;
    adj_gather_f64_kernel<<<dim3((unsigned)(iblocks * P)), dim3(256), 0, stream>>>(K64, W64, N0, nt, gbar, P, O, NS,
                                                                                  nt_max, iblocks, cbar);
    return hipGetLastError();
}

hipError_t launch_adj_gather_tuned(const PairRec *rec_po, const int32_t *nt, const float *gbar, int64_t P, int64_t O,
                                   int64_t NS, int64_t nt_max, float *cbar, hipStream_t stream) {
    dim3 grid((unsigned)((P + kAdjPanelsPerBlock - 1) / kAdjPanelsPerBlock), (unsigned)((NS + 63) / 64));
    adj_gather_tuned_kernel<<<grid, dim3(256), 0, stream>>>(rec_po, nt, gbar, P, O, NS, nt_max, cbar);
    return hipGetLastError();
}

}  // namespace fwh
