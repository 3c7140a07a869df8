// Post-processing of the observer signals on the device (gfx950): per-observer
// RMS pressure (the directivity plots of Sec. IV A-B) and the one-sided Welch
// power spectral density of Sec. IV C: segments of L samples with 50 % overlap,
// Hanning window, averaged squared DFT magnitudes, times the spanwise
// correction factor b_exp / b_m of Eq. (PSD_corr).
//
// One workgroup per observer.  RMS: strided sum of squares in FP64, block
// reduction.  Welch: each segment is windowed (periodic Hann, w_n = (1 -
// cos(2 pi n / L)) / 2) into LDS in bit-reversed order, transformed by an
// in-place radix-2 decimation-in-time FFT (log2 L stages of L/2 butterflies,
// twiddles exp(-2 pi i j / len) from sincospi of an exact argument), and
// |X_f|^2 for f = 0 .. L/2 is added to an FP64 accumulator in LDS.  Scaling:
// c_f / (n_seg f_s sum w^2) with c_f = 2 except at f = 0 and L/2, sum w^2 =
// 3L/8.  Deterministic (fixed order everywhere).
#include "fwh_internal.h"

namespace fwh {
namespace {

__device__ __forceinline__ int bit_reverse(int i, int bits) { return (int)(__brev((unsigned)i) >> (32 - bits)); }

template <typename T>
__global__ __launch_bounds__(256) void post_kernel(const T *__restrict__ p, int64_t ld, const int32_t *__restrict__ nt,
                                                   int L, int logL, double dt, double span_ratio,
                                                   float *__restrict__ psd, float *__restrict__ rms) {
    extern __shared__ __align__(16) unsigned char smem_post[];
    float *re = reinterpret_cast<float *>(smem_post);
    float *im = re + L;
    double *acc = reinterpret_cast<double *>(im + L);  // L/2 + 1
    double *red = acc + (L / 2 + 1);                    // 256
    const int tid = threadIdx.x;
    const int64_t o = blockIdx.x;
    const int n = nt[o];
    const T *x = p + o * ld;

    // RMS over the observer's window
    double s = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double v = (double)x[i];
        s += v * v;
    }
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) rms[o] = (float)sqrt(red[0] / (double)n);

    // Welch
    const int half_L = L / 2;
    const int nseg = n >= L ? (n - L) / half_L + 1 : 0;
    for (int f = tid; f <= half_L; f += 256) acc[f] = 0.0;
    for (int sgm = 0; sgm < nseg; ++sgm) {
        const T *xs = x + (int64_t)sgm * half_L;
        for (int i = tid; i < L; i += 256) {
            const float w = 0.5f - 0.5f * cospif(2.0f * (float)i / (float)L);
            const int j = bit_reverse(i, logL);
            re[j] = (float)xs[i] * w;
            im[j] = 0.f;
        }
        __syncthreads();
        for (int len = 2; len <= L; len <<= 1) {
            const int hl = len >> 1;
            for (int bf = tid; bf < half_L; bf += 256) {
                const int grp = bf / hl, j = bf - grp * hl;
                const int k = grp * len + j;
                float sn, cs;
                sincospif(-2.0f * (float)j / (float)len, &sn, &cs);
                const float br = re[k + hl], bi = im[k + hl];
                const float vr = br * cs - bi * sn, vi = br * sn + bi * cs;
                const float ur = re[k], ui = im[k];
                re[k] = ur + vr;
                im[k] = ui + vi;
                re[k + hl] = ur - vr;
                im[k + hl] = ui - vi;
            }
            __syncthreads();
        }
        for (int f = tid; f <= half_L; f += 256) acc[f] += (double)re[f] * re[f] + (double)im[f] * im[f];
        __syncthreads();
    }
    const double fs = 1.0 / dt, sumw2 = 3.0 * (double)L / 8.0;
    for (int f = tid; f <= half_L; f += 256) {
        const double c = (f == 0 || f == half_L) ? 1.0 : 2.0;
        psd[o * (half_L + 1) + f] =
            nseg > 0 ? (float)(span_ratio * c * acc[f] / ((double)nseg * fs * sumw2)) : 0.f;
    }
}

}  // namespace

size_t post_shmem(int L) { return (size_t)2 * L * sizeof(float) + (size_t)(L / 2 + 1 + 256) * sizeof(double); }

hipError_t launch_post(int real_type, const void *p, int64_t ld, const int32_t *nt, int64_t O, int L, double dt,
                       double span_ratio, float *psd, float *rms, hipStream_t stream) {
    int logL = 0;
    while ((1 << logL) < L) ++logL;
    const size_t shmem = post_shmem(L);
    if (real_type == 0)
        post_kernel<double><<<dim3((unsigned)O), dim3(256), shmem, stream>>>(static_cast<const double *>(p), ld, nt, L,
                                                                            logL, dt, span_ratio, psd, rms);
    else
        post_kernel<float><<<dim3((unsigned)O), dim3(256), shmem, stream>>>(static_cast<const float *>(p), ld, nt, L,
                                                                           logL, dt, span_ratio, psd, rms);
    return hipGetLastError();
}

}  // namespace fwh
