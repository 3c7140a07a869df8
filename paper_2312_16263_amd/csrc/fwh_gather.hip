// Gather kernels (gfx950): the surface sum of Sec. III C as a fixed
// fractional-delay gather, and its transpose for the adjoint.
//
// Coefficients are stored panel-major with the 4 channels of each of the two
// channel groups interleaved: coef[P][2][NS][4] (channel c = 4 g + cc).
//
// After the setup every (observer o, panel p) pair has a fixed delay index
// s0 = n0 + frac, fixed cubic B-spline taps w_0..w_3 (acting on spline
// coefficients c[n0+k-1 .. n0+k+2], storage indices n0+k .. n0+k+3) and fixed
// weights K_c of the 8 source channels, so
//   p'(o, k) = sum_p sum_jj w_jj(o,p) g_{o,p}(n0 + k + jj),
//   g_{o,p}(i) = sum_c K_c(o,p) coef_c(p, i).
// The forward kernels combine the channels first (8 FMA per new index) and then
// apply the 4 taps (4 FMA per output): 12 FMA per (panel, observer, sample); the
// contraction over channels has length 8 and each pair has its own shift.  The
// transposed gather sums over observers, a contraction of length O for every
// (panel, index): it runs on the matrix cores.
#include <type_traits>

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
            for (int c = 0; c < 8; ++c) g += K64[pr * 8 + c] * coef[((p * 2 + (c >> 2)) * NS + base + jj) * 4 + (c & 3)];
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
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130 /* wave_shl:1 */, 0xF, 0xF, true));
}

// a0 += w0 * (x of the next lane), a1 += w1 * (x of the next lane): two FMAs whose first source is
// read through a DPP wave_shl:1 (lane 63 reads 0), so the lane shift costs no instruction of its
// own (the compiler does not fold a DPP move into an FMA with a tied accumulator by itself).  The
// s_nop gives the two wait states a DPP read needs after the VALU write of x.
__device__ __forceinline__ void fmac2_next_lane(float &a0, float &a1, float x, float w0, float w1) {
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %2, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %2, %4 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "+v"(a0), "+v"(a1)
        : "v"(x), "v"(w0), "v"(w1));
}

constexpr int kChunk = 64;  // panels summed in FP32 before adding into the FP64 accumulator
// the LDS-staged gather keeps no accumulators beyond one FP32 sum per output in registers: it adds
// its sums over kLdsChunk panels into the split's partial signal in memory (a split of at most
// kLdsChunk panels is one FP32 sum; the splits are added in FP64 by the reduction)
constexpr int kLdsChunk = 256;

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
                                                           float *__restrict__ partial) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t o = (int64_t)blockIdx.x * kGatherObsPerBlock + wv;
    if (o >= O) return;
    const int64_t k0 = (int64_t)blockIdx.y * kGatherK;
    const int64_t z = blockIdx.z;
    const int64_t pb = z * p_chunk;
    const int64_t pe = pb + p_chunk < P ? pb + p_chunk : P;
    const int64_t kl = k0 + kGatherKT * lane;
    const PairRec *rr = rec + o * P;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    double accd[4] = {0.0, 0.0, 0.0, 0.0};
    int cnt = 0;
    for (int64_t p = pb; p < pe; ++p) {
        const PairRec r = rr[p];
        int64_t base = (int64_t)r.n0 + kl;
        if (base > NS - 4) base = NS - 4;  // only lanes whose samples are past N_t(o) reach the clamp
        const TS *c0 = coef + ((p * 2) * NS + base) * 4;   // group 0 quads at base .. base+3
        const TS *c1 = c0 + NS * 4;                        // group 1
        float g[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                g[i] = fmaf(r.K[cc], load_coef(c0 + i * 4 + cc), g[i]);
                g[i] = fmaf(r.K[4 + cc], load_coef(c1 + i * 4 + cc), g[i]);
            }
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
            if (k < nt_max) partial[(z * O + o) * nt_max + k] = (k < ntl) ? (float)(accd[m] + (double)acc[m]) : 0.f;
        }
    }
}


// A staged element: the 4 channels of one group at one time index (float4 in
// FP32, four bfloat16 in BF16) and its expansion to FP32.
template <typename TS>
struct Quad;
template <>
struct Quad<float> {
    using T = float4;
    static __device__ __forceinline__ void unpack(const float4 &v, float o[4]) {
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};
template <>
struct Quad<uint16_t> {
    using T = uint2;  // four bfloat16
    static __device__ __forceinline__ void unpack(const uint2 &v, float o[4]) {
        o[0] = __uint_as_float(v.x << 16);
        o[1] = __uint_as_float(v.x & 0xffff0000u);
        o[2] = __uint_as_float(v.y << 16);
        o[3] = __uint_as_float(v.y & 0xffff0000u);
    }
};

// Element of a staged window: the 4 channels of one group at one time index
// (16 bytes in FP32, 8 bytes in BF16); copied to LDS by direct global->LDS loads
// of 16 bytes per lane: one element (FP32) or two (BF16; the staged window
// length is then a multiple of 128 elements, so a group is whole 64-lane copies).
template <typename TS>
struct Stage;
template <>
struct Stage<float> {
    static constexpr int kElemPerUnit = 1;
};
template <>
struct Stage<uint16_t> {
    static constexpr int kElemPerUnit = 2;
};

typedef __attribute__((address_space(3))) void *lds_ptr_t;

// Row of observer o in the partial signal of split z ([splits][O][nt_max]).
__device__ __forceinline__ float *partial_row(float *partial, int64_t z, int64_t O, int64_t o, int64_t nt_max) {
    return partial + (z * O + o) * nt_max;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
// a.lo * b.lo + a.hi * b.hi + c for two bfloat16 pairs (v_dot2_f32_bf16)
__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c, false);
}

// Direct global -> LDS copy of `count` units of Stage::kBytesPerLoad bytes from
// src (byte address of unit u: src + u*bytes, clamped to unit `last`) to LDS at
// dst (unit u at dst + u*bytes), wave w handling 64-unit chunks w, w + 8, ...
template <int BYTES, int WAVES = kLdsWaves>  // 16 or 4 bytes per lane; waves sharing the copy
__device__ __forceinline__ void copy_to_lds(const unsigned char *src, int64_t last, unsigned char *dst, int count,
                                            int wv, int lane) {
    for (int ci = wv; ci * 64 < count; ci += WAVES) {
        int64_t u = (int64_t)ci * 64 + lane;
        u = u < last ? u : last;
        if constexpr (BYTES == 16)
            __builtin_amdgcn_global_load_lds((const void *)(src + u * 16), (lds_ptr_t)(dst + ci * 64 * 16), 16, 0, 0);
        else
            __builtin_amdgcn_global_load_lds((const void *)(src + u * 4), (lds_ptr_t)(dst + ci * 64 * 4), 4, 0, 0);
    }
}

// LDS-staged gather.  Block = kLdsWaves waves; a wave shape OPW x SUBW: each wave
// takes OPW observers of the block's tile (TILE = kLdsWaves * OPW observers, the
// first TILE of the 32-observer tile t) and SUBW sub-rows of kLdsLanesOut samples,
// so the block covers samples k0 .. k0 + SUBW * kLdsLanesOut - 1; panels
// [z*p_chunk, ...) in stages of PT panels, double-buffered: while the waves work
// on one stage the direct global->LDS loads of the next are in flight.  Per panel
// a stage holds the coefficient windows [lo + k0, lo + k0 + NW) of both channel
// groups ([2][NW][4], lo = min n0 over the tile's observers, NW >= max width +
// block samples + kLdsHalo) and the TILE pair records.  Every wave, for each of
// its observers and sub-rows, lets lane l combine the 8 channels at window
// position n0 - lo + 61 m + l (two vector LDS reads) and adds the combined value
// into two tap-pair accumulators (below).  Shapes: 4 x 4 (32 observers x 244
// samples) for full tiles; 2 x 8 (16 observers x 488 samples) for a last tile of
// at most 16 observers, whose waves would otherwise hold one or two observers
// each while the block still staged the full window for 244 samples (the same
// 32 accumulators per lane, about half the staged bytes per output).
// The two stage buffers are separate static LDS arrays (stA, stB): the compiler
// can then tell that the direct global->LDS loads into one buffer do not alias
// the LDS reads of the other, and does not make those reads wait for the loads.
template <typename TS, int OPW = kObsPerWave, int SUBW = kLdsSub, bool ADJ = false>
__device__ __forceinline__ void gather_lds_body(const GatherArgs &a, int64_t t, int64_t kb, int64_t z,
                                                unsigned char *stA, unsigned char *stB) {
    constexpr int TILE = kLdsWaves * OPW;         // observer slots of the block
    constexpr int KB = SUBW * kLdsLanesOut;       // samples of the block
    const PairRec *__restrict__ rec = a.rec;
    const int2 *__restrict__ tw = a.tw;
    const int32_t *__restrict__ nt = a.nt;
    const TS *__restrict__ coef = static_cast<const TS *>(a.coef);
    const int64_t P = a.P, O = a.O, NS = a.NS, nt_max = a.nt_max, p_chunk = a.p_chunk;
    const int NW = a.NW, PT = a.PT;
    float *__restrict__ partial = a.partial;
    using QT = typename Quad<TS>::T;
    constexpr int EB = 4 * (int)sizeof(TS);  // bytes per element (4 channels)
    constexpr bool kBf = std::is_same<TS, uint16_t>::value;
    const size_t win_bytes = (size_t)2 * NW * EB;                    // one panel, both groups
    // stage buffer: PT windows, then PT x TILE records, then (BF16) PT x TILE split weights
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t k0 = kb * KB;
    const int64_t pb = z * p_chunk;
    const int64_t pe = pb + p_chunk < P ? pb + p_chunk : P;
    const int64_t tbase = t * kObsTile;
    const int2 *twt = tw + t * P;
    const int64_t ot_last = (O - 1 - tbase) < TILE - 1 ? (O - 1 - tbase) : TILE - 1;
    // observer slot (offset in the tile) of the wave's j-th observer.  ADJ: the wave takes OPW
    // adjacent observers, whose windows are alike, so fewer of its sub-rows lie past the shorter
    // ones (the single-case 4 x 4 launch, whose tiles are full but for the last).  Otherwise
    // observers wv, wv + 8, ..., which spreads the few observers of a partly filled tile over all
    // waves (the 2 x 8 shape, for a last tile of at most 16 observers, and the batched gather,
    // where many cases end in such a tile).  Either way a wave's valid observers are a prefix
    // j < nobs.
    auto slot_of = [&](int j) { return ADJ ? wv * OPW + j : j * kLdsWaves + wv; };

    // issue the loads of the stage starting at panel ps into the stage buffer `base`
    auto fill = [&](int64_t ps, unsigned char *base) {
        const int np = (int)(pe - ps < PT ? pe - ps : PT);
        for (int q = 0; q < np; ++q) {
            const int64_t p = ps + q;
            const int64_t start = (int64_t)twt[p].x + k0;
            constexpr int EU = Stage<TS>::kElemPerUnit;
            const int units = NW / EU;
            for (int g = 0; g < 2; ++g) {
                const unsigned char *src =
                    reinterpret_cast<const unsigned char *>(coef + ((p * 2 + g) * NS + start) * 4);
                // units past the row end are clamped to its last unit (never read by valid outputs; in
                // BF16 a last unit may take one element of the next row, or of the region after the
                // coefficients, which are never read either)
                const int64_t last = (NS - start + EU - 1) / EU - 1;
                copy_to_lds<16>(src, last, base + q * win_bytes + g * NW * EB, units, wv, lane);
            }
        }
        // records: for panel q, observer slot j -> 64 bytes at [q][j]
        unsigned char *rbase = base + (size_t)PT * win_bytes;
        const int runits = np * TILE * 4;  // 16-byte units
        for (int ci = wv; ci * 64 < runits; ci += kLdsWaves) {
            int u = ci * 64 + lane;
            u = u < runits ? u : runits - 1;
            const int q = u / (TILE * 4), r = u - q * (TILE * 4);
            const int64_t jj = (r >> 2) < ot_last ? (r >> 2) : ot_last;
            const float4 *srec = reinterpret_cast<const float4 *>(rec + (tbase + jj) * P + ps + q) + (r & 3);
            __builtin_amdgcn_global_load_lds((const void *)srec, (lds_ptr_t)(rbase + ci * 64 * 16), 16, 0, 0);
        }
        if constexpr (kBf) {
            // split weights: for panel q, observer slot j -> 32 bytes at [q][j]
            unsigned char *bbase = rbase + (size_t)PT * TILE * sizeof(PairRec);
            const int bunits = np * TILE * 2;
            for (int ci = wv; ci * 64 < bunits; ci += kLdsWaves) {
                int u = ci * 64 + lane;
                u = u < bunits ? u : bunits - 1;
                const int q = u / (TILE * 2), r = u - q * (TILE * 2);
                const int64_t jj = (r >> 1) < ot_last ? (r >> 1) : ot_last;
                const uint4 *sb = reinterpret_cast<const uint4 *>(a.rbf + (tbase + jj) * P + ps + q) + (r & 1);
                __builtin_amdgcn_global_load_lds((const void *)sb, (lds_ptr_t)(bbase + ci * 64 * 16), 16, 0, 0);
            }
        }
    };

    // FP32 sums over kLdsChunk panels, added into the wave's own outputs of the split's partial signal
    // (no other wave writes them)
    // Per (observer slot j, sub-row m) two tap-pair accumulators: with g the lane's combined value
    // and g' = g of the next lane, acc[j][m][0] sums w_0 g + w_1 g' and acc[j][m][1] sums
    // w_2 g + w_3 g' over panels (the next-lane operand is a DPP source of the FMA, no extra
    // instruction).  The output of lane l is acc[j][m][0] at l plus acc[j][m][1] at l + 2; that
    // shift is the same for every panel, so it is applied once per flush (tap_sum).
    float acc[OPW][SUBW][2];
#pragma unroll
    for (int j = 0; j < OPW; ++j)
#pragma unroll
        for (int m = 0; m < SUBW; ++m) acc[j][m][0] = acc[j][m][1] = 0.f;
    // acc[j][m][0] + acc[j][m][1] two lanes up (every lane must take part: lane shifts)
    auto tap_sum = [&](int j, int m) {
        return acc[j][m][0] + from_next_lane(from_next_lane(acc[j][m][1]));
    };
    // this wave's output element of observer slot j, sub-row m (null outside the output)
    auto out_ptr = [&](int j, int m) -> float * {
        const int64_t o = tbase + slot_of(j);
        const int64_t k = k0 + m * kLdsLanesOut + lane;
        return (lane < kLdsLanesOut && o < O && k < nt_max) ? partial + (z * O + o) * nt_max + k : nullptr;
    };
    // this wave's valid observers (a prefix j < nobs) and the sub-rows of 61 samples below the
    // largest of their windows (0: nothing to do)
    int nt_wave = 0, nobs = 0;
#pragma unroll
    for (int j = 0; j < OPW; ++j) {
        const int64_t o = tbase + slot_of(j);
        if (o < O) {
            nt_wave = nt[o] > nt_wave ? nt[o] : nt_wave;
            nobs = j + 1;
        }
    }
    nobs = __builtin_amdgcn_readfirstlane(nobs);
    int nsub = (int)((nt_wave - k0 + kLdsLanesOut - 1) / kLdsLanesOut);
    nsub = __builtin_amdgcn_readfirstlane(nsub < 0 ? 0 : (nsub > SUBW ? SUBW : nsub));
    // one panel of the stage for this wave's first NOBS observers, NSUB sub-rows.  The window
    // elements are addressed by one byte offset from the stage buffer `sb` (qb: the byte offset of
    // the lane's element in panel slot q's first channel group at n0 = lo; the pair record carries
    // n0 - lo in bytes; the second group is NW elements later): a longer chain of pointer
    // arithmetic hides from the compiler which of the two buffers a read touches, and it then makes
    // the read wait for the copies into the other one.
    auto panel_work = [&](auto nobs_c, auto nsub_c, const float4 *lrec, const unsigned char *sb, int qb, int q) {
        constexpr int NOBS = decltype(nobs_c)::value;
        constexpr int NSUB = decltype(nsub_c)::value;
#pragma unroll
        for (int j = 0; j < NOBS; ++j) {
            const int slot = q * TILE + slot_of(j);
            const float4 *R = lrec + slot * 4;
            const float4 W = R[2];
            const int b0 = qb + __float_as_int(R[3].y);
            const QT *P0 = reinterpret_cast<const QT *>(sb + b0);
            const QT *P1 = reinterpret_cast<const QT *>(sb + (b0 + NW * EB));
            float4 Ka, Kb;
            uint4 Kh, Kl;
            if constexpr (kBf) {
                const uint4 *B = reinterpret_cast<const uint4 *>(lrec + PT * TILE * 4) + slot * 2;
                Kh = B[0];
                Kl = B[1];
            } else {
                Ka = R[0];
                Kb = R[1];
            }
#pragma unroll
            for (int m = 0; m < NSUB; ++m) {
                float g;
                if constexpr (kBf) {
                    // packed bf16 dot products: channel pairs of the four-channel elements against the
                    // high and low parts of their weights
                    const uint2 e0 = P0[m * kLdsLanesOut], e1 = P1[m * kLdsLanesOut];
                    g = dot2_bf16(Kh.x, e0.x, 0.f);
                    g = dot2_bf16(Kh.y, e0.y, g);
                    g = dot2_bf16(Kh.z, e1.x, g);
                    g = dot2_bf16(Kh.w, e1.y, g);
                    g = dot2_bf16(Kl.x, e0.x, g);
                    g = dot2_bf16(Kl.y, e0.y, g);
                    g = dot2_bf16(Kl.z, e1.x, g);
                    g = dot2_bf16(Kl.w, e1.y, g);
                } else {
                    float a[4], c[4];
                    Quad<TS>::unpack(P0[m * kLdsLanesOut], a);
                    Quad<TS>::unpack(P1[m * kLdsLanesOut], c);
                    g = Ka.x * a[0];
                    g = fmaf(Ka.y, a[1], g);
                    g = fmaf(Ka.z, a[2], g);
                    g = fmaf(Ka.w, a[3], g);
                    g = fmaf(Kb.x, c[0], g);
                    g = fmaf(Kb.y, c[1], g);
                    g = fmaf(Kb.z, c[2], g);
                    g = fmaf(Kb.w, c[3], g);
                }
                acc[j][m][0] = fmaf(W.x, g, acc[j][m][0]);
                acc[j][m][1] = fmaf(W.z, g, acc[j][m][1]);
                fmac2_next_lane(acc[j][m][0], acc[j][m][1], g, W.y, W.w);
            }
        }
    };
    // The stage loop, compiled once per (observers, sub-rows) of the wave: both are fixed for the
    // whole block, so the accumulators keep their registers across panels.  A wave without work
    // (NOBS = 0) still issues its share of the copies and meets every barrier.
    auto stage_loop = [&](auto nobs_c, auto nsub_c) {
        constexpr int NOBS = decltype(nobs_c)::value;
        constexpr int NSUB = decltype(nsub_c)::value;
        int cnt = 0;
        bool flushed = false;  // some chunk sum is already in the outputs
        if (pb < pe) fill(pb, stA);
        // one stage from buffer `cur` while the next one is copied into `nxt`
        auto stage = [&](int64_t ps, const unsigned char *cur, unsigned char *nxt) __attribute__((always_inline)) {
            const int np = (int)(pe - ps < PT ? pe - ps : PT);
            __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of stage ps have landed
            __syncthreads();                // ... and every wave's; the other buffer is free
            if (ps + PT < pe) fill(ps + PT, nxt);
            const unsigned char *base = cur;
            const float4 *lrec = reinterpret_cast<const float4 *>(base + (size_t)PT * win_bytes);
            for (int q = 0; q < np; ++q) {
                panel_work(nobs_c, nsub_c, lrec, base, (int)(q * win_bytes) + lane * EB, q);
                if (++cnt == kLdsChunk) {
#pragma unroll
                    for (int j = 0; j < NOBS; ++j)
#pragma unroll
                        for (int m = 0; m < NSUB; ++m) {
                            const float v = tap_sum(j, m);
                            float *dst = out_ptr(j, m);
                            if (dst) *dst = (flushed ? *dst : 0.f) + v;
                            acc[j][m][0] = acc[j][m][1] = 0.f;
                        }
                    flushed = true;
                    cnt = 0;
                }
            }
        };
        for (int64_t ps = pb; ps < pe; ps += 2 * PT) {
            stage(ps, stA, stB);
            if (ps + PT < pe) stage(ps + PT, stB, stA);
        }
        // final sums; outputs past an observer's window are zero
#pragma unroll
        for (int j = 0; j < OPW; ++j) {
            const int64_t o = tbase + slot_of(j);
            const int64_t ntl = o < O ? nt[o] : 0;
#pragma unroll
            for (int m = 0; m < SUBW; ++m) {
                const float v = tap_sum(j, m);
                float *dst = out_ptr(j, m);
                if (dst) {
                    const int64_t k = k0 + m * kLdsLanesOut + lane;
                    const float prev = (j < NOBS && m < NSUB && flushed) ? *dst : 0.f;
                    *dst = k < ntl ? prev + v : 0.f;
                }
            }
        }
    };
    // every record slot of the tile holds a valid record (slots past the last observer repeat
    // it); the wave skips the sub-rows past its observers' windows and the observer slots past its
    // last valid one.  Compiled (observers, sub-rows) pairs: 4 x 4 shape: observers 1, 2, 4 (3 runs
    // as 4), sub-rows 1 .. 4; 2 x 8 shape: observers 1, 2, sub-rows 2, 4, 6, 8 (odd counts run one
    // more sub-row, whose outputs lie past the windows and are not kept)
    auto by_sub = [&](auto nobs_c) {
        if constexpr (SUBW == 4) {
            switch (nsub) {
                case 1: stage_loop(nobs_c, std::integral_constant<int, 1>{}); break;
                case 2: stage_loop(nobs_c, std::integral_constant<int, 2>{}); break;
                case 3: stage_loop(nobs_c, std::integral_constant<int, 3>{}); break;
                default: stage_loop(nobs_c, std::integral_constant<int, 4>{}); break;
            }
        } else {
            static_assert(SUBW == 8, "wave shapes: 4 x 4 and 2 x 8");
            switch ((nsub + 1) >> 1) {
                case 1: stage_loop(nobs_c, std::integral_constant<int, 2>{}); break;
                case 2: stage_loop(nobs_c, std::integral_constant<int, 4>{}); break;
                case 3: stage_loop(nobs_c, std::integral_constant<int, 6>{}); break;
                default: stage_loop(nobs_c, std::integral_constant<int, 8>{}); break;
            }
        }
    };
    if (nobs == 0 || nsub == 0) {
        stage_loop(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    } else if constexpr (OPW == 4) {
        switch (nobs) {
            case 1: by_sub(std::integral_constant<int, 1>{}); break;
            case 2: by_sub(std::integral_constant<int, 2>{}); break;
            default: by_sub(std::integral_constant<int, 4>{}); break;
        }
    } else {
        static_assert(OPW == 2, "wave shapes: 4 x 4 and 2 x 8");
        if (nobs == 1) by_sub(std::integral_constant<int, 1>{});
        else by_sub(std::integral_constant<int, 2>{});
    }
}

// SB: bytes of each of the two stage buffers (a size class chosen at setup).  Up to 24 KiB
// three 8-wave blocks fit a CU (80 registers per lane, six waves per SIMD); 32 KiB buffers
// leave room for two.
constexpr int lds_waves_per_eu(int SB) { return SB <= 24576 ? 6 : 4; }

// SHAPE 0: 4 observers x 4 sub-rows per wave; SHAPE 1: 2 x 8.  Tiles t0 .. t0 + tiles - 1.
template <typename TS, int SB, int SHAPE>
__global__ __launch_bounds__(kLdsWaves * 64) __attribute__((amdgpu_waves_per_eu(lds_waves_per_eu(SB))))
void gather_lds_kernel(GatherArgs a, int64_t t0, int64_t tiles, int64_t kblocks) {
    __shared__ __align__(16) unsigned char stA[SB];
    __shared__ __align__(16) unsigned char stB[SB];
    // 1-D grid, block order (tile fastest, k block, split) regrouped per XCD
    const int64_t L = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = L % tiles, rest = L / tiles;
    if constexpr (SHAPE == 0)
        gather_lds_body<TS, 4, 4, true>(a, t0 + t, rest % kblocks, rest / kblocks, stA, stB);
    else
        gather_lds_body<TS, 2, 8>(a, t0 + t, rest % kblocks, rest / kblocks, stA, stB);
}

// Persistent batched gather: blocks pull work items (case, tile, k-block, split)
// in list order (longest first) through an atomic counter until the list is
// exhausted; every block ends when it draws an index past the list.
template <typename TS, int SB>
__global__ __launch_bounds__(kLdsWaves * 64) __attribute__((amdgpu_waves_per_eu(lds_waves_per_eu(SB)))) void gather_lds_persistent(const BatchCase *__restrict__ cases,
                                                                        const int4 *__restrict__ items,
                                                                        int n_items, int *__restrict__ counter) {
    __shared__ __align__(16) unsigned char stA[SB];
    __shared__ __align__(16) unsigned char stB[SB];
    __shared__ int cur;
    for (;;) {
        __syncthreads();  // the previous item is finished with LDS
        if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(cur);
        if (it >= n_items) break;
        const int4 w = items[it];
        const int c = __builtin_amdgcn_readfirstlane(w.x);
        gather_lds_body<TS>(cases[c].gat, __builtin_amdgcn_readfirstlane(w.y), __builtin_amdgcn_readfirstlane(w.z),
                            __builtin_amdgcn_readfirstlane(w.w), stA, stB);
    }
}

// Streaming gather for at most kLdsWaves observers: every panel's whole
// coefficient rows (both channel groups, NS indices) are staged once into LDS by
// direct global->LDS loads, double-buffered, and the block computes all samples
// of every observer from them: waves w and w + 8 share observer w, wave w taking
// the rows of 61 samples [0, NRH) and wave w + 8 the rows [NRH, 2 NRH), in
// registers.  Each coefficient leaves HBM once per panel split, which is what an
// HBM-bound case (few observers: about 4 bytes per panel-observer-sample against
// 24 flop) needs; the tiled gathers re-read overlapping windows per block of 244
// samples.  The two stage buffers are separate static arrays of BUF bytes (a
// size class of NS), so that reads of one do not wait for the copies into the other.
constexpr int kStreamWaves = 2 * kLdsWaves;
template <typename TS, int NRH, int BUF>
__global__ __launch_bounds__(kStreamWaves * 64) void gather_stream_kernel(GatherArgs a) {
    __shared__ __align__(16) unsigned char stA[BUF];
    __shared__ __align__(16) unsigned char stB[BUF];
    using QT = typename Quad<TS>::T;
    constexpr int EB = 4 * (int)sizeof(TS);  // bytes per element (4 channels of one group)
    constexpr bool kBf = std::is_same<TS, uint16_t>::value;
    const PairRec *__restrict__ rec = a.rec;
    const int32_t *__restrict__ nt = a.nt;
    const int64_t P = a.P, O = a.O, NS = a.NS, nt_max = a.nt_max, p_chunk = a.p_chunk;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jo = wv & (kLdsWaves - 1), half = wv / kLdsWaves;  // observer and row half of this wave
    const int64_t z = xcd_block(blockIdx.x, gridDim.x);
    const int64_t pb = z * p_chunk;
    const int64_t pe = pb + p_chunk < P ? pb + p_chunk : P;
    const int64_t o_last = O - 1;
    const size_t row_bytes = (size_t)NS * EB;  // one channel group of one panel
    const bool valid = jo <= o_last;
    const int ntw = valid ? nt[jo] : 0;
    const int r0 = half * NRH;  // first row of this wave
    int nrow = (ntw + kLdsLanesOut - 1) / kLdsLanesOut - r0;
    nrow = __builtin_amdgcn_readfirstlane(nrow < 0 ? 0 : (nrow > NRH ? NRH : nrow));

    auto fill = [&](int64_t p, unsigned char *base) {
        const unsigned char *src = reinterpret_cast<const unsigned char *>(a.coef) + (size_t)p * 2 * row_bytes;
        const int units = (int)(2 * row_bytes / 16);
        copy_to_lds<16, kStreamWaves>(src, units - 1, base, units, wv, lane);
        // records of the observers (slots past the last observer repeat it): 4 pieces of 16 bytes each
        unsigned char *rb = base + 2 * row_bytes;
        if (wv == 0 && lane < kLdsWaves * 4) {
            const int64_t j = (lane >> 2) < o_last ? (lane >> 2) : o_last;
            const float4 *sr = reinterpret_cast<const float4 *>(rec + j * P + p) + (lane & 3);
            __builtin_amdgcn_global_load_lds((const void *)sr, (lds_ptr_t)rb, 16, 0, 0);
        }
        if constexpr (kBf) {
            if (wv == 1 && lane < kLdsWaves * 2) {
                const int64_t j = (lane >> 1) < o_last ? (lane >> 1) : o_last;
                const uint4 *sb = reinterpret_cast<const uint4 *>(a.rbf + j * P + p) + (lane & 1);
                __builtin_amdgcn_global_load_lds((const void *)sb, (lds_ptr_t)(rb + kLdsWaves * sizeof(PairRec)),
                                                 16, 0, 0);
            }
        }
    };

    // BF16 (bound by VALU issue): four tap accumulators per row, the lane shifts of the taps applied
    // once per flush as in the LDS-staged gather.  FP32 (bound by HBM): one accumulator per row and
    // the shifts per panel, which keeps the 16-row form within its registers.
    constexpr int NT = kBf ? 4 : 1;
    float acc[NRH][NT];
#pragma unroll
    for (int r = 0; r < NRH; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[r][t] = 0.f;
    int cnt = 0;
    bool flushed = false;
    auto flush = [&](bool final_sums) {
        if (!valid) return;  // wave-uniform
        float *row = partial_row(a.partial, z, O, (int64_t)jo, nt_max);
#pragma unroll
        for (int r = 0; r < NRH; ++r) {
            float sum = acc[r][0];
            if constexpr (NT == 4) {
                float s3 = acc[r][3];
                s3 = acc[r][2] + from_next_lane(s3);
                s3 = acc[r][1] + from_next_lane(s3);
                sum = acc[r][0] + from_next_lane(s3);
            }
            const int k = (r0 + r) * kLdsLanesOut + lane;
            if (lane < kLdsLanesOut && k < nt_max) {
                const float prev = (flushed && r < nrow) ? row[k] : 0.f;
                const float v = r < nrow ? prev + sum : 0.f;
                row[k] = (!final_sums || k < ntw) ? v : 0.f;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[r][t] = 0.f;
        }
        flushed = true;
    };
    // panel p from buffer `cur` while panel p + 1 is copied into `nxt`
    auto panel = [&](int64_t p, const unsigned char *cur, unsigned char *nxt) __attribute__((always_inline)) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of panel p have landed
        __syncthreads();                // ... and every wave's; the other buffer is free
        if (p + 1 < pe) fill(p + 1, nxt);
        if (valid) {
            const int nr = nrow;
            const float4 *R = reinterpret_cast<const float4 *>(cur + 2 * row_bytes + (size_t)jo * sizeof(PairRec));
            const float4 W = R[2];
            // both groups' rows addressed from the buffer base (formed as P0 + NS, the second would make
            // the compiler wait for the copies into the other buffer before reading it)
            const int e0 = __float_as_int(R[3].x) + r0 * kLdsLanesOut + lane;
            const QT *P0 = reinterpret_cast<const QT *>(cur) + e0;
            const QT *P1 = reinterpret_cast<const QT *>(cur + row_bytes) + e0;
            float4 Ka, Kb;
            uint4 Kh, Kl;
            if constexpr (kBf) {
                const uint4 *B = reinterpret_cast<const uint4 *>(cur + 2 * row_bytes + kLdsWaves * sizeof(PairRec)) +
                                 jo * 2;
                Kh = B[0];
                Kl = B[1];
            } else {
                Ka = R[0];
                Kb = R[1];
            }
#pragma unroll
            for (int r = 0; r < NRH; ++r) {
                if (r < nr) {
                    float g;
                    if constexpr (kBf) {
                        const uint2 e0 = P0[r * kLdsLanesOut], e1 = P1[r * kLdsLanesOut];
                        g = dot2_bf16(Kh.x, e0.x, 0.f);
                        g = dot2_bf16(Kh.y, e0.y, g);
                        g = dot2_bf16(Kh.z, e1.x, g);
                        g = dot2_bf16(Kh.w, e1.y, g);
                        g = dot2_bf16(Kl.x, e0.x, g);
                        g = dot2_bf16(Kl.y, e0.y, g);
                        g = dot2_bf16(Kl.z, e1.x, g);
                        g = dot2_bf16(Kl.w, e1.y, g);
                    } else {
                        float c0[4], c1[4];
                        Quad<TS>::unpack(P0[r * kLdsLanesOut], c0);
                        Quad<TS>::unpack(P1[r * kLdsLanesOut], c1);
                        g = Ka.x * c0[0];
                        g = fmaf(Ka.y, c0[1], g);
                        g = fmaf(Ka.z, c0[2], g);
                        g = fmaf(Ka.w, c0[3], g);
                        g = fmaf(Kb.x, c1[0], g);
                        g = fmaf(Kb.y, c1[1], g);
                        g = fmaf(Kb.z, c1[2], g);
                        g = fmaf(Kb.w, c1[3], g);
                    }
                    if constexpr (NT == 4) {
                        acc[r][0] = fmaf(W.x, g, acc[r][0]);
                        acc[r][1] = fmaf(W.y, g, acc[r][1]);
                        acc[r][2] = fmaf(W.z, g, acc[r][2]);
                        acc[r][NT - 1] = fmaf(W.w, g, acc[r][NT - 1]);
                    } else {
                        const float g1 = from_next_lane(g);
                        const float g2 = from_next_lane(g1);
                        const float g3 = from_next_lane(g2);
                        float ac = acc[r][0];
                        ac = fmaf(W.x, g, ac);
                        ac = fmaf(W.y, g1, ac);
                        ac = fmaf(W.z, g2, ac);
                        ac = fmaf(W.w, g3, ac);
                        acc[r][0] = ac;
                    }
                }
            }
        }
        if (++cnt == kLdsChunk) {
            flush(false);
            cnt = 0;
        }
    };
    if (pb < pe) fill(pb, stA);
    for (int64_t p = pb; p < pe; p += 2) {
        panel(p, stA, stB);
        if (p + 1 < pe) panel(p + 1, stB, stA);
    }
    flush(true);
}

__global__ void reset_counter_kernel(int *counter) { counter[0] = 0; }

// Zero-padded copy of dJ/dp': gpad[o][k + padlo] = gbar[o][k] for 0 <= k < N_t(o), 0 elsewhere.
__device__ __forceinline__ void pad_grad_body(const PadArgs &a, int64_t i) {
    if (i >= a.O * a.LR) return;
    const int64_t o = i / a.LR;
    const int64_t k = i - o * a.LR - a.padlo;
    a.gpad[i] = (k >= 0 && k < a.nt[o]) ? a.gbar[o * a.nt_max + k] : 0.f;
}

__global__ __launch_bounds__(256) void pad_grad_kernel(PadArgs a) {
    pad_grad_body(a, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void pad_grad_batched(const BatchCase *__restrict__ cases,
                                                        const int64_t *__restrict__ start, int n) {
    const int c = find_case(start, n, blockIdx.x);
    pad_grad_body(cases[c].pad, ((int64_t)blockIdx.x - start[c]) * 256 + threadIdx.x);
}

// Transposed gather on the matrix cores.  For panel p and coefficient index i,
//   cbar_c(p, i) = sum_o K_c(o, p) H(o, i),  H(o, i) = sum_j w_j(o, p) gbar(o, i - n0(o, p) - j),
// a contraction over observers, one 16x16x4 FP32 MFMA per 4 observers and 16
// indices: A[m][k] = H(observer o + k, index m), B[k][n] = K_n(o + k, p) (zero for
// n >= 8), D[m][n] = the cbar contribution of channel n at index m.  The taps
// stay on the VALU: lane (q, s) of the wave (q = lane / 16, s = lane % 16) owns
// observer o + q and the 4 indices ib + 4 s + t (t = 0..3), loads gbar at the 4
// shifted positions with one 16-byte load, takes the 3 positions below from lane
// s - 1 of its row (a row shift; lane s = 0 takes them from lane 15's load of
// the previous block of 64, by a row rotation, and loads them for the first
// block), and forms H for its 4 indices.  MFMA t takes the rows m = s as index ib + 4 m + t, so lane (q', n)
// of its output holds channel n at indices ib + 16 q' + 4 r + t (r = 0..3): 16
// consecutive indices per lane over t and r, stored as 4 float4.
//
// A wave owns panel p and kAdjMW blocks of 64 indices.  Waves go in tiles of
// kAdjPT panels x all index blocks, panels fastest: the 4 waves of a block (and
// neighbouring blocks on one XCD) read the same observers' gbar windows a few
// samples apart and adjacent pair records, and a tile's records stay in L2 for
// all its index blocks.  Each row q fetches its pair record with one dword per lane (lane s:
// dword s of the 64-byte record, so lanes s < 8 hold K_s) and takes the taps and
// n0 from lanes 8..12 of the row by row broadcasts.
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float adj_row_rot(float x) {
    // lane s of each row of 16 receives lane s - 1 (mod 16); every lane has a source, so no old value
    // (and no move to set one) is needed
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x121 /* row_ror:1 */, 0xF, 0xF, false));
}

__device__ __forceinline__ float adj_row_prev(float x, float old) {
    // lane s of each row of 16 receives lane s - 1's x; lane 0 keeps `old`
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), 0x111 /* row_shr:1 */,
                                                      0xF, 0xF, false));
}

template <int LANE>
__device__ __forceinline__ float adj_row_bcast(float x) {
    // every lane of each row of 16 receives lane LANE of its row (no old value needed)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x150 + LANE /* row_newbcast */, 0xF, 0xF, false));
}

struct __attribute__((packed, aligned(4))) AdjF4 {
    float x, y, z, w;
};

// One group of 4 observers (one per row q of the wave): the row's pair record
// spread over its 16 lanes, and the gbar windows.
struct AdjGroup {
    float rv;          // dword s of the record of (o + q, p)
    AdjF4 x[kAdjMW];   // gbar at e .. e + 3, e = ib + 64 u + 4 s - n0
    AdjF4 pv;          // gbar at e - 4 .. e - 1 of block u = 0 (lane s = 0 only)
};

__device__ __forceinline__ void adj_gather_mfma_body(const AdjArgs &a, int64_t wave_id) {
    const int64_t P = a.P, O = a.O, NS = a.NS, LR = a.LR, nib = a.nib;
    if (wave_id >= P * nib) return;
    // tile of kAdjPT panels (the last one narrower) x nib index blocks, panels fastest
    const int64_t tile = wave_id / (kAdjPT * nib);
    const int64_t r = wave_id - tile * (kAdjPT * nib);
    const int64_t tw = min<int64_t>(kAdjPT, P - tile * kAdjPT);
    const int64_t bi = r / tw;
    const int64_t p = tile * kAdjPT + (r - bi * tw);
    const int64_t ib = bi * (64 * kAdjMW);
    const int nsub = (int)min<int64_t>(kAdjMW, (NS - ib) >> 6);  // NS is a multiple of 64
    const int lane = threadIdx.x & 63, q = lane >> 4, s = lane & 15;
    const float *g = a.gpad + a.padlo + ib + 4 * s;
    const float *rp = reinterpret_cast<const float *>(a.rec + p) + s;
    // index blocks past nsub load the last one again (in bounds) and skip their MFMAs
    int uoff[kAdjMW];
#pragma unroll
    for (int u = 0; u < kAdjMW; ++u) uoff[u] = 64 * min(u, nsub - 1);
    floatx4_t acc[kAdjMW][4];
#pragma unroll
    for (int u = 0; u < kAdjMW; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[u][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    // Loads run ahead of the arithmetic: while group o is on the VALU and the matrix cores, the
    // gbar windows of group o + 4 and the records of group o + 8 are in flight.  Observers past O
    // are clamped to O - 1 for the loads and get K = 0.
    constexpr int64_t kRecDwords = sizeof(PairRec) / 4;
    auto load_rec = [&](int64_t o) { return rp[min(o + q, O - 1) * P * kRecDwords]; };
    auto load_x = [&](int64_t o, AdjGroup &b) {
        const int n0 = __float_as_int(adj_row_bcast<12>(b.rv));
        const float *go = g + min(o + q, O - 1) * LR - n0;
#pragma unroll
        for (int u = 0; u < kAdjMW; ++u) b.x[u] = *reinterpret_cast<const AdjF4 *>(go + uoff[u]);
        // only lane 0 of each row uses pv; every lane loads it (in bounds: the row's lead pad holds
        // N + 4 floats and n0 <= N), so the register is not merged with its old value
        b.pv = *reinterpret_cast<const AdjF4 *>(go - 4);
    };
    // Waves near either end of the index range (check): 64-index blocks u_lo .. u_hi, those
    // that some observer of the group reaches (observer o + q adds to indices [n0, n0 + N_t + 2]
    // only; n0 from dword 12 of each row's record, N_t bounded by the longest window); the others
    // would get exact zeros and are skipped.  Inside [edge_lo, edge_hi] every block is reached.
    const bool check = ib < a.edge_lo || ib + 64 * kAdjMW - 1 > a.edge_hi;  // wave-uniform
    auto compute = [&](int64_t o, const AdjGroup &b) {
        const float kb = (o + q < O && s < 8) ? b.rv : 0.f;
        const float w0 = adj_row_bcast<8>(b.rv), w1 = adj_row_bcast<9>(b.rv), w2 = adj_row_bcast<10>(b.rv),
                    w3 = adj_row_bcast<11>(b.rv);
        int u_lo = 0, u_hi = nsub - 1;
        if (check) {
            int n0lo = __builtin_amdgcn_readlane(__float_as_int(b.rv), 12), n0hi = n0lo;
#pragma unroll
            for (int r = 1; r < 4; ++r) {
                const int v = __builtin_amdgcn_readlane(__float_as_int(b.rv), 16 * r + 12);
                n0lo = min(n0lo, v);
                n0hi = max(n0hi, v);
            }
            const int ibi = (int)ib;
            u_lo = max(0, (n0lo - ibi) >> 6);
            u_hi = min(nsub - 1, (n0hi + (int)a.nt_max + 2 - ibi) >> 6);
        }
#pragma unroll
        for (int u = 0; u < kAdjMW; ++u) {
            if (u >= u_lo && u <= u_hi) {
                const AdjF4 xv = b.x[u];
                // lane 0's values below e: its own load (u = 0) or lane 15's of block u - 1
                const AdjF4 &xp = b.x[u > 0 ? u - 1 : 0];
                const float o1 = u == 0 ? b.pv.w : adj_row_rot(xp.w);
                const float o2 = u == 0 ? b.pv.z : adj_row_rot(xp.z);
                const float o3 = u == 0 ? b.pv.y : adj_row_rot(xp.y);
                const float m1 = adj_row_prev(xv.w, o1);  // gbar at e - 1
                const float m2 = adj_row_prev(xv.z, o2);  // e - 2
                const float m3 = adj_row_prev(xv.y, o3);  // e - 3
                const float h0 = fmaf(w3, m3, fmaf(w2, m2, fmaf(w1, m1, w0 * xv.x)));
                const float h1 = fmaf(w3, m2, fmaf(w2, m1, fmaf(w1, xv.x, w0 * xv.y)));
                const float h2 = fmaf(w3, m1, fmaf(w2, xv.x, fmaf(w1, xv.y, w0 * xv.z)));
                const float h3 = fmaf(w3, xv.x, fmaf(w2, xv.y, fmaf(w1, xv.z, w0 * xv.w)));
                acc[u][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(h0, kb, acc[u][0], 0, 0, 0);
                acc[u][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(h1, kb, acc[u][1], 0, 0, 0);
                acc[u][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(h2, kb, acc[u][2], 0, 0, 0);
                acc[u][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(h3, kb, acc[u][3], 0, 0, 0);
            }
        }
    };
    // before step(o, cur, nxt): cur holds the record and windows of group o, nxt the record of
    // group o + 4.  Loads complete in issue order, so the record of o + 8 goes first: the next
    // step waits for it without waiting for the windows issued after it.
    auto step = [&](int64_t o, AdjGroup &cur, AdjGroup &nxt) {
        const float rnew = load_rec(o + 8);
        load_x(o + 4, nxt);
        compute(o, cur);
        cur.rv = rnew;
    };
    AdjGroup A, B;
    A.pv = B.pv = AdjF4{0.f, 0.f, 0.f, 0.f};
    A.rv = load_rec(0);
    B.rv = load_rec(4);
    load_x(0, A);
#pragma unroll 1
    for (int64_t o = 0; o < O; o += 8) {
        step(o, A, B);
        if (o + 4 >= O) break;
        step(o + 4, B, A);
    }
    if (s < 8) {
        float *out = a.cbar + ((int64_t)s * P + p) * NS + ib + 16 * q;
#pragma unroll
        for (int u = 0; u < kAdjMW; ++u)
            if (u < nsub) {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    *reinterpret_cast<float4 *>(out + 64 * u + 4 * rr) =
                        make_float4(acc[u][0][rr], acc[u][1][rr], acc[u][2][rr], acc[u][3][rr]);
            }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void adj_gather_mfma_kernel(AdjArgs a) {
    // consecutive blocks (neighbouring index blocks and panels) regrouped per XCD
    adj_gather_mfma_body(a, xcd_block(blockIdx.x, gridDim.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
}

// Batched transposed gather over a longest-first work list: block b runs item b,
// (case c, group g) = the waves 4 g .. 4 g + 3 of case c, wave w being (panel
// w / nib, index block w % nib); waves past the case's P * nib return at once.
// The items are sorted by their work (the paper's greedy partition by size) and
// blocks are dispatched in order, so every compute unit takes the longest item
// left when one of its blocks ends.  (A persistent form pulling items through a
// counter keeps the case arguments live across items: it needs more registers per
// lane than the three waves per SIMD this launch runs with allow.)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void adj_gather_listed(const BatchCase *__restrict__ cases,
                                                         const int2 *__restrict__ items) {
    const int2 w = items[blockIdx.x];
    const int c = __builtin_amdgcn_readfirstlane(w.x);
    const int64_t g = __builtin_amdgcn_readfirstlane(w.y);
    adj_gather_mfma_body(cases[c].adj, g * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
}

// out[o][k] = sum_z partial[z][o][k] in fixed order.  Eight loads are issued before they are
// added (the sum keeps its order), so each thread has eight reads in flight instead of one.
__device__ __forceinline__ float sum_splits(const float *__restrict__ partial, int splits, int64_t total,
                                            int64_t i) {
    double s = 0.0;
    int z = 0;
    for (; z + 8 <= splits; z += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = partial[(int64_t)(z + j) * total + i];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += (double)v[j];
    }
    for (; z < splits; ++z) s += (double)partial[(int64_t)z * total + i];
    return (float)s;
}

__device__ __forceinline__ void reduce_body(const ReduceArgs &a, int64_t i) {
    if (i >= a.total) return;
    a.out[i] = sum_splits(a.partial, a.splits, a.total, i);
}

__global__ __launch_bounds__(256) void reduce_batched(const BatchCase *__restrict__ cases,
                                                      const int64_t *__restrict__ start, int n) {
    const int c = find_case(start, n, blockIdx.x);
    reduce_body(cases[c].red, ((int64_t)blockIdx.x - start[c]) * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void reduce_splits_kernel(const float *__restrict__ partial, int splits,
                                                            int64_t total, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    out[i] = sum_splits(partial, splits, total, i);
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
                               int64_t O, int64_t NS, int64_t nt_max, int splits, float *partial,
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

hipError_t launch_gather_lds(int coef_type, const PairRec *rec_op, const PairBf *rbf, const int2 *tw, const int32_t *nt,
                             const void *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max, int splits, int NW,
                             int PT, float *partial, hipStream_t stream, int64_t t0, int64_t t1, int shape) {
    const int64_t p_chunk = (P + splits - 1) / splits;
    const GatherArgs a{rec_op, rbf, tw, nt, coef, P, O, NS, nt_max, p_chunk, NW, PT, splits, partial};
    const int64_t n_tiles = (O + kObsTile - 1) / kObsTile;
    if (t1 < 0) t1 = n_tiles;
    if (t0 < 0 || t1 > n_tiles || t0 >= t1 || shape < 0 || shape > 1) return hipErrorInvalidValue;
    const int64_t kb_len = shape == 0 ? kLdsK : 2 * kLdsK;
    const int64_t tiles = t1 - t0, kblocks = (nt_max + kb_len - 1) / kb_len;
    const dim3 n1((unsigned)(tiles * kblocks * splits)), blk(kLdsWaves * 64);
    const int sb = gather_lds_stage_class(coef_type, NW, PT, shape);
#define FWH_LDS_LAUNCH(T, S)                                                                   \
    (shape == 0 ? gather_lds_kernel<T, S, 0><<<n1, blk, 0, stream>>>(a, t0, tiles, kblocks)   \
                : gather_lds_kernel<T, S, 1><<<n1, blk, 0, stream>>>(a, t0, tiles, kblocks))
    if (coef_type == 1) {
        switch (sb) {
            case 8192: FWH_LDS_LAUNCH(float, 8192); break;
            case 12288: FWH_LDS_LAUNCH(float, 12288); break;
            case 16384: FWH_LDS_LAUNCH(float, 16384); break;
            case 24576: FWH_LDS_LAUNCH(float, 24576); break;
            case 32768: FWH_LDS_LAUNCH(float, 32768); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (sb) {
            case 8192: FWH_LDS_LAUNCH(uint16_t, 8192); break;
            case 12288: FWH_LDS_LAUNCH(uint16_t, 12288); break;
            case 16384: FWH_LDS_LAUNCH(uint16_t, 16384); break;
            case 24576: FWH_LDS_LAUNCH(uint16_t, 24576); break;
            case 32768: FWH_LDS_LAUNCH(uint16_t, 32768); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef FWH_LDS_LAUNCH
    return hipGetLastError();
}

// Stage buffer size classes of the streaming gather: both channel groups of a
// panel's row (NS <= NSMAX indices) plus the records of kLdsWaves observers.
constexpr int kStreamNs32[2] = {1216, 2496};   // FP32 storage
constexpr int kStreamNs16[2] = {2496, 5056};   // BF16 storage
constexpr int stream_buf(int eb, int nsmax, int rb) { return 2 * nsmax * eb + rb; }
constexpr int kRb32 = kLdsWaves * (int)sizeof(PairRec);
constexpr int kRb16 = kLdsWaves * (int)(sizeof(PairRec) + sizeof(PairBf));

size_t gather_stream_shmem(int coef_type, int64_t NS) {
    const int *cls = coef_type == 1 ? kStreamNs32 : kStreamNs16;
    for (int i = 0; i < 2; ++i)
        if (NS <= cls[i])
            return 2 * (size_t)stream_buf(coef_type == 1 ? 16 : 8, cls[i], coef_type == 1 ? kRb32 : kRb16);
    return 0;
}

// rows of 61 samples per wave (two waves per observer), 0 when an observer has more than 32 rows
// (the row loop is fully unrolled with the accumulators in registers)
int gather_stream_rows(int64_t nt_max) {
    const int64_t r = (nt_max + kLdsLanesOut - 1) / kLdsLanesOut;
    return r <= 16 ? 8 : r <= 32 ? 16 : 0;
}

// kernel of (storage, rows, NS class), null when the combination is not compiled
template <typename TS>
static const void *stream_kernel(int nr, int cls) {
#define FWH_SK(N, C) reinterpret_cast<const void *>(&gather_stream_kernel<TS, N, C>)
    constexpr bool f32 = std::is_same<TS, float>::value;
    constexpr int eb = f32 ? 16 : 8, rb = f32 ? kRb32 : kRb16;
    constexpr int c0 = stream_buf(eb, f32 ? kStreamNs32[0] : kStreamNs16[0], rb);
    constexpr int c1 = stream_buf(eb, f32 ? kStreamNs32[1] : kStreamNs16[1], rb);
    if (cls == 0) return nr == 8 ? FWH_SK(8, c0) : nr == 16 ? FWH_SK(16, c0) : nullptr;
    return nr == 8 ? FWH_SK(8, c1) : nr == 16 ? FWH_SK(16, c1) : nullptr;
#undef FWH_SK
}

static int stream_class(int coef_type, int64_t NS) {
    const int *cls = coef_type == 1 ? kStreamNs32 : kStreamNs16;
    return NS <= cls[0] ? 0 : NS <= cls[1] ? 1 : -1;
}

hipError_t launch_gather_stream(int coef_type, const PairRec *rec_op, const PairBf *rbf, const int32_t *nt,
                                const void *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max, int splits,
                                float *partial, hipStream_t stream) {
    const int nr = gather_stream_rows(nt_max), cls = stream_class(coef_type, NS);
    if (O > kLdsWaves || nr == 0 || cls < 0) return hipErrorInvalidValue;
    const void *k = coef_type == 1 ? stream_kernel<float>(nr, cls) : stream_kernel<uint16_t>(nr, cls);
    if (!k) return hipErrorInvalidValue;
    const int64_t p_chunk = (P + splits - 1) / splits;
    GatherArgs a{rec_op, rbf, nullptr, nt, coef, P, O, NS, nt_max, p_chunk, 0, 0, splits, partial, 0};
    void *args[] = {&a};
    return hipLaunchKernel(k, dim3((unsigned)splits), dim3(kStreamWaves * 64), args, 0, stream);
}

int gather_stream_blocks_per_cu(int coef_type, int64_t NS, int64_t nt_max) {
    const int nr = gather_stream_rows(nt_max), cls = stream_class(coef_type, NS);
    if (nr == 0 || cls < 0) return 0;
    const void *k = coef_type == 1 ? stream_kernel<float>(nr, cls) : stream_kernel<uint16_t>(nr, cls);
    if (!k) return 0;
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kStreamWaves * 64, 0);
    return e == hipSuccess && n > 0 ? n : 0;
}

int gather_lds_stage_class(int coef_type, int NW, int PT, int shape) {
    const size_t need = gather_lds_shmem(coef_type, NW, PT, shape) / 2;  // one of the two stage buffers
    for (int sb : {8192, 12288, 16384, 24576, 32768})
        if (need <= (size_t)sb) return sb;
    return 0;
}

template <typename T, int SHAPE>
static const void *lds_kernel_ptr(int sb) {
    switch (sb) {
        case 8192: return reinterpret_cast<const void *>(&gather_lds_kernel<T, 8192, SHAPE>);
        case 12288: return reinterpret_cast<const void *>(&gather_lds_kernel<T, 12288, SHAPE>);
        case 16384: return reinterpret_cast<const void *>(&gather_lds_kernel<T, 16384, SHAPE>);
        case 24576: return reinterpret_cast<const void *>(&gather_lds_kernel<T, 24576, SHAPE>);
        default: return reinterpret_cast<const void *>(&gather_lds_kernel<T, 32768, SHAPE>);
    }
}

int gather_lds_blocks_per_cu(int coef_type, int NW, int PT, int shape) {
    const int sb = gather_lds_stage_class(coef_type, NW, PT, shape);
    if (sb == 0) return 1;
    const void *k = coef_type == 1 ? (shape == 0 ? lds_kernel_ptr<float, 0>(sb) : lds_kernel_ptr<float, 1>(sb))
                                   : (shape == 0 ? lds_kernel_ptr<uint16_t, 0>(sb) : lds_kernel_ptr<uint16_t, 1>(sb));
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kLdsWaves * 64, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_reduce_splits(const float *partial, int splits, int64_t total, float *out, hipStream_t stream) {
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

hipError_t launch_adj_gather(const PairRec *rec_op, const int32_t *nt, const float *gbar, int64_t P, int64_t O,
                                 int64_t N, int64_t NS, int64_t nt_min, int64_t nt_max, float *gpad, float *cbar,
                                 hipStream_t stream) {
    const int64_t edge_lo = N - nt_min, edge_hi = nt_min + 2;
    const int64_t LR = adj_pad_row(N, NS), padlo = adj_pad_lo(N);
    const PadArgs pa{gbar, nt, O, nt_max, LR, padlo, gpad};
    pad_grad_kernel<<<dim3((unsigned)((O * LR + 255) / 256)), dim3(256), 0, stream>>>(pa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nib = adj_blocks(NS);
    const AdjArgs aa{rec_op, gpad, P, O, NS, LR, padlo, nib, cbar, nt_max, edge_lo, edge_hi};
    adj_gather_mfma_kernel<<<dim3((unsigned)((P * nib + 3) / 4)), dim3(256), 0, stream>>>(aa);
    return hipGetLastError();
}

hipError_t launch_batch_forward(int in_dtype, int coef_type, int umax, const BatchCase *cases, BatchIndex idx,
                                const int4 *items, int n_items, int *counter, int grid, size_t shmem,
                                int64_t blocks_src, int64_t blocks_srcg, int64_t blocks_red, hipStream_t stream) {
    hipError_t e =
        launch_batch_source(in_dtype, coef_type, cases, idx.src, idx.srcg, idx.n, blocks_src, blocks_srcg, stream);
    if (e != hipSuccess) return e;
    reset_counter_kernel<<<1, 1, 0, stream>>>(counter);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (umax > 0)
        e = launch_gather_mfma_persistent(coef_type, umax, cases, items, n_items, counter, grid, shmem, stream);
    else {
        // stage buffers of the widest case: shmem holds both of them
        int sb = 0;
        for (int c : {8192, 12288, 16384, 24576, 32768})
            if (sb == 0 && shmem / 2 <= (size_t)c) sb = c;
        const dim3 g((unsigned)grid), blk(kLdsWaves * 64);
#define FWH_LDS_PERSIST(T, S) gather_lds_persistent<T, S><<<g, blk, 0, stream>>>(cases, items, n_items, counter)
        if (coef_type == 1) {
            switch (sb) {
                case 8192: FWH_LDS_PERSIST(float, 8192); break;
                case 12288: FWH_LDS_PERSIST(float, 12288); break;
                case 16384: FWH_LDS_PERSIST(float, 16384); break;
                case 24576: FWH_LDS_PERSIST(float, 24576); break;
                case 32768: FWH_LDS_PERSIST(float, 32768); break;
                default: return hipErrorInvalidValue;
            }
        } else {
            switch (sb) {
                case 8192: FWH_LDS_PERSIST(uint16_t, 8192); break;
                case 12288: FWH_LDS_PERSIST(uint16_t, 12288); break;
                case 16384: FWH_LDS_PERSIST(uint16_t, 16384); break;
                case 24576: FWH_LDS_PERSIST(uint16_t, 24576); break;
                case 32768: FWH_LDS_PERSIST(uint16_t, 32768); break;
                default: return hipErrorInvalidValue;
            }
        }
#undef FWH_LDS_PERSIST
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    reduce_batched<<<dim3((unsigned)blocks_red), dim3(256), 0, stream>>>(cases, idx.red, idx.n);
    return hipGetLastError();
}

hipError_t launch_batch_adjoint(int in_dtype, const BatchCase *cases, BatchIndex idx, int64_t blocks_pad,
                                const int2 *adj_items, int n_adj_items, int64_t blocks_sadj, int64_t blocks_sadjg,
                                hipStream_t stream) {
    pad_grad_batched<<<dim3((unsigned)blocks_pad), dim3(256), 0, stream>>>(cases, idx.pad, idx.n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    adj_gather_listed<<<dim3((unsigned)n_adj_items), dim3(256), 0, stream>>>(cases, adj_items);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_batch_source_adjoint(in_dtype, cases, idx.sadj, idx.sadjg, idx.n, blocks_sadj, blocks_sadjg, stream);
}

}  // namespace fwh
