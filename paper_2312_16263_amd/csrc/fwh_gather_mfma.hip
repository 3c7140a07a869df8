// Forward gather with the channel combine on the matrix cores (gfx950).
//
// The surface sum of Sec. III C after the change of frame is, per observer o
// and sample k,
//   p'(o, k) = sum_p sum_jj w_jj(o,p) Y_p(o, n0(o,p) + k + jj),
//   Y_p(o, i) = sum_c K_c(o,p) coef_c(p, i),
// with fixed taps w, weights K and delay index n0 per (observer, panel) pair.
// For one panel and a tile of 32 observers, Y_p over a window of coefficient
// indices is a small dense product (32 observers x 8 channels) x (8 channels x
// window): that part runs as matrix-core instructions, 16 observers x 16
// indices per unit (v_mfma_f32_16x16x4f32, twice, in FP32 storage;
// v_mfma_f32_16x16x16bf16_1k with the weights split into bfloat16 high and low
// parts, once, in BF16 storage: products of bfloat16 values are exact in FP32,
// so both forms accumulate exact products in FP32).  Y goes through LDS; each
// observer then reads it at its own delay index and applies the four taps on
// the vector ALU (one LDS read, three wavefront shifts, four FMA per lane and
// 61 outputs), where the LDS-staged gather spent two 16-byte LDS reads and 12
// FMA per output.
//
// Block = kLdsWaves waves, observer tile t (32 observers), samples k0 ..
// k0 + 61 * kLdsSub - 1, panels [z*p_chunk, ...).  Per panel:
//   1. matrix units: unit u = (observer half u & 1, index block u >> 1) of the
//      panel's window [lo + k0, lo + k0 + 16 * nblk), lo = min n0 over the tile;
//      wave w takes u = w, w + 8, ...; operands were loaded during the previous
//      panel; the 16 x 16 result goes to Y[observer][index] in LDS;
//   2. barrier; the operands of the next panel are loaded meanwhile;
//   3. taps: wave w, observers w, w + 8, w + 16, w + 24 of the tile (the valid
//      ones), lane l of row m reads Y[j][n0_j - lo + 61 m + l];
//   4. barrier (Y is rewritten by the next panel).
// FP32 sums over kLdsChunk panels go into the split's partial signal, as in the
// other gathers; the split sums are added in FP64 by the reduction kernel.
#include <type_traits>

#include "fwh_internal.h"

namespace fwh {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaChunk = 256;  // panels summed in FP32 before adding into the partial signal

// Value of lane l+1 (wavefront shift by one lane; lane 63 receives 0).
__device__ __forceinline__ float next_lane(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130 /* wave_shl:1 */, 0xF, 0xF, true));
}

// Barrier for LDS data only: the waves' LDS writes are complete and visible
// after it; outstanding global loads (the next panel's operands) stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Operands of one matrix unit: the lane's coefficient values (A) for the unit's
// 16 indices.  FP32: lane (li, lq) holds channel lq of group 0 and of group 1 at
// index li; BF16: the four channels of group lq & 1 at index li (lanes 32..63
// repeat lanes 0..31 against the low parts of the weights).
template <typename TS>
struct MfmaA;
template <>
struct MfmaA<float> {
    float a0, a1;
};
template <>
struct MfmaA<uint16_t> {
    uint2 a;
};

template <typename TS, int UMAX>
__device__ __forceinline__ void gather_mfma_body(const GatherArgs &a, int64_t t, int64_t kb, int64_t z,
                                                 float *__restrict__ Y) {
    constexpr bool kBf = std::is_same<TS, uint16_t>::value;
    const PairRec *__restrict__ rec = a.rec;
    const int2 *__restrict__ tw = a.tw;
    const int32_t *__restrict__ nt = a.nt;
    const TS *__restrict__ coef = static_cast<const TS *>(a.coef);
    const int64_t P = a.P, O = a.O, NS = a.NS, nt_max = a.nt_max, p_chunk = a.p_chunk;
    const int YR = a.NW;      // row length (floats) of the Y tile
    const int rows = a.rows;  // rows of 61 samples per block
    float *__restrict__ partial = a.partial;
    // the tile's pair records (and BF16 split weights) of one panel, two buffers after the Y tile
    unsigned char *recs = reinterpret_cast<unsigned char *>(Y + kObsTile * YR);
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lq = lane >> 4;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t k0 = kb * kLdsLanesOut * rows;
    const int64_t pb = z * p_chunk;
    const int64_t pe = pb + p_chunk < P ? pb + p_chunk : P;
    const int64_t tbase = t * kObsTile;
    const int2 *twt = tw + t * P;
    const int64_t ot_last = (O - 1 - tbase) < kObsTile - 1 ? (O - 1 - tbase) : kObsTile - 1;

    // rows of 61 samples below the longest window of the tile (the matrix units cover them) and,
    // for this wave's observers (a prefix j < nobs of wv, wv + 8, ...), below the longest of theirs
    int nt_tile = 0, nt_wave = 0, nobs = 0;
    for (int j = 0; j <= ot_last; ++j) {
        const int n = nt[tbase + j];
        nt_tile = n > nt_tile ? n : nt_tile;
        if ((j & (kLdsWaves - 1)) == wv) {
            nt_wave = n > nt_wave ? n : nt_wave;
            nobs = j / kLdsWaves + 1;
        }
    }
    auto rows_below = [&](int n) {
        int r = (int)((n - k0 + kLdsLanesOut - 1) / kLdsLanesOut);
        return __builtin_amdgcn_readfirstlane(r < 0 ? 0 : (r > rows ? rows : r));
    };
    const int nsub_blk = rows_below(nt_tile);
    const int nsub = rows_below(nt_wave);
    nobs = __builtin_amdgcn_readfirstlane(nobs);

    // this wave's outputs of observer slot j: the split's partial signal row (uniform) and the lane's
    // sample offsets k0 + 61 m + lane; the row address is formed where it is used (an empty asm makes
    // it opaque, so that it is not kept live across the panel loop)
    auto out_row = [&](int j) -> float * {
        float *row = partial + (z * O + tbase + j * kLdsWaves + wv) * nt_max;
        asm volatile("" : "+s"(row));
        return row;
    };
    const int k_lane = (int)k0 + lane;
    const bool lane_out = lane < kLdsLanesOut;

    // window start and width of panel p (lane q of `win` holds panel ps + q)
    auto load_win = [&](int64_t ps) {
        const int64_t q = ps + lane < pe ? ps + lane : pe - 1;
        return twt[q];
    };
    auto n_units = [&](int width) {
        return 2 * ((width + kLdsLanesOut * nsub_blk + kLdsHalo + 15) / 16);
    };

    // Records of a panel through registers: waves 0 and 1 load the 32 records (128 pieces of 16
    // bytes), wave 2 in BF16 the 32 split weights (64 pieces), while the taps of the previous panel
    // run, and write them to the panel's record buffer afterwards.  (Direct global->LDS loads would
    // make the compiler wait for them before the taps' LDS reads.)
    constexpr int kRecBytes = kObsTile * (int)sizeof(PairRec);
    constexpr int kRecBuf = kRecBytes + (kBf ? kObsTile * (int)sizeof(PairBf) : 0);
    uint4 rstage = make_uint4(0u, 0u, 0u, 0u);
    auto load_recs = [&](int64_t p) {
        if (wv < 2) {
            const int u = wv * 64 + lane, j = u >> 2;
            const int64_t o = tbase + (j < ot_last ? j : ot_last);
            rstage = reinterpret_cast<const uint4 *>(rec + o * P + p)[u & 3];
        } else if (kBf && wv == 2) {
            const int j = lane >> 1;
            const int64_t o = tbase + (j < ot_last ? j : ot_last);
            rstage = reinterpret_cast<const uint4 *>(a.rbf + o * P + p)[lane & 1];
        }
    };
    auto store_recs = [&](int b) {
        unsigned char *rb = recs + b * kRecBuf;
        if (wv < 2) reinterpret_cast<uint4 *>(rb)[wv * 64 + lane] = rstage;
        else if (kBf && wv == 2) reinterpret_cast<uint4 *>(rb + kRecBytes)[lane] = rstage;
    };

    MfmaA<TS> A[UMAX];
    // issue the coefficient loads of panel p (window start lo, width) for this wave's units: a
    // uniform base per channel group and 32-bit byte offsets within the panel's rows
    const uint32_t row_bytes = (uint32_t)NS * 4u * (uint32_t)sizeof(TS);
    const int ci_max = (int)NS - 1;
    const int ci_lane = (int)k0 + li;
    auto load_ops = [&](int64_t p, int lo, int width) {
        const int nu = n_units(width);
        const unsigned char *g0 = reinterpret_cast<const unsigned char *>(coef) + (size_t)p * 2 * row_bytes;
        const unsigned char *g1 = g0 + row_bytes;
#pragma unroll
        for (int s = 0; s < UMAX; ++s) {
            const int u = wv + kLdsWaves * s;
            if (u < nu) {
                int ci = lo + ci_lane + 16 * (u >> 1);
                ci = ci < ci_max ? ci : ci_max;  // indices past the row are never read by valid outputs
                if constexpr (kBf) {
                    const uint32_t off = (uint32_t)ci * 8u;
                    A[s].a = *reinterpret_cast<const uint2 *>(((lq & 1) ? g1 : g0) + off);
                } else {
                    const uint32_t off = ((uint32_t)ci * 4u + (uint32_t)lq) * 4u;
                    A[s].a0 = *reinterpret_cast<const float *>(g0 + off);
                    A[s].a1 = *reinterpret_cast<const float *>(g1 + off);
                }
            }
        }
    };
    // matrix units of the panel whose operands are loaded: Y[16 h + li][16 (u >> 1) + 4 lq + r], the
    // weights (B operand) of observer 16 h + li read from the record buffer: FP32 channels lq and
    // 4 + lq; BF16 the high (lq < 2) or low parts of channel block lq & 1.  All products are issued
    // before the first result is written.
    const int h = wv & 1;
    float *ybase = Y + (16 * h + li) * YR + 4 * lq;
    auto mma_units = [&](int width, int b) {
        const int nu = n_units(width);
        const unsigned char *rb = recs + b * kRecBuf;
        uint2 bb = make_uint2(0u, 0u);
        float b0 = 0.f, b1 = 0.f;
        if constexpr (kBf) {
            bb = reinterpret_cast<const uint2 *>(rb + kRecBytes + (16 * h + li) * sizeof(PairBf))[lq];
        } else {
            const float *K = reinterpret_cast<const float *>(rb + (16 * h + li) * sizeof(PairRec));
            b0 = K[lq];
            b1 = K[4 + lq];
        }
        // two units at a time: their products are issued before either result is written
#pragma unroll
        for (int s = 0; s < UMAX; s += 2) {
            const bool v0 = wv + kLdsWaves * s < nu, v1 = wv + kLdsWaves * (s + 1) < nu;
            floatx4 d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
            if constexpr (kBf) {
                if (v0)
                    d0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(shortx4, A[s].a),
                                                                   __builtin_bit_cast(shortx4, bb), d0, 0, 0, 0);
                if (v1)
                    d1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(shortx4, A[s + 1].a),
                                                                   __builtin_bit_cast(shortx4, bb), d1, 0, 0, 0);
            } else {
                if (v0) d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(A[s].a0, b0, d0, 0, 0, 0);
                if (v1) d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(A[s + 1].a0, b0, d1, 0, 0, 0);
                if (v0) d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(A[s].a1, b1, d0, 0, 0, 0);
                if (v1) d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(A[s + 1].a1, b1, d1, 0, 0, 0);
            }
            if (v0) *reinterpret_cast<floatx4 *>(ybase + 16 * ((wv + kLdsWaves * s) >> 1)) = d0;
            if (v1) *reinterpret_cast<floatx4 *>(ybase + 16 * ((wv + kLdsWaves * (s + 1)) >> 1)) = d1;
        }
    };

    float acc[kObsPerWave][kLdsSub];
#pragma unroll
    for (int j = 0; j < kObsPerWave; ++j)
#pragma unroll
        for (int m = 0; m < kLdsSub; ++m) acc[j][m] = 0.f;

    // the panel loop, compiled once per (observers, rows) of the wave; a wave without taps (NOBS = 0)
    // still does its matrix units and record staging and meets every barrier
    auto panel_loop = [&](auto nobs_c, auto nsub_c) {
        constexpr int NOBS = decltype(nobs_c)::value;
        constexpr int NSUB = decltype(nsub_c)::value;
        int cnt = 0;
        bool flushed = false;
        int2 win = make_int2(0, 0);
        if (pb < pe) {  // an empty split (possible when P < splits * p_chunk) loads nothing
            load_recs(pb);
            win = load_win(pb);
            const int lo = __builtin_amdgcn_readlane(win.x, 0), hi = __builtin_amdgcn_readlane(win.y, 0);
            load_ops(pb, lo, hi - lo);
            store_recs(0);
            lds_barrier();
        }
        for (int64_t p = pb; p < pe; ++p) {
            const int q = (int)((p - pb) & 63), b = (int)((p - pb) & 1);
            const int lo = __builtin_amdgcn_readlane(win.x, q), hi = __builtin_amdgcn_readlane(win.y, q);
            mma_units(hi - lo, b);
            // next panel's records, window and operands, in flight during the taps
            const bool more = p + 1 < pe;
            if (more) {
                load_recs(p + 1);
                if (q == 63) win = load_win(p + 1);
                const int q1 = (int)((p + 1 - pb) & 63);
                const int lo1 = __builtin_amdgcn_readlane(win.x, q1), hi1 = __builtin_amdgcn_readlane(win.y, q1);
                load_ops(p + 1, lo1, hi1 - lo1);
            }
            lds_barrier();
            // taps, weights and delay indices of this wave's observers from the record buffer
            const unsigned char *rb = recs + b * kRecBuf;
#pragma unroll
            for (int j = 0; j < NOBS; ++j) {
                const unsigned char *r = rb + (j * kLdsWaves + wv) * sizeof(PairRec);
                const float4 W = *reinterpret_cast<const float4 *>(r + 32);
                const int d = *reinterpret_cast<const int *>(r + 48) - lo;
                const float *y = Y + (j * kLdsWaves + wv) * YR + d + lane;
#pragma unroll
                for (int m = 0; m < NSUB; ++m) {
                    const float g = y[m * kLdsLanesOut];
                    const float g1 = next_lane(g);
                    const float g2 = next_lane(g1);
                    const float g3 = next_lane(g2);
                    float ac = acc[j][m];
                    ac = fmaf(W.x, g, ac);
                    ac = fmaf(W.y, g1, ac);
                    ac = fmaf(W.z, g2, ac);
                    ac = fmaf(W.w, g3, ac);
                    acc[j][m] = ac;
                }
            }
            if (more) store_recs(b ^ 1);
            lds_barrier();
            if (++cnt == kMfmaChunk) {
#pragma unroll
                for (int j = 0; j < NOBS; ++j) {
                    float *row = out_row(j);
#pragma unroll
                    for (int m = 0; m < NSUB; ++m) {
                        const int k = k_lane + m * kLdsLanesOut;
                        if (lane_out && k < nt_max) row[k] = (flushed ? row[k] : 0.f) + acc[j][m];
                        acc[j][m] = 0.f;
                    }
                }
                flushed = true;
                cnt = 0;
            }
        }
        // final sums; outputs past an observer's window are zero (only this block's `rows` rows: the
        // next ones belong to the next k block)
#pragma unroll
        for (int j = 0; j < kObsPerWave; ++j) {
            if (tbase + j * kLdsWaves + wv >= O) continue;
            const int ntl = nt[tbase + j * kLdsWaves + wv];
            float *row = out_row(j);
#pragma unroll
            for (int m = 0; m < kLdsSub; ++m) {
                const int k = k_lane + m * kLdsLanesOut;
                if (m < rows && lane_out && k < nt_max) {
                    const float prev = (j < NOBS && m < NSUB && flushed) ? row[k] : 0.f;
                    row[k] = k < ntl ? prev + acc[j][m] : 0.f;
                }
            }
        }
    };
    auto by_sub = [&](auto nobs_c) {
        switch (nsub) {
            case 1: panel_loop(nobs_c, std::integral_constant<int, 1>{}); break;
            case 2: panel_loop(nobs_c, std::integral_constant<int, 2>{}); break;
            case 3: panel_loop(nobs_c, std::integral_constant<int, 3>{}); break;
            default: panel_loop(nobs_c, std::integral_constant<int, kLdsSub>{}); break;
        }
    };
    if (nsub_blk == 0) {
        // no sample of this block lies in a window of the tile: zeros (every wave, no barrier)
#pragma unroll
        for (int j = 0; j < kObsPerWave; ++j) {
            if (tbase + j * kLdsWaves + wv >= O) continue;
            float *row = out_row(j);
#pragma unroll
            for (int m = 0; m < kLdsSub; ++m) {
                const int k = k_lane + m * kLdsLanesOut;
                if (m < rows && lane_out && k < nt_max) row[k] = 0.f;
            }
        }
        return;
    }
    if (nobs == 0 || nsub == 0) {
        panel_loop(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    } else {
        switch (nobs) {
            case 1: by_sub(std::integral_constant<int, 1>{}); break;
            case 2: by_sub(std::integral_constant<int, 2>{}); break;
            default: by_sub(std::integral_constant<int, kObsPerWave>{}); break;
        }
    }
}

// four waves per SIMD (two blocks per compute unit): at most 128 VGPRs, a few of them spilled
template <typename TS, int UMAX>
__global__ __launch_bounds__(kLdsWaves * 64) __attribute__((amdgpu_waves_per_eu(4))) void gather_mfma_kernel(
    GatherArgs a, int64_t tiles, int64_t kblocks) {
    extern __shared__ __align__(16) float ysm[];
    // 1-D grid, block order (tile fastest, k block, split) regrouped per XCD
    const int64_t L = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = L % tiles, rest = L / tiles;
    gather_mfma_body<TS, UMAX>(a, t, rest % kblocks, rest / kblocks, ysm);
}

// Persistent batched form: blocks pull work items (case, tile, k block, split) in
// list order (longest first) through an atomic counter until the list is
// exhausted; each item runs the body above on its case's arguments.  The Y tile
// is reused from item to item (the loop-top barrier orders the last reads of one
// item before the first writes of the next).
template <typename TS, int UMAX>
__global__ __launch_bounds__(kLdsWaves * 64) __attribute__((amdgpu_waves_per_eu(4))) void gather_mfma_persistent(
    const BatchCase *__restrict__ cases,
                                                                         const int4 *__restrict__ items, int n_items,
                                                                         int *__restrict__ counter) {
    extern __shared__ __align__(16) float ysm[];
    __shared__ int cur;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(cur);
        if (it >= n_items) break;
        const int4 w = items[it];
        const int c = __builtin_amdgcn_readfirstlane(w.x);
        gather_mfma_body<TS, UMAX>(cases[c].gat, __builtin_amdgcn_readfirstlane(w.y),
                                   __builtin_amdgcn_readfirstlane(w.z), __builtin_amdgcn_readfirstlane(w.w), ysm);
    }
}

template <typename TS, int UMAX>
const void *persistent_ptr() {
    return reinterpret_cast<const void *>(&gather_mfma_persistent<TS, UMAX>);
}

template <typename TS, int UMAX>
const void *mfma_kernel_ptr() {
    return reinterpret_cast<const void *>(&gather_mfma_kernel<TS, UMAX>);
}

}  // namespace

int gather_mfma_umax(int wmax) {
    const int nu = 2 * ((wmax + kLdsK + kLdsHalo + 15) / 16);
    const int per_wave = (nu + kLdsWaves - 1) / kLdsWaves;
    return per_wave <= 4 ? 4 : (per_wave <= 6 ? 6 : (per_wave <= 8 ? 8 : 0));
}

int gather_mfma_blocks_per_cu(int coef_type, int wmax) {
    const int umax = gather_mfma_umax(wmax);
    if (umax == 0) return 0;
    const size_t shmem = gather_mfma_shmem(wmax);
    const void *k = nullptr;
    if (coef_type == 1) k = umax == 4 ? mfma_kernel_ptr<float, 4>() : umax == 6 ? mfma_kernel_ptr<float, 6>()
                                                                               : mfma_kernel_ptr<float, 8>();
    else k = umax == 4 ? mfma_kernel_ptr<uint16_t, 4>() : umax == 6 ? mfma_kernel_ptr<uint16_t, 6>()
                                                                    : mfma_kernel_ptr<uint16_t, 8>();
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kLdsWaves * 64, shmem);
    return e == hipSuccess && n > 0 ? n : 0;
}

hipError_t launch_gather_mfma(int coef_type, const PairRec *rec_op, const PairBf *rbf, const int2 *tw,
                              const int32_t *nt, const void *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max,
                              int splits, int wmax, float *partial, hipStream_t stream) {
    const int64_t p_chunk = (P + splits - 1) / splits;
    const int YR = gather_mfma_y_row(wmax);
    const GatherArgs a{rec_op, rbf, tw, nt, coef, P, O, NS, nt_max, p_chunk, YR, 0, splits, partial, kLdsSub};
    const int64_t tiles = (O + kObsTile - 1) / kObsTile, kblocks = (nt_max + kLdsK - 1) / kLdsK;
    const dim3 n1((unsigned)(tiles * kblocks * splits));
    const size_t shmem = gather_mfma_shmem(wmax);
    const int umax = gather_mfma_umax(wmax);
    const dim3 blk(kLdsWaves * 64);
    if (coef_type == 1) {
        if (umax == 4) gather_mfma_kernel<float, 4><<<n1, blk, shmem, stream>>>(a, tiles, kblocks);
        else if (umax == 6) gather_mfma_kernel<float, 6><<<n1, blk, shmem, stream>>>(a, tiles, kblocks);
        else if (umax == 8) gather_mfma_kernel<float, 8><<<n1, blk, shmem, stream>>>(a, tiles, kblocks);
        else return hipErrorInvalidValue;
    } else {
        if (umax == 4) gather_mfma_kernel<uint16_t, 4><<<n1, blk, shmem, stream>>>(a, tiles, kblocks);
        else if (umax == 6) gather_mfma_kernel<uint16_t, 6><<<n1, blk, shmem, stream>>>(a, tiles, kblocks);
        else if (umax == 8) gather_mfma_kernel<uint16_t, 8><<<n1, blk, shmem, stream>>>(a, tiles, kblocks);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fwh

namespace fwh {

int gather_mfma_persistent_blocks_per_cu(int coef_type, int umax, size_t shmem) {
    const void *k = nullptr;
    if (coef_type == 1) k = umax == 4 ? persistent_ptr<float, 4>() : umax == 6 ? persistent_ptr<float, 6>()
                                                                              : persistent_ptr<float, 8>();
    else k = umax == 4 ? persistent_ptr<uint16_t, 4>() : umax == 6 ? persistent_ptr<uint16_t, 6>()
                                                                   : persistent_ptr<uint16_t, 8>();
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kLdsWaves * 64, shmem);
    return e == hipSuccess && n > 0 ? n : 0;
}

hipError_t launch_gather_mfma_persistent(int coef_type, int umax, const BatchCase *cases, const int4 *items,
                                         int n_items, int *counter, int grid, size_t shmem, hipStream_t stream) {
    const dim3 g((unsigned)grid), blk(kLdsWaves * 64);
    if (coef_type == 1) {
        if (umax == 4) gather_mfma_persistent<float, 4><<<g, blk, shmem, stream>>>(cases, items, n_items, counter);
        else if (umax == 6) gather_mfma_persistent<float, 6><<<g, blk, shmem, stream>>>(cases, items, n_items, counter);
        else if (umax == 8) gather_mfma_persistent<float, 8><<<g, blk, shmem, stream>>>(cases, items, n_items, counter);
        else return hipErrorInvalidValue;
    } else {
        if (umax == 4) gather_mfma_persistent<uint16_t, 4><<<g, blk, shmem, stream>>>(cases, items, n_items, counter);
        else if (umax == 6)
            gather_mfma_persistent<uint16_t, 6><<<g, blk, shmem, stream>>>(cases, items, n_items, counter);
        else if (umax == 8)
            gather_mfma_persistent<uint16_t, 8><<<g, blk, shmem, stream>>>(cases, items, n_items, counter);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fwh
