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
    // byte offset of the pair's element n0 in its panel's staged window of the LDS-staged gather:
    // (n0 - lo) x 16 (FP32) or x 8 (BF16), lo = min n0 over the pair's 32-observer tile
    int32_t n0w;
    int32_t pad[2];
};
static_assert(sizeof(PairRec) == 64, "PairRec must be 64 bytes");

// BF16 mode: the 8 weights K_c of a pair as bfloat16 high and low parts
// (K ~ hi + lo to 2^-17 relative), channels (2i, 2i + 1) in word i (even channel
// in the low half), for the packed bf16 dot products of the forward gather.
struct alignas(32) PairBf {
    uint32_t hi[4];
    uint32_t lo[4];
};
static_assert(sizeof(PairBf) == 32, "PairBf must be 32 bytes");

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
constexpr int kMaxPanelSplits = 256;

// LDS-staged gather: a block of kLdsWaves waves owns kObsTile consecutive
// observers (kObsPerWave per wave) and kLdsK consecutive samples (kLdsSub
// sub-blocks of kLdsLanesOut lanes, one sample per lane; the last kLdsHalo
// lanes of a sub-block only supply combined values to their left neighbours).
// Panel coefficient windows are staged PT panels at a time, double-buffered.
constexpr int kObsTile = 32;
constexpr int kLdsWaves = 8;
constexpr int kObsPerWave = kObsTile / kLdsWaves;
constexpr int kLdsHalo = 3;
constexpr int kLdsLanesOut = 64 - kLdsHalo;
constexpr int kLdsSub = 4;
constexpr int kLdsK = kLdsSub * kLdsLanesOut;  // 244
constexpr size_t kLdsBudget = 64 * 1024;       // LDS bytes per block (two stage buffers)
constexpr int kMaxPanelsPerStage = 8;


// ------------------------------------------------------- per-stage arguments
// Workgroups are dispatched round-robin over the 8 XCDs (block h to XCD h mod 8),
// each with its own L2.  xcd_block(h, n) renumbers them so that XCD x runs the
// consecutive logical blocks [start(x), start(x) + count(x)): neighbouring
// logical blocks, which read the same panels' data, share an L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t h, int64_t n) {
    const int64_t x = h % kXcds, s = h / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + s;
}

// Every stage kernel is a body taking one of these; the single-case kernels
// pass them by value, the batched kernels pick them from a per-case array.

struct SrcFwdArgs {
    const void *rho, *u, *pp;  // time-major inputs
    const double *normal;
    int64_t P, N, NS;
    Flow f;
    const double *cp;
    void *scr;   // [8][N][P]
    void *coef;  // [P][2][NS][4]
};

struct GatherArgs {
    const PairRec *rec;
    const PairBf *rbf;  // BF16 mode: [O][P] split weights (null in FP32 mode)
    const int2 *tw;
    const int32_t *nt;
    const void *coef;
    int64_t P, O, NS, nt_max, p_chunk;
    int NW, PT, splits;
    float *partial;  // [splits][O][nt_max] partial signals of the panel splits
    int rows;        // matrix-core gather: rows of kLdsLanesOut samples per block (1..kLdsSub)
};

struct ReduceArgs {
    const float *partial;
    int splits;
    int64_t total;
    float *out;
};

struct PadArgs {
    const float *gbar;
    const int32_t *nt;
    int64_t O, nt_max, LR, padlo;
    float *gpad;
};

struct AdjArgs {
    const PairRec *rec;  // [O][P]
    const float *gpad;
    int64_t P, O, NS, LR, padlo, nib;
    float *cbar;
    int64_t nt_max;  // longest observer window (bounds the indices an observer's gradient reaches)
    // every observer's gradient reaches every index in [edge_lo, edge_hi] (N - shortest window, and
    // shortest window + 2): index blocks inside need no check for blocks that get only zeros
    int64_t edge_lo, edge_hi;
};

struct PreAdjArgs {
    const void *cbar;
    int64_t P, N, NS;
    const double *cp;
    void *scr;
};

struct ChainArgs {
    const void *scr;
    const void *rho, *u;
    const double *normal;
    int64_t P, N;
    Flow f;
    void *g_rho, *g_u, *g_p;
};

// One case of a batch (device-resident array) and the block counts of its stages.
// Chunked source adjoint (FP32/BF16 modes): cbar [8][P][NS] float -> gradients.
struct SrcAdjArgs {
    const float *cbar;
    const void *rho, *u;
    const double *normal;
    int64_t P, N, NS;
    Flow f;
    const double *cp;
    void *g_rho, *g_u, *g_p;
};

struct BatchCase {
    SrcFwdArgs src;
    GatherArgs gat;
    ReduceArgs red;
    PadArgs pad;
    AdjArgs adj;
    SrcAdjArgs sadj;
};

// Case of flattened block b: start[c] <= b < start[c+1] (start has n + 1 entries).
__device__ __forceinline__ int find_case(const int64_t *start, int n, int64_t b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Block/wave offsets of each case in the flattened batched grids: start[c] .. start[c+1].
struct BatchIndex {
    const int64_t *src, *srcg, *red, *pad, *adj, *sadj, *sadjg;  // block starts per case
    int n;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return the launch status.

hipError_t launch_delay(const double *y, const double *x_obs, int64_t P, int64_t O, Flow f, double *D,
                        hipStream_t stream);
hipError_t launch_minmax(const double *D, int64_t P, int64_t O, double *dmm, hipStream_t stream);
// mode 0: FP64 tables (K64 [O][P][8], W64 [O][P][4], N0 [O][P]); mode 1/2: PairRec [O][P] (and
// rbf, if not null), plus per (observer tile t, panel p) the lo/hi of n0 over the tile's observers
// -> tw[t][p], and per block of tile_window_panels() panels of one tile the largest hi - lo ->
// wblk[block] (tile_window_blocks(P, O) blocks, tile-major).
hipError_t launch_tables(int mode, const double *y, const double *dS, const double *x_obs, const double *t_start,
                         const int32_t *nt, int64_t P, int64_t O, int64_t N, Flow f, double *K64, double *W64,
                         int32_t *N0, PairRec *rec_op, PairBf *rbf, int2 *tw, int32_t *wblk, hipStream_t stream);
// blocks of the FP32/BF16 table kernel, which also reduces the tile windows: ceil(P / 8) per tile of
// kObsTile observers (8 panels x 32 observers per block)
inline int64_t tile_window_panels() { return 256 / kObsTile; }
inline int64_t tile_window_blocks(int64_t P, int64_t O) {
    return (O + kObsTile - 1) / kObsTile * ((P + tile_window_panels() - 1) / tile_window_panels());
}

// Chunked source stage (FP32/BF16 modes).  A block owns kSrcPanels panels and
// the kSrcTC coefficient indices [i0, i0 + kSrcTC) (NS is a multiple of 64); its
// recurrences run over the rows [i0 - 1 - kSrcH, i0 + kSrcTC - 1 + kSrcH].
// Interior chunks (every row, and every source term read, away from the record
// ends and past the first kSrcPivotRows rows) take a branch-free unrolled
// kernel; the others (the first chunk, the last one or two, all of them for
// short records) a general kernel.
constexpr int kSrcPanels = 32;
constexpr int kSrcTC = 64;
constexpr int kSrcH = 16;
constexpr int kSrcW = kSrcTC + 2 * kSrcH + 1;
constexpr int kSrcPivotRows = 16;
// interior chunks are k = 1 .. src_interior_chunks(N): i0 >= kSrcPivotRows + kSrcH + 1
// and i0 - 1 - kSrcH + kSrcW + 2 <= N - 1
__host__ __device__ inline int64_t src_interior_chunks(int64_t N) {
    const int64_t top = N - 1 - (kSrcW + 2) + 1 + kSrcH;  // largest admissible i0
    return top >= kSrcTC ? top / kSrcTC : 0;
}
// general chunk g -> chunk index: the first chunk, then those above the interior ones
__host__ __device__ inline int64_t src_general_chunk(int64_t g, int64_t n_interior) {
    return g == 0 ? 0 : n_interior + g;
}

// Chunked source adjoint: a block owns kSrcPanels panels and the frames
// [m0, m0 + kSrcTC); its recurrences run over the rows [m0 - kAdjLo, m0 - kAdjLo + kAdjW),
// whose coefficient adjoints are the 16-byte aligned storage indices
// [m0 - kAdjLo + 1, m0 - kAdjLo + 1 + kAdjW).  Interior chunks: rows inside
// [kSrcPivotRows, N - 3].
constexpr int kAdjLo = 17;
constexpr int kAdjW = 96;
__host__ __device__ inline int64_t adj_interior_chunks(int64_t N) {
    const int64_t top = N - 3 - (kAdjW - kAdjLo - 1);  // largest admissible m0
    return top >= kSrcTC ? top / kSrcTC : 0;
}
__host__ __device__ inline int64_t adj_chunks(int64_t N) { return (N + kSrcTC - 1) / kSrcTC; }

// Source terms + derivatives + natural-spline prefilter -> coefficients [P][2][NS][4]
// (channel c = 4 g + cc at ((p*2 + g)*NS + i)*4 + cc).
// in_dtype 0 = double, 1 = float; coef_type 0 = double, 1 = float, 2 = bf16; scratch is
// [8][N][P] of double (coef_type 0) or float (otherwise).
hipError_t launch_source(int in_dtype, int coef_type, const void *rho, const void *u, const void *pp,
                         const double *normal, int64_t P, int64_t N, int64_t NS, Flow f, const double *cp,
                         void *scratch, void *coef, hipStream_t stream);

hipError_t launch_gather_f64(const double *K64, const double *W64, const int32_t *N0, const int32_t *nt,
                             const double *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max, double *out,
                             hipStream_t stream);
// coef_type 1 = float, 2 = bf16.  partial: [splits][O][nt_max] floats.
hipError_t launch_gather_tuned(int coef_type, const PairRec *rec_op, const int32_t *nt, const void *coef, int64_t P,
                               int64_t O, int64_t NS, int64_t nt_max, int splits, float *partial,
                               hipStream_t stream);
// LDS-staged gather; NW = staged window length per channel group (multiple of 64, >= max
// width + block samples + kLdsHalo), PT = panels per stage (two stages fit in kLdsBudget).
// Wave shapes: 0 = 4 observers x 4 sub-rows (tiles of 32 observers, kLdsK samples per block);
// 1 = 2 observers x 8 sub-rows (a last tile of at most 16 observers, 2 kLdsK samples per block).
constexpr int kLdsShapeTile[2] = {kObsTile, kObsTile / 2};
constexpr int kLdsShapeK[2] = {kLdsK, 2 * kLdsK};
// Per panel of a stage: both windows, the tile's records and, in BF16 mode, its split weights.
inline size_t gather_lds_panel_bytes(int coef_type, int NW, int shape = 0) {
    const size_t esz = coef_type == 1 ? 4 : 2;
    return (size_t)8 * NW * esz +
           (size_t)kLdsShapeTile[shape] * (sizeof(PairRec) + (coef_type == 1 ? 0 : sizeof(PairBf)));
}
inline size_t gather_lds_shmem(int coef_type, int NW, int PT, int shape = 0) {
    return 2 * (size_t)PT * gather_lds_panel_bytes(coef_type, NW, shape);
}
// size class (bytes) of each of the two static stage buffers for this staging size (0: too large)
int gather_lds_stage_class(int coef_type, int NW, int PT, int shape = 0);
// blocks of the LDS-staged gather resident per CU at this staging size (registers and LDS)
int gather_lds_blocks_per_cu(int coef_type, int NW, int PT, int shape = 0);
// tiles t0 .. t1 - 1 of 32 observers (t1 < 0: all) with wave shape `shape`
hipError_t launch_gather_lds(int coef_type, const PairRec *rec_op, const PairBf *rbf, const int2 *tw, const int32_t *nt,
                             const void *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max, int splits, int NW,
                             int PT, float *partial, hipStream_t stream, int64_t t0 = 0, int64_t t1 = -1,
                             int shape = 0);
// Matrix-core gather (fwh_gather_mfma.hip): per panel a Y tile [kObsTile][YR] floats in LDS covering
// the window of the widest tile (wmax = largest n0 spread over a tile's observers).
inline int gather_mfma_y_row(int wmax) { return ((wmax + kLdsK + kLdsHalo + 15) / 16) * 16 + 4; }
// Y tile, then two record buffers of the tile (pair records and, in BF16, split weights)
inline size_t gather_mfma_shmem(int wmax) {
    return (size_t)kObsTile * gather_mfma_y_row(wmax) * sizeof(float) + 2 * (size_t)kObsTile * (sizeof(PairRec) + sizeof(PairBf));
}
// matrix units per wave and panel the kernel is compiled for (4, 6 or 8; 0: windows too wide)
int gather_mfma_umax(int wmax);
// resident blocks per CU (0 when the kernel does not apply)
int gather_mfma_blocks_per_cu(int coef_type, int wmax);
hipError_t launch_gather_mfma(int coef_type, const PairRec *rec_op, const PairBf *rbf, const int2 *tw,
                              const int32_t *nt, const void *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max,
                              int splits, int wmax, float *partial, hipStream_t stream);
// Persistent batched form: `grid` blocks pull (case, tile, k block, split) items through counter[0]
// (reset by the caller's stream order); every case's GatherArgs carries its Y row length in NW and
// its rows per block; umax as for the widest case, shmem its Y tile.
int gather_mfma_persistent_blocks_per_cu(int coef_type, int umax, size_t shmem);
hipError_t launch_gather_mfma_persistent(int coef_type, int umax, const BatchCase *cases, const int4 *items,
                                         int n_items, int *counter, int grid, size_t shmem, hipStream_t stream);
// Streaming gather for O <= kLdsWaves observers: whole coefficient rows of each panel staged in LDS
// (two buffers), two waves per observer, every sample in registers (rows of 61, up to 32 rows).
// Grid: one block per panel split.  0 blocks per CU when it does not apply (rows or LDS).
size_t gather_stream_shmem(int coef_type, int64_t NS);
int gather_stream_rows(int64_t nt_max);  // rows per wave it is compiled for (0: record too long)
int gather_stream_blocks_per_cu(int coef_type, int64_t NS, int64_t nt_max);
hipError_t launch_gather_stream(int coef_type, const PairRec *rec_op, const PairBf *rbf, const int32_t *nt,
                                const void *coef, int64_t P, int64_t O, int64_t NS, int64_t nt_max, int splits,
                                float *partial, hipStream_t stream);
// out[i] = sum over splits of partial[z][i], in FP64 and fixed order, rounded to float.
hipError_t launch_reduce_splits(const float *partial, int splits, int64_t total, float *out, hipStream_t stream);

hipError_t launch_adj_gather_f64(const double *K64, const double *W64, const int32_t *N0, const int32_t *nt,
                                 const double *gbar, int64_t P, int64_t O, int64_t NS, int64_t nt_max, double *cbar,
                                 hipStream_t stream);
// Transposed gather via a zero-padded copy of gbar (gpad: [O][adj_pad_row(N, NS)] floats).
inline int64_t adj_pad_lo(int64_t N) { return N + 4; }
// blocks of 64 coefficient indices per wave of the transposed gather; a gpad row covers every
// position it reads (from -n0 - 4 to NS - 1 - n0 past padlo, n0 < N)
constexpr int kAdjMW = 5;
constexpr int kAdjPT = 64;  // panels per tile of the transposed gather's wave order
inline int64_t adj_blocks(int64_t NS) { return (NS + 64 * kAdjMW - 1) / (64 * kAdjMW); }
inline int64_t adj_pad_row(int64_t N, int64_t NS) { return ((N + NS + 8 + 64 * (kAdjMW + 1) + 63) / 64) * 64; }
// nt_min, nt_max: shortest and longest observer window
hipError_t launch_adj_gather(const PairRec *rec_op, const int32_t *nt, const float *gbar, int64_t P, int64_t O,
                                 int64_t N, int64_t NS, int64_t nt_min, int64_t nt_max, float *gpad, float *cbar,
                                 hipStream_t stream);

// Adjoint of the source stage: coefficient adjoints [8][P][NS] -> gradients (time-major, in_dtype).
// real_type 0 = double (cbar and scratch double), 1 = float.
hipError_t launch_source_adjoint(int real_type, int in_dtype, const void *cbar, const void *rho, const void *u,
                                 const double *normal, int64_t P, int64_t N, int64_t NS, Flow f, const double *cp,
                                 void *scratch, void *g_rho, void *g_u, void *g_p, hipStream_t stream);

// Batched launches over n cases (device arrays `cases`, prefix tables in `idx`).
// coef_type 1 = float, 2 = bf16; in_dtype 0 = double, 1 = float.  The forward gather
// is persistent: `grid` blocks pull work items (case, tile, k-block, split) from
// items[0..n_items) through counter[0], which the launch resets first.
// interior-chunk blocks then general-chunk blocks of the chunked source stage
hipError_t launch_batch_source(int in_dtype, int coef_type, const BatchCase *cases, const int64_t *start_int,
                               const int64_t *start_gen, int n, int64_t blocks_int, int64_t blocks_gen,
                               hipStream_t stream);
hipError_t launch_batch_source_adjoint(int in_dtype, const BatchCase *cases, const int64_t *start_int,
                                       const int64_t *start_gen, int n, int64_t blocks_int, int64_t blocks_gen,
                                       hipStream_t stream);
// forward: chunked source stage of all cases, counter reset, the persistent gather (matrix-core with
// `umax` units per wave, or LDS-staged when umax is 0), then the split sums of all cases
hipError_t launch_batch_forward(int in_dtype, int coef_type, int umax, const BatchCase *cases, BatchIndex idx,
                                const int4 *items, int n_items, int *counter, int grid, size_t shmem,
                                int64_t blocks_src, int64_t blocks_srcg, int64_t blocks_red, hipStream_t stream);
// adjoint: zero-padded dJ/dp' of all cases, then the transposed gather over adj_items (case, group of
// 4 waves) in their longest-first order, one block per item, then the chunked source adjoint
hipError_t launch_batch_adjoint(int in_dtype, const BatchCase *cases, BatchIndex idx, int64_t blocks_pad,
                                const int2 *adj_items, int n_adj_items, int64_t blocks_sadj, int64_t blocks_sadjg,
                                hipStream_t stream);

// Post-processing: per-observer RMS and one-sided Welch PSD (segments of L
// samples, 50 % overlap, Hann window), times span_ratio; psd [O][L/2+1], rms [O].
// real_type 0 = double signals, 1 = float.  L is a power of two in [16, 4096].
size_t post_shmem(int L);
hipError_t launch_post(int real_type, const void *p, int64_t ld, const int32_t *nt, int64_t O, int L, double dt,
                       double span_ratio, float *psd, float *rms, hipStream_t stream);

// ------------------------------------------------ general motion (fwh_gm.hip)
constexpr int kGmPivots = 64;  // inv_beta[n] = 1 / beta_n of tridiag(1, 4, 1), n < 64 (constant past 64)
constexpr int kGmRows = 19;    // channel rows per panel: A, Q_n, L_1..3, Ld_1..3, L_M, M_1..3, Md_1..3, M^2, y_1..3

struct GmChanArgs {
    const double *y, *normal, *vel;  // [N][P][3]
    const double *rho, *u, *pp;      // [N][P], [3][N][P], [N][P]
    double mach, dtau;
    int64_t P, N, NS;                // NS = N + 2 coefficients per row
    double *coef;                    // [P][kGmRows][NS]
};
struct GmWinArgs {
    const double *y, *x_obs;
    double mach, dtau, tau0;
    int64_t P, O, N;
    double *t_start;
    int32_t *n_t;
};
struct GmGatherArgs {
    const double *coef, *dS, *x_obs, *t_start;
    const int32_t *n_t;
    double mach, dtau, tau0;
    int64_t P, O, N, NS, nkb, nt_stride, p_chunk;
    int splits;
    double *part;                    // [splits][O][nt_stride]
};
hipError_t launch_gm_source(const GmChanArgs &a, const double *inv_beta, hipStream_t stream);
hipError_t launch_gm_window(const GmWinArgs &a, hipStream_t stream);
hipError_t launch_gm_gather(const GmGatherArgs &a, double *out, hipStream_t stream);

}  // namespace fwh
