// Host side of the C ABI declared in include/fwh.h: argument validation,
// workspace layout, the observer window (Eqs. (t_start), (t_end)) and the
// launch sequence of setup, forward and adjoint.  No device memory is
// allocated here: every device buffer, including the workspace, is the caller's.
#include "../../include/fwh.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>
#include <new>

#include "fwh_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;

// Workspace of fwh_forward_noalloc: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never uses the
// array's name as an address: the device address of each GPU's copy is taken
// once per device with hipGetSymbolAddress and kept in g_noalloc_ptr.
constexpr size_t kNoAllocBytes = (size_t)FWH_NOALLOC_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocMaxDevices] = {};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct fwh_plan {
    int64_t P = 0, O = 0, N = 0, NS = 0;
    double mach = 0, aoa_deg = 0, dtau = 0, tau0 = 0;
    int mode = 0;
    fwh::Flow flow{};
    std::vector<double> y, normal, dS, x_obs, cp;
    // window (valid after setup)
    std::vector<double> t_start;
    std::vector<int64_t> n_t;
    std::vector<int32_t> n_t32;
    int64_t n_t_max = 0;
    int splits = 1;
    int max_splits = 1;          // panel splits the partial-signal region holds
    int gather_variant = FWH_GATHER_AUTO, forced_splits = 0;  // fwh_plan_tune
    int gather_kind = FWH_GATHER_AUTO;  // kernel chosen by fwh_setup (FP32/BF16 modes)
    int lds_nw = 0, lds_pt = 0;  // staged window length and panels per stage of the LDS gather (0: not usable)
    int tail_nw = 0, tail_pt = 0;  // the same for a last tile of at most 16 observers (2 x 8 wave shape; 0: none)
    int wmax = 0;                // widest delay-index window over a tile of observers
    int mfma_bpc = 0;            // resident blocks per CU of the matrix-core gather (0: not usable)
    int stream_bpc = 0;          // resident blocks per CU of the streaming gather (0: not usable)
    bool ready = false;
    // workspace layout (byte offsets) and binding
    size_t off_y = 0, off_n = 0, off_dS = 0, off_x = 0, off_D = 0, off_dmm = 0, off_ts = 0, off_nt = 0, off_cp = 0;
    size_t off_K64 = 0, off_W64 = 0, off_N0 = 0, off_rec_op = 0, off_rbf = 0, off_tw = 0, off_wblk = 0;
    size_t off_coef = 0, off_scr = SIZE_MAX, off_part = 0, off_gpad = 0, ws_bytes = 0;
    char *ws = nullptr;
    // optional per-stage event timing
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events[FWH_NUM_STAGES];

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    void *scratch() const { return off_scr == SIZE_MAX ? nullptr : ws + off_scr; }
    fwh::PairBf *rbf() const { return mode == FWH_MODE_BF16 ? at<fwh::PairBf>(off_rbf) : nullptr; }
};

namespace {

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Largest number of panel splits of the FP32/BF16 gathers (single-case and batched): at most
// kMaxPanelSplits and at least kMinSplitPanels panels per split.  The partial-signal region is sized for it.
constexpr int64_t kMinSplitPanels = 128;
int64_t split_cap(int64_t P) {
    return std::max<int64_t>(1, std::min<int64_t>(fwh::kMaxPanelSplits, (P + kMinSplitPanels - 1) / kMinSplitPanels));
}

// shortest observer window of a set-up plan (every observer's gradient reaches the coefficient
// indices [N - shortest, shortest + 2])
int64_t nt_min(const fwh_plan *pl) {
    int64_t m = pl->n_t_max;
    for (int64_t v : pl->n_t) m = v < m ? v : m;
    return m;
}

int layout(fwh_plan *pl) {
    const size_t P = (size_t)pl->P, O = (size_t)pl->O, N = (size_t)pl->N, NS = (size_t)pl->NS;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    pl->off_y = take(P * 3 * sizeof(double));
    pl->off_n = take(P * 3 * sizeof(double));
    pl->off_dS = take(P * sizeof(double));
    pl->off_x = take(O * 3 * sizeof(double));
    pl->off_dmm = take(O * 2 * sizeof(double));
    pl->off_ts = take(O * sizeof(double));
    pl->off_nt = take(O * sizeof(int32_t));
    pl->off_cp = take(N * sizeof(double));
    if (pl->mode == FWH_MODE_F64) {
        pl->off_K64 = take(O * P * 8 * sizeof(double));
        pl->off_W64 = take(O * P * 4 * sizeof(double));
        pl->off_N0 = take(O * P * sizeof(int32_t));
    } else {
        pl->off_rec_op = take(O * P * sizeof(fwh::PairRec));
        if (pl->mode == FWH_MODE_BF16) pl->off_rbf = take(O * P * sizeof(fwh::PairBf));
        pl->off_tw = take((O + fwh::kObsTile - 1) / fwh::kObsTile * P * sizeof(int2));
        pl->off_wblk = take((size_t)fwh::tile_window_blocks(pl->P, pl->O) * sizeof(int32_t));
    }
    // coefficient channels (forward) and coefficient adjoints (adjoint) share one region; the pair
    // delays [O][P], needed only between the delay kernel and the window reduction of fwh_setup, live
    // in it too when they fit (the forward writes the coefficients after the setup)
    const size_t real_sz = pl->mode == FWH_MODE_F64 ? sizeof(double) : sizeof(float);
    pl->off_coef = take(8 * P * NS * real_sz);
    pl->off_D = O * P * sizeof(double) <= 8 * P * NS * real_sz ? pl->off_coef : take(O * P * sizeof(double));
    // time-major scratch of the sequential FP64 source stage, forward and adjoint
    // (the chunked FP32/BF16 stages need none)
    if (pl->mode == FWH_MODE_F64) pl->off_scr = take(8 * N * P * real_sz);
    if (pl->mode != FWH_MODE_F64) {
        // FP32 partial signals of the panel splits, [max_splits][O][n_t_max <= N]
        pl->max_splits = (int)split_cap(pl->P);
        pl->off_part = take((size_t)pl->max_splits * O * N * sizeof(float));
        pl->off_gpad = take((size_t)O * fwh::adj_pad_row(pl->N, pl->NS) * sizeof(float));
    }
    pl->ws_bytes = off;
    return FWH_OK;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Brackets one stage with events when profiling is on.
struct StageScope {
    fwh_plan *pl;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    StageScope(fwh_plan *p, int s, hipStream_t stream) : pl(p), stage(s), st(stream) {
        if (pl->profiling && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, st);
    }
    ~StageScope() {
        if (a && b) {
            (void)hipEventRecord(b, st);
            pl->events[stage].emplace_back(a, b);
        }
    }
};

int hip_fail(const char *what, hipError_t e) {
    return fail(FWH_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" {

int fwh_plan_create(const fwh_setup_args *a, fwh_plan **out, size_t *workspace_bytes) {
    g_last_error.clear();
    if (out) *out = nullptr;
    if (!a || !out) return fail(FWH_EINVAL, "fwh_plan_create: null argument");
    if (a->n_panels < 1 || a->n_obs < 1 || a->n_tau < 4)
        return fail(FWH_ESIZE, "fwh_plan_create: need n_panels >= 1, n_obs >= 1, n_tau >= 4 (got %lld, %lld, %lld)",
                    (long long)a->n_panels, (long long)a->n_obs, (long long)a->n_tau);
    if (a->n_tau > 65535 || a->n_panels > (int64_t)1 << 30 || a->n_obs > (int64_t)1 << 24 ||
        a->n_panels * a->n_obs > (int64_t)1 << 36)
        return fail(FWH_ESIZE, "fwh_plan_create: sizes beyond the supported range (n_tau <= 65535, P*O <= 2^36)");
    if (!a->y || !a->normal || !a->dS || !a->x_obs) return fail(FWH_EINVAL, "fwh_plan_create: null geometry pointer");
    if (a->mode != FWH_MODE_F64 && a->mode != FWH_MODE_F32 && a->mode != FWH_MODE_BF16)
        return fail(FWH_EINVAL, "fwh_plan_create: unknown mode %d", (int)a->mode);
    if (!(std::isfinite(a->mach) && a->mach > 0.0 && a->mach < 1.0))
        return fail(FWH_EDOMAIN, "fwh_plan_create: Mach number must be in (0, 1), got %g", a->mach);
    if (!(std::isfinite(a->dtau) && a->dtau > 0.0))
        return fail(FWH_EDOMAIN, "fwh_plan_create: dtau must be positive, got %g", a->dtau);
    if (!std::isfinite(a->tau0) || !std::isfinite(a->aoa_deg))
        return fail(FWH_EINVAL, "fwh_plan_create: tau0 and aoa_deg must be finite");
    for (int64_t p = 0; p < a->n_panels; ++p) {
        const double *y = a->y + 3 * p, *n = a->normal + 3 * p;
        if (!finite3(y) || !finite3(n) || !std::isfinite(a->dS[p]))
            return fail(FWH_EINVAL, "fwh_plan_create: non-finite geometry at panel %lld", (long long)p);
        if (!(a->dS[p] > 0.0)) return fail(FWH_EINVAL, "fwh_plan_create: dS must be > 0 (panel %lld)", (long long)p);
        const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (std::fabs(nn - 1.0) > 1e-6)
            return fail(FWH_EINVAL, "fwh_plan_create: normal of panel %lld is not unit (|n| = %g)", (long long)p, nn);
    }
    for (int64_t o = 0; o < a->n_obs; ++o)
        if (!finite3(a->x_obs + 3 * o))
            return fail(FWH_EINVAL, "fwh_plan_create: non-finite observer %lld", (long long)o);

    fwh_plan *pl = new (std::nothrow) fwh_plan();
    if (!pl) return fail(FWH_EINVAL, "fwh_plan_create: out of host memory");
    pl->P = a->n_panels;
    pl->O = a->n_obs;
    pl->N = a->n_tau;
    pl->NS = fwh::coef_row_stride(a->n_tau);
    pl->mach = a->mach;
    pl->aoa_deg = a->aoa_deg;
    pl->dtau = a->dtau;
    pl->tau0 = a->tau0;
    pl->mode = a->mode;
    const double aoa = a->aoa_deg * (kPi / 180.0);
    pl->flow.M0 = a->mach;
    pl->flow.ca = std::cos(aoa);
    pl->flow.sa = std::sin(aoa);
    pl->flow.beta2 = 1.0 - a->mach * a->mach;
    pl->flow.dtau = a->dtau;
    pl->flow.tau0 = a->tau0;
    pl->y.assign(a->y, a->y + 3 * a->n_panels);
    pl->normal.assign(a->normal, a->normal + 3 * a->n_panels);
    pl->dS.assign(a->dS, a->dS + a->n_panels);
    pl->x_obs.assign(a->x_obs, a->x_obs + 3 * a->n_obs);
    // Thomas pivots of the constant (1, 4, 1) system of the spline prefilter
    pl->cp.assign((size_t)a->n_tau, 0.0);
    pl->cp[1] = 0.25;
    for (int64_t r = 2; r < a->n_tau; ++r) pl->cp[r] = 1.0 / (4.0 - pl->cp[r - 1]);
    layout(pl);
    *out = pl;
    if (workspace_bytes) *workspace_bytes = pl->ws_bytes;
    return FWH_OK;
}

int fwh_setup(fwh_plan *pl, void *workspace, size_t workspace_bytes, void *stream_) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_setup: null plan");
    if (!workspace) return fail(FWH_EWORKSPACE, "fwh_setup: null workspace");
    if (workspace_bytes < pl->ws_bytes)
        return fail(FWH_EWORKSPACE, "fwh_setup: workspace of %zu bytes, need %zu", workspace_bytes, pl->ws_bytes);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(FWH_EWORKSPACE, "fwh_setup: workspace must be %zu-byte aligned", kAlign);
    hipStream_t st = as_stream(stream_);
    pl->ready = false;
    pl->ws = static_cast<char *>(workspace);
    const int64_t P = pl->P, O = pl->O, N = pl->N;
    hipError_t e;
    if ((e = hipMemcpyAsync(pl->at<double>(pl->off_y), pl->y.data(), P * 3 * sizeof(double), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(pl->at<double>(pl->off_n), pl->normal.data(), P * 3 * sizeof(double), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(pl->at<double>(pl->off_dS), pl->dS.data(), P * sizeof(double), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(pl->at<double>(pl->off_x), pl->x_obs.data(), O * 3 * sizeof(double), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(pl->at<double>(pl->off_cp), pl->cp.data(), N * sizeof(double), hipMemcpyHostToDevice, st)))
        return hip_fail("fwh_setup: copy of the geometry", e);
    StageScope scope_a(pl, FWH_STAGE_SETUP, st);
    if ((e = fwh::launch_delay(pl->at<double>(pl->off_y), pl->at<double>(pl->off_x), P, O, pl->flow,
                               pl->at<double>(pl->off_D), st)))
        return hip_fail("fwh_setup: delay kernel", e);
    if ((e = fwh::launch_minmax(pl->at<double>(pl->off_D), P, O, pl->at<double>(pl->off_dmm), st)))
        return hip_fail("fwh_setup: min/max kernel", e);
    std::vector<double> dmm((size_t)(2 * O));
    if ((e = hipMemcpyAsync(dmm.data(), pl->at<double>(pl->off_dmm), 2 * O * sizeof(double), hipMemcpyDeviceToHost, st)))
        return hip_fail("fwh_setup: read-back of the delay extremes", e);
    if ((e = hipStreamSynchronize(st))) return hip_fail("fwh_setup: stream synchronize", e);
    // observer window, Eqs. (t_start), (t_end) per observer with a general tau0
    pl->t_start.assign((size_t)O, 0.0);
    pl->n_t.assign((size_t)O, 0);
    pl->n_t32.assign((size_t)O, 0);
    pl->n_t_max = 0;
    for (int64_t o = 0; o < O; ++o) {
        const double ts = pl->tau0 + dmm[2 * o];
        const double te = pl->tau0 + (double)(N - 1) * pl->dtau + dmm[2 * o + 1];
        pl->t_start[o] = ts;
        if (!(te >= ts))
            return fail(FWH_EWINDOW,
                        "fwh_setup: observer %lld has an empty window (t_end %.17g < t_start %.17g): the record is "
                        "shorter than the delay spread over the surface",
                        (long long)o, te, ts);
        const int64_t nt = (int64_t)std::floor((te - ts) / pl->dtau + 1e-9) + 1;
        pl->n_t[o] = nt;
        pl->n_t32[o] = (int32_t)nt;
        if (nt > pl->n_t_max) pl->n_t_max = nt;
    }
    if ((e = hipMemcpyAsync(pl->at<double>(pl->off_ts), pl->t_start.data(), O * sizeof(double), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(pl->at<int32_t>(pl->off_nt), pl->n_t32.data(), O * sizeof(int32_t), hipMemcpyHostToDevice, st)))
        return hip_fail("fwh_setup: copy of the window", e);
    const bool f64 = pl->mode == FWH_MODE_F64;
    StageScope scope_b(pl, FWH_STAGE_SETUP, st);
    if ((e = fwh::launch_tables(f64 ? 0 : 1, pl->at<double>(pl->off_y), pl->at<double>(pl->off_dS),
                                pl->at<double>(pl->off_x), pl->at<double>(pl->off_ts), pl->at<int32_t>(pl->off_nt), P,
                                O, N, pl->flow, f64 ? pl->at<double>(pl->off_K64) : nullptr,
                                f64 ? pl->at<double>(pl->off_W64) : nullptr, f64 ? pl->at<int32_t>(pl->off_N0) : nullptr,
                                f64 ? nullptr : pl->at<fwh::PairRec>(pl->off_rec_op), pl->rbf(),
                                f64 ? nullptr : pl->at<int2>(pl->off_tw), f64 ? nullptr : pl->at<int32_t>(pl->off_wblk),
                                st)))
        return hip_fail("fwh_setup: table kernel", e);
    if (!f64) {
        // per (observer tile, panel) windows of n0 (from the table kernel) and their largest width
        // -> LDS staging geometry
        const int64_t nb = fwh::tile_window_blocks(P, O);
        std::vector<int32_t> wblk((size_t)nb);
        if ((e = hipMemcpyAsync(wblk.data(), pl->at<int32_t>(pl->off_wblk), nb * sizeof(int32_t),
                                hipMemcpyDeviceToHost, st)) ||
            (e = hipStreamSynchronize(st)))
            return hip_fail("fwh_setup: read-back of the tile windows", e);
        int wmax = 0;
        for (int32_t w : wblk) wmax = w > wmax ? w : wmax;
        const size_t esz = pl->mode == FWH_MODE_F32 ? sizeof(float) : sizeof(uint16_t);
        // window length per channel group: a multiple of 64 elements (whole wave-wide direct loads)
        // (BF16: a multiple of 128, two elements per 16-byte copy unit)
        const int nwq = pl->mode == FWH_MODE_F32 ? 64 : 128;
        const int nw = ((wmax + fwh::kLdsK + fwh::kLdsHalo + nwq - 1) / nwq) * nwq;
        // two stage buffers of PT panels: windows of both groups plus the tile's pair records (and,
        // in BF16, split weights), at most kLdsBudget; the largest PT that keeps as many blocks per CU
        // resident as a one-panel stage (more waves in flight hide the staging latency better than
        // longer stages)
        const int ctype = esz == sizeof(float) ? 1 : 2;
        int64_t pt = (int64_t)(fwh::kLdsBudget / (2 * fwh::gather_lds_panel_bytes(ctype, nw)));
        if (pt > fwh::kMaxPanelsPerStage) pt = fwh::kMaxPanelsPerStage;
        if (pt > 1) {
            const int occ1 = fwh::gather_lds_blocks_per_cu(ctype, nw, 1);
            while (pt > 1 && fwh::gather_lds_blocks_per_cu(ctype, nw, (int)pt) < occ1) --pt;
        }
        pl->lds_nw = nw;
        pl->lds_pt = (int)pt;  // 0 when one panel's window does not fit
        // a last tile of at most 16 observers runs with the 2 x 8 wave shape (16 observers x 488
        // samples per block) and its own window length: the widest window over that tile's panels
        pl->tail_nw = pl->tail_pt = 0;
        const int64_t n_tiles = (O + fwh::kObsTile - 1) / fwh::kObsTile,
                      bpt = (P + fwh::tile_window_panels() - 1) / fwh::tile_window_panels();
        if (O - (n_tiles - 1) * fwh::kObsTile <= fwh::kObsTile / 2) {
            int wt = 0;
            for (int64_t b = (n_tiles - 1) * bpt; b < n_tiles * bpt; ++b) wt = wblk[b] > wt ? wblk[b] : wt;
            const int nwt = ((wt + fwh::kLdsShapeK[1] + fwh::kLdsHalo + nwq - 1) / nwq) * nwq;
            int64_t ptt = (int64_t)(fwh::kLdsBudget / (2 * fwh::gather_lds_panel_bytes(ctype, nwt, 1)));
            if (ptt > fwh::kMaxPanelsPerStage) ptt = fwh::kMaxPanelsPerStage;
            if (ptt > 1) {
                const int occ1 = fwh::gather_lds_blocks_per_cu(ctype, nwt, 1, 1);
                while (ptt > 1 && fwh::gather_lds_blocks_per_cu(ctype, nwt, (int)ptt, 1) < occ1) --ptt;
            }
            pl->tail_nw = nwt;
            pl->tail_pt = (int)ptt;
        }
        pl->wmax = wmax;
        pl->mfma_bpc = fwh::gather_mfma_blocks_per_cu(ctype, wmax);
        pl->stream_bpc = O <= fwh::kLdsWaves ? fwh::gather_stream_blocks_per_cu(ctype, pl->NS, pl->n_t_max) : 0;
        // kernel: the streaming gather for a few observers, else the LDS-staged one when a panel's
        // window over a tile fits its staging, else the matrix-core one, else direct loads
        switch (pl->gather_variant) {
            case FWH_GATHER_STREAM:
                if (pl->stream_bpc <= 0)
                    return fail(FWH_EINVAL, "fwh_setup: the streaming gather takes at most %d observers and %d "
                                            "samples per observer", fwh::kLdsWaves, 32 * fwh::kLdsLanesOut);
                pl->gather_kind = FWH_GATHER_STREAM;
                break;
            case FWH_GATHER_MFMA:
                if (pl->mfma_bpc <= 0)
                    return fail(FWH_EINVAL, "fwh_setup: the delay windows (%d samples) are too wide for the "
                                            "matrix-core gather", wmax);
                pl->gather_kind = FWH_GATHER_MFMA;
                break;
            case FWH_GATHER_LDS:
                if (pl->lds_pt <= 0)
                    return fail(FWH_EINVAL, "fwh_setup: the delay windows (%d samples) are too wide for the "
                                            "LDS-staged gather", wmax);
                pl->gather_kind = FWH_GATHER_LDS;
                break;
            case FWH_GATHER_DIRECT: pl->gather_kind = FWH_GATHER_DIRECT; break;
            default:
                pl->gather_kind = pl->stream_bpc > 0 ? FWH_GATHER_STREAM
                                  : pl->lds_pt > 0   ? FWH_GATHER_LDS
                                  : pl->mfma_bpc > 0 ? FWH_GATHER_MFMA
                                                     : FWH_GATHER_DIRECT;
        }
    }
    // panel splits of the tuned gathers.  A split's block takes P/s panels, so a launch of B*s blocks
    // on R resident blocks (the LDS gather's occupancy at its staging size times the CU count; 2 per
    // CU for the direct-load gather) lasts about ceil(B*s/R)/s block-times of the unsplit work.  Among
    // the s (at most kMaxPanelSplits, at least 128 panels per split) within 3 % of its minimum, take
    // the largest that keeps B*s within 32 rounds: whole rounds (no last round that leaves most CUs
    // idle), and enough of them that blocks of unequal work even out
    int64_t blocks;
    const bool tiled = !f64 && pl->gather_kind != FWH_GATHER_DIRECT;  // 32-observer x 244-sample blocks
    if (!f64 && pl->gather_kind == FWH_GATHER_STREAM)
        blocks = 1;  // one block per split covers every observer and sample
    else if (tiled)
        blocks = ((O + fwh::kObsTile - 1) / fwh::kObsTile) * ((pl->n_t_max + fwh::kLdsK - 1) / fwh::kLdsK);
    else
        blocks = ((O + fwh::kGatherObsPerBlock - 1) / fwh::kGatherObsPerBlock) *
                 ((pl->n_t_max + fwh::kGatherK - 1) / fwh::kGatherK);
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) || (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)))
        return hip_fail("fwh_setup: device query", e);
    const int ctype_s = pl->mode == FWH_MODE_F32 ? 1 : 2;
    const int64_t resident =
        (int64_t)cus * (pl->gather_kind == FWH_GATHER_STREAM ? pl->stream_bpc
                        : pl->gather_kind == FWH_GATHER_MFMA  ? pl->mfma_bpc
                        : pl->gather_kind == FWH_GATHER_LDS ? fwh::gather_lds_blocks_per_cu(ctype_s, pl->lds_nw,
                                                                                            pl->lds_pt)
                                                            : 2);
    const int64_t smax = split_cap(P);
    auto rounds = [&](int64_t c) { return (double)((blocks * c + resident - 1) / resident) / (double)c; };
    double best = 1e300;
    for (int64_t c = 1; c <= smax; ++c) best = std::min(best, rounds(c));
    int64_t s = 1;
    for (int64_t c = 1; c <= smax; ++c)
        if (rounds(c) <= best * 1.03 && (c == 1 || blocks * c <= 32 * resident)) s = c;
    if (pl->forced_splits > 0) s = pl->forced_splits;
    pl->splits = (int)s;
    if (!f64) {
        // one launch: a 1-D grid of at most 2^32 work-items
        const int64_t threads = blocks * s * (tiled ? (int64_t)2 * fwh::kLdsWaves * 64 : 256);
        if (blocks * s > INT32_MAX || threads >= ((int64_t)1 << 32))
            return fail(FWH_ESIZE, "fwh_setup: %lld observers x %lld samples x %lld panel splits exceed one gather launch",
                        (long long)O, (long long)pl->n_t_max, (long long)s);
    }
    pl->ready = true;
    return FWH_OK;
}

int fwh_plan_tune(fwh_plan *pl, int32_t gather, int32_t splits) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_plan_tune: null plan");
    if (gather != FWH_GATHER_AUTO && gather != FWH_GATHER_LDS && gather != FWH_GATHER_DIRECT &&
        gather != FWH_GATHER_MFMA && gather != FWH_GATHER_STREAM)
        return fail(FWH_EINVAL, "fwh_plan_tune: unknown gather variant %d", (int)gather);
    if (pl->mode == FWH_MODE_F64 && (gather != FWH_GATHER_AUTO || splits != 0))
        return fail(FWH_EINVAL, "fwh_plan_tune: the plain FP64 form has one gather and no panel splits");
    if (splits < 0 || splits > pl->max_splits)
        return fail(FWH_ESIZE, "fwh_plan_tune: splits must be in 0 .. %d for %lld panels (got %d)", pl->max_splits,
                    (long long)pl->P, (int)splits);
    pl->gather_variant = gather;
    pl->forced_splits = splits;
    pl->ready = false;
    return FWH_OK;
}

int fwh_plan_info(const fwh_plan *pl, int32_t *gather, int32_t *splits) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_plan_info: null plan");
    if (!pl->ready) return fail(FWH_ESTATE, "fwh_plan_info: plan is not set up");
    if (gather)
        *gather = pl->mode == FWH_MODE_F64 ? FWH_GATHER_AUTO : pl->gather_kind;
    if (splits) *splits = pl->mode == FWH_MODE_F64 ? 1 : pl->splits;
    return FWH_OK;
}

int fwh_obs_window(const fwh_plan *pl, double *t_start, int64_t *n_t, int64_t *n_t_max) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_obs_window: null plan");
    if (!pl->ready) return fail(FWH_ESTATE, "fwh_obs_window: plan is not set up");
    if (t_start) std::memcpy(t_start, pl->t_start.data(), pl->O * sizeof(double));
    if (n_t) std::memcpy(n_t, pl->n_t.data(), pl->O * sizeof(int64_t));
    if (n_t_max) *n_t_max = pl->n_t_max;
    return FWH_OK;
}

int fwh_forward(fwh_plan *pl, int32_t in_dtype, const void *rho, const void *u, const void *pp, void *p_out,
                void *stream_) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_forward: null plan");
    if (!pl->ready) return fail(FWH_ESTATE, "fwh_forward: plan is not set up");
    if (!rho || !u || !pp || !p_out) return fail(FWH_EINVAL, "fwh_forward: null data pointer");
    if (in_dtype != FWH_F64 && in_dtype != FWH_F32) return fail(FWH_EINVAL, "fwh_forward: bad in_dtype %d", in_dtype);
    hipStream_t st = as_stream(stream_);
    const int coef_type = pl->mode == FWH_MODE_F64 ? 0 : (pl->mode == FWH_MODE_F32 ? 1 : 2);
    hipError_t e;
    {
        StageScope sc(pl, FWH_STAGE_SOURCE, st);
        e = fwh::launch_source(in_dtype == FWH_F64 ? 0 : 1, coef_type, rho, u, pp, pl->at<double>(pl->off_n), pl->P,
                               pl->N, pl->NS, pl->flow, pl->at<double>(pl->off_cp), pl->scratch(),
                               pl->ws + pl->off_coef, st);
    }
    if (e) return hip_fail("fwh_forward: source kernel", e);
    if (pl->mode == FWH_MODE_F64) {
        StageScope sc(pl, FWH_STAGE_GATHER, st);
        e = fwh::launch_gather_f64(pl->at<double>(pl->off_K64), pl->at<double>(pl->off_W64),
                                   pl->at<int32_t>(pl->off_N0), pl->at<int32_t>(pl->off_nt),
                                   pl->at<double>(pl->off_coef), pl->P, pl->O, pl->NS, pl->n_t_max,
                                   static_cast<double *>(p_out), st);
    } else {
        {
            StageScope sc(pl, FWH_STAGE_GATHER, st);
            if (pl->gather_kind == FWH_GATHER_STREAM)
                e = fwh::launch_gather_stream(coef_type, pl->at<fwh::PairRec>(pl->off_rec_op), pl->rbf(),
                                              pl->at<int32_t>(pl->off_nt), pl->ws + pl->off_coef, pl->P, pl->O,
                                              pl->NS, pl->n_t_max, pl->splits, pl->at<float>(pl->off_part), st);
            else if (pl->gather_kind == FWH_GATHER_MFMA)
                e = fwh::launch_gather_mfma(coef_type, pl->at<fwh::PairRec>(pl->off_rec_op), pl->rbf(),
                                            pl->at<int2>(pl->off_tw), pl->at<int32_t>(pl->off_nt),
                                            pl->ws + pl->off_coef, pl->P, pl->O, pl->NS, pl->n_t_max, pl->splits,
                                            pl->wmax, pl->at<float>(pl->off_part), st);
            else if (pl->gather_kind == FWH_GATHER_LDS) {
                // full tiles with the 4 x 4 wave shape; a last tile of at most 16 observers with 2 x 8
                const int64_t n_tiles = (pl->O + fwh::kObsTile - 1) / fwh::kObsTile;
                const int64_t t_full = pl->tail_pt > 0 ? n_tiles - 1 : n_tiles;
                e = hipSuccess;
                if (t_full > 0)
                    e = fwh::launch_gather_lds(coef_type, pl->at<fwh::PairRec>(pl->off_rec_op), pl->rbf(),
                                               pl->at<int2>(pl->off_tw), pl->at<int32_t>(pl->off_nt),
                                               pl->ws + pl->off_coef, pl->P, pl->O, pl->NS, pl->n_t_max, pl->splits,
                                               pl->lds_nw, pl->lds_pt, pl->at<float>(pl->off_part), st, 0, t_full, 0);
                if (!e && t_full < n_tiles)
                    e = fwh::launch_gather_lds(coef_type, pl->at<fwh::PairRec>(pl->off_rec_op), pl->rbf(),
                                               pl->at<int2>(pl->off_tw), pl->at<int32_t>(pl->off_nt),
                                               pl->ws + pl->off_coef, pl->P, pl->O, pl->NS, pl->n_t_max, pl->splits,
                                               pl->tail_nw, pl->tail_pt, pl->at<float>(pl->off_part), st, t_full,
                                               n_tiles, 1);
            }
            else
                e = fwh::launch_gather_tuned(coef_type, pl->at<fwh::PairRec>(pl->off_rec_op),
                                             pl->at<int32_t>(pl->off_nt), pl->ws + pl->off_coef, pl->P, pl->O,
                                             pl->NS, pl->n_t_max, pl->splits, pl->at<float>(pl->off_part), st);
        }
        if (!e) {
            StageScope sc(pl, FWH_STAGE_REDUCE, st);
            e = fwh::launch_reduce_splits(pl->at<float>(pl->off_part), pl->splits, pl->O * pl->n_t_max,
                                          static_cast<float *>(p_out), st);
        }
    }
    if (e) return hip_fail("fwh_forward: gather kernel", e);
    return FWH_OK;
}

int fwh_adjoint(fwh_plan *pl, int32_t in_dtype, const void *rho, const void *u, const void *pp, const void *grad_p,
                void *g_rho, void *g_u, void *g_p, void *stream_) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_adjoint: null plan");
    if (!pl->ready) return fail(FWH_ESTATE, "fwh_adjoint: plan is not set up");
    if (!rho || !u || !pp || !grad_p || !g_rho || !g_u || !g_p)
        return fail(FWH_EINVAL, "fwh_adjoint: null data pointer");
    if (in_dtype != FWH_F64 && in_dtype != FWH_F32) return fail(FWH_EINVAL, "fwh_adjoint: bad in_dtype %d", in_dtype);
    hipStream_t st = as_stream(stream_);
    hipError_t e;
    const bool f64 = pl->mode == FWH_MODE_F64;
    {
    StageScope sc(pl, FWH_STAGE_ADJ_GATHER, st);
    if (f64)
        e = fwh::launch_adj_gather_f64(pl->at<double>(pl->off_K64), pl->at<double>(pl->off_W64),
                                       pl->at<int32_t>(pl->off_N0), pl->at<int32_t>(pl->off_nt),
                                       static_cast<const double *>(grad_p), pl->P, pl->O, pl->NS, pl->n_t_max,
                                       pl->at<double>(pl->off_coef), st);
    else
        e = fwh::launch_adj_gather(pl->at<fwh::PairRec>(pl->off_rec_op), pl->at<int32_t>(pl->off_nt),
                                       static_cast<const float *>(grad_p), pl->P, pl->O, pl->N, pl->NS,
                                       nt_min(pl), pl->n_t_max, pl->at<float>(pl->off_gpad),
                                       pl->at<float>(pl->off_coef), st);
    }
    if (e) return hip_fail("fwh_adjoint: transposed gather", e);
    {
        StageScope sc(pl, FWH_STAGE_SOURCE_ADJ, st);
        e = fwh::launch_source_adjoint(f64 ? 0 : 1, in_dtype == FWH_F64 ? 0 : 1, pl->ws + pl->off_coef, rho, u,
                                       pl->at<double>(pl->off_n), pl->P, pl->N, pl->NS, pl->flow,
                                       pl->at<double>(pl->off_cp), pl->scratch(), g_rho, g_u, g_p, st);
    }
    if (e) return hip_fail("fwh_adjoint: source adjoint", e);
    (void)pp;
    return FWH_OK;
}

int fwh_post(const fwh_plan *pl, const void *p_out, int64_t seg_len, double span_ratio, float *psd, float *rms,
             void *stream_) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_post: null plan");
    if (!pl->ready) return fail(FWH_ESTATE, "fwh_post: plan is not set up");
    if (!p_out || !psd || !rms) return fail(FWH_EINVAL, "fwh_post: null pointer");
    if (seg_len < 16 || seg_len > 4096 || (seg_len & (seg_len - 1)))
        return fail(FWH_ESIZE, "fwh_post: seg_len must be a power of two in [16, 4096] (got %lld)",
                    (long long)seg_len);
    if (!(span_ratio > 0.0) || !std::isfinite(span_ratio)) return fail(FWH_EINVAL, "fwh_post: span_ratio must be > 0");
    for (int64_t o = 0; o < pl->O; ++o)
        if (pl->n_t[o] < seg_len)
            return fail(FWH_ESIZE, "fwh_post: observer %lld has %lld samples, fewer than seg_len %lld", (long long)o,
                        (long long)pl->n_t[o], (long long)seg_len);
    hipError_t e = fwh::launch_post(pl->mode == FWH_MODE_F64 ? 0 : 1, p_out, pl->n_t_max, pl->at<int32_t>(pl->off_nt),
                                    pl->O, (int)seg_len, pl->flow.dtau, span_ratio, psd, rms, as_stream(stream_));
    if (e) return hip_fail("fwh_post", e);
    return FWH_OK;
}

int fwh_profile_enable(fwh_plan *pl, int enable) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_profile_enable: null plan");
    pl->profiling = enable != 0;
    return FWH_OK;
}

int fwh_profile_read(fwh_plan *pl, int32_t stage, double *total_ms, int64_t *launches) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_profile_read: null plan");
    if (stage < 0 || stage >= FWH_NUM_STAGES) return fail(FWH_EINVAL, "fwh_profile_read: bad stage %d", stage);
    double sum = 0.0;
    int64_t n = 0;
    int status = FWH_OK;
    for (auto &ab : pl->events[stage]) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(ab.second);
        if (!e) e = hipEventElapsedTime(&ms, ab.first, ab.second);
        if (e && status == FWH_OK) status = hip_fail("fwh_profile_read", e);
        sum += ms;
        ++n;
        (void)hipEventDestroy(ab.first);
        (void)hipEventDestroy(ab.second);
    }
    pl->events[stage].clear();
    if (total_ms) *total_ms = sum;
    if (launches) *launches = n;
    return status;
}

}  // extern "C"

struct fwh_batch {
    std::vector<fwh_batch_case> cases;
    int in_dtype = 0, mode = 0, n = 0;
    double item_units = 4.0e6;
    int blocks_per_cu = 2;
    int kind = FWH_GATHER_MFMA;        // forward gather of every case (matrix-core or LDS-staged)
    int umax = 0;                      // matrix units per wave the persistent kernel is compiled for
    std::vector<double> case_units;    // per case: target panel-observer-samples per forward item
    std::vector<int> case_rows;        // per case: rows of 61 samples per block (matrix-core gather)
    int64_t max_items = 0, n_items = 0, units = 0, grid = 0;
    int64_t max_adj_items = 0, n_adj_items = 0;
    int64_t blocks_src = 0, blocks_srcg = 0, blocks_red = 0, blocks_pad = 0, waves_adj = 0, blocks_sadj = 0,
            blocks_sadjg = 0;
    size_t shmem = 0;
    size_t off_cases = 0, off_idx = 0, off_items = 0, off_adj_items = 0, off_counter = 0, ws_bytes = 0;
    char *ws = nullptr;
    bool bound = false;
    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

extern "C" {

int fwh_batch_create(const fwh_batch_case *cases, int32_t n, int32_t in_dtype, fwh_batch **out,
                     size_t *workspace_bytes) {
    g_last_error.clear();
    if (out) *out = nullptr;
    if (!cases || !out || n < 1) return fail(FWH_EINVAL, "fwh_batch_create: need cases, out and n_cases >= 1");
    if (in_dtype != FWH_F64 && in_dtype != FWH_F32) return fail(FWH_EINVAL, "fwh_batch_create: bad in_dtype");
    int mode = -1;
    int64_t max_items = 0, max_adj_items = 0;
    for (int c = 0; c < n; ++c) {
        const fwh_batch_case &k = cases[c];
        if (!k.plan || !k.rho || !k.u || !k.p_prime || !k.p_out || !k.grad_p || !k.g_rho || !k.g_u || !k.g_p)
            return fail(FWH_EINVAL, "fwh_batch_create: case %d has a null pointer", c);
        if (!k.plan->ready) return fail(FWH_ESTATE, "fwh_batch_create: plan of case %d is not set up", c);
        if (k.plan->mode == FWH_MODE_F64)
            return fail(FWH_EINVAL, "fwh_batch_create: case %d uses the plain FP64 mode (batches run FP32/BF16)", c);
        if (mode < 0) mode = k.plan->mode;
        if (k.plan->mode != mode) return fail(FWH_EINVAL, "fwh_batch_create: cases mix FP32 and BF16 modes");
        if (k.plan->lds_pt <= 0 && k.plan->mfma_bpc <= 0)
            return fail(FWH_EINVAL, "fwh_batch_create: case %d has delay windows too wide for the batched gathers", c);
        // k blocks of at least 2 rows (matrix-core gather), 4 rows (LDS-staged gather)
        const int64_t tiles = ceil_div(k.plan->O, fwh::kObsTile),
                      kbs = ceil_div(k.plan->n_t_max, 2 * fwh::kLdsLanesOut);
        max_items += tiles * kbs * k.plan->max_splits;
        const int64_t nib = fwh::adj_blocks(k.plan->NS);
        max_adj_items += ceil_div(k.plan->P * nib, 4);
    }
    if (max_adj_items > INT32_MAX) return fail(FWH_ESIZE, "fwh_batch_create: too many adjoint work items");
    if (max_items > INT32_MAX) return fail(FWH_ESIZE, "fwh_batch_create: too many work items");
    fwh_batch *b = new (std::nothrow) fwh_batch();
    if (!b) return fail(FWH_EINVAL, "fwh_batch_create: out of host memory");
    b->cases.assign(cases, cases + n);
    b->n = n;
    b->in_dtype = in_dtype;
    b->mode = mode;
    b->max_items = max_items;
    b->max_adj_items = max_adj_items;
    // the LDS-staged gather when every case can take it, unless every plan asked for the matrix-core
    // one (fwh_plan_tune); the matrix-core gather when only it takes the windows of every case
    bool all_mfma = true, all_lds = true, want_mfma = true;
    for (int c = 0; c < n; ++c) {
        all_mfma = all_mfma && cases[c].plan->mfma_bpc > 0;
        all_lds = all_lds && cases[c].plan->lds_pt > 0;
        want_mfma = want_mfma && cases[c].plan->gather_variant == FWH_GATHER_MFMA;
        b->umax = std::max(b->umax, fwh::gather_mfma_umax(cases[c].plan->wmax));
    }
    if (!all_mfma && !all_lds) {
        delete b;
        return fail(FWH_EINVAL, "fwh_batch_create: no batched gather takes the delay windows of every case");
    }
    b->kind = all_mfma && (want_mfma || !all_lds) ? FWH_GATHER_MFMA : FWH_GATHER_LDS;
    b->case_units.assign((size_t)n, b->item_units);
    b->case_rows.assign((size_t)n, fwh::kLdsSub);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    b->off_cases = take((size_t)n * sizeof(fwh::BatchCase));
    b->off_idx = take((size_t)7 * (n + 1) * sizeof(int64_t));
    b->off_items = take((size_t)max_items * sizeof(int4));
    b->off_adj_items = take((size_t)max_adj_items * sizeof(int2));
    b->off_counter = take(sizeof(int));  // forward work-list counter
    b->ws_bytes = off;
    *out = b;
    if (workspace_bytes) *workspace_bytes = off;
    return FWH_OK;
}

int fwh_batch_tune(fwh_batch *b, double item_units, int32_t blocks_per_cu) {
    g_last_error.clear();
    if (!b) return fail(FWH_EINVAL, "fwh_batch_tune: null batch");
    if (blocks_per_cu < 1 || blocks_per_cu > 4) return fail(FWH_EINVAL, "fwh_batch_tune: blocks_per_cu in 1..4");
    if (item_units > 0.0) {
        b->item_units = item_units;
        b->case_units.assign((size_t)b->n, item_units);
    }
    b->blocks_per_cu = blocks_per_cu;
    b->bound = false;
    return FWH_OK;
}

int fwh_batch_tune_case(fwh_batch *b, int32_t c, double item_units, int32_t rows) {
    g_last_error.clear();
    if (!b) return fail(FWH_EINVAL, "fwh_batch_tune_case: null batch");
    if (c < 0 || c >= b->n) return fail(FWH_EINVAL, "fwh_batch_tune_case: case %d not in 0..%d", (int)c, b->n - 1);
    if (rows < 2 || rows > fwh::kLdsSub || (b->kind != FWH_GATHER_MFMA && rows != fwh::kLdsSub))
        return fail(FWH_EINVAL, "fwh_batch_tune_case: rows must be 2..%d (%d with the LDS-staged gather)",
                    fwh::kLdsSub, fwh::kLdsSub);
    if (item_units > 0.0) b->case_units[(size_t)c] = item_units;
    b->case_rows[(size_t)c] = rows;
    b->bound = false;
    return FWH_OK;
}

int fwh_batch_gather(const fwh_batch *b, int32_t *gather) {
    g_last_error.clear();
    if (!b) return fail(FWH_EINVAL, "fwh_batch_gather: null batch");
    if (gather) *gather = b->kind;
    return FWH_OK;
}

int fwh_batch_bind(fwh_batch *b, void *workspace, size_t workspace_bytes, void *stream_) {
    g_last_error.clear();
    if (!b) return fail(FWH_EINVAL, "fwh_batch_bind: null batch");
    if (!workspace || workspace_bytes < b->ws_bytes || reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(FWH_EWORKSPACE, "fwh_batch_bind: need a %zu-byte, 256-byte aligned workspace", b->ws_bytes);
    hipStream_t st = as_stream(stream_);
    const int n = b->n;
    const int coef_type = b->mode == FWH_MODE_F32 ? 1 : 2;
    std::vector<fwh::BatchCase> desc((size_t)n);
    std::vector<int64_t> idx((size_t)7 * (n + 1), 0);
    int64_t *s_src = idx.data(), *s_srcg = s_src + (n + 1), *s_red = s_srcg + (n + 1), *s_pad = s_red + (n + 1),
            *s_adj = s_pad + (n + 1), *s_sadj = s_adj + (n + 1), *s_sadjg = s_sadj + (n + 1);
    struct Item {
        double cost;
        int4 w;
    };
    std::vector<Item> items;
    struct AdjItem {
        double cost;
        int2 w;
    };
    std::vector<AdjItem> adj_items;
    b->units = 0;
    b->shmem = 0;
    for (int c = 0; c < n; ++c) {
        const fwh_batch_case &k = b->cases[c];
        fwh_plan *pl = k.plan;
        const int64_t P = pl->P, O = pl->O, N = pl->N, NS = pl->NS, ntm = pl->n_t_max;
        const bool mfma = b->kind == FWH_GATHER_MFMA;
        const int rows = mfma ? b->case_rows[(size_t)c] : fwh::kLdsSub;
        const int64_t kstep = (int64_t)fwh::kLdsLanesOut * rows;
        const int64_t tiles = ceil_div(O, fwh::kObsTile), kbs = ceil_div(ntm, kstep);
        // panel splits: work per item close to the case's target
        const double tile_units = (double)P * std::min<int64_t>(O, fwh::kObsTile) * std::min<int64_t>(ntm, kstep);
        int64_t S = (int64_t)std::ceil(tile_units / b->case_units[(size_t)c]);
        S = std::max<int64_t>(1, std::min<int64_t>(S, pl->max_splits));
        const int64_t p_chunk = ceil_div(P, S);
        const int64_t LR = fwh::adj_pad_row(N, NS), padlo = fwh::adj_pad_lo(N);
        const int64_t nib = fwh::adj_blocks(NS);
        fwh::BatchCase &d = desc[c];
        d.src = fwh::SrcFwdArgs{k.rho, k.u, k.p_prime, pl->at<double>(pl->off_n), P, N, NS, pl->flow,
                                pl->at<double>(pl->off_cp), pl->scratch(), pl->ws + pl->off_coef};
        d.gat = fwh::GatherArgs{pl->at<fwh::PairRec>(pl->off_rec_op), pl->rbf(), pl->at<int2>(pl->off_tw),
                                pl->at<int32_t>(pl->off_nt), pl->ws + pl->off_coef, P, O, NS, ntm, p_chunk,
                                mfma ? fwh::gather_mfma_y_row(pl->wmax) : pl->lds_nw, pl->lds_pt, (int)S,
                                pl->at<float>(pl->off_part), rows};
        d.red = fwh::ReduceArgs{pl->at<float>(pl->off_part), (int)S, O * ntm, static_cast<float *>(k.p_out)};
        d.pad = fwh::PadArgs{static_cast<const float *>(k.grad_p), pl->at<int32_t>(pl->off_nt), O, ntm, LR, padlo,
                             pl->at<float>(pl->off_gpad)};
        d.adj = fwh::AdjArgs{pl->at<fwh::PairRec>(pl->off_rec_op), pl->at<float>(pl->off_gpad), P, O, NS, LR, padlo,
                             nib, pl->at<float>(pl->off_coef), ntm, N - nt_min(pl), nt_min(pl) + 2};
        d.sadj = fwh::SrcAdjArgs{pl->at<float>(pl->off_coef), k.rho, k.u, pl->at<double>(pl->off_n), P, N, NS,
                                 pl->flow, pl->at<double>(pl->off_cp), k.g_rho, k.g_u, k.g_p};
        const int64_t src_int = fwh::src_interior_chunks(N);
        s_src[c + 1] = s_src[c] + ceil_div(P, fwh::kSrcPanels) * src_int;
        s_srcg[c + 1] = s_srcg[c] + ceil_div(P, fwh::kSrcPanels) * (NS / fwh::kSrcTC - src_int);
        s_red[c + 1] = s_red[c] + ceil_div(O * ntm, 256);
        s_pad[c + 1] = s_pad[c] + ceil_div(O * LR, 256);
        s_adj[c + 1] = s_adj[c] + P * nib;
        const int64_t adj_int = fwh::adj_interior_chunks(N);
        s_sadj[c + 1] = s_sadj[c] + ceil_div(P, fwh::kSrcPanels) * adj_int;
        s_sadjg[c + 1] = s_sadjg[c] + ceil_div(P, fwh::kSrcPanels) * (fwh::adj_chunks(N) - adj_int);
        b->shmem = std::max(b->shmem, mfma ? fwh::gather_mfma_shmem(pl->wmax)
                                           : fwh::gather_lds_shmem(coef_type, pl->lds_nw, pl->lds_pt));
        for (int64_t t = 0; t < tiles; ++t)
            for (int64_t kb = 0; kb < kbs; ++kb)
                for (int64_t z = 0; z < S; ++z) {
                    const int64_t np = std::max<int64_t>(0, std::min(P, (z + 1) * p_chunk) - z * p_chunk);
                    const int64_t no = std::min<int64_t>(fwh::kObsTile, O - t * fwh::kObsTile);
                    const int64_t nk = std::min<int64_t>(kstep, ntm - kb * kstep);
                    items.push_back({(double)np * no * nk, make_int4(c, (int)t, (int)kb, (int)z)});
                }
        // transposed gather: items of 4 (panel, index block) waves, each wave costing O x 244
        // panel-observer-samples (the last item of a case may be partly empty)
        const int64_t groups = ceil_div(P * nib, 4);
        for (int64_t g = 0; g < groups; ++g) {
            const int64_t waves = std::min<int64_t>(4, P * nib - 4 * g);
            adj_items.push_back({(double)waves * O, make_int2(c, (int)g)});
        }
        int64_t sum_nt = 0;
        for (int64_t o = 0; o < O; ++o) sum_nt += pl->n_t[o];
        b->units += P * sum_nt;
    }
    // longest first (the paper's greedy partition by size), ties in case order
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
    std::stable_sort(adj_items.begin(), adj_items.end(),
                     [](const AdjItem &x, const AdjItem &y) { return x.cost > y.cost; });
    std::vector<int4> wl(items.size());
    for (size_t i = 0; i < items.size(); ++i) wl[i] = items[i].w;
    std::vector<int2> wla(adj_items.size());
    for (size_t i = 0; i < adj_items.size(); ++i) wla[i] = adj_items[i].w;
    b->n_items = (int64_t)wl.size();
    b->n_adj_items = (int64_t)wla.size();
    b->blocks_src = s_src[n];
    b->blocks_srcg = s_srcg[n];
    b->blocks_red = s_red[n];
    b->blocks_pad = s_pad[n];
    b->waves_adj = s_adj[n];
    b->blocks_sadj = s_sadj[n];
    b->blocks_sadjg = s_sadjg[n];
    int dev = 0, cus = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) || (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)))
        return hip_fail("fwh_batch_bind: device query", e);
    b->grid = (int64_t)cus * b->blocks_per_cu;
    b->ws = static_cast<char *>(workspace);
    if ((e = hipMemcpyAsync(b->at<fwh::BatchCase>(b->off_cases), desc.data(), desc.size() * sizeof(fwh::BatchCase),
                            hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(b->at<int64_t>(b->off_idx), idx.data(), idx.size() * sizeof(int64_t),
                            hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(b->at<int4>(b->off_items), wl.data(), wl.size() * sizeof(int4), hipMemcpyHostToDevice,
                            st)) ||
        (e = hipMemcpyAsync(b->at<int2>(b->off_adj_items), wla.data(), wla.size() * sizeof(int2),
                            hipMemcpyHostToDevice, st)) ||
        (e = hipStreamSynchronize(st)))
        return hip_fail("fwh_batch_bind: upload", e);
    b->bound = true;
    return FWH_OK;
}

static fwh::BatchIndex batch_index(const fwh_batch *b) {
    const int64_t *base = b->at<int64_t>(b->off_idx);
    const int64_t m = b->n + 1;
    return fwh::BatchIndex{base,         base + m,     base + 2 * m, base + 3 * m,
                           base + 4 * m, base + 5 * m, base + 6 * m, b->n};
}

int fwh_batch_forward(fwh_batch *b, void *stream_) {
    g_last_error.clear();
    if (!b || !b->bound) return fail(FWH_ESTATE, "fwh_batch_forward: batch is not bound");
    hipError_t e = fwh::launch_batch_forward(b->in_dtype == FWH_F64 ? 0 : 1, b->mode == FWH_MODE_F32 ? 1 : 2,
                                             b->kind == FWH_GATHER_MFMA ? b->umax : 0,
                                             b->at<fwh::BatchCase>(b->off_cases), batch_index(b),
                                             b->at<int4>(b->off_items), (int)b->n_items, b->at<int>(b->off_counter),
                                             (int)b->grid, b->shmem, b->blocks_src, b->blocks_srcg, b->blocks_red,
                                             as_stream(stream_));
    if (e) return hip_fail("fwh_batch_forward", e);
    return FWH_OK;
}

int fwh_batch_adjoint(fwh_batch *b, void *stream_) {
    g_last_error.clear();
    if (!b || !b->bound) return fail(FWH_ESTATE, "fwh_batch_adjoint: batch is not bound");
    hipError_t e = fwh::launch_batch_adjoint(b->in_dtype == FWH_F64 ? 0 : 1, b->at<fwh::BatchCase>(b->off_cases),
                                             batch_index(b), b->blocks_pad, b->at<int2>(b->off_adj_items),
                                             (int)b->n_adj_items, b->blocks_sadj, b->blocks_sadjg,
                                             as_stream(stream_));
    if (e) return hip_fail("fwh_batch_adjoint", e);
    return FWH_OK;
}

int fwh_batch_info(const fwh_batch *b, int64_t *n_items, int64_t *units, int64_t *grid) {
    g_last_error.clear();
    if (!b) return fail(FWH_EINVAL, "fwh_batch_info: null batch");
    if (n_items) *n_items = b->n_items;
    if (units) *units = b->units;
    if (grid) *grid = b->grid;
    return FWH_OK;
}

void fwh_batch_destroy(fwh_batch *b) { delete b; }

void fwh_destroy(fwh_plan *pl) {
    if (!pl) return;
    for (auto &v : pl->events)
        for (auto &ab : v) {
            (void)hipEventDestroy(ab.first);
            (void)hipEventDestroy(ab.second);
        }
    delete pl;
}

}  // extern "C"

// ------------------------------------------------------------ general motion

struct fwh_gm_plan {
    fwh_gm_args a{};
    int64_t NS = 0, nt_cap = 0;
    int splits = 1;
    int64_t p_chunk = 0;
    std::vector<double> inv_beta;
    std::vector<double> t_start;
    std::vector<int64_t> n_t;
    int64_t n_t_max = 0;
    size_t off_coef = 0, off_ib = 0, off_ts = 0, off_nt = 0, off_part = 0, ws_bytes = 0;
    char *ws = nullptr;
    bool ready = false;
    // optional per-stage event timing (FWH_GM_STAGE_SOURCE, FWH_GM_STAGE_GATHER)
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events[FWH_GM_NUM_STAGES];
};

namespace {
struct GmStageScope {
    fwh_gm_plan *pl;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    GmStageScope(fwh_gm_plan *p, int s, hipStream_t stream) : pl(p), stage(s), st(stream) {
        if (pl->profiling && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, st);
    }
    ~GmStageScope() {
        if (a && b) {
            (void)hipEventRecord(b, st);
            pl->events[stage].emplace_back(a, b);
        }
    }
};
}  // namespace

extern "C" {

int fwh_gm_plan_create(const fwh_gm_args *a, fwh_gm_plan **out, size_t *workspace_bytes) {
    g_last_error.clear();
    if (!a || !out) return fail(FWH_EINVAL, "fwh_gm_plan_create: null argument");
    *out = nullptr;
    if (a->n_panels < 1 || a->n_obs < 1 || a->n_tau < 4)
        return fail(FWH_ESIZE, "fwh_gm_plan_create: need n_panels >= 1, n_obs >= 1, n_tau >= 4 (got %lld, %lld, %lld)",
                    (long long)a->n_panels, (long long)a->n_obs, (long long)a->n_tau);
    if (a->n_tau > (1 << 20) || a->n_panels > ((int64_t)1 << 26) || a->n_obs > ((int64_t)1 << 20) ||
        a->n_panels * a->n_tau > ((int64_t)1 << 36))
        return fail(FWH_ESIZE, "fwh_gm_plan_create: sizes beyond the supported range");
    if (!a->y || !a->normal || !a->vel || !a->dS || !a->x_obs)
        return fail(FWH_EINVAL, "fwh_gm_plan_create: null kinematics pointer");
    if (!(a->mach > 0.0 && a->mach < 1.0))
        return fail(FWH_EDOMAIN, "fwh_gm_plan_create: mach must be in (0, 1), got %g", a->mach);
    if (!(a->dtau > 0.0) || !std::isfinite(a->dtau))
        return fail(FWH_EDOMAIN, "fwh_gm_plan_create: dtau must be positive, got %g", a->dtau);
    if (!std::isfinite(a->tau0)) return fail(FWH_EINVAL, "fwh_gm_plan_create: tau0 must be finite");
    fwh_gm_plan *pl = new (std::nothrow) fwh_gm_plan;
    if (!pl) return fail(FWH_EINVAL, "fwh_gm_plan_create: out of host memory");
    pl->a = *a;
    const int64_t P = a->n_panels, O = a->n_obs, N = a->n_tau;
    pl->NS = N + 2;
    pl->nt_cap = 2 * N;
    // Thomas pivots of tridiag(1, 4, 1): c'_1 = 1/4, c'_n = 1 / (4 - c'_{n-1})
    pl->inv_beta.assign(fwh::kGmPivots, 0.0);
    double c = 0.0;
    for (int n = 1; n < fwh::kGmPivots; ++n) {
        c = 1.0 / (4.0 - c);
        pl->inv_beta[n] = c;
    }
    // panel splits: blocks of 4 observers x 64 samples x panel range (the record length stands in for
    // the window), 4 resident per CU.  As for the wind-tunnel gather, among the split counts within
    // 3 % of the fewest rounds per unit of work take the largest that keeps the launch within 32
    // rounds (at most 1024 splits, at least 16 panels each)
    const int64_t nkb = (N + 63) / 64;
    const int64_t gblocks = nkb * ((O + 3) / 4), gres = 4 * 256;
    const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(1024, P / 16));
    auto grounds = [&](int64_t c) { return (double)((gblocks * c + gres - 1) / gres) / (double)c; };
    double gbest = 1e300;
    for (int64_t c = 1; c <= smax; ++c) gbest = std::min(gbest, grounds(c));
    int64_t sp = 1;
    for (int64_t c = 1; c <= smax; ++c)
        if (grounds(c) <= gbest * 1.03 && (c == 1 || gblocks * c <= 32 * gres)) sp = c;
    pl->splits = (int)sp;
    pl->p_chunk = (P + pl->splits - 1) / pl->splits;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    pl->off_coef = take((size_t)P * fwh::kGmRows * pl->NS * sizeof(double));
    pl->off_ib = take(fwh::kGmPivots * sizeof(double));
    pl->off_ts = take((size_t)O * sizeof(double));
    pl->off_nt = take((size_t)O * sizeof(int32_t));
    pl->off_part = take((size_t)pl->splits * O * pl->nt_cap * sizeof(double));
    pl->ws_bytes = off;
    if (workspace_bytes) *workspace_bytes = pl->ws_bytes;
    *out = pl;
    return FWH_OK;
}

int fwh_gm_window(fwh_gm_plan *pl, void *workspace, size_t workspace_bytes, void *stream_) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_gm_window: null plan");
    if (!workspace) return fail(FWH_EWORKSPACE, "fwh_gm_window: null workspace");
    if (workspace_bytes < pl->ws_bytes)
        return fail(FWH_EWORKSPACE, "fwh_gm_window: workspace of %zu bytes, need %zu", workspace_bytes, pl->ws_bytes);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(FWH_EWORKSPACE, "fwh_gm_window: workspace must be %zu-byte aligned", kAlign);
    pl->ready = false;
    pl->ws = static_cast<char *>(workspace);
    hipStream_t st = as_stream(stream_);
    const int64_t O = pl->a.n_obs;
    hipError_t e = hipMemcpyAsync(pl->ws + pl->off_ib, pl->inv_beta.data(), fwh::kGmPivots * sizeof(double),
                                  hipMemcpyHostToDevice, st);
    if (e) return hip_fail("fwh_gm_window: pivot table copy", e);
    fwh::GmWinArgs w{};
    w.y = pl->a.y;
    w.x_obs = pl->a.x_obs;
    w.mach = pl->a.mach;
    w.dtau = pl->a.dtau;
    w.tau0 = pl->a.tau0;
    w.P = pl->a.n_panels;
    w.O = O;
    w.N = pl->a.n_tau;
    w.t_start = reinterpret_cast<double *>(pl->ws + pl->off_ts);
    w.n_t = reinterpret_cast<int32_t *>(pl->ws + pl->off_nt);
    e = fwh::launch_gm_window(w, st);
    if (e) return hip_fail("fwh_gm_window: window kernel", e);
    pl->t_start.assign(O, 0.0);
    std::vector<int32_t> nt32(O, 0);
    e = hipMemcpyAsync(pl->t_start.data(), w.t_start, O * sizeof(double), hipMemcpyDeviceToHost, st);
    if (!e) e = hipMemcpyAsync(nt32.data(), w.n_t, O * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (!e) e = hipStreamSynchronize(st);
    if (e) return hip_fail("fwh_gm_window: window copy", e);
    pl->n_t.assign(O, 0);
    pl->n_t_max = 0;
    for (int64_t o = 0; o < O; ++o) {
        if (nt32[o] < 1)
            return fail(FWH_EWINDOW, "fwh_gm_window: observer %lld has an empty window", (long long)o);
        if (nt32[o] >= pl->nt_cap)
            return fail(FWH_ESIZE, "fwh_gm_window: observer %lld has N_t = %d >= 2N (supersonic surface motion?)",
                        (long long)o, nt32[o]);
        pl->n_t[o] = nt32[o];
        pl->n_t_max = std::max<int64_t>(pl->n_t_max, nt32[o]);
    }
    pl->ready = true;
    return FWH_OK;
}

int fwh_gm_obs_window(const fwh_gm_plan *pl, double *t_start, int64_t *n_t, int64_t *n_t_max) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_gm_obs_window: null plan");
    if (!pl->ready) return fail(FWH_ESTATE, "fwh_gm_obs_window: no window computed");
    if (t_start) std::copy(pl->t_start.begin(), pl->t_start.end(), t_start);
    if (n_t) std::copy(pl->n_t.begin(), pl->n_t.end(), n_t);
    if (n_t_max) *n_t_max = pl->n_t_max;
    return FWH_OK;
}

int fwh_gm_forward(fwh_gm_plan *pl, const double *rho, const double *u, const double *pp, double *p_out,
                   void *stream_) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_gm_forward: null plan");
    if (!pl->ready) return fail(FWH_ESTATE, "fwh_gm_forward: no window computed");
    if (!rho || !u || !pp || !p_out) return fail(FWH_EINVAL, "fwh_gm_forward: null data pointer");
    // one launch of 256-thread blocks: at most 2^32 work-items
    if ((int64_t)pl->splits * ((pl->a.n_obs + 3) / 4) * ((pl->n_t_max + 63) / 64) * 256 >= ((int64_t)1 << 32))
        return fail(FWH_ESIZE, "fwh_gm_forward: %lld observers x %lld samples x %d panel ranges exceed one launch",
                    (long long)pl->a.n_obs, (long long)pl->n_t_max, pl->splits);
    hipStream_t st = as_stream(stream_);
    fwh::GmChanArgs c{};
    c.y = pl->a.y;
    c.normal = pl->a.normal;
    c.vel = pl->a.vel;
    c.rho = rho;
    c.u = u;
    c.pp = pp;
    c.mach = pl->a.mach;
    c.dtau = pl->a.dtau;
    c.P = pl->a.n_panels;
    c.N = pl->a.n_tau;
    c.NS = pl->NS;
    c.coef = reinterpret_cast<double *>(pl->ws + pl->off_coef);
    hipError_t e;
    {
        GmStageScope sc(pl, FWH_GM_STAGE_SOURCE, st);
        e = fwh::launch_gm_source(c, reinterpret_cast<const double *>(pl->ws + pl->off_ib), st);
    }
    if (e) return hip_fail("fwh_gm_forward: source stage", e);
    fwh::GmGatherArgs g{};
    g.coef = c.coef;
    g.dS = pl->a.dS;
    g.x_obs = pl->a.x_obs;
    g.t_start = reinterpret_cast<const double *>(pl->ws + pl->off_ts);
    g.n_t = reinterpret_cast<const int32_t *>(pl->ws + pl->off_nt);
    g.mach = pl->a.mach;
    g.dtau = pl->a.dtau;
    g.tau0 = pl->a.tau0;
    g.P = pl->a.n_panels;
    g.O = pl->a.n_obs;
    g.N = pl->a.n_tau;
    g.NS = pl->NS;
    g.nt_stride = pl->n_t_max;
    g.nkb = (pl->n_t_max + 63) / 64;
    g.p_chunk = pl->p_chunk;
    g.splits = pl->splits;
    g.part = reinterpret_cast<double *>(pl->ws + pl->off_part);
    {
        GmStageScope sc(pl, FWH_GM_STAGE_GATHER, st);
        e = fwh::launch_gm_gather(g, p_out, st);
    }
    if (e) return hip_fail("fwh_gm_forward: gather", e);
    return FWH_OK;
}

int fwh_gm_profile_enable(fwh_gm_plan *pl, int enable) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_gm_profile_enable: null plan");
    pl->profiling = enable != 0;
    return FWH_OK;
}

int fwh_gm_profile_read(fwh_gm_plan *pl, int32_t stage, double *total_ms, int64_t *launches) {
    g_last_error.clear();
    if (!pl) return fail(FWH_EINVAL, "fwh_gm_profile_read: null plan");
    if (stage < 0 || stage >= FWH_GM_NUM_STAGES) return fail(FWH_EINVAL, "fwh_gm_profile_read: bad stage %d", stage);
    double tot = 0.0;
    int64_t n = 0;
    for (auto &ab : pl->events[stage]) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(ab.second);
        if (!e) e = hipEventElapsedTime(&ms, ab.first, ab.second);
        if (e) return hip_fail("fwh_gm_profile_read", e);
        tot += ms;
        ++n;
        (void)hipEventDestroy(ab.first);
        (void)hipEventDestroy(ab.second);
    }
    pl->events[stage].clear();
    if (total_ms) *total_ms = tot;
    if (launches) *launches = n;
    return FWH_OK;
}

void fwh_gm_destroy(fwh_gm_plan *pl) {
    if (!pl) return;
    for (auto &v : pl->events)
        for (auto &ab : v) {
            (void)hipEventDestroy(ab.first);
            (void)hipEventDestroy(ab.second);
        }
    delete pl;
}

const char *fwh_last_error(void) { return g_last_error.c_str(); }

int fwh_forward_noalloc(const fwh_setup_args *args, int32_t in_dtype, const void *rho, const void *u,
                        const void *pp, void *p_out, int64_t out_capacity, int64_t *n_t_max, void *stream) {
    g_last_error.clear();
    if (!args || !rho || !u || !pp || !p_out || !n_t_max)
        return fail(FWH_EINVAL, "fwh_forward_noalloc: null argument");
    if (in_dtype != FWH_F64 && in_dtype != FWH_F32)
        return fail(FWH_EINVAL, "fwh_forward_noalloc: bad in_dtype %d", in_dtype);
    fwh_plan *pl = nullptr;
    size_t need = 0;
    int rc = fwh_plan_create(args, &pl, &need);
    if (rc != FWH_OK) return rc;
    struct Release {
        fwh_plan *p;
        ~Release() { fwh_destroy(p); }
    } release{pl};
    if (need > kNoAllocBytes)
        return fail(FWH_ESIZE,
                    "fwh_forward_noalloc: the case needs a %zu-byte workspace, more than the %zu bytes of the "
                    "static one (use fwh_plan_create / fwh_setup / fwh_forward with a caller workspace)",
                    need, kNoAllocBytes);
    // this device's copy of the static workspace, looked up once per device
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e) return hip_fail("fwh_forward_noalloc: hipGetDevice", e);
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(FWH_EINVAL, "fwh_forward_noalloc: device %d beyond the %d supported", dev, kNoAllocMaxDevices);
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return hip_fail("fwh_forward_noalloc: address of the static workspace", e);
            g_noalloc_ptr[dev] = p;
        }
        ws = g_noalloc_ptr[dev];
    }
    // setup writes every table it later reads, the forward every coefficient and partial it reads,
    // so nothing left by an earlier call is read and nothing needs clearing
    if ((rc = fwh_setup(pl, ws, kNoAllocBytes, stream)) != FWH_OK) return rc;
    *n_t_max = pl->n_t_max;
    if (pl->O * pl->n_t_max > out_capacity)
        return fail(FWH_ESIZE, "fwh_forward_noalloc: p_out holds %lld elements, the output needs %lld x %lld",
                    (long long)out_capacity, (long long)pl->O, (long long)pl->n_t_max);
    return fwh_forward(pl, in_dtype, rho, u, pp, p_out, stream);
}

const char *fwh_version(void) { return "fwh-mi355x 0.1 (gfx950)"; }

}  // extern "C"
