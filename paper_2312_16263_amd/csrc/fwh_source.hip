// Source stage (gfx950): per panel and source frame, the source terms of
// Eqs. (Qn_New_nd), (Li_New_nd); their 2nd-order source-time derivatives
// (one-sided at the first and last frame, central elsewhere; Sec. III B); and the
// B-spline coefficients of the natural cubic spline through each of the 8
// resulting series (the observer-independent half of the "interp pressure
// signal" step).  Plus the exact transpose of this stage for the adjoint.
//
// The natural cubic spline through f_0..f_{N-1} is sum_n c_n B((tau - tau_n)/dtau)
// with B the uniform cubic B-spline; natural end conditions give c_0 = f_0,
// c_{N-1} = f_{N-1}, c_{-1} = 2c_0 - c_1, c_N = 2c_{N-1} - c_{N-2} and, inside,
// (c_{n-1} + 4 c_n + c_{n+1})/6 = f_n, a constant tridiagonal system solved by
// the Thomas algorithm with the precomputed pivots cp[r] (cp[1] = 1/4,
// cp[r] = 1/(4 - cp[r-1])).
//
// Layout: one thread per (panel, channel), a wave = 64 consecutive panels of one
// channel and a block = the 4 channels of one channel group, so every time step
// is one coalesced load per input variable.  The forward elimination streams
// the inputs in time order and writes the reduced right-hand sides to a
// time-major scratch [8][N][P]; back substitution runs in reverse time order and
// the coefficients go out panel-major with the 4 channels of a group
// interleaved, coef[P][2][NS][4] (one 4-channel quad per time index), through a
// block-wide LDS transpose.  All arithmetic FP64.
#include "fwh_internal.h"

namespace fwh {
namespace {

struct bf16s {
    uint16_t bits;
};

template <typename T>
struct Store;
template <>
struct Store<double> {
    static __device__ __forceinline__ double put(double v) { return v; }
};
template <>
struct Store<float> {
    static __device__ __forceinline__ float put(double v) { return (float)v; }
};
template <>
struct Store<bf16s> {
    // double -> float (round to nearest even) -> bfloat16 (round to nearest even)
    static __device__ __forceinline__ bf16s put(double v) {
        const float x = (float)v;
        uint32_t u = __float_as_uint(x);
        bf16s r;
        if ((u & 0x7fffffffu) > 0x7f800000u) {
            r.bits = (uint16_t)((u >> 16) | 0x40u);
        } else {
            u += 0x7fffu + ((u >> 16) & 1u);
            r.bits = (uint16_t)(u >> 16);
        }
        return r;
    }
};

// Channel c: base quantity (0 = Q, 1..3 = L_i) and whether it is the derivative.
__device__ __forceinline__ int channel_base(int c) { return c <= 1 ? 0 : (c <= 4 ? c - 1 : c - 4); }
__device__ __forceinline__ bool channel_deriv(int c) { return c == 0 || (c >= 2 && c <= 4); }

struct PanelFrame {
    double nx, ny, nz, U0n;
};

// Source term of the given base at time-major index idx (Eqs. (Qn_New_nd), (Li_New_nd)):
//   Q = rho u.n - U0.n,  L_i = p' n_i + rho (u_i - U0_i) u.n
template <typename TIn>
__device__ __forceinline__ double source_term(int base, const TIn *__restrict__ rho, const TIn *__restrict__ u,
                                              const TIn *__restrict__ pp, int64_t idx, int64_t NP,
                                              const PanelFrame &pf, const Flow &f) {
    const double r = (double)rho[idx];
    const double u1 = (double)u[idx], u2 = (double)u[NP + idx], u3 = (double)u[2 * NP + idx];
    const double un = u1 * pf.nx + u2 * pf.ny + u3 * pf.nz;
    if (base == 0) return r * un - pf.U0n;
    const double pv = (double)pp[idx];
    if (base == 1) return pv * pf.nx + r * (u1 - f.ca) * un;
    if (base == 2) return pv * pf.ny + r * (u2 - f.sa) * un;
    return pv * pf.nz + r * u3 * un;
}

template <typename TIn, typename TScr, typename TOut>
__device__ __forceinline__ void source_fwd_body(const SrcFwdArgs &a, int64_t bx, int by) {
    const TIn *__restrict__ rho = static_cast<const TIn *>(a.rho);
    const TIn *__restrict__ u = static_cast<const TIn *>(a.u);
    const TIn *__restrict__ pp = static_cast<const TIn *>(a.pp);
    const double *__restrict__ normal = a.normal;
    const int64_t P = a.P, N = a.N, NS = a.NS;
    const Flow f = a.f;
    const double *__restrict__ cp = a.cp;
    TScr *__restrict__ scr = static_cast<TScr *>(a.scr);
    TOut *__restrict__ coef = static_cast<TOut *>(a.coef);
    constexpr int CH = 128 / (int)sizeof(TOut);  // time indices per flush (128-byte row segments per channel)
    constexpr int PF = 8;                        // time steps loaded ahead
    constexpr int RS = CH * 4 + 1;               // padded LDS row: [CH][4 channels] + 1
    __shared__ TOut stage[64 * RS];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int ch = by * 4 + wv;
    const int base = channel_base(ch);
    const bool deriv = channel_deriv(ch);
    const int64_t pbase = bx * 64;
    const int64_t p = pbase + lane;
    const bool active = p < P;
    const int64_t pc = active ? p : P - 1;
    const int64_t NP = N * P;
    PanelFrame pf;
    pf.nx = normal[3 * pc];
    pf.ny = normal[3 * pc + 1];
    pf.nz = normal[3 * pc + 2];
    pf.U0n = f.ca * pf.nx + f.sa * pf.ny;
    const double i2h = 1.0 / (2.0 * f.dtau);

    auto X = [&](int64_t n) { return source_term<TIn>(base, rho, u, pp, n * P + pc, NP, pf, f); };

    // ---- forward sweep: f_n for n = 0..N-1, Thomas row r = n-1 once f_n is known
    const double X0 = X(0), X1 = X(1), X2 = X(2);
    const double f0 = deriv ? (-3.0 * X0 + 4.0 * X1 - X2) * i2h : X0;
    double Xmm = 0.0, Xm = X0, Xc = X1, Xp = X2;
    double fprev = f0, fN1 = 0.0, dprev = 0.0;
    TScr *scr_ch = scr + (int64_t)ch * NP;
    for (int64_t nb = 1; nb < N; nb += PF) {
        double Xf[PF];
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int64_t n2 = nb + i + 2;
            Xf[i] = (n2 < N) ? X(n2) : 0.0;
        }
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int64_t n = nb + i;
            if (n < N) {
                double fn;
                if (n < N - 1) fn = deriv ? (Xp - Xm) * i2h : Xc;
                else fn = deriv ? (3.0 * Xc - 4.0 * Xm + Xmm) * i2h : Xc;
                const int64_t r = n - 1;
                if (r >= 1) {
                    double rhs = 6.0 * fprev;
                    if (r == 1) rhs -= f0;
                    if (r == N - 2) rhs -= fn;
                    const double d = (rhs - dprev) * cp[r];
                    if (active) scr_ch[r * P + p] = (TScr)d;
                    dprev = d;
                }
                if (n == N - 1) fN1 = fn;
                fprev = fn;
                Xmm = Xm;
                Xm = Xc;
                Xc = Xp;
                Xp = Xf[i];
            }
        }
    }

    // ---- back substitution in reverse order, coefficients by storage index i:
    // i = 0: c_{-1}; i = n+1: c_n (n = 0..N-1); i = N+1: c_N; i >= N+2: 0.
    const double xN2 = dprev;  // x_{N-2} = d'_{N-2}
    double x = xN2;            // x_{n+1} of the recurrence
    const int cc = ch & 3;  // channel within the group
    constexpr int SB = CH < 16 ? CH : 16;  // back-substitution steps loaded ahead
    for (int64_t b = NS / CH - 1; b >= 0; --b) {
        const int64_t i0 = b * CH;
        for (int sb = CH - SB; sb >= 0; sb -= SB) {
            double dpre[SB];
#pragma unroll
            for (int q = 0; q < SB; ++q) {
                const int64_t n = i0 + sb + q - 1;
                dpre[q] = (n >= 1 && n <= N - 3 && active) ? (double)scr_ch[n * P + p] : 0.0;
            }
#pragma unroll
            for (int q = SB - 1; q >= 0; --q) {
                const int64_t i = i0 + sb + q;
                double v;
                if (i >= N + 2) v = 0.0;
                else if (i == N + 1) v = 2.0 * fN1 - xN2;
                else if (i == N) v = fN1;
                else if (i >= 2) {
                    const int64_t n = i - 1;
                    if (n <= N - 3) x = dpre[q] - cp[n] * x;
                    v = x;
                } else if (i == 1) v = f0;
                else v = 2.0 * f0 - x;
                stage[lane * RS + (sb + q) * 4 + cc] = Store<TOut>::put(v);
            }
        }
        __syncthreads();
        // block-wide flush: for each of the 64 panels, CH quads of 4 channels, contiguous in memory
        for (int t = threadIdx.x; t < 64 * CH; t += 256) {
            const int r = t / CH, col = t - r * CH;
            const int64_t prow = pbase + r;
            if (prow < P) {
                TOut *dst = coef + (((prow * 2 + by) * NS) + i0 + col) * 4;
                const TOut *src = stage + r * RS + col * 4;
                dst[0] = src[0];
                dst[1] = src[1];
                dst[2] = src[2];
                dst[3] = src[3];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- chunked source stage
// FP32 and BF16 coefficient modes (the plain FP64 form keeps the exact
// sequential kernel above).  Geometry in fwh_internal.h: a block owns 32 panels
// and 64 coefficient indices; wave w handles base quantity w (Q, L_1, L_2, L_3)
// with lanes 0-31 on its derivative channel and lanes 32-63 on the channel
// itself, so the source terms are wave-uniform.  Each thread runs the forward
// elimination over the rows [R0, R0 + kSrcW) (pivots from the exact table, so a
// window that reaches row 1 is exact) and back-substitutes from the top of the
// window (exact when it reaches row N-2).  Starting elsewhere from zero moves
// the chunk's coefficients by about (2 - sqrt 3)^kSrcH = 7e-10 of their local
// scale, below the FP32/BF16 storage rounding.  No workspace buffer: the
// coefficients leave through an LDS tile [kSrcTC / 4][257], a quarter of the
// chunk at a time, as 16-byte (8-byte for BF16) quads of the interleaved layout.
constexpr int kSrcRS = 257;  // LDS row: 8 channels x 32 panels + 1

// Per-thread source-term form X = a p' + rho (b.u - g) u.n - d, which covers
// Q (a = 0, b = 0, g = -1, d = U0.n) and L_i (a = n_i, b = e_i, g = U0_i, d = 0).
template <typename TIn>
struct SrcLane {
    const TIn *rho, *u, *pp;
    int64_t NP;
    double nx, ny, nz, al, b1, b2, b3, gm, dl;
    double s_der, s_val;  // f = s_der (X+ - X-) + s_val X
    int ch;               // channel index (0..7)
    __device__ __forceinline__ SrcLane(const SrcFwdArgs &a, int64_t pc) {
        rho = static_cast<const TIn *>(a.rho) + pc;
        u = static_cast<const TIn *>(a.u) + pc;
        pp = static_cast<const TIn *>(a.pp) + pc;
        NP = a.N * a.P;
        const int w = threadIdx.x >> 6;
        const bool der = (threadIdx.x & 32) == 0;
        ch = w == 0 ? (der ? 0 : 1) : (der ? 1 + w : 4 + w);
        nx = a.normal[3 * pc];
        ny = a.normal[3 * pc + 1];
        nz = a.normal[3 * pc + 2];
        const double Ux = a.f.ca, Uy = a.f.sa;
        al = w == 1 ? nx : (w == 2 ? ny : (w == 3 ? nz : 0.0));
        b1 = w == 1 ? 1.0 : 0.0;
        b2 = w == 2 ? 1.0 : 0.0;
        b3 = w == 3 ? 1.0 : 0.0;
        gm = w == 0 ? -1.0 : (w == 1 ? Ux : (w == 2 ? Uy : 0.0));
        dl = w == 0 ? Ux * nx + Uy * ny : 0.0;
        s_der = der ? 1.0 / (2.0 * a.f.dtau) : 0.0;
        s_val = der ? 0.0 : 1.0;
    }
    // the five inputs at time row m (offset m * P from this panel)
    struct Raw {
        TIn r, u1, u2, u3, p;
    };
    __device__ __forceinline__ Raw load(int64_t off) const {
        return Raw{rho[off], u[off], u[NP + off], u[2 * NP + off], pp[off]};
    }
    __device__ __forceinline__ double X(const Raw &v) const {
        const double r = (double)v.r;
        const double u1 = (double)v.u1, u2 = (double)v.u2, u3 = (double)v.u3;
        const double un = u1 * nx + u2 * ny + u3 * nz;
        const double bu = b1 * u1 + b2 * u2 + b3 * u3 - gm;
        return al * (double)v.p + r * bu * un - dl;
    }
    __device__ __forceinline__ double X(int64_t off) const { return X(load(off)); }
};

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ void store_quad(float *dst, const float *v) {
    *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void store_quad(bf16s *dst, const float *v) {
    uint2 w;
    w.x = (uint32_t)bf16_rne(v[0]) | ((uint32_t)bf16_rne(v[1]) << 16);
    w.y = (uint32_t)bf16_rne(v[2]) | ((uint32_t)bf16_rne(v[3]) << 16);
    *reinterpret_cast<uint2 *>(dst) = w;
}

// tile[q * kSrcRS + c * 32 + pl] (q < TC) -> coef quads; a wave writes TC
// consecutive indices of one panel and channel group (64 / TC groups per wave).
template <typename TOut, int TC = kSrcTC>
__device__ __forceinline__ void src_flush(const float *tile, TOut *coef, int64_t pbase, int64_t P, int64_t NS,
                                          int64_t i0) {
    for (int e = threadIdx.x; e < kSrcPanels * 2 * TC; e += 256) {
        const int pl = e / (2 * TC);
        const int g = (e / TC) & 1;
        const int q = e & (TC - 1);
        const int64_t p = pbase + pl;
        if (p < P) {
            float v[4];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) v[cc] = tile[q * kSrcRS + (4 * g + cc) * 32 + pl];
            store_quad(coef + ((p * 2 + g) * NS + i0 + q) * 4, v);
        }
    }
}

// Chunk of kSrcTC coefficient indices i0 .. i0 + 63 for 32 panels: the
// Thomas forward elimination over the kSrcW rows [R0, R0 + kSrcW), R0 = i0 - 17,
// and the back substitution from the top of that window, reduced right-hand
// sides in registers, overwritten by the coefficients.  The block's inputs (5
// variables x 32 panels per source-term row, rows R0 - 3 .. R0 + kSrcW + 2) are
// loaded once, cooperatively, in groups of kSrcG rows by direct global -> LDS
// copies into two buffers: group m + 1 is in flight while group m is used, one
// barrier per group.  The four waves (four base quantities) read their inputs
// from LDS (both half-waves read the same panel's row: a broadcast).
//
// GEN = false: interior chunk (every row in [kSrcPivotRows, N - 3]): central
// differences, constant pivot, no end rows, no branches.  GEN = true: a chunk
// with a record end in reach: zero source terms outside the record, one-sided
// differences at the first and last frame, exact pivots, the end rows'
// right-hand-side corrections and the end coefficients c_{-1}, c_0, c_{N-1},
// c_N, zero padding past c_N.  Row positions are compile-time (unrolled) and
// the end rules block-uniform predicates, so both kinds keep the right-hand
// sides in registers.  The coefficients leave through a [kSrcTC / 4][kSrcRS]
// LDS tile in four quarters.
constexpr int kSrcG = 12;                       // rows per staged group
constexpr int kSrcNX = kSrcW + 6;               // source-term rows R0 - 3 .. R0 + kSrcW + 2
constexpr int kSrcNG = (kSrcNX + kSrcG - 1) / kSrcG;
constexpr int kSrcGV = kSrcG * 5 * kSrcPanels;  // values per group

typedef __attribute__((address_space(3))) void *src_lds_ptr_t;

// Direct global -> LDS copies of the staged groups.  Group m goes to
// dst[var][r][panel]: variables [rho, u1, u2, u3, p'], source-term rows k =
// m*kSrcG + r (record row R0 - 3 + k, clamped to [0, N-1]), panels pbase ..
// pbase + 31.  A piece of 64 dwords (4 bytes per lane) is one (variable, row) in
// FP64 and two rows of a variable in FP32; the lane's panel (clamped to P - 1),
// dword half and row within the piece are fixed.  Wave wv issues the pieces wv,
// wv + 4, ...; pieces whose first row lies past the staged rows are skipped.
template <typename TIn>
struct SrcDma {
    static constexpr int DW = (int)sizeof(TIn) / 4;  // dwords per value
    static constexpr int RPP = 2 / DW;               // rows per piece
    static constexpr int PPV = kSrcG / RPP;          // pieces per variable
    static constexpr int NPIECE = 5 * PPV;
    static constexpr int NI = (NPIECE + 3) / 4;      // pieces per wave (at most)
    const unsigned char *vbase[NI];                  // variable base of piece i (uniform)
    int r[NI];                                       // its first row in the group
    int64_t rowb;                                    // bytes per record row (P values)

    __device__ __forceinline__ SrcDma(const SrcFwdArgs &a, int wv) {
        rowb = a.P * (int64_t)sizeof(TIn);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            int pc = wv + 4 * i;
            pc = pc < NPIECE ? pc : NPIECE - 1;
            const int var = pc / PPV;
            r[i] = (pc - var * PPV) * RPP;
            vbase[i] = var == 0 ? static_cast<const unsigned char *>(a.rho)
                                : (var == 4 ? static_cast<const unsigned char *>(a.pp)
                                            : static_cast<const unsigned char *>(a.u) + (int64_t)(var - 1) * a.N * rowb);
        }
    }

    // lane_row: row of this lane within a piece (0, or lane >> 5 in FP32);
    // lane_off: byte offset of the lane's panel and dword half within a row
    __device__ __forceinline__ void issue(int m, TIn *dst, int wv, int lane_row, uint32_t lane_off, int64_t R0,
                                          int64_t N) const {
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int pc = wv + 4 * i;
            const int k0 = m * kSrcG + r[i];
            const bool go = (NPIECE % 4 == 0 || i + 1 < NI ? true : pc < NPIECE) && k0 < kSrcNX;
            if (go) {
                int64_t row = R0 - 3 + k0 + lane_row;
                row = row < 0 ? 0 : (row > N - 1 ? N - 1 : row);
                __builtin_amdgcn_global_load_lds((const void *)(vbase[i] + row * rowb + lane_off),
                                                 (src_lds_ptr_t)((unsigned char *)dst + pc * 256), 4, 0, 0);
            }
        }
    }
};

// ENDS (GEN): which record ends the chunk's rows can reach, bit 0 the first frame (R0 <= 3), bit 1
// the last (R0 + kSrcW >= N - 1); the rules of an end out of reach are compiled out (they would be
// false at run time).
template <typename TIn, typename TOut, bool GEN, int ENDS = 3>
__device__ __forceinline__ void src_chunk(const SrcFwdArgs &a, int64_t pbk, int64_t i0, TIn *ring0, TIn *ring1,
                                          float *tile, double *endv) {
    constexpr bool kStart = (ENDS & 1) != 0, kEnd = (ENDS & 2) != 0;
    const int64_t P = a.P, N = a.N;
    const int pl = threadIdx.x & 31;
    const int half = (threadIdx.x >> 5) & 1;  // row of a pair this half-wave computes X for
    const int64_t pbase = pbk * kSrcPanels;
    const int64_t pc = min(pbase + pl, P - 1);
    const SrcLane<TIn> L(a, pc);
    using Raw = typename SrcLane<TIn>::Raw;
    const double cpi = 2.0 - sqrt(3.0);
    const int64_t R0 = i0 - 1 - kSrcH;
    // Exact Thomas pivots of tridiag(1, 4, 1) (GEN): c'_1 = 1/4, c'_n = 1/(4 - c'_{n-1}), from the
    // plan's table a.cp (a uniform load; equal to cpi to double precision past n = 30, so rows from
    // 64 on take cpi)
    const double *__restrict__ cpt = a.cp;
    auto pivot = [&](int rr) { return rr < 64 ? cpt[rr] : cpi; };
    // 32-bit copies for the block-uniform end rules (records are far below 2^31 frames)
    const int R0i = (int)R0, Ni = (int)N;
    // two buffers of [rho, u1, u2, u3, p'] x kSrcG rows x 32 panels; group m in buffer m & 1
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    int lane_row;
    uint32_t lane_off;
    if constexpr (sizeof(TIn) == 8) {
        lane_row = 0;
        lane_off = (uint32_t)(min(pbase + (lane >> 1), P - 1) * 8 + (lane & 1) * 4);
    } else {
        lane_row = lane >> 5;
        lane_off = (uint32_t)(min(pbase + (lane & 31), P - 1) * 4);
    }
    const SrcDma<TIn> dma(a, wv);
    dma.issue(0, ring0, wv, lane_row, lane_off, R0, N);
    // reduced right-hand sides, then coefficients, of window rows s, in registers
    const int col = L.ch * 32 + pl;
    float dvr[kSrcW];
    auto DV = [&](int s_) -> float & { return dvr[s_]; };
    // Forward sweep over source-term rows k (record row R0 - 3 + k).  Step it (it = 0 .. kSrcW + 1,
    // right-hand side of frame n = R0 - 1 + it) takes X of frames n - 2 .. n + 2 = rows it .. it + 4.
    double Xa = 0.0, Xb = 0.0, Xc = 0.0, Xd = 0.0, Xe = 0.0;
    double fprev = 0.0, dprev = 0.0, f0 = 0.0;
#pragma unroll
    for (int m = 0; m < kSrcNG; ++m) {
        // this wave's copies of group m have landed; the barrier makes every wave's visible
        // and frees the other buffer (group m - 1 has been read), which then receives m + 1
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (m + 1 < kSrcNG) dma.issue(m + 1, ((m + 1) & 1) ? ring1 : ring0, wv, lane_row, lane_off, R0, N);
        const TIn *buf = (m & 1) ? ring1 : ring0;
        // Rows go in pairs: lanes 0-31 compute X of row k, lanes 32-63 (the same panel and base
        // quantity) X of row k + 1, and one swap of the halves (v_permlane32_swap, per dword) gives
        // every lane both, so each source term is computed once instead of once per half.
        auto row_step = [&](const int k, const double Xn) __attribute__((always_inline)) {
            Xa = Xb;
            Xb = Xc;
            Xc = Xd;
            Xd = Xe;
            Xe = Xn;
            if (k >= 4) {
                const int it = k - 4;
                const int n = R0i - 1 + it;
                double fn;
                if constexpr (!GEN) {
                    fn = L.s_der * (Xd - Xb) + L.s_val * Xc;
                } else {
                    fn = 0.0;
                    if ((unsigned)n < (unsigned)Ni) {
                        const double dx = (kStart && n == 0) ? -3.0 * Xc + 4.0 * Xd - Xe
                                          : ((kEnd && n == Ni - 1) ? 3.0 * Xc - 4.0 * Xb + Xa : Xd - Xb);
                        fn = L.s_der * dx + L.s_val * Xc;
                    }
                    if (kStart && n == 0) f0 = fn;
                    // f_{N-1} and (below) d_{N-2} wait in LDS for the end coefficients: held in
                    // registers across the back substitution they cost it about 110 registers
                    if (kEnd && n == Ni - 1) endv[col] = fn;
                }
                if (it >= 2) {
                    float dvs;
                    if constexpr (!GEN) {
                        const double d = (6.0 * fprev - dprev) * cpi;
                        dprev = d;
                        dvs = (float)d;
                    } else {
                        const int rr = n - 1;  // system row
                        dvs = 0.f;
                        if ((unsigned)(rr - 1) < (unsigned)(Ni - 2)) {
                            double rhs = 6.0 * fprev;
                            if (kStart && rr == 1) rhs -= f0;
                            if (kEnd && rr == Ni - 2) rhs -= fn;
                            const double piv = pivot(rr);
                            const double d = (rhs - dprev) * piv;
                            dprev = d;
                            dvs = (float)d;
                            if (kEnd && rr == Ni - 2) endv[256 + col] = d;
                        }
                    }
                    dvr[it - 2] = dvs;
                    // computed here, not sunk to the back substitution (which would keep every
                    // row's inputs live)
                    asm volatile("" : "+v"(dvr[it - 2]));
                }
                fprev = fn;
            }
        };
#pragma unroll
        for (int r = 0; r < kSrcG; r += 2) {
            const int k = m * kSrcG + r;
            if (k < kSrcNX) {
                const TIn *rw = buf + (r + half) * kSrcPanels + pl;
                constexpr int VS = kSrcG * kSrcPanels;  // variable stride
                const Raw v{rw[0], rw[VS], rw[2 * VS], rw[3 * VS], rw[4 * VS]};
                double Xm = L.X(v);
                if constexpr (GEN) {
                    const int mrow = R0i - 3 + k + half;
                    if ((unsigned)mrow >= (unsigned)Ni) Xm = 0.0;
                }
                const unsigned xl = (unsigned)__double2loint(Xm), xh = (unsigned)__double2hiint(Xm);
                const auto sl = __builtin_amdgcn_permlane32_swap(xl, xl, false, false);
                const auto sh = __builtin_amdgcn_permlane32_swap(xh, xh, false, false);
                row_step(k, __hiloint2double((int)sh[0], (int)sl[0]));  // row k (lanes 0-31's value)
                if (k + 1 < kSrcNX) row_step(k + 1, __hiloint2double((int)sh[1], (int)sl[1]));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // back substitution from the top of the window; window row s holds coefficient index i = R0 + s + 1
    double x = 0.0;
#pragma unroll
    for (int s = kSrcW - 1; s >= 0; --s) {
        if constexpr (!GEN) {
            x = (double)dvr[s] - cpi * x;
            dvr[s] = (float)x;
        } else {
            const int rr = R0i + s;
            if ((unsigned)(rr - 1) < (unsigned)(Ni - 2)) x = (double)DV(s) - pivot(rr) * x;
            if (s >= kSrcH && s < kSrcH + kSrcTC) {
                const int i = rr + 1;
                double v;
                if (kStart && i == 0) v = 2.0 * f0 - x;
                else if (kStart && i == 1) v = f0;
                else if (i < Ni) v = x;
                else v = 0.0;  // c_N and c_{N+1} are set as the coefficients leave (below)
                DV(s) = (float)v;
            }
        }
    }
    TOut *coef = static_cast<TOut *>(a.coef);
    constexpr int QT = kSrcTC / 4;
#pragma unroll
    for (int qt = 0; qt < 4; ++qt) {
        __syncthreads();  // the previous quarter's tile has been read
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            float c = dvr[kSrcH + qt * QT + q];
            if constexpr (GEN && kEnd) {
                // the last frame's end coefficients c_N = f_{N-1}, c_{N+1} = 2 f_{N-1} - d_{N-2} (both
                // rows lie in the window of a chunk that holds index N or N + 1)
                const int i = (int)i0 + qt * QT + q;
                if (i == Ni) c = (float)endv[col];
                else if (i == Ni + 1) c = (float)(2.0 * endv[col] - endv[256 + col]);
            }
            tile[q * kSrcRS + col] = c;
        }
        __syncthreads();
        src_flush<TOut, QT>(tile, coef, pbase, P, a.NS, i0 + qt * QT);
    }
}

template <typename TIn, typename TOut, bool GEN, int ENDS = 3>
__device__ __forceinline__ void src_chunk_block(const SrcFwdArgs &a, int64_t pbk, int64_t k) {
    __shared__ TIn ring0[kSrcGV];
    __shared__ TIn ring1[kSrcGV];
    __shared__ float tile[(kSrcTC / 4) * kSrcRS];
    __shared__ double endv[GEN && (ENDS & 2) ? 2 * 256 : 1];  // f_{N-1}, d_{N-2} per thread
    src_chunk<TIn, TOut, GEN, ENDS>(a, pbk, k * kSrcTC, ring0, ring1, tile, endv);
}

// ------------------------------------------------ chunked source adjoint stage
// FP32/BF16 modes: the exact transpose of the chunked source stage, fused with
// the derivative transpose and the chain rule (geometry in fwh_internal.h).
// With a_k the adjoint of coefficient c_k (storage index k + 1):
//   chat_r = a_r - [r = 1] a_{-1} - [r = N-2] a_N   (r = 1 .. N-2),  z = A^{-1} chat,
//   fbar_j = 6 z_j (1 <= j <= N-2),  fbar_0 = a_0 + 2 a_{-1} - z_1,
//   fbar_{N-1} = a_{N-1} + 2 a_N - z_{N-2}
// (A = tridiag(1, 4, 1) is symmetric, so its transpose solve is the same Thomas
// sweep); then Xbar = fbar (value channels) or D^T fbar (derivative channels)
// and the chain rule through the source terms at every frame of the chunk.
// Wave w, lanes 0-31 / 32-63: base w, derivative / value channel (as forward).

// Xbar of 8 channels at (frame m, panel) from tile[(m - m0) * kSrcRS + c * 32 + pl];
// chain rule; gradients out time-major (32 consecutive panels per frame).
template <typename TIn, int TC = kSrcTC>
__device__ __forceinline__ void src_adj_chain_out(const float *tile, const SrcAdjArgs &a, int64_t pbase, int64_t m0) {
    const int64_t P = a.P, N = a.N, NP = N * P;
    const TIn *__restrict__ rho = static_cast<const TIn *>(a.rho);
    const TIn *__restrict__ u = static_cast<const TIn *>(a.u);
    TIn *__restrict__ g_rho = static_cast<TIn *>(a.g_rho);
    TIn *__restrict__ g_u = static_cast<TIn *>(a.g_u);
    TIn *__restrict__ g_p = static_cast<TIn *>(a.g_p);
    const int pl = threadIdx.x & 31;
    const int64_t p = pbase + pl;
    if (p >= P) return;
    const double nx = a.normal[3 * p], ny = a.normal[3 * p + 1], nz = a.normal[3 * p + 2];
    const double Ux = a.f.ca, Uy = a.f.sa;
    // all of this thread's frames are loaded before any gradient is stored
    constexpr int NF = TC / 8;
    TIn vr[NF], v1[NF], v2[NF], v3[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int64_t m = m0 + (threadIdx.x >> 5) + 8 * f;
        const int64_t idx = (m < N ? m : N - 1) * P + p;
        vr[f] = rho[idx];
        v1[f] = u[idx];
        v2[f] = u[NP + idx];
        v3[f] = u[2 * NP + idx];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int ml = (threadIdx.x >> 5) + 8 * f;
        const int64_t m = m0 + ml;
        if (m < N) {
            const float *t = tile + ml * kSrcRS + pl;
            const double Qb = (double)t[0] + (double)t[32];
            const double L1 = (double)t[2 * 32] + (double)t[5 * 32];
            const double L2 = (double)t[3 * 32] + (double)t[6 * 32];
            const double L3 = (double)t[4 * 32] + (double)t[7 * 32];
            const int64_t idx = m * P + p;
            const double r = (double)vr[f];
            const double u1 = (double)v1[f], u2 = (double)v2[f], u3 = (double)v3[f];
            const double un = u1 * nx + u2 * ny + u3 * nz;
            const double w1 = u1 - Ux, w2 = u2 - Uy, w3 = u3;
            const double S = Qb + L1 * w1 + L2 * w2 + L3 * w3;
            g_rho[idx] = (TIn)(un * S);
            g_u[idx] = (TIn)(r * nx * S + r * un * L1);
            g_u[NP + idx] = (TIn)(r * ny * S + r * un * L2);
            g_u[2 * NP + idx] = (TIn)(r * nz * S + r * un * L3);
            g_p[idx] = (TIn)(L1 * nx + L2 * ny + L3 * nz);
        }
    }
}

struct AdjLane {
    double s_der, s_val;
    int ch;
    __device__ __forceinline__ explicit AdjLane(double dtau) {
        const int w = threadIdx.x >> 6;
        const bool der = (threadIdx.x & 32) == 0;
        ch = w == 0 ? (der ? 0 : 1) : (der ? 1 + w : 4 + w);
        s_der = der ? 1.0 / (2.0 * dtau) : 0.0;
        s_val = der ? 0.0 : 1.0;
    }
};

constexpr int kAdjSlab = 32;            // storage indices per staged slab
constexpr int kAdjSlabRS = kAdjSlab + 1;

// One chunk of kSrcTC frames m0 .. m0 + 63 for 32 panels: window rows s = 0 .. kAdjW - 1 are
// system rows r = m0 - kAdjLo + s (storage index r + 1).  The coefficient adjoints come in
// through LDS slabs of 32 indices x 256 rows (8 lanes per 128-byte row segment); the reduced
// right-hand sides, then z, then Xbar stay in registers (the window loops are unrolled, so every
// row position is a compile-time index).
// GEN = false (interior chunk, every row in [kSrcPivotRows, N - 3]): constant pivot, no end rows.
// GEN = true (either record end in reach, or a short record): the exact pivots cp[r], the end
// rows' right-hand-side corrections, fbar_0 and fbar_{N-1}, one-sided differences at the first
// and last frames, as block-uniform predicates on the row; slab indices outside the row are
// clamped into it (those rows are never used).
template <typename TIn, bool GEN>
__device__ __forceinline__ void src_adj_chunk(const SrcAdjArgs &a, int64_t pbk, int64_t k, float *lds) {
    const int64_t P = a.P, NS = a.NS;
    const int pl = threadIdx.x & 31;
    const int64_t pbase = pbk * kSrcPanels;
    const AdjLane L(a.f.dtau);
    const double cpi = 2.0 - sqrt(3.0);
    const int64_t m0 = k * kSrcTC;
    const int64_t i_lo = m0 - kAdjLo + 1;  // storage index of window row 0
    // cooperative slab loads: float4 e = tid + 256 j -> row e / 8 (channel-major rows c*32 + pl), quad e % 8
    auto slab_load = [&](int t, float4 *v) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int row = e >> 3, qd = e & 7;
            const int64_t pr = min(pbase + (row & 31), P - 1);
            int64_t idx = i_lo + t * kAdjSlab + 4 * qd;  // a multiple of 4, as NS is
            if constexpr (GEN) idx = idx < 0 ? 0 : (idx > NS - 4 ? NS - 4 : idx);
            const float *src = a.cbar + ((int64_t)(row >> 5) * P + pr) * NS + idx;
            v[j] = *reinterpret_cast<const float4 *>(src);
        }
    };
    auto slab_store = [&](const float4 *v) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = threadIdx.x + 256 * j;
            float *dst = lds + (e >> 3) * kAdjSlabRS + 4 * (e & 7);
            dst[0] = v[j].x;
            dst[1] = v[j].y;
            dst[2] = v[j].z;
            dst[3] = v[j].w;
        }
    };
    const int myrow = L.ch * 32 + pl;
    // GEN: end data of this thread's row (a_{-1}, a_0, a_{N-1}, a_N) and 32-bit row positions
    const int Ni = (int)a.N, R0i = (int)(m0 - kAdjLo);
    const double *__restrict__ cp = a.cp;
    double am1 = 0.0, a0 = 0.0, aN1 = 0.0, aN = 0.0;
    if constexpr (GEN) {
        const float *row = a.cbar + ((int64_t)L.ch * P + min(pbase + pl, P - 1)) * NS;
        am1 = row[0];
        a0 = row[1];
        aN1 = row[Ni];
        aN = row[Ni + 1];
    }
    auto inside = [&](int r) { return (unsigned)(r - 1) < (unsigned)(Ni - 2); };  // 1 <= r <= N - 2
    auto pivot = [&](int r) { return r < 64 ? cp[r] : cpi; };
    float dv[kAdjW];
    double dprev = 0.0;
    float4 cur[8], nxt[8];
    slab_load(0, cur);
#pragma unroll
    for (int t = 0; t < kAdjW / kAdjSlab; ++t) {
        if (t + 1 < kAdjW / kAdjSlab) slab_load(t + 1, nxt);
        __syncthreads();
        slab_store(cur);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kAdjSlab; ++q) {
            const double c = (double)lds[myrow * kAdjSlabRS + q];
            if constexpr (!GEN) {
                const double d = (c - dprev) * cpi;
                dprev = d;
                dv[t * kAdjSlab + q] = (float)d;
            } else {
                const int r = R0i + t * kAdjSlab + q;
                float v = 0.f;
                if (inside(r)) {
                    double cc = c;
                    if (r == 1) cc -= am1;
                    if (r == Ni - 2) cc -= aN;
                    const double d = (cc - dprev) * pivot(r);
                    dprev = d;
                    v = (float)d;
                }
                dv[t * kAdjSlab + q] = v;
            }
        }
        if (t + 1 < kAdjW / kAdjSlab) {
#pragma unroll
            for (int j = 0; j < 8; ++j) cur[j] = nxt[j];
        }
    }
    if constexpr (!GEN) {
        // back substitution; Xbar_m once fbar_{m-1} is known (window row s = m - m0 + kAdjLo - 1),
        // kept in place of the consumed right-hand side dv[s]
        double z = 0.0, fp1 = 0.0, fc = 0.0;
#pragma unroll
        for (int s = kAdjW - 1; s >= 0; --s) {
            z = (double)dv[s] - cpi * z;
            const double fm1 = 6.0 * z;
            const int ml = s - kAdjLo + 1;  // frame m = m0 + ml has fbar_{m-1} = fm1
            if (ml >= 0 && ml < kSrcTC) dv[s] = (float)(L.s_val * fc + L.s_der * (fm1 - fp1));
            fp1 = fc;
            fc = fm1;
        }
    } else {
        // back substitution (z rounded to FP32 in place), then fbar and Xbar_m, which overwrites
        // the row of fbar_{m-1} (no later frame needs it)
        double z = 0.0, z1 = 0.0, zN2 = 0.0;
#pragma unroll
        for (int s = kAdjW - 1; s >= 0; --s) {
            const int r = R0i + s;
            if (inside(r)) {
                z = (double)dv[s] - pivot(r) * z;
                dv[s] = (float)z;
                if (r == 1) z1 = z;
                if (r == Ni - 2) zN2 = z;
            }
        }
        const double fb0 = a0 + 2.0 * am1 - z1, fbN1 = aN1 + 2.0 * aN - zN2;
        // fbar_j of window row s = j - (m0 - kAdjLo)
        auto fbar = [&](int j, int s_) -> double {
            if (j == 0) return fb0;
            if (j == Ni - 1) return fbN1;
            if (inside(j)) return 6.0 * (double)dv[s_];
            return 0.0;
        };
        const double sd = L.s_der;
#pragma unroll
        for (int ml = 0; ml < kSrcTC; ++ml) {
            const int m = R0i + kAdjLo + ml;
            double xb = 0.0;
            if (m < Ni) {
                const double fm = fbar(m, ml + kAdjLo);
                double dx = 0.0;
                if (inside(m - 1)) dx += fbar(m - 1, ml + kAdjLo - 1);
                if (inside(m + 1)) dx -= fbar(m + 1, ml + kAdjLo + 1);
                if (m == 0) dx -= 3.0 * fb0;
                if (m == 1) dx += 4.0 * fb0;
                if (m == 2) dx -= fb0;
                if (m == Ni - 1) dx += 3.0 * fbN1;
                if (m == Ni - 2) dx -= 4.0 * fbN1;
                if (m == Ni - 3) dx += fbN1;
                xb = L.s_val * fm + sd * dx;
            }
            dv[ml + kAdjLo - 1] = (float)xb;
        }
    }
    // chain rule in two halves of kSrcTC / 2 frames through a [kSrcTC / 2][kSrcRS] tile
    constexpr int HT = kSrcTC / 2;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        __syncthreads();  // the slabs (first half) or the previous half's tile have been read
#pragma unroll
        for (int q = 0; q < HT; ++q) lds[q * kSrcRS + myrow] = dv[half * HT + q + kAdjLo - 1];
        __syncthreads();
        src_adj_chain_out<TIn, HT>(lds, a, pbase, m0 + half * HT);
    }
}

// slabs [256][kAdjSlabRS], then the Xbar tile [kSrcTC / 2][kSrcRS]
constexpr int kAdjWords = 256 * kAdjSlabRS > (kSrcTC / 2) * kSrcRS ? 256 * kAdjSlabRS : (kSrcTC / 2) * kSrcRS;
template <typename TIn>
__device__ __forceinline__ void src_adj_interior_block(const SrcAdjArgs &a, int64_t pbk, int64_t k) {
    __shared__ float lds[kAdjWords];
    src_adj_chunk<TIn, false>(a, pbk, k, lds);
}

template <typename TIn>
__device__ __forceinline__ void src_adj_general_block(const SrcAdjArgs &a, int64_t pbk, int64_t k) {
    __shared__ float lds[kAdjWords];
    src_adj_chunk<TIn, true>(a, pbk, k, lds);
}

// 1-D grid of (panel block, interior chunk) pairs, chunks fastest, renumbered per XCD: the chunks of
// one panel block run together on one XCD, so the coefficient-adjoint rows that neighbouring chunks
// both read (the recurrences' overlap) come from that XCD's L2 rather than from HBM twice.
template <typename TIn>
__global__ __launch_bounds__(256) void src_adj_interior_kernel(SrcAdjArgs a, int64_t nint) {
    const int64_t L = xcd_block(blockIdx.x, gridDim.x), pbk = L / nint;
    src_adj_interior_block<TIn>(a, pbk, 1 + L - pbk * nint);
}
// grid (panel blocks, general chunks)
template <typename TIn>
__global__ __launch_bounds__(256) void src_adj_general_kernel(SrcAdjArgs a) {
    src_adj_general_block<TIn>(a, blockIdx.x, src_general_chunk(blockIdx.y, adj_interior_chunks(a.N)));
}
template <typename TIn>
__global__ __launch_bounds__(256) void src_adj_interior_batched(const BatchCase *__restrict__ cases,
                                                                const int64_t *__restrict__ start, int n) {
    const int64_t h = xcd_block(blockIdx.x, gridDim.x);
    const int c = find_case(start, n, h);
    const int64_t local = h - start[c];
    const int64_t nk = adj_interior_chunks(cases[c].sadj.N);
    const int64_t pbk = local / nk;
    src_adj_interior_block<TIn>(cases[c].sadj, pbk, 1 + local - pbk * nk);
}
template <typename TIn>
__global__ __launch_bounds__(256) void src_adj_general_batched(const BatchCase *__restrict__ cases,
                                                               const int64_t *__restrict__ start, int n) {
    const int c = find_case(start, n, blockIdx.x);
    const int64_t local = (int64_t)blockIdx.x - start[c];
    const int64_t N = cases[c].sadj.N;
    const int64_t nint = adj_interior_chunks(N);
    const int64_t ng = adj_chunks(N) - nint;
    const int64_t pbk = local / ng;
    src_adj_general_block<TIn>(cases[c].sadj, pbk, src_general_chunk(local - pbk * ng, nint));
}

template <typename TIn>
hipError_t src_adj_chunk_launch_t(const SrcAdjArgs &a, hipStream_t stream) {
    const unsigned pb = (unsigned)((a.P + kSrcPanels - 1) / kSrcPanels);
    const int64_t nint = adj_interior_chunks(a.N);
    const int64_t ngen = adj_chunks(a.N) - nint;
    if (nint > 0) {
        src_adj_interior_kernel<TIn><<<dim3((unsigned)(pb * nint)), dim3(256), 0, stream>>>(a, nint);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    src_adj_general_kernel<TIn><<<dim3(pb, (unsigned)ngen), dim3(256), 0, stream>>>(a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ adjoint

// Transpose of the prefilter for one (panel, channel): coefficient adjoints
// a_{-1..N} (storage indices 0..N+1) -> adjoints of the channel values f_0..f_{N-1}:
//   end rows: a_0 += 2 a_{-1}, a_1 -= a_{-1}, a_{N-1} += 2 a_N, a_{N-2} -= a_N;
//   interior: z = T^{-1} a_{1..N-2} (T = tridiag(1,4,1), symmetric);
//   fbar_r = 6 z_r (r = 1..N-2), fbar_0 = a_0 - z_1, fbar_{N-1} = a_{N-1} - z_{N-2}.
// Result written time-major into scr [8][N][P].
template <typename TR>
__device__ __forceinline__ void prefilter_adj_body(const PreAdjArgs &a, int64_t bx, int by) {
    const TR *__restrict__ cbar = static_cast<const TR *>(a.cbar);
    const int64_t P = a.P, N = a.N, NS = a.NS;
    const double *__restrict__ cp = a.cp;
    TR *__restrict__ scr = static_cast<TR *>(a.scr);
    constexpr int CH = 128 / (int)sizeof(TR);
    constexpr int PF = 8;
    __shared__ TR stage[4][64][CH + 1];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int ch = by * 4 + wv;
    const int64_t pbase = bx * 64;
    const int64_t p = pbase + lane;
    const bool active = p < P;
    const int64_t pc = active ? p : P - 1;
    const TR *row = cbar + ((int64_t)ch * P + pc) * NS;
    const TR *cbar_ch = cbar + (int64_t)ch * P * NS;
    const double am1 = (double)row[0];
    const double aN = (double)row[N + 1];
    double a0 = 0.0, aN1 = 0.0, dprev = 0.0;
    TR *scr_ch = scr + (int64_t)ch * N * P;
    // forward elimination over rows r = 1..N-2 (storage index r+1), streaming the row through LDS
    const int64_t nblk = (N + CH - 1) / CH;  // storage indices 0..N cover a_{-1}..a_{N-1}
    for (int64_t b = 0; b < nblk + 1; ++b) {
        const int64_t i0 = b * CH;
        __syncthreads();
        for (int t = lane; t < 64 * CH; t += 64) {
            const int r = t / CH, col = t - r * CH;
            const int64_t prow = pbase + r;
            stage[wv][r][col] = (prow < P && i0 + col < NS) ? cbar_ch[prow * NS + i0 + col] : (TR)0;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < CH; ++q) {
            const int64_t i = i0 + q;
            const int64_t r = i - 1;  // coefficient index
            double a = (double)stage[wv][lane][q];
            if (r == 0) a0 = a + 2.0 * am1;
            if (r == N - 1) aN1 = a + 2.0 * aN;
            if (r >= 1 && r <= N - 2) {
                if (r == 1) a -= am1;
                if (r == N - 2) a -= aN;
                const double d = (a - dprev) * cp[r];
                if (active) scr_ch[r * P + p] = (TR)d;
                dprev = d;
            }
        }
    }
    // back substitution, fbar written in place
    double z = dprev;  // z_{N-2}
    const double zN2 = z;
    if (active) scr_ch[(N - 2) * P + p] = (TR)(6.0 * zN2);
    for (int64_t rb = N - 3; rb >= 1; rb -= PF) {
        double dpre[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int64_t r = rb - q;
            dpre[q] = (r >= 1 && active) ? (double)scr_ch[r * P + p] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int64_t r = rb - q;
            if (r >= 1) {
                z = dpre[q] - cp[r] * z;
                if (active) scr_ch[r * P + p] = (TR)(6.0 * z);
            }
        }
    }
    const double z1 = (N - 2 >= 1) ? z : 0.0;  // after the loop z = z_1
    if (active) {
        scr_ch[p] = (TR)(a0 - z1);
        scr_ch[(N - 1) * P + p] = (TR)(aN1 - zN2);
    }
}

// Per (frame n, panel p): source-term adjoints
//   Qbar = fbar_Q + D^T fbar_Qdot,  Lbar_i = fbar_Li + D^T fbar_Ldot_i
// (D the derivative matrix: central rows 1..N-2, one-sided rows 0 and N-1), then the
// chain rule through Q = rho u.n - U0.n and L_i = p' n_i + rho (u_i - U0_i) u.n:
//   drho = u.n (Qbar + Lbar.w),  du = rho n (Qbar + Lbar.w) + rho u.n Lbar,
//   dp' = Lbar.n,  with w = u - U0.
template <typename TR, typename TIn>
__device__ __forceinline__ void source_adj_chain_body(const ChainArgs &a, int64_t bx, int64_t n) {
    const TR *__restrict__ scr = static_cast<const TR *>(a.scr);
    const TIn *__restrict__ rho = static_cast<const TIn *>(a.rho);
    const TIn *__restrict__ u = static_cast<const TIn *>(a.u);
    const double *__restrict__ normal = a.normal;
    const int64_t P = a.P, N = a.N;
    const Flow f = a.f;
    TIn *__restrict__ g_rho = static_cast<TIn *>(a.g_rho);
    TIn *__restrict__ g_u = static_cast<TIn *>(a.g_u);
    TIn *__restrict__ g_p = static_cast<TIn *>(a.g_p);
    const int64_t p = bx * 256 + threadIdx.x;
    if (p >= P) return;
    const int64_t NP = N * P;
    const double i2h = 1.0 / (2.0 * f.dtau);
    auto S = [&](int c, int64_t m) { return (double)scr[(int64_t)c * NP + m * P + p]; };
    auto DT = [&](int c) {  // (D^T v)_n for channel c
        double s = 0.0;
        if (n - 1 >= 1 && n - 1 <= N - 2) s += S(c, n - 1);
        if (n + 1 >= 1 && n + 1 <= N - 2) s -= S(c, n + 1);
        if (n <= 2) s += (n == 0 ? -3.0 : (n == 1 ? 4.0 : -1.0)) * S(c, 0);
        if (n >= N - 3) s += (n == N - 1 ? 3.0 : (n == N - 2 ? -4.0 : 1.0)) * S(c, N - 1);
        return s * i2h;
    };
    const double Qb = S(1, n) + DT(0);
    double Lb[3];
    for (int i = 0; i < 3; ++i) Lb[i] = S(5 + i, n) + DT(2 + i);
    const double nx = normal[3 * p], ny = normal[3 * p + 1], nz = normal[3 * p + 2];
    const int64_t idx = n * P + p;
    const double r = (double)rho[idx];
    const double u1 = (double)u[idx], u2 = (double)u[NP + idx], u3 = (double)u[2 * NP + idx];
    const double un = u1 * nx + u2 * ny + u3 * nz;
    const double Lw = Lb[0] * (u1 - f.ca) + Lb[1] * (u2 - f.sa) + Lb[2] * u3;
    const double q = Qb + Lw;
    g_rho[idx] = (TIn)(un * q);
    g_u[idx] = (TIn)(r * nx * q + r * un * Lb[0]);
    g_u[NP + idx] = (TIn)(r * ny * q + r * un * Lb[1]);
    g_u[2 * NP + idx] = (TIn)(r * nz * q + r * un * Lb[2]);
    g_p[idx] = (TIn)(Lb[0] * nx + Lb[1] * ny + Lb[2] * nz);
}

template <typename TIn, typename TScr, typename TOut>
__global__ __launch_bounds__(256) void source_fwd_kernel(SrcFwdArgs a) {
    source_fwd_body<TIn, TScr, TOut>(a, blockIdx.x, blockIdx.y);
}

// grid (panel blocks, interior chunks): chunk k = 1 + blockIdx.y.  (Chunks of one panel block on one
// XCD, as the source adjoint runs them, did not cut this stage's HBM reads: a chunk reads the rows it
// shares with the next one last, the next chunk reads them first.)
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void src_interior_kernel(SrcFwdArgs a) {
    src_chunk_block<TIn, TOut, false>(a, blockIdx.x, 1 + (int64_t)blockIdx.y);
}
// one general chunk k for every panel block; ENDS as in src_chunk
template <typename TIn, typename TOut, int ENDS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void src_general_kernel(
    SrcFwdArgs a, int64_t k) {
    src_chunk_block<TIn, TOut, true, ENDS>(a, blockIdx.x, k);
}
// batched: blocks of case c are [start[c], start[c+1]), panel block major
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void src_interior_batched(const BatchCase *__restrict__ cases,
                                                            const int64_t *__restrict__ start, int n) {
    const int c = find_case(start, n, blockIdx.x);
    const int64_t local = (int64_t)blockIdx.x - start[c];
    const int64_t nk = src_interior_chunks(cases[c].src.N);
    const int64_t pbk = local / nk;
    src_chunk_block<TIn, TOut, false>(cases[c].src, pbk, 1 + local - pbk * nk);
}
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void src_general_batched(const BatchCase *__restrict__ cases,
                                                           const int64_t *__restrict__ start, int n) {
    const int c = find_case(start, n, blockIdx.x);
    const int64_t local = (int64_t)blockIdx.x - start[c];
    const int64_t nint = src_interior_chunks(cases[c].src.N);
    const int64_t ng = cases[c].src.NS / kSrcTC - nint;
    const int64_t pbk = local / ng;
    src_chunk_block<TIn, TOut, true>(cases[c].src, pbk, src_general_chunk(local - pbk * ng, nint));
}

template <typename TR>
__global__ __launch_bounds__(256) void prefilter_adj_kernel(PreAdjArgs a) {
    prefilter_adj_body<TR>(a, blockIdx.x, blockIdx.y);
}

template <typename TR, typename TIn>
__global__ __launch_bounds__(256) void source_adj_chain_kernel(ChainArgs a) {
    source_adj_chain_body<TR, TIn>(a, blockIdx.x, blockIdx.y);
}

template <typename TIn, typename TOut>
hipError_t source_chunk_launch_t(const SrcFwdArgs &a, hipStream_t stream) {
    const unsigned pb = (unsigned)((a.P + kSrcPanels - 1) / kSrcPanels);
    const int64_t nint = src_interior_chunks(a.N);
    const int64_t ngen = a.NS / kSrcTC - nint;
    if (nint > 0) {
        src_interior_kernel<TIn, TOut><<<dim3(pb, (unsigned)nint), dim3(256), 0, stream>>>(a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // one launch per general chunk, with the end rules it can reach
    for (int64_t g = 0; g < ngen; ++g) {
        const int64_t k = src_general_chunk(g, nint), R0 = k * kSrcTC - 1 - kSrcH;
        const bool s_in = R0 <= 3, e_in = R0 + kSrcW >= a.N - 1;
        if (s_in && e_in) src_general_kernel<TIn, TOut, 3><<<dim3(pb), dim3(256), 0, stream>>>(a, k);
        else if (e_in) src_general_kernel<TIn, TOut, 2><<<dim3(pb), dim3(256), 0, stream>>>(a, k);
        else src_general_kernel<TIn, TOut, 1><<<dim3(pb), dim3(256), 0, stream>>>(a, k);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TIn, typename TScr, typename TOut>
hipError_t source_launch_t(const SrcFwdArgs &a, hipStream_t stream) {
    dim3 grid((unsigned)((a.P + 63) / 64), 2);
    source_fwd_kernel<TIn, TScr, TOut><<<grid, dim3(256), 0, stream>>>(a);
    return hipGetLastError();
}

template <typename TR, typename TIn>
hipError_t source_adj_launch_t(const PreAdjArgs &pa, const ChainArgs &ca, hipStream_t stream) {
    dim3 grid1((unsigned)((pa.P + 63) / 64), 2);
    prefilter_adj_kernel<TR><<<grid1, dim3(256), 0, stream>>>(pa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid2((unsigned)((ca.P + 255) / 256), (unsigned)ca.N);
    source_adj_chain_kernel<TR, TIn><<<grid2, dim3(256), 0, stream>>>(ca);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_source(int in_dtype, int coef_type, const void *rho, const void *u, const void *pp,
                         const double *normal, int64_t P, int64_t N, int64_t NS, Flow f, const double *cp,
                         void *scratch, void *coef, hipStream_t stream) {
    const SrcFwdArgs a{rho, u, pp, normal, P, N, NS, f, cp, scratch, coef};
    if (in_dtype == 0) {
        if (coef_type == 0) return source_launch_t<double, double, double>(a, stream);
        if (coef_type == 1) return source_chunk_launch_t<double, float>(a, stream);
        return source_chunk_launch_t<double, bf16s>(a, stream);
    }
    if (coef_type == 0) return source_launch_t<float, double, double>(a, stream);
    if (coef_type == 1) return source_chunk_launch_t<float, float>(a, stream);
    return source_chunk_launch_t<float, bf16s>(a, stream);
}

hipError_t launch_source_adjoint(int real_type, int in_dtype, const void *cbar, const void *rho, const void *u,
                                 const double *normal, int64_t P, int64_t N, int64_t NS, Flow f, const double *cp,
                                 void *scratch, void *g_rho, void *g_u, void *g_p, hipStream_t stream) {
    const PreAdjArgs pa{cbar, P, N, NS, cp, scratch};
    const ChainArgs ca{scratch, rho, u, normal, P, N, f, g_rho, g_u, g_p};
    if (real_type == 0) {
        if (in_dtype == 0) return source_adj_launch_t<double, double>(pa, ca, stream);
        return source_adj_launch_t<double, float>(pa, ca, stream);
    }
    const SrcAdjArgs sa{static_cast<const float *>(cbar), rho, u, normal, P, N, NS, f, cp, g_rho, g_u, g_p};
    if (in_dtype == 0) return src_adj_chunk_launch_t<double>(sa, stream);
    return src_adj_chunk_launch_t<float>(sa, stream);
}

// Batched source stages (FP32/BF16 modes: float scratch).
hipError_t launch_batch_source(int in_dtype, int coef_type, const BatchCase *cases, const int64_t *start_int,
                               const int64_t *start_gen, int n, int64_t blocks_int, int64_t blocks_gen,
                               hipStream_t stream) {
    const dim3 b(256);
    if (blocks_int > 0) {
        const dim3 g((unsigned)blocks_int);
        if (in_dtype == 0) {
            if (coef_type == 1) src_interior_batched<double, float><<<g, b, 0, stream>>>(cases, start_int, n);
            else src_interior_batched<double, bf16s><<<g, b, 0, stream>>>(cases, start_int, n);
        } else {
            if (coef_type == 1) src_interior_batched<float, float><<<g, b, 0, stream>>>(cases, start_int, n);
            else src_interior_batched<float, bf16s><<<g, b, 0, stream>>>(cases, start_int, n);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 g((unsigned)blocks_gen);
    if (in_dtype == 0) {
        if (coef_type == 1) src_general_batched<double, float><<<g, b, 0, stream>>>(cases, start_gen, n);
        else src_general_batched<double, bf16s><<<g, b, 0, stream>>>(cases, start_gen, n);
    } else {
        if (coef_type == 1) src_general_batched<float, float><<<g, b, 0, stream>>>(cases, start_gen, n);
        else src_general_batched<float, bf16s><<<g, b, 0, stream>>>(cases, start_gen, n);
    }
    return hipGetLastError();
}

hipError_t launch_batch_source_adjoint(int in_dtype, const BatchCase *cases, const int64_t *start_int,
                                       const int64_t *start_gen, int n, int64_t blocks_int, int64_t blocks_gen,
                                       hipStream_t stream) {
    const dim3 b(256);
    if (blocks_int > 0) {
        if (in_dtype == 0) src_adj_interior_batched<double><<<dim3((unsigned)blocks_int), b, 0, stream>>>(cases, start_int, n);
        else src_adj_interior_batched<float><<<dim3((unsigned)blocks_int), b, 0, stream>>>(cases, start_int, n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (in_dtype == 0) src_adj_general_batched<double><<<dim3((unsigned)blocks_gen), b, 0, stream>>>(cases, start_gen, n);
    else src_adj_general_batched<float><<<dim3((unsigned)blocks_gen), b, 0, stream>>>(cases, start_gen, n);
    return hipGetLastError();
}

}  // namespace fwh
