"""FP64 CPU oracle of the wind-tunnel FW-H far-field integral.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code with
the GPU library.  The arithmetic lives in ``fwh_oracle.c`` (plain C, FP64,
OpenMP over panels, no fast-math); this module only builds/loads it and
marshals arrays (transposing the time-major interface layout [N][P] to the
oracle's panel-major [P][N]).

Functions pinned by the non-GPU tests (see tests/test_oracle_*.py):
  pair_geometry, source_terms, fd, spline_m/spline_eval, window, forward,
  forward_sources, adjoint, adjoint_sources; general motion (Sec. II B):
  gm_window, gm_forward, gm_forward_samples, gm_channels
  (tests/test_oracle_gm.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fwh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")

# FP64 throughout: no contraction of a*b+c into fused multiply-adds, no fast-math
BASE_FLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]
NATIVE_FLAGS = BASE_FLAGS + ["-march=native"]

_lib = None
_lib_path = _LIB


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -ffp-contract=off, no fast-math).
    native=True builds a copy tuned for the host CPU (-march=native) under
    another name: it is only for timing on the machine that built it, the
    portable build is the one the tests load."""
    path = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(path):
        cmd = ["gcc", *(NATIVE_FLAGS if native else BASE_FLAGS), _SRC, "-o", path + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(path + ".tmp", path)
    return path


def use_native() -> str:
    """Build the -march=native copy on this host and load it in place of the
    portable one for the calls that follow; returns the compile flags."""
    global _lib, _lib_path
    build(force=True, native=True)
    _lib, _lib_path = None, _LIB_NATIVE
    _load()
    return " ".join(NATIVE_FLAGS)


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            build(force=True, native=_lib_path == _LIB_NATIVE)
        _lib = ctypes.CDLL(_lib_path)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int64)
        i64, f64 = ctypes.c_int64, ctypes.c_double
        _lib.orc_pair_geometry.argtypes = [i64, i64, D, D, f64, f64, D, D, D, D, D]
        _lib.orc_pair_geometry.restype = None
        _lib.orc_source_terms.argtypes = [i64, i64, D, D, D, D, f64, D, D]
        _lib.orc_source_terms.restype = None
        _lib.orc_fd.argtypes = [i64, D, f64, D]
        _lib.orc_fd.restype = None
        _lib.orc_spline_m.argtypes = [i64, D, f64, D, D]
        _lib.orc_spline_m.restype = None
        _lib.orc_spline_eval.argtypes = [i64, D, D, f64, f64, f64]
        _lib.orc_spline_eval.restype = f64
        _lib.orc_obs_window.argtypes = [i64, i64, D, i64, f64, f64, D, I]
        _lib.orc_obs_window.restype = ctypes.c_int
        _lib.orc_window.argtypes = [i64, i64, i64, D, D, f64, f64, f64, f64, D, I]
        _lib.orc_window.restype = ctypes.c_int
        _lib.orc_forward.argtypes = [i64, i64, i64, D, D, D, D, f64, f64, f64, f64, D, D, D, I, i64, D, i64]
        _lib.orc_forward.restype = ctypes.c_int
        _lib.orc_forward_sources.argtypes = [i64, i64, i64, D, D, D, D, f64, f64, f64, f64, D, D, I, i64, D, i64]
        _lib.orc_forward_sources.restype = ctypes.c_int
        _lib.orc_adjoint.argtypes = [i64, i64, i64, D, D, D, D, f64, f64, f64, f64, D, D, D, D, i64, D, D, D]
        _lib.orc_adjoint.restype = ctypes.c_int
        _lib.orc_adjoint_panels.argtypes = [i64, i64, i64, D, D, D, D, f64, f64, f64, f64, I, i64, D, D, D, D, i64,
                                            D, D, D]
        _lib.orc_adjoint_panels.restype = ctypes.c_int
        _lib.orc_adjoint_sources.argtypes = [i64, i64, i64, D, D, D, D, f64, f64, f64, f64, D, i64, D, D]
        _lib.orc_adjoint_sources.restype = ctypes.c_int
        _lib.orc_gm_window.argtypes = [i64, i64, i64, D, D, f64, f64, f64, D, I]
        _lib.orc_gm_window.restype = ctypes.c_int
        _lib.orc_gm_forward.argtypes = [i64, i64, i64, D, D, D, D, D, f64, f64, f64, D, D, D, I, i64, D, i64]
        _lib.orc_gm_forward.restype = ctypes.c_int
        _lib.orc_gm_forward_samples.argtypes = [i64, i64, i64, D, D, D, D, D, f64, f64, f64, D, D, D, I, I, i64, D]
        _lib.orc_gm_forward_samples.restype = ctypes.c_int
        _lib.orc_gm_channels.argtypes = [i64, i64, D, D, D, f64, f64, D, D, D, D]
        _lib.orc_gm_channels.restype = None
        _lib.orc_num_threads.argtypes = []
        _lib.orc_num_threads.restype = ctypes.c_int
        _lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib.orc_set_num_threads.restype = None
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def pair_geometry(y, x_obs, mach, aoa_deg):
    """Per (observer, panel): R, R_s, Rhat [O,P,3], M_R, delay D = M0 R."""
    lib = _load()
    y, x_obs = _f64(y), _f64(x_obs)
    P, O = y.shape[0], x_obs.shape[0]
    R = np.empty((O, P)); Rs = np.empty((O, P)); Rh = np.empty((O, P, 3)); MR = np.empty((O, P)); D = np.empty((O, P))
    lib.orc_pair_geometry(P, O, _d(y), _d(x_obs), float(mach), float(aoa_deg), _d(R), _d(Rs), _d(Rh), _d(MR), _d(D))
    return R, Rs, Rh, MR, D


def source_terms(rho, u, pp, normal, aoa_deg):
    """Q [N,P] and L [3,N,P] from time-major rho [N,P], u [3,N,P], p' [N,P]."""
    lib = _load()
    rho_pm = _f64(np.asarray(rho).T)
    u_pm = _f64(np.transpose(np.asarray(u), (0, 2, 1)))
    pp_pm = _f64(np.asarray(pp).T)
    N, P = np.asarray(rho).shape
    nrm = _f64(normal)
    Q = np.empty((P, N)); L = np.empty((3, P, N))
    lib.orc_source_terms(N, P, _d(rho_pm), _d(u_pm), _d(pp_pm), _d(nrm), float(aoa_deg), _d(Q), _d(L))
    return np.ascontiguousarray(Q.T), np.ascontiguousarray(np.transpose(L, (0, 2, 1)))


def fd(f, h):
    lib = _load()
    f = _f64(f)
    out = np.empty_like(f)
    lib.orc_fd(f.shape[0], _d(f), float(h), _d(out))
    return out


def spline_m(f, h):
    lib = _load()
    f = _f64(f)
    m = np.empty_like(f)
    work = np.empty_like(f)
    lib.orc_spline_m(f.shape[0], _d(f), float(h), _d(m), _d(work))
    return m


def spline_eval(f, m, tau0, h, tau):
    lib = _load()
    f, m = _f64(f), _f64(m)
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    return np.array([lib.orc_spline_eval(f.shape[0], _d(f), _d(m), float(tau0), float(h), float(t)) for t in tau])


def window(y, x_obs, mach, aoa_deg, n_tau, dtau, tau0=0.0):
    """(status, t_start [O], n_t [O]) of Eqs. (t_start), (t_end)."""
    lib = _load()
    y, x_obs = _f64(y), _f64(x_obs)
    O = x_obs.shape[0]
    ts = np.empty(O); nt = np.empty(O, dtype=np.int64)
    st = lib.orc_window(y.shape[0], O, int(n_tau), _d(y), _d(x_obs), float(mach), float(aoa_deg), float(dtau),
                        float(tau0), _d(ts), _i(nt))
    return int(st), ts, nt


class OracleError(RuntimeError):
    pass


def _check(st):
    if st != 0:
        raise OracleError({-1: "empty observer window", -2: "output stride too small", -3: "bad sizes"}.get(st, st))


def forward(surf, x_obs, mach, aoa_deg, dtau, tau0, rho, u, pp, obs_idx=None, nt_stride=None):
    """p'(o, k) for the selected observers; returns (p [n_sel, nt_stride], t_start, n_t).

    surf: object with y, normal, dS.  rho [N,P], u [3,N,P], p' [N,P] time-major."""
    lib = _load()
    y, nrm, dS, x_obs = _f64(surf.y), _f64(surf.normal), _f64(surf.dS), _f64(x_obs)
    N, P = np.asarray(rho).shape
    O = x_obs.shape[0]
    st, ts, nt = window(y, x_obs, mach, aoa_deg, N, dtau, tau0)
    _check(st)
    if obs_idx is None:
        obs_idx = np.arange(O)
    obs_idx = np.ascontiguousarray(np.asarray(obs_idx, dtype=np.int64))
    if nt_stride is None:
        nt_stride = int(nt.max())
    out = np.empty((obs_idx.shape[0], nt_stride))
    rho_pm = _f64(np.asarray(rho).T)
    u_pm = _f64(np.transpose(np.asarray(u), (0, 2, 1)))
    pp_pm = _f64(np.asarray(pp).T)
    _check(lib.orc_forward(P, O, N, _d(y), _d(nrm), _d(dS), _d(x_obs), float(mach), float(aoa_deg), float(dtau),
                           float(tau0), _d(rho_pm), _d(u_pm), _d(pp_pm), _i(obs_idx), obs_idx.shape[0], _d(out),
                           int(nt_stride)))
    return out, ts, nt


def forward_sources(surf, x_obs, mach, aoa_deg, dtau, tau0, Q, L, obs_idx=None, nt_stride=None):
    """Linear part: p' from source terms Q [N,P], L [3,N,P] (time-major)."""
    lib = _load()
    y, nrm, dS, x_obs = _f64(surf.y), _f64(surf.normal), _f64(surf.dS), _f64(x_obs)
    N, P = np.asarray(Q).shape
    O = x_obs.shape[0]
    st, ts, nt = window(y, x_obs, mach, aoa_deg, N, dtau, tau0)
    _check(st)
    if obs_idx is None:
        obs_idx = np.arange(O)
    obs_idx = np.ascontiguousarray(np.asarray(obs_idx, dtype=np.int64))
    if nt_stride is None:
        nt_stride = int(nt.max())
    out = np.empty((obs_idx.shape[0], nt_stride))
    Q_pm = _f64(np.asarray(Q).T)
    L_pm = _f64(np.transpose(np.asarray(L), (0, 2, 1)))
    _check(lib.orc_forward_sources(P, O, N, _d(y), _d(nrm), _d(dS), _d(x_obs), float(mach), float(aoa_deg),
                                   float(dtau), float(tau0), _d(Q_pm), _d(L_pm), _i(obs_idx), obs_idx.shape[0],
                                   _d(out), int(nt_stride)))
    return out, ts, nt


def adjoint(surf, x_obs, mach, aoa_deg, dtau, tau0, rho, u, pp, gbar):
    """Gradient of J given gbar = dJ/dp' [O, nt_stride]; returns time-major
    (g_rho [N,P], g_u [3,N,P], g_p [N,P])."""
    lib = _load()
    y, nrm, dS, x_obs = _f64(surf.y), _f64(surf.normal), _f64(surf.dS), _f64(x_obs)
    N, P = np.asarray(rho).shape
    O = x_obs.shape[0]
    gbar = _f64(gbar)
    g_r = np.empty((P, N)); g_u = np.empty((3, P, N)); g_p = np.empty((P, N))
    rho_pm = _f64(np.asarray(rho).T)
    u_pm = _f64(np.transpose(np.asarray(u), (0, 2, 1)))
    pp_pm = _f64(np.asarray(pp).T)
    _check(lib.orc_adjoint(P, O, N, _d(y), _d(nrm), _d(dS), _d(x_obs), float(mach), float(aoa_deg), float(dtau),
                           float(tau0), _d(rho_pm), _d(u_pm), _d(pp_pm), _d(gbar), gbar.shape[1], _d(g_r), _d(g_u),
                           _d(g_p)))
    return (np.ascontiguousarray(g_r.T), np.ascontiguousarray(np.transpose(g_u, (0, 2, 1))),
            np.ascontiguousarray(g_p.T))


def adjoint_panels(surf, x_obs, mach, aoa_deg, dtau, tau0, rho, u, pp, gbar, panel_idx):
    """adjoint() restricted to the panels panel_idx: the observer windows come
    from the whole surface, the gradients of each listed panel from its own data.
    Returns time-major (g_rho [N,n], g_u [3,N,n], g_p [N,n]), columns in the
    order of panel_idx."""
    lib = _load()
    y, nrm, dS, x_obs = _f64(surf.y), _f64(surf.normal), _f64(surf.dS), _f64(x_obs)
    N, P = np.asarray(rho).shape
    O = x_obs.shape[0]
    idx = np.ascontiguousarray(np.asarray(panel_idx, dtype=np.int64))
    n = idx.shape[0]
    if n < 1 or idx.min() < 0 or idx.max() >= P:
        raise ValueError(f"panel_idx must list panels in [0, {P})")
    gbar = _f64(gbar)
    g_r = np.empty((n, N)); g_u = np.empty((3, n, N)); g_p = np.empty((n, N))
    rho_pm = _f64(np.asarray(rho)[:, idx].T)
    u_pm = _f64(np.transpose(np.asarray(u)[:, :, idx], (0, 2, 1)))
    pp_pm = _f64(np.asarray(pp)[:, idx].T)
    _check(lib.orc_adjoint_panels(P, O, N, _d(y), _d(nrm), _d(dS), _d(x_obs), float(mach), float(aoa_deg),
                                  float(dtau), float(tau0), _i(idx), n, _d(rho_pm), _d(u_pm), _d(pp_pm), _d(gbar),
                                  gbar.shape[1], _d(g_r), _d(g_u), _d(g_p)))
    return (np.ascontiguousarray(g_r.T), np.ascontiguousarray(np.transpose(g_u, (0, 2, 1))),
            np.ascontiguousarray(g_p.T))


def adjoint_sources(surf, x_obs, mach, aoa_deg, dtau, tau0, n_tau, gbar):
    """Transpose of forward_sources: (Qbar [N,P], Lbar [3,N,P])."""
    lib = _load()
    y, nrm, dS, x_obs = _f64(surf.y), _f64(surf.normal), _f64(surf.dS), _f64(x_obs)
    P, N, O = y.shape[0], int(n_tau), x_obs.shape[0]
    gbar = _f64(gbar)
    Qb = np.empty((P, N)); Lb = np.empty((3, P, N))
    _check(lib.orc_adjoint_sources(P, O, N, _d(y), _d(nrm), _d(dS), _d(x_obs), float(mach), float(aoa_deg),
                                   float(dtau), float(tau0), _d(gbar), gbar.shape[1], _d(Qb), _d(Lb)))
    return np.ascontiguousarray(Qb.T), np.ascontiguousarray(np.transpose(Lb, (0, 2, 1)))


# ------------------------------------------------------------ general motion
# Moving surface, medium and observers at rest (Sec. II B).  Interface layout
# (time-major): y, normal, vel [N,P,3]; rho, p' [N,P]; u [3,N,P].

GM_CHANNELS = ("A", "Qn", "L1", "L2", "L3", "Ld1", "Ld2", "Ld3", "LM", "M1", "M2", "M3",
               "Md1", "Md2", "Md3", "Msq", "Y1", "Y2", "Y3")


def _gm_pm(ms, rho, u, pp):
    vec = lambda a: _f64(np.transpose(np.asarray(a), (2, 1, 0)))      # [N,P,3] -> [3,P,N]
    return (vec(ms.y), vec(ms.normal), vec(ms.vel), _f64(ms.dS), _f64(np.asarray(rho).T),
            _f64(np.transpose(np.asarray(u), (0, 2, 1))), _f64(np.asarray(pp).T))


def gm_window(ms, x_obs, mach, dtau, tau0=0.0):
    """(status, t_start [O], n_t [O]) of the general-motion observer window."""
    lib = _load()
    y = _f64(np.transpose(np.asarray(ms.y), (2, 1, 0)))
    x_obs = _f64(x_obs)
    N, P = ms.y.shape[0], ms.y.shape[1]
    O = x_obs.shape[0]
    ts = np.empty(O)
    nt = np.empty(O, dtype=np.int64)
    st = lib.orc_gm_window(P, O, N, _d(y), _d(x_obs), float(mach), float(dtau), float(tau0), _d(ts), _i(nt))
    return int(st), ts, nt


def gm_forward(ms, x_obs, mach, dtau, tau0, rho, u, pp, obs_idx=None, nt_stride=None):
    """p' [n_sel, nt_stride] (zero padded), t_start [O], n_t [O]."""
    lib = _load()
    x_obs = _f64(x_obs)
    O = x_obs.shape[0]
    N, P = ms.y.shape[0], ms.y.shape[1]
    st, ts, nt = gm_window(ms, x_obs, mach, dtau, tau0)
    if st != 0:
        raise ValueError("empty observer window")
    if obs_idx is None:
        obs_idx = np.arange(O)
    obs_idx = np.ascontiguousarray(np.asarray(obs_idx, dtype=np.int64))
    if nt_stride is None:
        nt_stride = int(nt.max())
    y, n, v, dS, r, uu, p = _gm_pm(ms, rho, u, pp)
    out = np.empty((obs_idx.size, nt_stride))
    st = lib.orc_gm_forward(P, O, N, _d(y), _d(n), _d(v), _d(dS), _d(x_obs), float(mach), float(dtau), float(tau0),
                            _d(r), _d(uu), _d(p), _i(obs_idx), obs_idx.size, _d(out), int(nt_stride))
    if st != 0:
        raise ValueError(f"orc_gm_forward status {st}")
    return out, ts, nt


def gm_forward_samples(ms, x_obs, mach, dtau, tau0, rho, u, pp, s_obs, s_k):
    """p'(o, k) at the listed (observer, sample) pairs."""
    lib = _load()
    x_obs = _f64(x_obs)
    O = x_obs.shape[0]
    N, P = ms.y.shape[0], ms.y.shape[1]
    s_obs = np.ascontiguousarray(np.asarray(s_obs, dtype=np.int64))
    s_k = np.ascontiguousarray(np.asarray(s_k, dtype=np.int64))
    y, n, v, dS, r, uu, p = _gm_pm(ms, rho, u, pp)
    out = np.empty(s_obs.size)
    st = lib.orc_gm_forward_samples(P, O, N, _d(y), _d(n), _d(v), _d(dS), _d(x_obs), float(mach), float(dtau),
                                    float(tau0), _d(r), _d(uu), _d(p), _i(s_obs), _i(s_k), s_obs.size, _d(out))
    if st != 0:
        raise ValueError(f"orc_gm_forward_samples status {st}")
    return out


def gm_channels(ms, mach, dtau, rho, u, pp):
    """The 19 observer-independent channels, [19, N, P] (order GM_CHANNELS)."""
    lib = _load()
    N, P = ms.y.shape[0], ms.y.shape[1]
    y, n, v, _, r, uu, p = _gm_pm(ms, rho, u, pp)
    out = np.empty((len(GM_CHANNELS), P, N))
    lib.orc_gm_channels(P, N, _d(y), _d(n), _d(v), float(mach), float(dtau), _d(r), _d(uu), _d(p), _d(out))
    return np.ascontiguousarray(np.transpose(out, (0, 2, 1)))

