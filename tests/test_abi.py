"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/fwh.h and include/fwh_io.h declare, and fwh_plan_create / fwh_setup /
fwh_forward reject bad arguments with the documented codes before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2312_16263_amd as fwh
from workloads import surfaces

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="fwh.h"):
    text = open(os.path.join(ROOT, "include", name)).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(fwh_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    L = fwh.lib()
    names = header_functions()
    assert set(names) == set(fwh.EXPORTED), names
    for n in names:
        assert hasattr(L, n), n
    assert "gfx950" in fwh.version()


def test_library_exports_every_file_io_function():
    L = fwh.lib()
    names = header_functions("fwh_io.h")
    assert set(names) == set(fwh.IO_EXPORTED), names
    for n in names:
        assert hasattr(L, n), n


def test_headers_cover_every_include():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["fwh.h", "fwh_io.h"]


def _args(**kw):
    s = surfaces.sphere(1.0, 4, 8)
    x = surfaces.observer_circle(3, 10.0)
    d = dict(y=s.y, normal=s.normal, dS=s.dS, x_obs=x, mach=0.3, aoa_deg=5.0, dtau=0.01, tau0=0.0, n_tau=64,
             mode=fwh.MODE_F32)
    d.update(kw)
    keep = [np.ascontiguousarray(np.asarray(d[k], dtype=np.float64)) for k in ("y", "normal", "dS", "x_obs")]
    a = fwh.SetupArgs(keep[0].shape[0], keep[3].shape[0], d["n_tau"], fwh._dptr(keep[0]), fwh._dptr(keep[1]),
                      fwh._dptr(keep[2]), fwh._dptr(keep[3]), d["mach"], d["aoa_deg"], d["dtau"], d["tau0"], d["mode"])
    return a, keep


def _create(a):
    h = ctypes.c_void_p()
    nb = ctypes.c_size_t()
    code = fwh.lib().fwh_plan_create(ctypes.byref(a), ctypes.byref(h), ctypes.byref(nb))
    return code, h, nb.value


@pytest.mark.parametrize("mode", [fwh.MODE_F64, fwh.MODE_F32, fwh.MODE_BF16])
def test_plan_create_reports_workspace(mode):
    a, keep = _args(mode=mode)
    code, h, nb = _create(a)
    assert code == fwh.FWH_OK
    assert nb > 0 and nb % 256 == 0
    fwh.lib().fwh_destroy(h)


@pytest.mark.parametrize("kw,code", [
    (dict(mach=0.0), fwh.FWH_EDOMAIN), (dict(mach=1.0), fwh.FWH_EDOMAIN), (dict(mach=float("nan")), fwh.FWH_EDOMAIN),
    (dict(dtau=0.0), fwh.FWH_EDOMAIN), (dict(dtau=-1.0), fwh.FWH_EDOMAIN),
    (dict(n_tau=3), fwh.FWH_ESIZE), (dict(n_tau=70000), fwh.FWH_ESIZE),
    (dict(mode=7), fwh.FWH_EINVAL), (dict(aoa_deg=float("inf")), fwh.FWH_EINVAL),
])
def test_plan_create_rejects(kw, code):
    a, keep = _args(**kw)
    c, h, nb = _create(a)
    assert c == code
    assert not h.value
    assert len(fwh.lib().fwh_last_error()) > 0


def test_plan_create_rejects_bad_geometry():
    s = surfaces.sphere(1.0, 4, 8)
    dS = s.dS.copy()
    dS[3] = 0.0
    a, keep = _args(dS=dS)
    assert _create(a)[0] == fwh.FWH_EINVAL
    n = s.normal.copy()
    n[2] *= 1.5
    a, keep = _args(normal=n)
    assert _create(a)[0] == fwh.FWH_EINVAL
    y = s.y.copy()
    y[0, 1] = np.nan
    a, keep = _args(y=y)
    assert _create(a)[0] == fwh.FWH_EINVAL
    assert fwh.lib().fwh_plan_create(None, None, None) == fwh.FWH_EINVAL


def test_setup_and_forward_state_checks():
    a, keep = _args()
    code, h, nb = _create(a)
    assert code == fwh.FWH_OK
    L = fwh.lib()
    assert L.fwh_setup(h, None, nb, None) == fwh.FWH_EWORKSPACE
    assert L.fwh_setup(h, ctypes.c_void_p(256), nb - 1, None) == fwh.FWH_EWORKSPACE
    assert L.fwh_setup(h, ctypes.c_void_p(257), nb, None) == fwh.FWH_EWORKSPACE
    dummy = ctypes.c_void_p(1 << 20)
    assert L.fwh_forward(h, fwh.FWH_F64, dummy, dummy, dummy, dummy, None) == fwh.FWH_ESTATE
    assert L.fwh_adjoint(h, fwh.FWH_F64, dummy, dummy, dummy, dummy, dummy, dummy, dummy, None) == fwh.FWH_ESTATE
    assert L.fwh_obs_window(h, None, None, None) == fwh.FWH_ESTATE
    assert b"not set up" in L.fwh_last_error()
    assert L.fwh_post(h, dummy, 256, 1.0, dummy, dummy, None) == fwh.FWH_ESTATE
    assert L.fwh_post(None, dummy, 256, 1.0, dummy, dummy, None) == fwh.FWH_EINVAL
    L.fwh_destroy(h)


# ------------------------------------------------------------ general motion

def _gm_args(**kw):
    d = dict(P=10, O=3, N=32, mach=0.3, dtau=0.01, tau0=0.0, ptr=0x1000)
    d.update(kw)
    p = d["ptr"]
    return fwh.GmArgs(d["P"], d["O"], d["N"], d["mach"], d["dtau"], d["tau0"], p, p, p, p, p)


def test_gm_plan_create_reports_workspace():
    """The device pointers are not read by plan creation (host only); the
    workspace covers the coefficient rows [P][19][N+2] FP64 at least."""
    L = fwh.lib()
    h, nb = ctypes.c_void_p(), ctypes.c_size_t()
    assert L.fwh_gm_plan_create(ctypes.byref(_gm_args(P=100, N=64)), ctypes.byref(h), ctypes.byref(nb)) == 0
    assert nb.value >= 100 * 19 * 66 * 8 and nb.value % 256 == 0
    # no window yet: state errors, not HIP calls
    assert L.fwh_gm_obs_window(h, None, None, None) == fwh.FWH_ESTATE
    assert L.fwh_gm_forward(h, ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1),
                            None) == fwh.FWH_ESTATE
    assert L.fwh_gm_window(h, None, nb.value, None) == fwh.FWH_EWORKSPACE
    assert L.fwh_gm_window(h, ctypes.c_void_p(256), nb.value - 1, None) == fwh.FWH_EWORKSPACE
    assert L.fwh_gm_window(h, ctypes.c_void_p(257), nb.value, None) == fwh.FWH_EWORKSPACE
    L.fwh_gm_destroy(h)


@pytest.mark.parametrize("kw,code", [
    (dict(P=0), fwh.FWH_ESIZE), (dict(O=0), fwh.FWH_ESIZE), (dict(N=3), fwh.FWH_ESIZE),
    (dict(N=1 << 21), fwh.FWH_ESIZE), (dict(mach=0.0), fwh.FWH_EDOMAIN), (dict(mach=1.0), fwh.FWH_EDOMAIN),
    (dict(dtau=0.0), fwh.FWH_EDOMAIN), (dict(dtau=float("nan")), fwh.FWH_EDOMAIN),
    (dict(tau0=float("inf")), fwh.FWH_EINVAL), (dict(ptr=0), fwh.FWH_EINVAL)])
def test_gm_plan_create_rejects(kw, code):
    L = fwh.lib()
    h, nb = ctypes.c_void_p(), ctypes.c_size_t()
    assert L.fwh_gm_plan_create(ctypes.byref(_gm_args(**kw)), ctypes.byref(h), ctypes.byref(nb)) == code
    assert not h.value
    assert fwh.lib().fwh_last_error().decode()


def test_gm_profile_entry_points_host_only():
    """Enabling and reading the stage timers needs no GPU while nothing was recorded."""
    L = fwh.lib()
    h, nb = ctypes.c_void_p(), ctypes.c_size_t()
    assert L.fwh_gm_plan_create(ctypes.byref(_gm_args()), ctypes.byref(h), ctypes.byref(nb)) == 0
    assert L.fwh_gm_profile_enable(h, 1) == 0
    ms, n = ctypes.c_double(-1.0), ctypes.c_int64(-1)
    for stage in (0, 1):
        assert L.fwh_gm_profile_read(h, stage, ctypes.byref(ms), ctypes.byref(n)) == 0
        assert ms.value == 0.0 and n.value == 0
    assert L.fwh_gm_profile_read(h, 2, ctypes.byref(ms), ctypes.byref(n)) == fwh.FWH_EINVAL
    assert L.fwh_gm_profile_enable(None, 1) == fwh.FWH_EINVAL
    L.fwh_gm_destroy(h)


def test_plan_tune_host_checks():
    """fwh_plan_tune validates on the host: unknown variants, split counts beyond
    min(256, ceil(P/128)), any choice in the plain FP64 form; fwh_plan_info needs
    a set-up plan."""
    L = fwh.lib()
    s = surfaces.sphere(1.0, 91, 183)                 # 16653 panels: split cap ceil(P/128) = 131
    a, keep = _args(y=s.y, normal=s.normal, dS=s.dS)
    code, h, nb = _create(a)
    assert code == fwh.FWH_OK
    assert L.fwh_plan_tune(h, fwh.GATHER_DIRECT, 131) == fwh.FWH_OK
    assert L.fwh_plan_tune(h, fwh.GATHER_LDS, 0) == fwh.FWH_OK
    assert L.fwh_plan_tune(h, fwh.GATHER_AUTO, 132) == fwh.FWH_ESIZE
    assert L.fwh_plan_tune(h, fwh.GATHER_AUTO, -1) == fwh.FWH_ESIZE
    assert L.fwh_plan_tune(h, 7, 0) == fwh.FWH_EINVAL
    assert L.fwh_plan_tune(None, 0, 0) == fwh.FWH_EINVAL
    g, sp = ctypes.c_int32(), ctypes.c_int32()
    assert L.fwh_plan_info(h, ctypes.byref(g), ctypes.byref(sp)) == fwh.FWH_ESTATE
    L.fwh_destroy(h)
    a, keep = _args(mode=fwh.MODE_F64)
    code, h, nb = _create(a)
    assert L.fwh_plan_tune(h, fwh.GATHER_AUTO, 0) == fwh.FWH_OK
    assert L.fwh_plan_tune(h, fwh.GATHER_LDS, 0) == fwh.FWH_EINVAL
    assert L.fwh_plan_tune(h, fwh.GATHER_AUTO, 1) == fwh.FWH_EINVAL
    L.fwh_destroy(h)


def test_partial_region_follows_split_cap():
    """The FP32/BF16 workspace holds FP32 partial signals for at most
    min(256, ceil(P/128)) panel splits: doubling P below 128 * 256 panels grows
    the workspace by more than the coefficient region alone would need."""
    sizes = {}
    for nth in (8, 16):
        s = surfaces.sphere(1.0, nth, 2 * nth)
        a, keep = _args(y=s.y, normal=s.normal, dS=s.dS, mode=fwh.MODE_F32, n_tau=64)
        code, h, nb = _create(a)
        assert code == fwh.FWH_OK
        sizes[s.n_panels] = nb
        fwh.lib().fwh_destroy(h)
    (p1, b1), (p2, b2) = sorted(sizes.items())
    assert b2 > b1
