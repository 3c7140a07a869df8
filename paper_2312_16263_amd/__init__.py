"""Python binding of libfwh (the gfx950 FW-H far-field library, C ABI in
include/fwh.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libfwh.so``.  PyTorch provides device memory (the workspace and the output
tensors) and the current HIP stream.  If the library is missing, every entry
point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfwh.so")

FWH_OK, FWH_EINVAL, FWH_EDOMAIN, FWH_EWINDOW, FWH_ESIZE, FWH_EWORKSPACE, FWH_EHIP, FWH_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
FWH_F64, FWH_F32 = 0, 1
GATHER_AUTO, GATHER_LDS, GATHER_DIRECT, GATHER_MFMA, GATHER_STREAM = 0, 1, 2, 3, 4
GATHERS = {"auto": GATHER_AUTO, "lds": GATHER_LDS, "direct": GATHER_DIRECT, "mfma": GATHER_MFMA,
           "stream": GATHER_STREAM}
MODE_F64, MODE_F32, MODE_BF16 = 0, 1, 2
MODES = {"f64": MODE_F64, "f32": MODE_F32, "bf16": MODE_BF16}
ERROR_NAMES = {FWH_EINVAL: "FWH_EINVAL", FWH_EDOMAIN: "FWH_EDOMAIN", FWH_EWINDOW: "FWH_EWINDOW",
               FWH_ESIZE: "FWH_ESIZE", FWH_EWORKSPACE: "FWH_EWORKSPACE", FWH_EHIP: "FWH_EHIP",
               FWH_ESTATE: "FWH_ESTATE"}

# names declared in include/fwh.h
EXPORTED = ["fwh_plan_create", "fwh_plan_tune", "fwh_plan_info", "fwh_setup", "fwh_obs_window", "fwh_forward", "fwh_adjoint", "fwh_post", "fwh_profile_enable",
            "fwh_profile_read", "fwh_batch_create", "fwh_batch_tune", "fwh_batch_tune_case", "fwh_batch_gather", "fwh_batch_bind", "fwh_batch_forward",
            "fwh_batch_adjoint", "fwh_batch_info", "fwh_batch_destroy", "fwh_destroy", "fwh_gm_plan_create",
            "fwh_gm_window", "fwh_gm_obs_window", "fwh_gm_forward", "fwh_gm_profile_enable",
            "fwh_gm_profile_read", "fwh_gm_destroy", "fwh_forward_noalloc", "fwh_last_error",
            "fwh_version"]
NOALLOC_BYTES = 64 << 20  # FWH_NOALLOC_BYTES
# names declared in include/fwh_io.h
IO_EXPORTED = ["fwh_io_control_read", "fwh_io_geometry_read", "fwh_io_geometry_write", "fwh_io_observers_read",
               "fwh_io_frame_path", "fwh_io_frames_read", "fwh_io_frame_write", "fwh_io_last_error"]
STAGES = {"setup": 0, "source": 1, "gather": 2, "reduce": 3, "adj_gather": 4, "source_adj": 5}


class FwhError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class SetupArgs(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int64), ("n_obs", ctypes.c_int64), ("n_tau", ctypes.c_int64),
                ("y", ctypes.POINTER(ctypes.c_double)), ("normal", ctypes.POINTER(ctypes.c_double)),
                ("dS", ctypes.POINTER(ctypes.c_double)), ("x_obs", ctypes.POINTER(ctypes.c_double)),
                ("mach", ctypes.c_double), ("aoa_deg", ctypes.c_double), ("dtau", ctypes.c_double),
                ("tau0", ctypes.c_double), ("mode", ctypes.c_int32)]


class GmArgs(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int64), ("n_obs", ctypes.c_int64), ("n_tau", ctypes.c_int64),
                ("mach", ctypes.c_double), ("dtau", ctypes.c_double), ("tau0", ctypes.c_double),
                ("y", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("vel", ctypes.c_void_p),
                ("dS", ctypes.c_void_p), ("x_obs", ctypes.c_void_p)]


class BatchCaseC(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("rho", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("p_prime", ctypes.c_void_p), ("p_out", ctypes.c_void_p), ("grad_p", ctypes.c_void_p),
                ("g_rho", ctypes.c_void_p), ("g_u", ctypes.c_void_p), ("g_p", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libfwh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libfwh.so not found at {LIB_PATH}; build it with __graft_entry__.build() "
                               "or python paper_2312_16263_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.fwh_plan_create.argtypes = [ctypes.POINTER(SetupArgs), ctypes.POINTER(vp), ctypes.POINTER(sz)]
        L.fwh_plan_create.restype = ctypes.c_int
        L.fwh_plan_tune.argtypes = [vp, i32, i32]
        L.fwh_plan_tune.restype = ctypes.c_int
        L.fwh_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.fwh_plan_info.restype = ctypes.c_int
        L.fwh_setup.argtypes = [vp, vp, sz, vp]
        L.fwh_setup.restype = ctypes.c_int
        L.fwh_obs_window.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.fwh_obs_window.restype = ctypes.c_int
        L.fwh_forward.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.fwh_forward.restype = ctypes.c_int
        L.fwh_adjoint.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.fwh_adjoint.restype = ctypes.c_int
        L.fwh_post.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp, vp]
        L.fwh_post.restype = ctypes.c_int
        L.fwh_profile_enable.argtypes = [vp, ctypes.c_int]
        L.fwh_profile_enable.restype = ctypes.c_int
        L.fwh_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.fwh_profile_read.restype = ctypes.c_int
        L.fwh_batch_create.argtypes = [ctypes.POINTER(BatchCaseC), i32, i32, ctypes.POINTER(vp), ctypes.POINTER(sz)]
        L.fwh_batch_create.restype = ctypes.c_int
        L.fwh_batch_tune.argtypes = [vp, ctypes.c_double, i32]
        L.fwh_batch_tune.restype = ctypes.c_int
        L.fwh_batch_tune_case.argtypes = [vp, i32, ctypes.c_double, i32]
        L.fwh_batch_tune_case.restype = ctypes.c_int
        L.fwh_batch_gather.argtypes = [vp, ctypes.POINTER(i32)]
        L.fwh_batch_gather.restype = ctypes.c_int
        L.fwh_batch_bind.argtypes = [vp, vp, sz, vp]
        L.fwh_batch_bind.restype = ctypes.c_int
        L.fwh_batch_forward.argtypes = [vp, vp]
        L.fwh_batch_forward.restype = ctypes.c_int
        L.fwh_batch_adjoint.argtypes = [vp, vp]
        L.fwh_batch_adjoint.restype = ctypes.c_int
        L.fwh_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.fwh_batch_info.restype = ctypes.c_int
        L.fwh_batch_destroy.argtypes = [vp]
        L.fwh_batch_destroy.restype = None
        L.fwh_gm_plan_create.argtypes = [ctypes.POINTER(GmArgs), ctypes.POINTER(vp), ctypes.POINTER(sz)]
        L.fwh_gm_plan_create.restype = ctypes.c_int
        L.fwh_gm_window.argtypes = [vp, vp, sz, vp]
        L.fwh_gm_window.restype = ctypes.c_int
        L.fwh_gm_obs_window.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.fwh_gm_obs_window.restype = ctypes.c_int
        L.fwh_gm_forward.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fwh_gm_forward.restype = ctypes.c_int
        L.fwh_gm_profile_enable.argtypes = [vp, ctypes.c_int]
        L.fwh_gm_profile_enable.restype = ctypes.c_int
        L.fwh_gm_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.fwh_gm_profile_read.restype = ctypes.c_int
        L.fwh_gm_destroy.argtypes = [vp]
        L.fwh_gm_destroy.restype = None
        L.fwh_destroy.argtypes = [vp]
        L.fwh_destroy.restype = None
        L.fwh_forward_noalloc.argtypes = [ctypes.POINTER(SetupArgs), i32, vp, vp, vp, vp, i64, ctypes.POINTER(i64), vp]
        L.fwh_forward_noalloc.restype = ctypes.c_int
        L.fwh_last_error.argtypes = []
        L.fwh_last_error.restype = ctypes.c_char_p
        L.fwh_version.argtypes = []
        L.fwh_version.restype = ctypes.c_char_p
        # host-side file readers, include/fwh_io.h
        cs = ctypes.c_char_p
        for name, args in (("fwh_io_control_read", [cs, vp, i32, ctypes.POINTER(i32)]),
                           ("fwh_io_geometry_read", [cs, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp, vp,
                                                     i64, i64]),
                           ("fwh_io_geometry_write", [cs, i64, vp, vp, vp, vp]),
                           ("fwh_io_observers_read", [cs, ctypes.POINTER(i64), vp, i64]),
                           ("fwh_io_frame_path", [cs, i64, ctypes.c_char_p, i64]),
                           ("fwh_io_frames_read", [cs, i64, i64, i64, i32, i64, vp, i32, vp, vp, vp, i32]),
                           ("fwh_io_frame_write", [cs, i32, i64, vp, vp, vp, vp, vp, vp])):
            getattr(L, name).argtypes = args
            getattr(L, name).restype = ctypes.c_int
        L.fwh_io_last_error.argtypes = []
        L.fwh_io_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code: int):
    if code != FWH_OK:
        raise FwhError(code, lib().fwh_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Window:
    t_start: np.ndarray
    n_t: np.ndarray
    n_t_max: int


class Plan:
    """A set-up FW-H plan on the current CUDA(HIP) device.

    y, normal [P,3], dS [P], x_obs [O,3]: geometry (host arrays);
    mach, aoa_deg, dtau, tau0, n_tau: flow and time grid; mode: 'f64' | 'f32' | 'bf16';
    gather: forward gather kernel of the FP32/BF16 modes, 'auto' | 'stream' | 'lds' | 'mfma' | 'direct';
    splits: panel splits of that gather (0: chosen at setup).
    """

    def __init__(self, y, normal, dS, x_obs, mach, aoa_deg, dtau, tau0, n_tau, mode="f32", device=None,
                 gather="auto", splits=0):
        import torch
        L = lib()
        self._keep = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (y, normal, dS, x_obs)]
        yy, nn, ds, xx = self._keep
        self.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        args = SetupArgs(yy.shape[0], xx.shape[0], int(n_tau), _dptr(yy), _dptr(nn), _dptr(ds), _dptr(xx),
                         float(mach), float(aoa_deg), float(dtau), float(tau0), self.mode)
        h = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        _check(L.fwh_plan_create(ctypes.byref(args), ctypes.byref(h), ctypes.byref(nbytes)))
        self._h = h
        self._free = lib().fwh_destroy  # kept: at interpreter exit the module globals may be gone
        if gather != "auto" or splits:
            _check(L.fwh_plan_tune(h, GATHERS[gather], int(splits)))
        self.P, self.O, self.N = yy.shape[0], xx.shape[0], int(n_tau)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.workspace_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self.setup()
        self.out_dtype = torch.float64 if self.mode == MODE_F64 else torch.float32

    def setup(self):
        """(Re-)run the device setup: delays, observer window, pair tables."""
        import torch
        L = lib()
        with torch.cuda.device(self.device):
            _check(L.fwh_setup(self._h, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace_bytes,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        ts = np.empty(self.O)
        nt = np.empty(self.O, dtype=np.int64)
        ntm = ctypes.c_int64()
        _check(L.fwh_obs_window(self._h, _dptr(ts), nt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                ctypes.byref(ntm)))
        self.window = Window(ts, nt, int(ntm.value))

    def info(self):
        """(gather kernel, panel splits) chosen at setup: ('mfma' | 'lds' | 'direct' | 'f64', splits)."""
        g, s = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fwh_plan_info(self._h, ctypes.byref(g), ctypes.byref(s)))
        names = {GATHER_LDS: "lds", GATHER_DIRECT: "direct", GATHER_MFMA: "mfma", GATHER_STREAM: "stream"}
        return names.get(g.value, "f64"), int(s.value)

    def profile(self, enable: bool = True):
        """Bracket every stage of this plan with HIP events on its stream."""
        _check(lib().fwh_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{stage: (total_ms, launches)} of the events recorded since the last read."""
        out = {}
        for name, st in STAGES.items():
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            _check(lib().fwh_profile_read(self._h, st, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, int(n.value))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None

    def _in_dtype(self, t):
        import torch
        if t.dtype == torch.float64:
            return FWH_F64
        if t.dtype == torch.float32:
            return FWH_F32
        raise TypeError(f"surface data must be float64 or float32, got {t.dtype}")

    def _check_inputs(self, rho, u, pp):
        for name, t, shape in (("rho", rho, (self.N, self.P)), ("u", u, (3, self.N, self.P)),
                               ("p", pp, (self.N, self.P))):
            if tuple(t.shape) != shape:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
            if not t.is_contiguous() or t.device != self.device:
                raise ValueError(f"{name} must be contiguous on {self.device}")
        if not (rho.dtype == u.dtype == pp.dtype):
            raise TypeError("rho, u and p must have one dtype")

    def forward(self, rho, u, pp, out=None):
        """p'(o, k) as a [O, n_t_max] tensor (float64 in mode f64, float32 otherwise)."""
        import torch
        self._check_inputs(rho, u, pp)
        if out is None:
            out = torch.empty((self.O, self.window.n_t_max), dtype=self.out_dtype, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().fwh_forward(self._h, self._in_dtype(rho), ctypes.c_void_p(rho.data_ptr()),
                                     ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(pp.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return out

    def adjoint(self, rho, u, pp, grad_p, out=None):
        """(dJ/drho, dJ/du, dJ/dp') for grad_p = dJ/dp' [O, n_t_max]."""
        import torch
        self._check_inputs(rho, u, pp)
        grad_p = grad_p.to(self.out_dtype).contiguous()
        if tuple(grad_p.shape) != (self.O, self.window.n_t_max):
            raise ValueError(f"grad_p has shape {tuple(grad_p.shape)}, expected {(self.O, self.window.n_t_max)}")
        if out is None:
            out = (torch.empty_like(rho), torch.empty_like(u), torch.empty_like(pp))
        g_r, g_u, g_p = out
        with torch.cuda.device(self.device):
            _check(lib().fwh_adjoint(self._h, self._in_dtype(rho), ctypes.c_void_p(rho.data_ptr()),
                                     ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(pp.data_ptr()),
                                     ctypes.c_void_p(grad_p.data_ptr()), ctypes.c_void_p(g_r.data_ptr()),
                                     ctypes.c_void_p(g_u.data_ptr()), ctypes.c_void_p(g_p.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return g_r, g_u, g_p

    def post(self, p, seg_len, span_ratio=1.0):
        """Per-observer RMS [O] and one-sided Welch PSD [O, seg_len/2 + 1] (Hann window, 50 % overlap,
        times span_ratio) of a forward result p; frequencies k / (seg_len * dtau).  float32 tensors."""
        import torch
        if tuple(p.shape) != (self.O, self.window.n_t_max) or p.dtype != self.out_dtype or not p.is_contiguous():
            raise ValueError("p must be a contiguous forward result of this plan")
        psd = torch.empty((self.O, seg_len // 2 + 1), dtype=torch.float32, device=self.device)
        rms = torch.empty((self.O,), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().fwh_post(self._h, ctypes.c_void_p(p.data_ptr()), int(seg_len), float(span_ratio),
                                  ctypes.c_void_p(psd.data_ptr()), ctypes.c_void_p(rms.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return psd, rms


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Batch:
    """Many set-up plans (FP32 or BF16 mode) run as one batch: forward and
    adjoint of every case are each a fixed sequence of batched launches (the
    gathers persistent over longest-first work lists), so `capture()` records a
    whole step (forward, dJ/dp' = 2 p', adjoint) in one HIP graph.  `inputs`
    holds (rho, u, p) device tensors per plan, one dtype."""

    def __init__(self, plans, inputs, item_units=None, blocks_per_cu=2):
        import torch
        L = lib()
        self.plans = list(plans)
        self.inputs = [tuple(t) for t in inputs]
        dt = self.inputs[0][0].dtype
        self.in_dtype = FWH_F64 if dt == torch.float64 else FWH_F32
        self.p_out, self.grad_p, self.grads = [], [], []
        arr = (BatchCaseC * len(self.plans))()
        for i, (pl, (rho, u, pp)) in enumerate(zip(self.plans, self.inputs)):
            pl._check_inputs(rho, u, pp)
            if rho.dtype != dt:
                raise TypeError("all cases of a batch need one input dtype")
            po = torch.zeros((pl.O, pl.window.n_t_max), dtype=torch.float32, device=pl.device)
            gp = torch.zeros_like(po)
            g = (torch.empty_like(rho), torch.empty_like(u), torch.empty_like(pp))
            self.p_out.append(po)
            self.grad_p.append(gp)
            self.grads.append(g)
            arr[i] = BatchCaseC(pl._h.value, rho.data_ptr(), u.data_ptr(), pp.data_ptr(), po.data_ptr(),
                                gp.data_ptr(), g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr())
        h = ctypes.c_void_p()
        nb = ctypes.c_size_t()
        _check(L.fwh_batch_create(arr, len(self.plans), self.in_dtype, ctypes.byref(h), ctypes.byref(nb)))
        self._h = h
        self._free = lib().fwh_batch_destroy  # kept: at interpreter exit the module globals may be gone
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.plans[0].device)
        self.blocks_per_cu = blocks_per_cu
        self.tune(item_units, blocks_per_cu)

    @property
    def gather(self):
        """'mfma' or 'lds': the forward gather of every case."""
        g = ctypes.c_int32()
        _check(lib().fwh_batch_gather(self._h, ctypes.byref(g)))
        return {GATHER_MFMA: "mfma", GATHER_LDS: "lds"}[g.value]

    def tune(self, item_units=None, blocks_per_cu=None):
        """Batch-wide work granularity (None keeps each case's) and resident blocks per CU; rebinds."""
        bpc = self.blocks_per_cu if blocks_per_cu is None else blocks_per_cu
        _check(lib().fwh_batch_tune(self._h, float(item_units or 0.0), int(bpc)))
        self.blocks_per_cu = bpc
        self.bind()

    def tune_case(self, i, item_units=None, rows=4, bind=True):
        """Tiles of case i: forward work per item and rows of 61 samples per block (2..4)."""
        _check(lib().fwh_batch_tune_case(self._h, int(i), float(item_units or 0.0), int(rows)))
        if bind:
            self.bind()

    def bind(self):
        _check(lib().fwh_batch_bind(self._h, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                    _stream()))

    def info(self):
        n_items, units, grid = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fwh_batch_info(self._h, ctypes.byref(n_items), ctypes.byref(units), ctypes.byref(grid)))
        return {"items": int(n_items.value), "units": int(units.value), "grid": int(grid.value)}

    def forward(self):
        _check(lib().fwh_batch_forward(self._h, _stream()))
        return self.p_out

    def adjoint(self):
        _check(lib().fwh_batch_adjoint(self._h, _stream()))
        return self.grads

    def step(self):
        """forward, dJ/dp' = 2 p' for J = sum p'^2 (elementwise, no memset), adjoint."""
        import torch
        self.forward()
        for po, gp in zip(self.p_out, self.grad_p):
            torch.mul(po, 2.0, out=gp)
        self.adjoint()

    def capture(self):
        """Record one step in a HIP graph (torch.cuda.CUDAGraph) and return it."""
        import torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        return g

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None


# per-class candidates: (rows of 61 samples per block, target panel-observer-samples per forward item)
DEFAULT_CASE_CANDIDATES = [(4, 1e6), (4, 4e6), (4, 16e6), (2, 1e6), (2, 4e6), (2, 16e6)]
DEFAULT_BPC_CANDIDATES = (2, 3)


def batch_signature(batch: "Batch") -> str:
    parts = [f"m{batch.plans[0].mode}", f"d{batch.in_dtype}"]
    parts += [f"{p.P}x{p.O}x{p.N}" for p in batch.plans]
    return "|".join(parts)


def size_class(plan) -> str:
    """Tuning class of a case: mode, panels (nearest power of two), observers
    (<= 32, <= 96, <= 192, more) and record length (<= 1024, <= 2048, more)."""
    import math
    ob = 0 if plan.O <= 32 else 1 if plan.O <= 96 else 2 if plan.O <= 192 else 3
    nb = 0 if plan.N <= 1024 else 1 if plan.N <= 2048 else 2
    return f"m{plan.mode}|P2^{int(round(math.log2(plan.P)))}|O{ob}|N{nb}"


def _time_forward(batch, reps):
    import torch
    batch.forward()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        batch.forward()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def autotune(batch: "Batch", candidates=None, bpc_candidates=None, reps=2, cache_path=None):
    """Tile choice per class of case sizes (size_class): the cases of one class
    run alone as a batch under each (rows, item_units) candidate, timed with HIP
    events over the batched forward; the fastest is applied to those cases.
    Then the resident blocks per CU of the persistent gathers are timed on the
    whole batch.  Choices are cached in `cache_path` (JSON) per class and, for
    the grid, per batch signature.  Returns {"classes": {class: {"choice": [rows,
    item_units], "table": [[rows, item_units, ms], ...]}}, "blocks_per_cu": b,
    "grid_table": [[b, ms], ...]}."""
    import json
    import os
    cands = list(candidates or DEFAULT_CASE_CANDIDATES)
    if batch.gather != "mfma":
        cands = sorted({(4, iu) for _, iu in cands})
    cache = json.load(open(cache_path)) if cache_path and os.path.exists(cache_path) else {}
    groups = {}
    for i, pl in enumerate(batch.plans):
        groups.setdefault(f"{batch.gather}|{size_class(pl)}", []).append(i)
    out = {"classes": {}}
    for key, idx in groups.items():
        if key in cache:
            rows, iu = cache[key]["choice"]
            table = cache[key]["table"]
        else:
            sub = Batch([batch.plans[i] for i in idx], [batch.inputs[i] for i in idx],
                        blocks_per_cu=batch.blocks_per_cu)
            table = []
            for rows, iu in cands:
                for j in range(len(idx)):
                    sub.tune_case(j, iu, rows, bind=False)
                sub.bind()
                table.append([rows, iu, _time_forward(sub, reps)])
            del sub
            rows, iu, _ = min(table, key=lambda r: r[2])
            cache[key] = {"choice": [rows, iu], "table": table}
        for i in idx:
            batch.tune_case(i, iu, rows, bind=False)
        out["classes"][key] = {"choice": [rows, iu], "table": table, "cases": len(idx)}
    sig = batch_signature(batch)
    if sig in cache:
        bpc, gtable = cache[sig]["choice"], cache[sig]["table"]
    else:
        gtable = []
        for bpc in (bpc_candidates or DEFAULT_BPC_CANDIDATES):
            batch.tune(None, bpc)
            gtable.append([bpc, _time_forward(batch, reps)])
        bpc = min(gtable, key=lambda r: r[1])[0]
        cache[sig] = {"choice": bpc, "table": gtable}
    batch.tune(None, bpc)
    out["blocks_per_cu"], out["grid_table"] = bpc, gtable
    if cache_path:
        json.dump(cache, open(cache_path, "w"))
    return out


def _autograd_function():
    import torch

    class FwhFunction(torch.autograd.Function):
        """p' = FW-H(rho, u, p) on a set-up plan; backward runs the hand-written
        transposed gather and source adjoint (fwh_adjoint)."""

        @staticmethod
        def forward(ctx, plan, rho, u, pp):
            ctx.plan = plan
            ctx.save_for_backward(rho, u, pp)
            return plan.forward(rho, u, pp)

        @staticmethod
        def backward(ctx, grad):
            rho, u, pp = ctx.saved_tensors
            g_r, g_u, g_p = ctx.plan.adjoint(rho, u, pp, grad.contiguous())
            return None, g_r, g_u, g_p

    return FwhFunction


_fn = None


def fwh_apply(plan: Plan, rho, u, pp):
    """Differentiable forward: torch.autograd sees p' as a function of (rho, u, p)."""
    global _fn
    if _fn is None:
        _fn = _autograd_function()
    return _fn.apply(plan, rho, u, pp)


def version() -> str:
    return lib().fwh_version().decode()


class GMPlan:
    """General-motion plan (moving surface, medium and observers at rest) on
    the current CUDA(HIP) device.

    y, normal, vel [N,P,3], dS [P], x_obs [O,3]: float64 tensors on the device
    (kept referenced by the plan); mach, dtau, tau0: scalars.  The observer
    window is computed at construction (``self.window``)."""

    def __init__(self, y, normal, vel, dS, x_obs, mach, dtau, tau0=0.0):
        import torch
        L = lib()
        N, P = int(y.shape[0]), int(y.shape[1])
        O = int(x_obs.shape[0])
        for name, t, shape in (("y", y, (N, P, 3)), ("normal", normal, (N, P, 3)), ("vel", vel, (N, P, 3)),
                               ("dS", dS, (P,)), ("x_obs", x_obs, (O, 3))):
            if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {shape}")
        self.device = y.device
        self._keep = (y, normal, vel, dS, x_obs)
        args = GmArgs(P, O, N, float(mach), float(dtau), float(tau0), y.data_ptr(), normal.data_ptr(),
                      vel.data_ptr(), dS.data_ptr(), x_obs.data_ptr())
        h = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        _check(L.fwh_gm_plan_create(ctypes.byref(args), ctypes.byref(h), ctypes.byref(nbytes)))
        self._h = h
        self._free = lib().fwh_gm_destroy  # kept: at interpreter exit the module globals may be gone
        self.P, self.O, self.N = P, O, N
        self.workspace_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            _check(L.fwh_gm_window(self._h, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace_bytes,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        ts = np.empty(O)
        nt = np.empty(O, dtype=np.int64)
        ntm = ctypes.c_int64()
        _check(L.fwh_gm_obs_window(self._h, _dptr(ts), nt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   ctypes.byref(ntm)))
        self.window = Window(ts, nt, int(ntm.value))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None

    def profile(self, enable: bool = True):
        """Bracket the source and gather stages of forward() with HIP events."""
        _check(lib().fwh_gm_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{stage: (total ms, launches)} of the recorded events (then cleared)."""
        out = {}
        for name, st in (("source", 0), ("gather", 1)):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            _check(lib().fwh_gm_profile_read(self._h, st, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def forward(self, rho, u, pp, out=None):
        """p'(o, k) as a float64 [O, n_t_max] tensor (0 past each observer's N_t)."""
        import torch
        for name, t, shape in (("rho", rho, (self.N, self.P)), ("u", u, (3, self.N, self.P)),
                               ("p", pp, (self.N, self.P))):
            if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
                raise ValueError(f"{name} must be a contiguous float64 tensor of shape {shape} on {self.device}")
        if out is None:
            out = torch.empty((self.O, self.window.n_t_max), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().fwh_gm_forward(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                        ctypes.c_void_p(pp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return out

