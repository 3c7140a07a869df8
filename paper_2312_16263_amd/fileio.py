"""Readers and writers of the OpenCFD-FWH input files (Sec. III A and
Appendix A of the paper): the control file, the surface geometry file, the
observer file and the per-step FW-H dataset.  Binding of include/fwh_io.h:
the parsing runs in libfwh.so's host code (frames on a pool of threads, straight
into the caller's time-major arrays); this module marshals arguments, types
the namelist values and gathers one case.

Readings where the text leaves a choice (the example control file and the
dataset figure are unavailable):
* the number of frames is (Kstep_end - Kstep_start) / delta_step + 1, the k-th
  frame being solver step Kstep_start + k*delta_step;
* the control file's time step is the solver's; frames are dt*delta_step apart
  in source time, and frame 0 lies at tau0 = Kstep_start*dt;
* the Mach number, angle of attack (degrees), time step, observer count, frame
  count and thread count are taken under the key names of CONTROL_KEYS (case
  folded); counts present in the file must agree with the files read;
* dataset files hold, per Face, its dimensions then (rho, u1, u2, u3, p') per
  subface (layouts in include/fwh_io.h).
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass, field

import numpy as np

from . import lib

FWH_IO_OK, FWH_IO_EINVAL, FWH_IO_ESIZE, FWH_IO_EFILE, FWH_IO_EFORMAT = 0, -1, -4, -8, -9
BINARY, ASCII = 0, 1
IO_ERROR_NAMES = {FWH_IO_EINVAL: "FWH_IO_EINVAL", FWH_IO_ESIZE: "FWH_IO_ESIZE", FWH_IO_EFILE: "FWH_IO_EFILE",
                  FWH_IO_EFORMAT: "FWH_IO_EFORMAT"}

CONTROL_FILE, GEOMETRY_FILE, OBSERVER_FILE = "control.fwh", "FWH_Surface_Geo.dat", "observers.dat"

# accepted key names (lower case) of each control quantity; the first is the one written
CONTROL_KEYS = {
    "mach": ("mach", "ma", "mach_number", "m0"),
    "aoa": ("aoa", "alpha", "angle_of_attack", "aoa_deg"),
    "dt": ("dt", "time_step", "delta_t", "dt_step"),
    "kstep_start": ("kstep_start",),
    "kstep_end": ("kstep_end",),
    "delta_step": ("delta_step",),
    "format": ("fwh_data_format",),
    "n_observers": ("n_observers", "num_observers", "nobs", "n_obs", "number_of_observers"),
    "n_frames": ("n_frames", "num_frames", "nframes", "number_of_frames"),
    "threads": ("num_threads", "omp_threads", "n_threads", "nthreads"),
}


class FwhIOError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{IO_ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code: int):
    if code != FWH_IO_OK:
        raise FwhIOError(code, lib().fwh_io_last_error().decode())


def _b(path) -> bytes:
    return os.fsencode(os.fspath(path))


def _ptr(a) -> int:
    """Address of a C-contiguous numpy array or a contiguous CPU torch tensor."""
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        if a.device.type != "cpu" or not a.is_contiguous():
            raise ValueError("tensor must be a contiguous host tensor")
        return a.data_ptr()
    raise TypeError(type(a))


# ---------------------------------------------------------------- control file
class _KV(ctypes.Structure):
    _fields_ = [("group", ctypes.c_char * 64), ("key", ctypes.c_char * 64), ("value", ctypes.c_char * 192)]


def read_control_entries(path):
    """[(group, key, value text)] of a namelist file, in file order."""
    L = lib()
    n = ctypes.c_int32(0)
    _check(L.fwh_io_control_read(_b(path), None, 0, ctypes.byref(n)))
    kv = (_KV * max(n.value, 1))()
    _check(L.fwh_io_control_read(_b(path), kv, n.value, ctypes.byref(n)))
    return [(e.group.decode(), e.key.decode(), e.value.decode()) for e in kv[: n.value]]


_INT = re.compile(r"^[+-]?\d+$")
_REAL = re.compile(r"^[+-]?(\d+\.?\d*|\.\d+)([eEdD][+-]?\d+)?$")


def _split_items(text: str):
    """Comma/blank-separated items of a value, quoted text kept whole."""
    items, cur, q, i = [], "", None, 0
    while i < len(text):
        ch = text[i]
        if q:
            cur += ch
            if ch == q:
                if i + 1 < len(text) and text[i + 1] == q:
                    cur += q
                    i += 1
                else:
                    q = None
        elif ch in "'\"":
            q = ch
            cur += ch
        elif ch == "," or ch.isspace():
            if cur:
                items.append(cur)
            cur = ""
        else:
            cur += ch
        i += 1
    if cur:
        items.append(cur)
    return items


def _scalar(p: str):
    if p[:1] in ("'", '"'):
        return p[1:-1].replace(p[0] * 2, p[0])
    low = p.lower()
    if low in (".true.", "t", ".t.", "true"):
        return True
    if low in (".false.", "f", ".f.", "false"):
        return False
    if _INT.match(p):
        return int(p)
    if _REAL.match(p):
        return float(re.sub("[dD]", "e", p))
    return p


def parse_value(text: str):
    """Fortran namelist value text -> bool, int, float, str or a list of them
    (r*v repeats v r times)."""
    out = []
    for p in _split_items(text):
        m = re.match(r"^(\d+)\*(.+)$", p)
        if m:
            out.extend([_scalar(m.group(2))] * int(m.group(1)))
        else:
            out.append(_scalar(p))
    if not out:
        return ""
    return out if len(out) > 1 else out[0]


def read_control(path) -> dict:
    """{key: typed value} of every entry (keys lower case; a later entry wins)."""
    return {k: parse_value(v) for _, k, v in read_control_entries(path)}


def control_value(ctl: dict, name: str, default=None):
    for k in CONTROL_KEYS[name]:
        if k in ctl:
            return ctl[k]
    return default


def write_control(path, values: dict, group: str = "control_fwh"):
    """Writes a namelist group; bool as .true./.false., str quoted, float with
    17 significant digits."""
    def fmt(v):
        if isinstance(v, bool):
            return ".true." if v else ".false."
        if isinstance(v, (int, np.integer)):
            return str(int(v))
        if isinstance(v, (float, np.floating)):
            return repr(float(v))
        return "'" + str(v).replace("'", "''") + "'"
    with open(path, "w") as f:
        f.write(f"&{group}\n")
        for k, v in values.items():
            f.write(f"  {k} = {fmt(v)}\n")
        f.write("/\n")


# -------------------------------------------------------- geometry, observers
@dataclass
class Geometry:
    face_dims: np.ndarray  # [F][3] int64 (nx, ny, nz)
    y: np.ndarray          # [P][3]
    normal: np.ndarray     # [P][3]
    dS: np.ndarray         # [P]

    @property
    def n_panels(self) -> int:
        return int(self.dS.shape[0])

    @property
    def face_id(self) -> np.ndarray:
        """Face of each panel (file order), the case/surface id of a panel."""
        return np.repeat(np.arange(self.face_dims.shape[0], dtype=np.int32), np.prod(self.face_dims, axis=1))


def read_geometry(path) -> Geometry:
    L = lib()
    nf, npn = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(L.fwh_io_geometry_read(_b(path), ctypes.byref(nf), ctypes.byref(npn), None, None, None, None, 0, 0))
    dims = np.zeros((nf.value, 3), dtype=np.int64)
    y = np.zeros((npn.value, 3))
    nrm = np.zeros((npn.value, 3))
    dS = np.zeros(npn.value)
    _check(L.fwh_io_geometry_read(_b(path), ctypes.byref(nf), ctypes.byref(npn), dims.ctypes.data, y.ctypes.data,
                                  nrm.ctypes.data, dS.ctypes.data, dims.shape[0], dS.shape[0]))
    return Geometry(dims, y, nrm, dS)


def write_geometry(path, geom: Geometry):
    dims = np.ascontiguousarray(geom.face_dims, dtype=np.int64)
    y, nrm, dS = (np.ascontiguousarray(a, dtype=np.float64) for a in (geom.y, geom.normal, geom.dS))
    if y.shape != (int(np.prod(dims, axis=1).sum()), 3) or nrm.shape != y.shape or dS.shape != y.shape[:1]:
        raise ValueError("geometry arrays do not match the Face dimensions")
    _check(lib().fwh_io_geometry_write(_b(path), dims.shape[0], dims.ctypes.data, y.ctypes.data, nrm.ctypes.data,
                                       dS.ctypes.data))


def read_observers(path) -> np.ndarray:
    L = lib()
    n = ctypes.c_int64(0)
    _check(L.fwh_io_observers_read(_b(path), ctypes.byref(n), None, 0))
    x = np.zeros((n.value, 3))
    _check(L.fwh_io_observers_read(_b(path), ctypes.byref(n), x.ctypes.data, x.shape[0]))
    return x


def write_observers(path, x_obs):
    np.savetxt(path, np.asarray(x_obs, dtype=np.float64).reshape(-1, 3), fmt="%.17g")


# -------------------------------------------------------------------- dataset
def frame_path(directory, step: int) -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(lib().fwh_io_frame_path(_b(directory), int(step), buf, len(buf)))
    return os.fsdecode(buf.value)


def write_frame(path, fmt: int, face_dims, rho, u, pp):
    """One dataset file from per-panel arrays rho [P], u [3][P], pp [P]."""
    dims = np.ascontiguousarray(face_dims, dtype=np.int64)
    P = int(np.prod(dims, axis=1).sum())
    r, p = (np.ascontiguousarray(a, dtype=np.float64).reshape(P) for a in (rho, pp))
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(3, P)
    _check(lib().fwh_io_frame_write(_b(path), int(fmt), dims.shape[0], dims.ctypes.data, r.ctypes.data,
                                    uu[0].ctypes.data, uu[1].ctypes.data, uu[2].ctypes.data, p.ctypes.data))


def read_frames(directory, kstep_start: int, delta_step: int, n_frames: int, fmt: int, face_dims,
                dtype: str = "f64", out=None, threads: int = 0):
    """Reads n_frames dataset files into time-major host arrays
    (rho [N][P], u [3][N][P], pp [N][P]).  `out`, if given, is such a triple of
    contiguous host buffers (numpy arrays or CPU torch tensors, pinned ones
    included) of the matching type; else numpy arrays are allocated."""
    dims = np.ascontiguousarray(face_dims, dtype=np.int64)
    P = int(np.prod(dims, axis=1).sum())
    npdt = {"f64": np.float64, "f32": np.float32}[dtype]
    if out is None:
        out = (np.empty((n_frames, P), npdt), np.empty((3, n_frames, P), npdt), np.empty((n_frames, P), npdt))
    rho, u, pp = out
    for a, shape in ((rho, (n_frames, P)), (u, (3, n_frames, P)), (pp, (n_frames, P))):
        if tuple(a.shape) != shape or (a.itemsize if isinstance(a, np.ndarray) else a.element_size()) != \
                np.dtype(npdt).itemsize:
            raise ValueError(f"output buffer of shape {tuple(a.shape)} does not hold {shape} {dtype}")
    _check(lib().fwh_io_frames_read(_b(directory), int(kstep_start), int(delta_step), int(n_frames), int(fmt),
                                    dims.shape[0], dims.ctypes.data, 0 if dtype == "f64" else 1, _ptr(rho), _ptr(u),
                                    _ptr(pp), int(threads)))
    return rho, u, pp


def read_frames_to_device(directory, kstep_start: int, delta_step: int, n_frames: int, fmt: int, face_dims,
                          dtype: str = "f32", device="cuda", block: int = 128, threads: int = 0):
    """Reads n_frames dataset files straight into time-major device tensors
    (rho [N][P], u [3][N][P], pp [N][P]) in blocks of `block` frames: each block
    is parsed by the library's reader threads into one of two page-locked
    buffers while the previous block is copied to the device on a side stream.
    Host memory stays at two blocks whatever the record length, for records
    larger than the host can pin.  Returns after the copies are ordered before
    later work on the current stream."""
    import torch
    dims = np.ascontiguousarray(face_dims, dtype=np.int64)
    P = int(np.prod(dims, axis=1).sum())
    tdt = {"f64": torch.float64, "f32": torch.float32}[dtype]
    dev = torch.device(device)
    rho = torch.empty((n_frames, P), dtype=tdt, device=dev)
    u = torch.empty((3, n_frames, P), dtype=tdt, device=dev)
    pp = torch.empty((n_frames, P), dtype=tdt, device=dev)
    block = max(1, min(block, n_frames))
    bufs = [(torch.empty(block * P, dtype=tdt, pin_memory=True), torch.empty(3 * block * P, dtype=tdt, pin_memory=True),
             torch.empty(block * P, dtype=tdt, pin_memory=True)) for _ in range(2)]
    done = [None, None]
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))  # the outputs' allocation is ordered before the copies
    for bi, k0 in enumerate(range(0, n_frames, block)):
        nb = min(block, n_frames - k0)
        rb, ub, pb = bufs[bi % 2]
        if done[bi % 2] is not None:
            done[bi % 2].synchronize()  # this buffer's previous copy has finished
        views = (rb[:nb * P].view(nb, P), ub[:3 * nb * P].view(3, nb, P), pb[:nb * P].view(nb, P))
        read_frames(directory, kstep_start + k0 * delta_step, delta_step, nb, fmt, dims, dtype=dtype, out=views,
                    threads=threads)
        with torch.cuda.stream(side):
            rho[k0:k0 + nb].copy_(views[0], non_blocking=True)
            for c in range(3):
                u[c, k0:k0 + nb].copy_(views[1][c], non_blocking=True)
            pp[k0:k0 + nb].copy_(views[2], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(side)
        done[bi % 2] = ev
    torch.cuda.current_stream(dev).wait_stream(side)
    # the pinned buffers must outlive their copies
    for ev in done:
        if ev is not None:
            ev.synchronize()
    return rho, u, pp


# ----------------------------------------------------------------- whole case
@dataclass
class Case:
    """One case directory: flow, geometry, observers and the surface data."""
    mach: float
    aoa_deg: float
    dt: float
    kstep_start: int
    kstep_end: int
    delta_step: int
    fmt: int
    geometry: Geometry
    x_obs: np.ndarray
    rho: object = None
    u: object = None
    pp: object = None
    control: dict = field(default_factory=dict)

    @property
    def n_frames(self) -> int:
        return (self.kstep_end - self.kstep_start) // self.delta_step + 1

    @property
    def dtau(self) -> float:
        return self.dt * self.delta_step

    @property
    def tau0(self) -> float:
        return self.kstep_start * self.dt

    def plan(self, mode: str = "f32", device=None):
        """A wind-tunnel Plan (fwh_plan_create) for this case."""
        from . import Plan
        g = self.geometry
        return Plan(g.y, g.normal, g.dS, self.x_obs, self.mach, self.aoa_deg, self.dtau, self.tau0, self.n_frames,
                    mode=mode, device=device)


def load_case(directory, dtype: str = "f64", threads=None, pinned: bool = False, frames: bool = True,
              device=None) -> Case:
    """Reads control.fwh, FWH_Surface_Geo.dat, observers.dat and the dataset
    files of `directory`.  pinned=True reads the frames into page-locked torch
    host tensors (ready for an asynchronous copy to the device); device="cuda"
    streams them into device tensors (read_frames_to_device)."""
    ctl = read_control(os.path.join(directory, CONTROL_FILE))

    def need(name):
        v = control_value(ctl, name)
        if v is None:
            raise FwhIOError(FWH_IO_EFORMAT, f"{CONTROL_FILE}: no value for {name} (keys {CONTROL_KEYS[name]})")
        return v

    geom = read_geometry(os.path.join(directory, GEOMETRY_FILE))
    x_obs = read_observers(os.path.join(directory, OBSERVER_FILE))
    case = Case(mach=float(need("mach")), aoa_deg=float(control_value(ctl, "aoa", 0.0)), dt=float(need("dt")),
                kstep_start=int(need("kstep_start")), kstep_end=int(need("kstep_end")),
                delta_step=int(control_value(ctl, "delta_step", 1)), fmt=int(control_value(ctl, "format", BINARY)),
                geometry=geom, x_obs=x_obs, control=ctl)
    if case.delta_step < 1 or case.kstep_end < case.kstep_start or \
            (case.kstep_end - case.kstep_start) % case.delta_step != 0:
        raise FwhIOError(FWH_IO_EFORMAT, f"{CONTROL_FILE}: Kstep_start {case.kstep_start}, Kstep_end "
                         f"{case.kstep_end}, delta_step {case.delta_step} do not give whole frames")
    for name, have in (("n_observers", x_obs.shape[0]), ("n_frames", case.n_frames)):
        want = control_value(ctl, name)
        if want is not None and int(want) != have:
            raise FwhIOError(FWH_IO_EFORMAT, f"{CONTROL_FILE}: {name} = {want} but the files give {have}")
    if frames:
        if threads is None:
            threads = int(control_value(ctl, "threads", 0))
        if device is not None:
            case.rho, case.u, case.pp = read_frames_to_device(directory, case.kstep_start, case.delta_step,
                                                              case.n_frames, case.fmt, geom.face_dims, dtype=dtype,
                                                              device=device, threads=threads)
            return case
        out = None
        if pinned:
            import torch
            tdt = {"f64": torch.float64, "f32": torch.float32}[dtype]
            N, P = case.n_frames, geom.n_panels
            out = (torch.empty((N, P), dtype=tdt, pin_memory=True), torch.empty((3, N, P), dtype=tdt, pin_memory=True),
                   torch.empty((N, P), dtype=tdt, pin_memory=True))
        case.rho, case.u, case.pp = read_frames(directory, case.kstep_start, case.delta_step, case.n_frames, case.fmt,
                                                geom.face_dims, dtype=dtype, out=out, threads=threads)
    return case


def save_case(directory, mach, aoa_deg, dt, kstep_start, delta_step, geometry: Geometry, x_obs, rho, u, pp,
              fmt: int = BINARY, threads: int = 0, extra: dict | None = None):
    """Writes a case directory that load_case reads back: time-major rho [N][P],
    u [3][N][P], pp [N][P] become the files of steps kstep_start + k*delta_step."""
    os.makedirs(directory, exist_ok=True)
    rho, u, pp = (np.asarray(a, dtype=np.float64) for a in (rho, u, pp))
    N = rho.shape[0]
    values = {"Mach": float(mach), "AoA": float(aoa_deg), "dt": float(dt), "Kstep_start": int(kstep_start),
              "Kstep_end": int(kstep_start + (N - 1) * delta_step), "delta_step": int(delta_step),
              "FWH_data_Format": int(fmt), "n_observers": int(np.asarray(x_obs).reshape(-1, 3).shape[0]),
              "num_threads": int(threads)}
    values.update(extra or {})
    write_control(os.path.join(directory, CONTROL_FILE), values)
    write_geometry(os.path.join(directory, GEOMETRY_FILE), geometry)
    write_observers(os.path.join(directory, OBSERVER_FILE), x_obs)
    for k in range(N):
        write_frame(frame_path(directory, kstep_start + k * delta_step), fmt, geometry.face_dims, rho[k], u[:, k],
                    pp[k])
