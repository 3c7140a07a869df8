"""The benchmark/parity workloads as seeded synthetic inputs.

  monopole_small   convected monopole, sphere r = 1, 32 x 64 panels, M0 0.3, AoA 5 deg,
                   w = 2 pi, 256 samples per period over 2 periods (N = 512),
                   8 observers on a circle of radius 50; FP64 data.
  dipole_sphere    convected dipole (axis x2), sphere r = 1, 128 x 256 = 32768 panels,
                   M0 0.5, AoA 10 deg, N = 2048 at dtau = 1/256, 360 observers every
                   1 deg on a circle of radius 100; FP64 data.
  airfoil_broadband  Joukowski contour (1200 points, chord 1) extruded over 200 stations
                   across a span of 1/9 chord: 240000 panels, M0 0.17, AoA 5.5 deg,
                   N = 4096 at the 30P30N sampling interval 1e-5 s in units of
                   c_s/U0 (dtau = 1.2642e-3), 72 observers every 5 deg at R = 10 about
                   mid-chord; seeded broadband data, RMS 1 % of freestream, FP32.

The constructors take the panel grid, samples and observers as arguments, so
parity tests build the same workloads at sizes the FP64 oracle finishes in
seconds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import analytic, broadband, surfaces

# nondimensional amplitude of the analytic sources (|u'| ~ 1e-3 at r = 1)
ANALYTIC_AMPLITUDE = 4.0 * math.pi * 1e-4


@dataclass
class Case:
    name: str
    surface: surfaces.Surface
    x_obs: np.ndarray
    mach: float
    aoa_deg: float
    dtau: float
    n_tau: int
    tau0: float = 0.0
    kind: str = "monopole"          # 'monopole' | 'dipole' | 'broadband'
    omega: float = 2.0 * math.pi
    amplitude: float = ANALYTIC_AMPLITUDE
    seed: int = 0
    data_dtype: type = np.float64
    meta: dict = field(default_factory=dict)

    @property
    def n_panels(self) -> int:
        return self.surface.n_panels

    @property
    def n_obs(self) -> int:
        return int(self.x_obs.shape[0])

    def data(self):
        """(rho [N,P], u [3,N,P], p' [N,P]) time-major numpy arrays."""
        if self.kind == "broadband":
            return broadband.surface_data(self.n_panels, self.n_tau, self.aoa_deg, self.seed, dtype=self.data_dtype)
        return analytic.surface_series(self.kind, self.surface.y, analytic.Flow(self.mach, self.aoa_deg),
                                       self.amplitude, self.omega, self.n_tau, self.dtau, self.tau0,
                                       dtype=self.data_dtype)

    def data_device(self, device="cuda"):
        """Surface data as device tensors; broadband data are generated on the
        device (torch generator), analytic data on the host then copied."""
        if self.kind == "broadband":
            return broadband.surface_data_torch(self.n_panels, self.n_tau, self.aoa_deg, self.seed, device=device)
        return analytic.surface_series_torch(self.kind, self.surface.y, analytic.Flow(self.mach, self.aoa_deg),
                                             self.amplitude, self.omega, self.n_tau, self.dtau, self.tau0,
                                             dtype=self.data_dtype, device=device)

    def exact(self, t):
        """Closed-form p'(x_o, t) of the analytic source ([O, K] times)."""
        return analytic.far_field_pressure(self.kind, self.x_obs, analytic.Flow(self.mach, self.aoa_deg),
                                           self.amplitude, self.omega, t)


def monopole_small() -> Case:
    return Case("monopole_small", surfaces.sphere(1.0, 32, 64), surfaces.observer_circle(8, 50.0), 0.3, 5.0,
                1.0 / 256.0, 512, kind="monopole")


def dipole_sphere(n_theta=128, n_phi=256, n_tau=2048, n_obs=360) -> Case:
    return Case("dipole_sphere", surfaces.sphere(1.0, n_theta, n_phi),
                surfaces.observer_circle(n_obs, 100.0, step_deg=360.0 / n_obs), 0.5, 10.0, 1.0 / 256.0, n_tau,
                kind="dipole")


AIRFOIL_DTAU = 1e-5 * (0.17 * 340.0) / 0.4572   # 1e-5 s sampling, L_ref = stowed chord, U0 = M0 c0


def airfoil_broadband(n_points=1200, n_stations=200, n_tau=4096, n_obs=72, seed=2312, dtype=np.float32) -> Case:
    contour = surfaces.joukowski_contour(n_points)
    surf = surfaces.extruded_contour(contour, n_stations, 1.0 / 9.0)
    x = surfaces.observer_circle(n_obs, 10.0, center=(0.5, 0.0, 0.0), step_deg=360.0 / n_obs)
    return Case("airfoil_broadband", surf, x, 0.17, 5.5, AIRFOIL_DTAU, n_tau, kind="broadband", seed=seed,
                data_dtype=dtype)


def by_name(name: str) -> Case:
    return {"monopole_small": monopole_small, "dipole_sphere": dipole_sphere,
            "dipole_sphere_obs8": lambda: dipole_sphere(n_obs=8),
            "airfoil_broadband": airfoil_broadband}[name]()


def batched_cases(n_cases=64, seed=4, p_range=(2048, 65536), n_range=(512, 4096), o_range=(8, 360),
                  mach_range=(0.1, 0.5), aoa_range=(0.0, 10.0), dtau=1.0 / 128.0):
    """Seeded uneven cases for the batched launch: surface kind (analytic sphere
    with a monopole or dipole, or an extruded Joukowski contour with broadband
    data), panel count log-uniform in p_range, record length uniform in
    n_range, observer count uniform in o_range, Mach number and AoA uniform.
    Spheres have n_phi = 2 n_theta; contours use about 6 points per station.
    Observers sit on a circle of radius 10 to 100 (spheres) or 10 chords
    (contours).  FP32 surface data."""
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(n_cases):
        P_target = float(np.exp(rng.uniform(np.log(p_range[0]), np.log(p_range[1]))))
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        O = int(rng.integers(o_range[0], o_range[1] + 1))
        mach = float(rng.uniform(*mach_range))
        aoa = float(rng.uniform(*aoa_range))
        kind = ["monopole", "dipole", "broadband"][int(rng.integers(0, 3))]
        if kind == "broadband":
            stations = max(4, int(round(np.sqrt(P_target / 6.0))))
            points = max(16, int(round(P_target / stations)))
            surf = surfaces.extruded_contour(surfaces.joukowski_contour(points), stations, 1.0 / 9.0)
            x = surfaces.observer_circle(O, 10.0, center=(0.5, 0.0, 0.0), start_deg=float(rng.uniform(0, 360)))
        else:
            nth = max(4, int(round(np.sqrt(P_target / 2.0))))
            surf = surfaces.sphere(1.0, nth, 2 * nth)
            x = surfaces.observer_circle(O, float(rng.uniform(10.0, 100.0)), start_deg=float(rng.uniform(0, 360)))
        cases.append(Case(f"batch{i:02d}_{kind}", surf, x, mach, aoa, dtau, N, kind=kind,
                          seed=int(seed * 1000 + i), data_dtype=np.float32))
    return cases
