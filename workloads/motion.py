"""Seeded moving-surface inputs for the general-motion form of the method
(Sec. II B): panel kinematics sampled at the source frames and closed-form
acoustic fields, nondimensional as in Sec. II D (rho0 = 1, reference speed 1,
c0 = 1/M0).  Input generation and exact reference fields only; nothing here
evaluates the FW-H integral.

Kinematics (time-major, [N][P][3]): panel centre y, unit outward normal n and
velocity v of a rigid surface whose body-frame panels (y0, n0) are carried by

    y(tau) = c(tau) + Rz(W tau) (y0 - c0_body),   n(tau) = Rz(W tau) n0,

with the centre path c(tau) of the motion kind:
  'static'     c = c0;                                   W = 0
  'translate'  c = c0 + V tau (uniform, V given);        W = 0
  'orbit'      c = c0 (fixed) and spin W about the z axis through the origin,
               i.e. the body centre c0 circles the origin (panels both
               translate and rotate: v.n != 0, dn/dtau != 0, dM/dtau != 0)
  'oscillate'  c = c0 + a sin(w_m tau) e_x and spin W about the body centre.
The velocity is the exact derivative of y(tau).

Fields:
  * quiescent monopole at x_s in still air: phi = Re[A/(4 pi r) exp(i w (t - M0 r))],
    u = grad phi, p' = -d phi / dt, rho = 1 + M0^2 p' (linear acoustics);
  * translating convected monopole: the Sec. IV A monopole (workloads.analytic,
    mean flow U0 along Uhat in the source frame) seen from the medium, in which
    source and surface move at -Uhat: p'_med(x, t) = p'_src(x + Uhat t, t),
    rho unchanged, u_med = u_src - Uhat.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import analytic, surfaces


@dataclass
class MovingSurface:
    y: np.ndarray       # [N,P,3] panel centres at the source frames
    normal: np.ndarray  # [N,P,3] unit outward normals
    vel: np.ndarray     # [N,P,3] panel velocities
    dS: np.ndarray      # [P]     panel areas (rigid panels)

    @property
    def n_panels(self) -> int:
        return int(self.dS.shape[0])

    @property
    def n_tau(self) -> int:
        return int(self.y.shape[0])


def _rz(a: np.ndarray) -> np.ndarray:
    """Rotation matrices about z, a [N] -> [N,3,3]."""
    c, s = np.cos(a), np.sin(a)
    R = np.zeros(a.shape + (3, 3))
    R[:, 0, 0] = c
    R[:, 0, 1] = -s
    R[:, 1, 0] = s
    R[:, 1, 1] = c
    R[:, 2, 2] = 1.0
    return R


def moving_surface(body: surfaces.Surface, kind: str, n_tau: int, dtau: float, tau0: float = 0.0,
                   velocity=(0.0, 0.0, 0.0), spin: float = 0.0, amplitude: float = 0.0,
                   omega_m: float = 0.0) -> MovingSurface:
    """Kinematics of the rigid body surface `body` (panel centres about its own
    centre of mass, which is taken as the body centre c0) for the motion kind."""
    tau = tau0 + dtau * np.arange(n_tau, dtype=np.float64)
    y0 = np.asarray(body.y, dtype=np.float64)
    n0 = np.asarray(body.normal, dtype=np.float64)
    c0 = np.average(y0, axis=0, weights=body.dS)
    if kind == "static":
        y = np.broadcast_to(y0, (n_tau,) + y0.shape).copy()
        n = np.broadcast_to(n0, (n_tau,) + n0.shape).copy()
        v = np.zeros_like(y)
    elif kind == "translate":
        V = np.asarray(velocity, dtype=np.float64)
        y = y0[None] + tau[:, None, None] * V[None, None, :]
        n = np.broadcast_to(n0, (n_tau,) + n0.shape).copy()
        v = np.broadcast_to(V, y.shape).copy()
    elif kind == "orbit":
        R = _rz(spin * tau)
        y = np.einsum("nij,pj->npi", R, y0)
        n = np.einsum("nij,pj->npi", R, n0)
        w = np.array([0.0, 0.0, spin])
        v = np.cross(np.broadcast_to(w, y.shape), y)
    elif kind == "oscillate":
        R = _rz(spin * tau)
        rel = np.einsum("nij,pj->npi", R, y0 - c0)
        c = c0[None, :] + np.outer(amplitude * np.sin(omega_m * tau), [1.0, 0.0, 0.0])
        cd = np.outer(amplitude * omega_m * np.cos(omega_m * tau), [1.0, 0.0, 0.0])
        y = c[:, None, :] + rel
        n = np.einsum("nij,pj->npi", R, n0)
        w = np.array([0.0, 0.0, spin])
        v = cd[:, None, :] + np.cross(np.broadcast_to(w, rel.shape), rel)
    else:
        raise ValueError(kind)
    return MovingSurface(np.ascontiguousarray(y), np.ascontiguousarray(n), np.ascontiguousarray(v),
                         np.ascontiguousarray(body.dS, dtype=np.float64))


# ---------------------------------------------------------------- fields

def quiescent_monopole_amplitudes(x: np.ndarray, mach: float, amplitude: float, omega: float,
                                  source=(0.0, 0.0, 0.0)):
    """Complex amplitudes (Phi, grad Phi, p_hat) of the still-air monopole
    Phi = A/(4 pi r) exp(-i w M0 r) at points x [...,3]."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(source, dtype=np.float64)
    r = np.linalg.norm(d, axis=-1)
    Phi = amplitude / (4.0 * math.pi * r) * np.exp(-1j * omega * mach * r)
    grad = (Phi * (-1.0 / r - 1j * omega * mach))[..., None] * d / r[..., None]
    return Phi, grad, -1j * omega * Phi


def quiescent_monopole_series(ms: MovingSurface, mach: float, amplitude: float, omega: float, dtau: float,
                              tau0: float = 0.0, source=(0.0, 0.0, 0.0)):
    """Surface data seen by the moving panels: rho [N,P], u [3,N,P], p' [N,P]."""
    tau = tau0 + dtau * np.arange(ms.n_tau, dtype=np.float64)
    _, grad, p_hat = quiescent_monopole_amplitudes(ms.y, mach, amplitude, omega, source)
    e = np.exp(1j * omega * tau)[:, None]
    pp = (p_hat * e).real
    u = np.stack([(grad[..., i] * e).real for i in range(3)], axis=0)
    rho = 1.0 + mach * mach * pp
    return np.ascontiguousarray(rho), np.ascontiguousarray(u), np.ascontiguousarray(pp)


def quiescent_monopole_pressure(x_obs: np.ndarray, mach: float, amplitude: float, omega: float, t: np.ndarray,
                                source=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Exact p'(x_o, t) of the still-air monopole, t [O,K] -> [O,K]."""
    _, _, p_hat = quiescent_monopole_amplitudes(x_obs, mach, amplitude, omega, source)
    return (p_hat[:, None] * np.exp(1j * omega * np.asarray(t))).real


def translating_convected_series(body: surfaces.Surface, flow: analytic.Flow, amplitude: float, omega: float,
                                 n_tau: int, dtau: float, tau0: float = 0.0, kind: str = "monopole"):
    """Surface and data of a body and a convected source moving together at
    -Uhat through still air (the Galilean image of the Sec. IV A/B fields):
    returns (MovingSurface, rho [N,P], u [3,N,P], p' [N,P])."""
    U = flow.U
    ms = moving_surface(body, "translate", n_tau, dtau, tau0, velocity=-U)
    rho, u, pp = analytic.surface_series(kind, body.y, flow, amplitude, omega, n_tau, dtau, tau0)
    u = u - U[:, None, None]
    return ms, rho, np.ascontiguousarray(u), pp


def translating_convected_pressure(x_obs: np.ndarray, flow: analytic.Flow, amplitude: float, omega: float,
                                   t: np.ndarray, kind: str = "monopole") -> np.ndarray:
    """Exact p' at observers at rest in the medium, t [O,K] -> [O,K]."""
    U = flow.U
    t = np.asarray(t, dtype=np.float64)
    pts = x_obs[:, None, :] + t[..., None] * U[None, None, :]
    _, p_hat = analytic.field_amplitudes(kind, pts.reshape(-1, 3), flow, amplitude, omega)
    return (p_hat.reshape(t.shape) * np.exp(1j * omega * t)).real


@dataclass
class GMCase:
    """A general-motion case: kinematics, observers, surface data."""
    name: str
    ms: MovingSurface
    x_obs: np.ndarray   # [O,3]
    mach: float
    dtau: float
    tau0: float
    rho: np.ndarray     # [N,P]
    u: np.ndarray       # [3,N,P]
    pp: np.ndarray      # [N,P]
    amplitude: float = 0.0
    omega: float = 0.0
    source: tuple = (0.0, 0.0, 0.0)

    def exact(self, t: np.ndarray) -> np.ndarray:
        """Closed-form p' of the still-air monopole at the observers, t [O,K]."""
        return quiescent_monopole_pressure(self.x_obs, self.mach, self.amplitude, self.omega, t, self.source)


def orbiting_sphere_case(n_theta: int = 64, n_phi: int = 128, n_tau: int = 1024, dtau: float = 1 / 128,
                         n_obs: int = 72, mach: float = 0.3, spin: float = 0.5, amplitude: float = 4 * math.pi * 1e-3,
                         omega: float = 2 * math.pi, obs_radius: float = 20.0, obs_height: float = 3.0) -> GMCase:
    """Sphere of radius 1.2 centred at (0.3, 0, 0) spinning at `spin` about the z
    axis through the origin (its centre circles the origin), around a still-air
    monopole at (0.05, 0.02, 0); observers on a circle of radius obs_radius at
    height obs_height.  Default size: 8192 panels, 1024 frames, 72 observers."""
    body = surfaces.sphere(1.2, n_theta, n_phi, center=(0.3, 0.0, 0.0))
    ms = moving_surface(body, "orbit", n_tau, dtau, spin=spin)
    src = (0.05, 0.02, 0.0)
    rho, u, pp = quiescent_monopole_series(ms, mach, amplitude, omega, dtau, source=src)
    x = surfaces.observer_circle(n_obs, obs_radius, start_deg=2.5)
    x[:, 2] = obs_height
    return GMCase(f"orbiting_sphere_{n_theta * n_phi}", ms, x, mach, dtau, 0.0, rho, u, pp, amplitude, omega, src)
