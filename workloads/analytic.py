"""Closed-form convected monopole and dipole fields (input generation + exact
far field), nondimensional as in Sec. II D (rho0 = U0 = 1, c0 = 1/M0).

The potentials are those of Sec. IV A (convected monopole, with the Garrick
distances of the angle-of-attack form, Eqs. (R_New) and (R_s_New)) and Sec. IV B
(dipole = derivative of the monopole potential along x2).  Velocity, pressure
and density pulsations follow the relations given there:
u' = grad(phi), p' = -(d/dt + U0 . grad) phi, rho' = p'/c0^2 = M0^2 p'.

Every field is harmonic, phi(x, t) = Re[Phi(x) exp(i w t)], so a surface
time series is the real part of a complex spatial amplitude times exp(i w tau).
Derivatives are written out analytically; tests cross-check them against
high-order finite differences.  Nothing here evaluates the FW-H integral.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Flow:
    mach: float
    aoa_deg: float

    @property
    def U(self) -> np.ndarray:
        a = math.radians(self.aoa_deg)
        return np.array([math.cos(a), math.sin(a), 0.0])


def _garrick(d: np.ndarray, flow: Flow):
    """Distances of the convected free-space Green's function for the mean flow
    M0*U: returns (R_s, R, grad R_s, grad R, Hess R_s) at separations d [...,3]."""
    M0 = flow.mach
    U = flow.U
    b2 = 1.0 - M0 * M0
    m = M0 * (d @ U)
    Rs = np.sqrt(m * m + b2 * np.sum(d * d, axis=-1))
    R = (Rs - m) / b2
    gRs = (m[..., None] * M0 * U + b2 * d) / Rs[..., None]
    gR = (gRs - M0 * U) / b2
    eye = np.eye(3)
    HRs = (M0 * M0 * np.outer(U, U) + b2 * eye - gRs[..., :, None] * gRs[..., None, :]) / Rs[..., None, None]
    return Rs, R, gRs, gR, HRs


def monopole_amplitudes(x: np.ndarray, flow: Flow, amplitude: float, omega: float,
                        source=(0.0, 0.0, 0.0), order: int = 1):
    """Complex amplitude Phi of the convected monopole potential
    Phi = A/(4 pi R_s) exp(-i w M0 R) at points x [...,3], its gradient and
    (order >= 2) its Hessian."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(source, dtype=np.float64)
    M0 = flow.mach
    b2 = 1.0 - M0 * M0
    Rs, R, gRs, gR, HRs = _garrick(d, flow)
    Phi = amplitude / (4.0 * math.pi * Rs) * np.exp(-1j * omega * M0 * R)
    G = -gRs / Rs[..., None] - 1j * omega * M0 * gR
    grad = Phi[..., None] * G
    if order < 2:
        return Phi, grad, None
    dG = (-HRs / Rs[..., None, None] + gRs[..., :, None] * gRs[..., None, :] / (Rs * Rs)[..., None, None]
          - 1j * omega * M0 * HRs / b2)
    hess = Phi[..., None, None] * (G[..., :, None] * G[..., None, :] + dG)
    return Phi, grad, hess


def field_amplitudes(kind: str, x: np.ndarray, flow: Flow, amplitude: float, omega: float,
                     source=(0.0, 0.0, 0.0)):
    """Complex amplitudes (u_hat [...,3], p_hat [...]) of the velocity and
    pressure pulsation of a 'monopole' or 'dipole' (axis x2) source."""
    U = flow.U
    if kind == "monopole":
        Phi, grad, _ = monopole_amplitudes(x, flow, amplitude, omega, source, order=1)
        phi, gphi = Phi, grad
    elif kind == "dipole":
        Phi, grad, hess = monopole_amplitudes(x, flow, amplitude, omega, source, order=2)
        phi = grad[..., 1]
        gphi = hess[..., :, 1]
    else:
        raise ValueError(kind)
    p_hat = -(1j * omega * phi + gphi @ U)
    return gphi, p_hat


def surface_series(kind: str, y: np.ndarray, flow: Flow, amplitude: float, omega: float,
                   n_tau: int, dtau: float, tau0: float = 0.0, source=(0.0, 0.0, 0.0),
                   dtype=np.float64):
    """Surface data of the analytic field at panel centres y [P,3] and source
    times tau_n = tau0 + n*dtau, time-major: rho [N,P], u [3,N,P], p' [N,P].

    rho and u are full values (rho = 1 + rho', u = U0 + u'); the pressure is the
    pulsation p' (reading of Sec. II C: 'density, velocity, and pressure
    pulsation')."""
    u_hat, p_hat = field_amplitudes(kind, y, flow, amplitude, omega, source)
    tau = tau0 + dtau * np.arange(n_tau, dtype=np.float64)
    c = np.cos(omega * tau)[:, None]
    s = np.sin(omega * tau)[:, None]

    def re(a):  # Re(a exp(i w tau)) as [N, P]
        return a.real[None, :] * c - a.imag[None, :] * s

    pp = re(p_hat)
    rho = 1.0 + flow.mach ** 2 * pp
    U = flow.U
    u = np.stack([U[i] + re(u_hat[:, i]) for i in range(3)], axis=0)
    return (np.ascontiguousarray(rho, dtype=dtype), np.ascontiguousarray(u, dtype=dtype),
            np.ascontiguousarray(pp, dtype=dtype))


def surface_series_torch(kind: str, y: np.ndarray, flow: Flow, amplitude: float, omega: float,
                         n_tau: int, dtau: float, tau0: float = 0.0, source=(0.0, 0.0, 0.0),
                         dtype=np.float64, device="cuda"):
    """surface_series built on a torch device: the spatial amplitudes and the
    time factors come from the host (numpy, as above), the [N, P] products are
    formed on the device with the same separately rounded FP64 operations, so
    the values equal surface_series bit for bit."""
    import torch
    u_hat, p_hat = field_amplitudes(kind, y, flow, amplitude, omega, source)
    tau = tau0 + dtau * np.arange(n_tau, dtype=np.float64)
    c = torch.from_numpy(np.cos(omega * tau)).to(device)[:, None]
    s = torch.from_numpy(np.sin(omega * tau)).to(device)[:, None]
    tdt = {np.float64: torch.float64, np.float32: torch.float32}[np.dtype(dtype).type]

    def re(a):  # Re(a exp(i w tau)) as [N, P], FP64
        ar = torch.from_numpy(np.ascontiguousarray(a.real)).to(device)[None, :]
        ai = torch.from_numpy(np.ascontiguousarray(a.imag)).to(device)[None, :]
        return torch.sub(torch.mul(ar, c), torch.mul(ai, s))

    pp = re(p_hat)
    rho = torch.add(torch.mul(pp, flow.mach ** 2), 1.0).to(tdt)
    U = flow.U
    u = torch.empty((3, n_tau, y.shape[0]), dtype=tdt, device=device)
    for i in range(3):
        u[i] = torch.add(re(u_hat[:, i]), float(U[i])).to(tdt)
    return rho.contiguous(), u, pp.to(tdt).contiguous()


def far_field_pressure(kind: str, x_obs: np.ndarray, flow: Flow, amplitude: float, omega: float,
                       t: np.ndarray, source=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Exact pressure pulsation p'(x_o, t) of the analytic field at observers
    x_obs [O,3] and times t [O,K] (or [K]); returns [O,K]."""
    _, p_hat = field_amplitudes(kind, x_obs, flow, amplitude, omega, source)
    t = np.asarray(t, dtype=np.float64)
    if t.ndim == 1:
        t = np.broadcast_to(t[None, :], (x_obs.shape[0], t.shape[0]))
    return (p_hat[:, None] * np.exp(1j * omega * t)).real
