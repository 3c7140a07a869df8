"""Seeded synthetic FW-H surfaces and observer arrays (input generation only).

A surface is a set of panels, each given by its centre y [P,3], unit outward
normal n [P,3] and area dS [P] -- the geometric inputs the method asks the CFD
solver for (Sec. II C, last paragraph).  Nothing here evaluates the FW-H
integral; these arrays are consumed both by the FP64 oracle and by the GPU path.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Surface:
    y: np.ndarray       # [P,3] panel centres
    normal: np.ndarray  # [P,3] unit outward normals
    dS: np.ndarray      # [P]   panel areas

    @property
    def n_panels(self) -> int:
        return int(self.y.shape[0])

    def subset(self, idx) -> "Surface":
        return Surface(self.y[idx].copy(), self.normal[idx].copy(), self.dS[idx].copy())


def sphere(radius: float, n_theta: int, n_phi: int, center=(0.0, 0.0, 0.0)) -> Surface:
    """Latitude-longitude sphere, polar axis x3 (the monopole/dipole validation
    surface of Sec. IV A is an 18 x 36 sphere of this kind).

    Panel (i, j) spans theta in [i, i+1]*dtheta, phi in [j, j+1]*dphi.  The centre
    is the surface point at the mid angles, the normal is radial there and dS is
    the exact area of the spherical patch r^2 (cos th_i - cos th_{i+1}) dphi.
    Panels are ordered theta-major (index i*n_phi + j).
    """
    dth = math.pi / n_theta
    dph = 2.0 * math.pi / n_phi
    i = np.arange(n_theta, dtype=np.float64)
    j = np.arange(n_phi, dtype=np.float64)
    th = (i + 0.5) * dth
    ph = (j + 0.5) * dph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    nrm = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=-1).reshape(-1, 3)
    area_row = radius * radius * (np.cos(i * dth) - np.cos((i + 1) * dth)) * dph
    dS = np.repeat(area_row, n_phi)
    y = radius * nrm + np.asarray(center, dtype=np.float64)[None, :]
    return Surface(np.ascontiguousarray(y), np.ascontiguousarray(nrm), np.ascontiguousarray(dS))


def joukowski_contour(n_points: int, center=(-0.08, 0.04), chord: float = 1.0):
    """Closed Joukowski profile z = zeta + 1/zeta of the circle through zeta = 1
    with the given centre, sampled at n_points angles uniformly, then shifted so
    the leading edge is at x = 0 and scaled to the requested chord.

    Returns the contour vertices [n_points, 2], ordered counter-clockwise.
    """
    c = complex(center[0], center[1])
    a = abs(1.0 - c)
    th0 = math.atan2(-c.imag, 1.0 - c.real)  # angle of the trailing-edge point zeta = 1
    th = th0 + 2.0 * math.pi * np.arange(n_points) / n_points
    zeta = c + a * np.exp(1j * th)
    z = zeta + 1.0 / zeta
    x = z.real
    yv = z.imag
    span_x = x.max() - x.min()
    x = (x - x.min()) / span_x * chord
    yv = yv / span_x * chord
    pts = np.stack([x, yv], axis=-1)
    # enforce counter-clockwise order (positive signed area)
    area = 0.5 * np.sum(pts[:, 0] * np.roll(pts[:, 1], -1) - np.roll(pts[:, 0], -1) * pts[:, 1])
    if area < 0:
        pts = pts[::-1].copy()
    return pts


def extruded_contour(contour: np.ndarray, n_stations: int, span: float) -> Surface:
    """Extrude a closed counter-clockwise 2-D contour (x1, x2) along x3.

    Panels are the contour edges times spanwise strips: centre at the edge
    midpoint and strip centre, outward normal = edge tangent rotated by -90 deg
    (outward for a counter-clockwise contour), dS = edge length * span/n_stations.
    Panels are ordered station-major (station s, edge e -> s*E + e).  There are
    no end caps, as for the airfoil surface of Sec. IV C.
    """
    p0 = contour
    p1 = np.roll(contour, -1, axis=0)
    mid = 0.5 * (p0 + p1)
    t = p1 - p0
    length = np.hypot(t[:, 0], t[:, 1])
    n2 = np.stack([t[:, 1], -t[:, 0]], axis=-1) / length[:, None]
    dz = span / n_stations
    zc = (np.arange(n_stations) + 0.5) * dz - 0.5 * span
    E = contour.shape[0]
    y = np.empty((n_stations, E, 3))
    y[:, :, 0] = mid[None, :, 0]
    y[:, :, 1] = mid[None, :, 1]
    y[:, :, 2] = zc[:, None]
    nrm = np.zeros((n_stations, E, 3))
    nrm[:, :, 0] = n2[None, :, 0]
    nrm[:, :, 1] = n2[None, :, 1]
    dS = np.broadcast_to(length[None, :] * dz, (n_stations, E))
    return Surface(np.ascontiguousarray(y.reshape(-1, 3)), np.ascontiguousarray(nrm.reshape(-1, 3)),
                   np.ascontiguousarray(dS.reshape(-1)).copy())


def observer_circle(n_obs: int, radius: float, center=(0.0, 0.0, 0.0), start_deg: float = 0.0,
                    step_deg: float | None = None) -> np.ndarray:
    """Observers on a circle in the x1-x2 plane (Sec. IV A/B place them on such a
    circle around the source).  Angle of observer i: start + i*step degrees;
    step defaults to 360/n_obs."""
    if step_deg is None:
        step_deg = 360.0 / n_obs
    ang = np.deg2rad(start_deg + step_deg * np.arange(n_obs))
    x = np.stack([radius * np.cos(ang), radius * np.sin(ang), np.zeros(n_obs)], axis=-1)
    return np.ascontiguousarray(x + np.asarray(center, dtype=np.float64)[None, :])
