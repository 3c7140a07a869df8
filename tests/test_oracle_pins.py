"""Pins of the oracle's building blocks against facts that do not come from the
oracle itself: the emission condition in the medium frame, special cases of
the paper's formulas, a library spline, a library finite difference and
brute-force window checks.  CPU only."""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import oracle

rng = np.random.default_rng(1234)


def _rand_geometry(n):
    d = rng.normal(size=(n, 3)) * rng.uniform(0.1, 50.0, size=(n, 1))
    return d


@pytest.mark.parametrize("mach,aoa", [(0.05, 0.0), (0.3, 5.0), (0.5, 10.0), (0.6, 45.0), (0.9, -20.0), (0.17, 5.5)])
def test_garrick_emission_condition(mach, aoa):
    """R solves the emission condition of a source and observer moving together
    at -U0 through a medium at rest: |d - M0 R Uhat| = R, with the radiation
    direction (d - M0 R Uhat)/R (Sec. II C, Garrick triangle)."""
    d = _rand_geometry(400)
    y = np.zeros((1, 3))
    R, Rs, Rh, MR, D = oracle.pair_geometry(y, d, mach, aoa)
    R, Rs, Rh, MR, D = R[:, 0], Rs[:, 0], Rh[:, 0], MR[:, 0], D[:, 0]
    a = math.radians(aoa)
    U = np.array([math.cos(a), math.sin(a), 0.0])
    r_vec = d - mach * R[:, None] * U[None, :]
    np.testing.assert_allclose(np.linalg.norm(r_vec, axis=1), R, rtol=1e-13)
    np.testing.assert_allclose(Rh, r_vec / R[:, None], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(Rh, axis=1), 1.0, rtol=1e-13)
    # Doppler factor: R (1 - M_R) equals R_* with M = -M0 Uhat
    np.testing.assert_allclose(R * (1.0 - MR), Rs, rtol=1e-12)
    np.testing.assert_allclose(MR, -mach * (Rh @ U), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(D, mach * R, rtol=1e-15)
    assert np.all(R > 0)


def test_zero_aoa_reduces_to_flow_along_x1():
    """With AoA = 0 the rotated forms reduce to Eqs. (R), (R_s), (R1)-(R3)."""
    d = _rand_geometry(200)
    M0 = 0.4
    R, Rs, Rh, _, _ = oracle.pair_geometry(np.zeros((1, 3)), d, M0, 0.0)
    b2 = 1 - M0 ** 2
    Rs_ref = np.sqrt(d[:, 0] ** 2 + b2 * (d[:, 1] ** 2 + d[:, 2] ** 2))
    R_ref = (-M0 * d[:, 0] + Rs_ref) / b2
    np.testing.assert_allclose(Rs[:, 0], Rs_ref, rtol=1e-13)
    np.testing.assert_allclose(R[:, 0], R_ref, rtol=1e-13)
    np.testing.assert_allclose(Rh[:, 0, 0], (-M0 * Rs_ref + d[:, 0]) / (b2 * R_ref), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Rh[:, 0, 1], d[:, 1] / R_ref, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Rh[:, 0, 2], d[:, 2] / R_ref, rtol=1e-12, atol=1e-14)


def test_geometry_rotation_covariance_and_static_limit():
    """Rotating d about x3 by theta and the AoA by theta rotates Rhat and keeps
    R; as M0 -> 0 the distance becomes |d|."""
    d = _rand_geometry(200)
    th = 0.7
    c, s = math.cos(th), math.sin(th)
    Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    R1, _, Rh1, MR1, _ = oracle.pair_geometry(np.zeros((1, 3)), d, 0.45, 3.0)
    R2, _, Rh2, MR2, _ = oracle.pair_geometry(np.zeros((1, 3)), d @ Rz.T, 0.45, 3.0 + math.degrees(th))
    np.testing.assert_allclose(R2, R1, rtol=1e-12)
    np.testing.assert_allclose(Rh2[:, 0], Rh1[:, 0] @ Rz.T, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(MR2, MR1, rtol=1e-11, atol=1e-14)
    R0, _, Rh0, _, _ = oracle.pair_geometry(np.zeros((1, 3)), d, 1e-9, 17.0)
    np.testing.assert_allclose(R0[:, 0], np.linalg.norm(d, axis=1), rtol=1e-8)


def test_source_terms_freestream_is_zero():
    """Uniform freestream (rho = 1, u = U0, p' = 0) gives Q = L = 0 (Eqs. (Qn_New_nd), (Li_New_nd))."""
    N, P = 7, 33
    aoa = 5.5
    a = math.radians(aoa)
    nrm = rng.normal(size=(P, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    rho = np.ones((N, P))
    u = np.stack([np.full((N, P), math.cos(a)), np.full((N, P), math.sin(a)), np.zeros((N, P))])
    pp = np.zeros((N, P))
    Q, L = oracle.source_terms(rho, u, pp, nrm, aoa)
    assert np.all(Q == 0.0) and np.all(L == 0.0)


def test_source_terms_match_general_moving_surface_definitions():
    """The wind-tunnel source terms equal the general permeable-surface
    definitions Eqs. (Qn), (Li) written in the medium frame, where the surface
    moves at v = -U0 and the fluid at u - U0 (rho0 = 1, P_ij = p' delta_ij)."""
    N, P = 5, 40
    aoa = -7.0
    a = math.radians(aoa)
    U = np.array([math.cos(a), math.sin(a), 0.0])
    nrm = rng.normal(size=(P, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    rho = 1 + 0.1 * rng.normal(size=(N, P))
    u = U[:, None, None] + 0.2 * rng.normal(size=(3, N, P))
    pp = 0.05 * rng.normal(size=(N, P))
    Q, L = oracle.source_terms(rho, u, pp, nrm, aoa)
    v = -U[:, None, None]
    u_med = u - U[:, None, None]
    nT = nrm.T[:, None, :]
    Q_ref = np.sum((1.0 * v + rho[None] * (u_med - v)) * nT, axis=0)
    L_ref = pp[None] * nT + rho[None] * u_med * np.sum((u_med - v) * nT, axis=0)[None]
    np.testing.assert_allclose(Q, Q_ref, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(L, L_ref, rtol=1e-12, atol=1e-14)


def test_fd_matches_library_second_order_gradient():
    """Second-order derivative with one-sided ends = numpy.gradient(edge_order=2)."""
    for N in (3, 4, 17, 200):
        f = rng.normal(size=N)
        h = 0.37
        np.testing.assert_allclose(oracle.fd(f, h), np.gradient(f, h, edge_order=2), rtol=1e-12, atol=1e-12)


def test_fd_exact_on_quadratics():
    N, h = 50, 0.01
    t = h * np.arange(N)
    f = 3.0 - 2.0 * t + 7.0 * t * t
    np.testing.assert_allclose(oracle.fd(f, h), -2.0 + 14.0 * t, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("N", [4, 5, 16, 300])
def test_spline_matches_scipy_natural(N):
    """Natural cubic spline = scipy CubicSpline(bc_type='natural'), at knots,
    inside intervals and at the ends."""
    h, tau0 = 0.013, -0.4
    f = rng.normal(size=N)
    m = oracle.spline_m(f, h)
    knots = tau0 + h * np.arange(N)
    cs = CubicSpline(knots, f, bc_type="natural")
    tau = np.concatenate([knots, tau0 + h * (N - 1) * rng.uniform(size=200)])
    np.testing.assert_allclose(oracle.spline_eval(f, m, tau0, h, tau), cs(tau), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(m, cs(knots, 2), rtol=1e-9, atol=1e-9 * np.abs(m).max())


def test_spline_reproduces_linear_data_and_clamps_ends():
    N, h = 20, 0.5
    f = 2.0 - 0.25 * np.arange(N)
    m = oracle.spline_m(f, h)
    assert np.max(np.abs(m)) < 1e-12
    tau = np.linspace(0, h * (N - 1), 77)
    np.testing.assert_allclose(oracle.spline_eval(f, m, 0.0, h, tau), 2.0 - 0.25 * tau / h, rtol=1e-13)
    # beyond the ends the interval index and t are clamped: value of the end sample
    assert oracle.spline_eval(f, m, 0.0, h, [-3.0])[0] == pytest.approx(f[0], rel=1e-15)
    assert oracle.spline_eval(f, m, 0.0, h, [h * N + 5])[0] == pytest.approx(f[-1], rel=1e-15)


def test_window_brute_force():
    """Every pair's retarded time tau_k = t_k - delay lies inside the record for
    k < N_t, and N_t is maximal (Eqs. (t_start), (t_end))."""
    y = rng.normal(size=(60, 3))
    x = rng.normal(size=(9, 3)) * 20
    M0, aoa, N, h, tau0 = 0.35, 8.0, 400, 0.02, 1.5
    st, ts, nt = oracle.window(y, x, M0, aoa, N, h, tau0)
    assert st == 0
    _, _, _, _, D = oracle.pair_geometry(y, x, M0, aoa)
    t_end_rec = tau0 + (N - 1) * h
    for o in range(x.shape[0]):
        tk = ts[o] + h * np.arange(nt[o])
        tau = tk[:, None] - D[o][None, :]
        assert tau.min() >= tau0 - 1e-12
        assert tau.max() <= t_end_rec + 1e-9 * h + 1e-12
        # one more observer sample would leave the record for the nearest panel
        tnext = ts[o] + h * nt[o] - D[o].min()
        assert tnext > t_end_rec
        assert ts[o] == pytest.approx(tau0 + D[o].max(), rel=1e-15)


def test_window_empty_is_reported():
    y = np.array([[0, 0, 0], [30.0, 0, 0]])
    x = np.array([[100.0, 0, 0]])
    st, ts, nt = oracle.window(y, x, 0.5, 0.0, 10, 0.1, 0.0)  # delay spread >> record length
    assert st == -1 and nt[0] == 0
