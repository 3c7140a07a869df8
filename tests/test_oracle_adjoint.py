"""Pins of the oracle's adjoint (not in the paper: the transpose of its forward
map, used for the gradient of J = sum p'^2): the dot-product identity of the
linear part and central finite differences of J through the full nonlinear
chain.  Also checks the analytic input generator (its derivatives and the
convected wave equation).  CPU only."""
import math

import numpy as np
import pytest

import oracle
from workloads import analytic, surfaces


def _case(seed, P_theta=5, N=48):
    rng = np.random.default_rng(seed)
    s = surfaces.sphere(1.0, P_theta, 2 * P_theta, center=(0.05, -0.1, 0.2))
    x = np.array([[7.0, 2.0, 0.5], [-5.0, 4.0, -1.0], [1.0, -9.0, 2.0]])
    return rng, s, x


def test_adjoint_dot_product_identity():
    """<A x, y> = <x, A^T y> for the map from source terms (Q, L) to p'."""
    rng, s, x = _case(3)
    N, P = 48, s.n_panels
    M0, aoa, h, tau0 = 0.45, 17.0, 0.05, -0.2
    Q, L = rng.normal(size=(N, P)), rng.normal(size=(3, N, P))
    p, ts, nt = oracle.forward_sources(s, x, M0, aoa, h, tau0, Q, L)
    g = rng.normal(size=p.shape)
    g[np.arange(p.shape[1])[None, :] >= nt[:, None]] = 0.0
    Qb, Lb = oracle.adjoint_sources(s, x, M0, aoa, h, tau0, N, g)
    lhs = np.sum(p * g)
    rhs = np.sum(Q * Qb) + np.sum(L * Lb)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.sqrt(np.sum(p * p) * np.sum(g * g)))


def test_adjoint_ignores_padding():
    rng, s, x = _case(4)
    N, P = 40, s.n_panels
    args = (s, x, 0.3, 5.0, 0.05, 0.0)
    Q, L = rng.normal(size=(N, P)), rng.normal(size=(3, N, P))
    p, ts, nt = oracle.forward_sources(*args, Q, L, nt_stride=None)
    g = rng.normal(size=(x.shape[0], p.shape[1] + 5))
    Qb1, Lb1 = oracle.adjoint_sources(*args, N, g)
    g2 = g.copy()
    for o in range(x.shape[0]):
        g2[o, nt[o]:] = 1e30
    Qb2, Lb2 = oracle.adjoint_sources(*args, N, g2)
    assert np.array_equal(Qb1, Qb2) and np.array_equal(Lb1, Lb2)


def test_adjoint_gradient_central_fd():
    """dJ/d(rho, u, p') of J = sum_{o,k} p'(o,k)^2 against central finite
    differences on seeded random entries, through the nonlinear source terms."""
    rng, s, x = _case(5)
    N, P = 48, s.n_panels
    M0, aoa, h, tau0 = 0.5, 10.0, 0.05, 0.0
    a = math.radians(aoa)
    U = np.array([math.cos(a), math.sin(a), 0])
    rho = 1 + 0.05 * rng.normal(size=(N, P))
    u = U[:, None, None] + 0.05 * rng.normal(size=(3, N, P))
    pp = 0.05 * rng.normal(size=(N, P))
    geo = (s, x, M0, aoa, h, tau0)
    p, ts, nt = oracle.forward(*geo, rho, u, pp)
    g_r, g_u, g_p = oracle.adjoint(*geo, rho, u, pp, 2 * p)
    arrays = {"rho": rho, "u": u, "p": pp}
    grads = {"rho": g_r, "u": g_u, "p": g_p}
    for trial in range(24):
        var = ["rho", "u", "p"][trial % 3]
        arr = arrays[var]
        idx = tuple(int(rng.integers(0, d)) for d in arr.shape)
        eps = 1e-6 * max(1.0, abs(arr[idx]))
        plus = {k: v.copy() for k, v in arrays.items()}
        minus = {k: v.copy() for k, v in arrays.items()}
        plus[var][idx] += eps
        minus[var][idx] -= eps
        pa, _, _ = oracle.forward(*geo, plus["rho"], plus["u"], plus["p"])
        pb, _, _ = oracle.forward(*geo, minus["rho"], minus["u"], minus["p"])
        dJ = np.sum((pa - pb) * (pa + pb)) / (2 * eps)   # (J+ - J-)/(2 eps) without cancellation against J
        ref = grads[var][idx]
        scale = np.max(np.abs(grads[var]))
        assert abs(dJ - ref) <= 1e-6 * scale + 1e-7 * abs(ref), (var, idx, dJ, ref)


@pytest.mark.parametrize("kind", ["monopole", "dipole"])
def test_analytic_generator_derivatives_and_wave_equation(kind):
    """The closed-form velocity is the gradient of the potential, and the
    potential satisfies the convected wave equation
    M0^2 (i w + U0.grad)^2 Phi = lap Phi away from the source."""
    fl = analytic.Flow(0.45, 23.0)
    w, A = 2 * math.pi * 0.8, 1.0
    rng = np.random.default_rng(9)
    pts = rng.normal(size=(20, 3))
    pts *= (1.5 + 2 * rng.uniform(size=(20, 1))) / np.linalg.norm(pts, axis=1, keepdims=True)
    eps = 1e-3

    def phi(xx):
        Phi, grad, _ = analytic.monopole_amplitudes(xx, fl, A, w, order=1)
        return Phi if kind == "monopole" else grad[..., 1]

    c8 = np.array([1 / 280, -4 / 105, 1 / 5, -4 / 5, 0, 4 / 5, -1 / 5, 4 / 105, -1 / 280])
    offs = np.arange(-4, 5)
    grad_fd = np.zeros((20, 3), dtype=complex)
    lap = np.zeros(20, dtype=complex)
    e = np.eye(3)
    for i in range(3):
        vals = np.stack([phi(pts + o * eps * e[i]) for o in offs])
        grad_fd[:, i] = np.tensordot(c8, vals, axes=1) / eps
    u_hat, p_hat = analytic.field_amplitudes(kind, pts, fl, A, w)
    np.testing.assert_allclose(u_hat, grad_fd, rtol=1e-9, atol=1e-12)
    # Laplacian and the convective second derivative with 8th-order stencils
    d2 = np.array([-1 / 560, 8 / 315, -1 / 5, 8 / 5, -205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560])
    for i in range(3):
        vals = np.stack([phi(pts + o * eps * e[i]) for o in offs])
        lap += np.tensordot(d2, vals, axes=1) / eps ** 2
    U = fl.U
    valsU = np.stack([phi(pts + o * eps * U[None, :]) for o in offs])
    dUU = np.tensordot(d2, valsU, axes=1) / eps ** 2
    dU = np.tensordot(c8, valsU, axes=1) / eps
    ph = phi(pts)
    lhs = fl.mach ** 2 * (-(w ** 2) * ph + 2j * w * dU + dUU)
    np.testing.assert_allclose(lhs, lap, rtol=1e-5, atol=1e-7 * np.abs(lap).max())
    # p' = -(d/dt + U0.grad) phi
    np.testing.assert_allclose(p_hat, -(1j * w * ph + dU), rtol=1e-9, atol=1e-12)


def test_adjoint_panel_subset_matches_full():
    """adjoint_panels on a subset (unsorted, with a repeat) returns exactly the
    columns of the full adjoint: the windows come from the whole surface."""
    rng, s, x = _case(6)
    N, P = 40, s.n_panels
    args = (s, x, 0.4, 8.0, 0.05, 0.1)
    rho = 1 + 0.05 * rng.normal(size=(N, P))
    u = 0.1 * rng.normal(size=(3, N, P))
    pp = 0.01 * rng.normal(size=(N, P))
    p, ts, nt = oracle.forward(*args, rho, u, pp)
    g = 2.0 * p
    full = oracle.adjoint(*args, rho, u, pp, g)
    idx = np.array([P - 1, 0, 7, 7, 3 * P // 5])
    sub = oracle.adjoint_panels(*args, rho, u, pp, g, idx)
    for f, s_ in zip(full, sub):
        assert np.array_equal(f[..., idx], s_)
    with pytest.raises(ValueError):
        oracle.adjoint_panels(*args, rho, u, pp, g, np.array([P]))
