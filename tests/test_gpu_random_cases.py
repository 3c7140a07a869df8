"""Seeded random sweep of the wind-tunnel path against the FP64 oracle: panel,
observer and sample counts that fall on and between the tile sizes (32-panel
source chunks, 32-observer tiles, 61-sample sub-rows, 244-sample blocks),
random Mach numbers, angles of attack, tau0, observer distances (delay spreads
from a few samples to hundreds) and surfaces (spheres, extruded contours,
random panel subsets).  Forward in the three forms and the FP32 adjoint, with
the tolerances of the parity tests."""
import numpy as np
import pytest

from gpu_common import make_plan, oracle_adjoint, oracle_forward, rel_l2, to_device, valid_mask
from workloads import configs, surfaces

pytestmark = pytest.mark.gpu

TOL_FWD = {"f64": 1e-11, "f32": 1e-5, "bf16": 2e-3}
N_CASES = 10


def _random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    kind = ["sphere", "contour", "subset"][seed % 3]
    if kind == "sphere":
        nt = int(rng.integers(2, 14))
        surf = surfaces.sphere(float(rng.uniform(0.5, 1.5)), nt, 2 * nt)
    elif kind == "contour":
        surf = surfaces.extruded_contour(surfaces.joukowski_contour(int(rng.integers(20, 120))),
                                         int(rng.integers(1, 6)), float(rng.uniform(0.05, 0.3)))
    else:
        full = surfaces.sphere(1.0, 12, 24)
        idx = np.sort(rng.choice(full.n_panels, size=int(rng.integers(1, full.n_panels)), replace=False))
        surf = full.subset(idx)
    O = int(rng.choice([1, 7, 31, 32, 33, 40, 65]))
    R = float(rng.uniform(3.0, 60.0))
    x = rng.normal(size=(O, 3))
    x *= (R / np.linalg.norm(x, axis=1))[:, None]
    mach = float(rng.uniform(0.05, 0.6))
    aoa = float(rng.uniform(-30.0, 30.0))
    n_tau = int(rng.choice([4, 61, 62, 244, 245, 300, 489]))
    # a record long enough for every observer's window: delay spread <= 2 M0 (diameter) / (1 - M0)
    dtau = float(rng.uniform(0.01, 0.2))
    n_tau = max(n_tau, int(4.0 * mach / (1.0 - mach) / dtau) + 8)
    tau0 = float(rng.uniform(-2.0, 2.0))
    dk = ["monopole", "dipole"][seed % 2]
    return configs.Case(f"rand{seed}", surf, x, mach, aoa, dtau, n_tau, tau0=tau0, kind=dk,
                        omega=float(rng.uniform(1.0, 8.0)))


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_case(seed):
    import torch
    c = _random_case(seed)
    print(f"[random case] seed={seed} P={c.n_panels} O={c.n_obs} N={c.n_tau} M0={c.mach:.3f} "
          f"AoA={c.aoa_deg:.1f} dtau={c.dtau:.3f} tau0={c.tau0:.2f}", flush=True)
    rho, u, pp = c.data()
    p_ref, ts_ref, nt_ref = oracle_forward(c, rho, u, pp)
    m = valid_mask(nt_ref, p_ref.shape[1])
    for mode in ("f64", "f32", "bf16"):
        plan = make_plan(c, mode)
        assert np.array_equal(plan.window.n_t, nt_ref)
        p = plan.forward(*to_device((rho, u, pp))).double().cpu().numpy()
        assert np.all(p[m == 0] == 0.0)
        err = rel_l2(p, p_ref, m)
        print(f"    {mode}: rel L2 {err:.2e}", flush=True)
        assert err <= TOL_FWD[mode], (mode, err)
    plan = make_plan(c, "f32")
    gbar = 2.0 * p_ref
    g_ref = oracle_adjoint(c, rho, u, pp, gbar)
    g = plan.adjoint(*to_device((rho, u, pp)), torch.from_numpy(gbar).float().cuda())
    torch.cuda.synchronize()
    for gv, gr in zip(g, g_ref):
        err = rel_l2(gv.double().cpu().numpy(), gr)
        assert err <= 1e-5, err
