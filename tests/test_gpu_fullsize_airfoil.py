"""Parity at the largest workload, the stand-in for the airfoil case of
Sec. IV C: a Joukowski contour of 1200 points extruded over 200 stations
(240000 panels), 4096 source samples, 72 observers every 5 deg at 10 chords,
M0 0.17, AoA 5.5 deg, seeded broadband FP32 surface data, in the launch
configuration the benchmark times.  The FP64 oracle computes a sample of
observers one by one, among them observers 64..71, the partly filled third
32-observer tile: the forward in FP32 and BF16 coefficient storage, and the
FP32 adjoint with dJ/dp' non-zero only on three of them (an observer's
window and pairs do not depend on the other observers, so the oracle runs the
same geometry restricted to them), compared on 4096 sampled panels (the
gradient of a panel depends only on its own data and the observer windows,
which the oracle takes from the whole surface)."""
import numpy as np
import pytest

import oracle
from gpu_common import make_plan, rel_l2, valid_mask
from workloads import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SAMPLED = np.array([0, 9, 20, 35, 47, 58, 64, 67, 71])
ADJ_SAMPLED = np.array([9, 47, 67])
ADJ_PANELS = 4096
TOL_FWD = {"f32": 1e-5, "bf16": 2e-3}
TOL_ADJ = 1e-5

_state = {}


def _setup():
    import torch
    if not _state:
        c = configs.airfoil_broadband()
        print(f"\n[airfoil fullsize] {c.name}: P={c.n_panels} O={c.n_obs} N={c.n_tau}; data on the device", flush=True)
        d = c.data_device("cuda")
        torch.cuda.synchronize()
        host = [t.cpu().numpy() for t in d]
        print("[airfoil fullsize] oracle forward on observers " + str(SAMPLED.tolist()), flush=True)
        p_ref, ts, nt = oracle.forward(c.surface, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0, *host,
                                       obs_idx=SAMPLED)
        print("[airfoil fullsize] oracle forward done", flush=True)
        _state.update(case=c, dev=d, host=host, p_ref=p_ref, nt=nt)
    return _state


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_airfoil_forward_sampled(mode):
    import torch
    st = _setup()
    c = st["case"]
    plan = make_plan(c, mode)
    assert np.array_equal(plan.window.n_t, st["nt"])
    out = plan.forward(*st["dev"])
    torch.cuda.synchronize()
    p = out.double().cpu().numpy()[SAMPLED]
    ref = st["p_ref"]
    w = min(p.shape[1], ref.shape[1])
    m = valid_mask(st["nt"][SAMPLED], w)
    err = rel_l2(p[:, :w], ref[:, :w], m)
    per = [rel_l2(p[i, :w], ref[i, :w], m[i]) for i in range(len(SAMPLED))]
    print(f"    airfoil {mode} forward ({plan.info()[0]} gather, {plan.info()[1]} splits): rel L2 vs oracle on "
          f"observers {SAMPLED.tolist()} = {err:.3e}; per observer max {max(per):.3e}", flush=True)
    assert err <= TOL_FWD[mode], err
    del plan
    torch.cuda.empty_cache()


def test_airfoil_adjoint_sampled():
    import torch
    st = _setup()
    c = st["case"]
    plan = make_plan(c, "f32")
    gbar = np.zeros((c.n_obs, plan.window.n_t_max))
    w = min(gbar.shape[1], st["p_ref"].shape[1])
    rows = np.searchsorted(SAMPLED, ADJ_SAMPLED)
    gbar[ADJ_SAMPLED, :w] = 2.0 * st["p_ref"][rows, :w]
    g = plan.adjoint(*st["dev"], torch.from_numpy(gbar).float().cuda())
    torch.cuda.synchronize()
    del plan
    torch.cuda.empty_cache()
    # sampled panels: both ends of the panel order, the rest seeded uniform
    rng = np.random.default_rng(5)
    P = c.n_panels
    idx = np.unique(np.concatenate([np.arange(8), np.arange(P - 8, P),
                                    rng.choice(P, ADJ_PANELS - 16, replace=False)]))
    print(f"[airfoil fullsize] oracle adjoint, observers {ADJ_SAMPLED.tolist()}, {idx.size} panels", flush=True)
    g_ref = oracle.adjoint_panels(c.surface, c.x_obs[ADJ_SAMPLED], c.mach, c.aoa_deg, c.dtau, c.tau0, *st["host"],
                                  gbar[ADJ_SAMPLED], idx)
    print("[airfoil fullsize] oracle adjoint done", flush=True)
    it = torch.from_numpy(idx).cuda()
    for name, gv, gr in zip(("rho", "u", "p"), g, g_ref):
        gs = gv.index_select(-1, it).double().cpu().numpy()
        err = rel_l2(gs, gr, 1.0)
        print(f"    airfoil FP32 adjoint d/d{name} on {idx.size} panels: rel L2 vs oracle = {err:.3e}", flush=True)
        assert err <= TOL_ADJ, (name, err)
    del g
    _state.clear()
