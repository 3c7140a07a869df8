"""Parity at the largest workload, the stand-in for the airfoil case of
Sec. IV C: a Joukowski contour of 1200 points extruded over 200 stations
(240000 panels), 4096 source samples, 72 observers every 5 deg at 10 chords,
M0 0.17, AoA 5.5 deg, seeded broadband FP32 surface data, in the launch
configuration the benchmark times.  The FP64 oracle computes a sample of
observers one by one, among them observers 64..71, the partly filled third
32-observer tile: the forward in FP32 and BF16 coefficient storage, and the
FP32 adjoint with dJ/dp' non-zero only on three of them (an observer's
window and pairs do not depend on the other observers, so the oracle runs the
same geometry restricted to them)."""
import numpy as np
import pytest

import oracle
from gpu_common import make_plan, rel_l2, valid_mask
from workloads import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SAMPLED = np.array([0, 9, 20, 35, 47, 58, 64, 67, 71])
ADJ_SAMPLED = np.array([9, 67])   # the oracle adjoint takes about a minute per observer here
TOL_FWD = {"f32": 1e-5, "bf16": 2e-3}
TOL_ADJ = 1e-5

_state = {}


def _rel_l2_rows(t, ref, rows=256):
    """rel_l2 of a device tensor against a host array of the same shape, a few
    rows at a time (the full-size gradients are 8-24 GB in FP64)."""
    t = t.reshape(-1, t.shape[-1])
    ref = ref.reshape(-1, ref.shape[-1])
    num = den = 0.0
    for r in range(0, t.shape[0], rows):
        a = t[r:r + rows].double().cpu().numpy()
        b = ref[r:r + rows]
        num += float(np.sum((a - b) ** 2))
        den += float(np.sum(b * b))
    return (num / den) ** 0.5 if den > 0 else num ** 0.5


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
    # the adjoint is linear in dJ/dp': the oracle's gradient is the sum of one call per observer
    g_ref = None
    for o in ADJ_SAMPLED:
        print(f"[airfoil fullsize] oracle adjoint, observer {o}", flush=True)
        g1 = oracle.adjoint(c.surface, c.x_obs[[o]], c.mach, c.aoa_deg, c.dtau, c.tau0, *st["host"], gbar[[o]])
        g_ref = list(g1) if g_ref is None else [a + b for a, b in zip(g_ref, g1)]
        del g1
    print("[airfoil fullsize] oracle adjoint done", flush=True)
    for name, gv, gr in zip(("rho", "u", "p"), g, g_ref):
        err = _rel_l2_rows(gv, gr)
        print(f"    airfoil FP32 adjoint d/d{name}: rel L2 vs oracle = {err:.3e}", flush=True)
        assert err <= TOL_ADJ, (name, err)
    _state.clear()
