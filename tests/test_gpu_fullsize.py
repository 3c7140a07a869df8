"""Parity at the full benchmark size (convected dipole, 32768-panel sphere,
2048 samples, 360 observers), in the launch configuration the benchmark times,
on sampled outputs the FP64 oracle computes one by one: a few observers for
the forward; for the adjoint, dJ/dp' non-zero only on those observers, where
the oracle runs the same geometry restricted to them (an observer's window and
pairs do not depend on the other observers)."""
import numpy as np
import pytest

import oracle
from gpu_common import make_plan, rel_l2, to_device, valid_mask
from workloads import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SAMPLED = np.array([0, 97, 180, 271, 359])
TOL_FWD = {"f64": 1e-11, "f32": 1e-5, "bf16": 2e-3}
TOL_ADJ = {"f64": 1e-11, "f32": 1e-5}

_state = {}


def _setup():
    if not _state:
        c = configs.dipole_sphere()
        print(f"[fullsize] generating {c.name}: P={c.n_panels} O={c.n_obs} N={c.n_tau}", flush=True)
        rho, u, pp = c.data()
        p_ref, ts, nt = oracle.forward(c.surface, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0, rho, u, pp,
                                       obs_idx=SAMPLED)
        _state.update(case=c, data=(rho, u, pp), p_ref=p_ref, nt=nt)
        print("[fullsize] oracle forward on sampled observers done", flush=True)
    return _state


@pytest.mark.parametrize("mode", ["f32", "bf16", "f64"])
def test_fullsize_forward_sampled(mode):
    import torch
    st = _setup()
    c = st["case"]
    print(f"[fullsize forward] mode={mode}", flush=True)
    plan = make_plan(c, mode)
    assert np.array_equal(plan.window.n_t, st["nt"])
    d = to_device(st["data"])
    out = plan.forward(*d)
    torch.cuda.synchronize()
    p = out.double().cpu().numpy()[SAMPLED]
    ref = st["p_ref"]
    w = min(p.shape[1], ref.shape[1])
    m = valid_mask(st["nt"][SAMPLED], w)
    err = rel_l2(p[:, :w], ref[:, :w], m)
    print(f"    rel L2 vs oracle on observers {SAMPLED.tolist()} = {err:.3e}", flush=True)
    assert err <= TOL_FWD[mode], err


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_fullsize_adjoint_sampled(mode):
    import torch
    st = _setup()
    c = st["case"]
    rho, u, pp = st["data"]
    print(f"[fullsize adjoint] mode={mode}", flush=True)
    plan = make_plan(c, mode)
    gbar = np.zeros((c.n_obs, plan.window.n_t_max))
    w = min(gbar.shape[1], st["p_ref"].shape[1])
    gbar[SAMPLED, :w] = 2.0 * st["p_ref"][:, :w]
    d = to_device((rho, u, pp))
    g = plan.adjoint(*d, torch.from_numpy(gbar).to(plan.out_dtype).cuda())
    torch.cuda.synchronize()
    g_ref = oracle.adjoint(c.surface, c.x_obs[SAMPLED], c.mach, c.aoa_deg, c.dtau, c.tau0, rho, u, pp,
                           gbar[SAMPLED])
    for name, gv, gr in zip(("rho", "u", "p"), g, g_ref):
        err = rel_l2(gv.double().cpu().numpy(), gr)
        print(f"    d/d{name}: rel L2 vs oracle = {err:.3e}", flush=True)
        assert err <= TOL_ADJ[mode], (name, err)
