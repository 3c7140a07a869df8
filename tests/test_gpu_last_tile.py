"""The LDS-staged forward gather runs a last tile of at most 16 observers in a
second launch with the 2 x 8 wave shape, after the launch of the full tiles.
A 40-observer case (one full tile of 32 and a last tile of 8) against the FP64
oracle in both storage modes, repeat runs bit for bit, and the single-case
forward recorded in a HIP graph: every replay, with the program's own eager
work between replays, equal to the eager result."""
import numpy as np
import pytest

from gpu_common import make_plan, oracle_forward, rel_l2, to_device, valid_mask
from workloads import configs, surfaces

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-3}
_cache = {}


def _case():
    surf = surfaces.sphere(1.0, 16, 32)
    return configs.Case("tail40", surf, surfaces.observer_circle(40, 30.0, step_deg=9.0), 0.4, 8.0, 1.0 / 64.0,
                        700, kind="dipole", omega=2.0)


def _data():
    if "d" not in _cache:
        c = _case()
        rho, u, pp = c.data()
        p_ref, _, nt_ref = oracle_forward(c, rho, u, pp)
        _cache["d"] = (c, rho, u, pp, p_ref, nt_ref)
    return _cache["d"]


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_last_tile_launch_matches_oracle(mode):
    import torch
    c, rho, u, pp, p_ref, nt_ref = _data()
    plan = make_plan(c, mode, gather="lds")
    assert plan.info()[0] == "lds"
    d = to_device((rho, u, pp))
    p1 = plan.forward(*d)
    p2 = plan.forward(*d)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2), "repeat forward differs"
    p = p1.double().cpu().numpy()
    err = rel_l2(p, p_ref, valid_mask(nt_ref, p.shape[1]))
    # the last tile's 8 observers alone
    err_tail = rel_l2(p[32:], p_ref[32:], valid_mask(nt_ref[32:], p.shape[1]))
    print(f"    tail40 {mode}: rel L2 vs oracle = {err:.3e} (last tile {err_tail:.3e})", flush=True)
    assert err <= TOL[mode], err
    assert err_tail <= TOL[mode], err_tail


def test_single_case_forward_graph_replays():
    import torch
    c, rho, u, pp, _, _ = _data()
    plan = make_plan(c, "f32", gather="lds")
    d = to_device((rho, u, pp))
    out = torch.empty((c.n_obs, plan.window.n_t_max), dtype=torch.float32, device="cuda")
    plan.forward(*d, out=out)
    torch.cuda.synchronize()
    ref = out.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.forward(*d, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.forward(*d, out=out)
    for rep in range(3):
        out.fill_(float("nan"))  # the program's own eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep} differs from the eager forward"
        print(f"    replay {rep} matches the eager forward", flush=True)
