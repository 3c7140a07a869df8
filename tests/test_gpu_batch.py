"""The batched launch (many uneven cases; persistent forward gather over a
longest-first work list; forward + dJ/dp' + adjoint captured in one HIP graph)
against the FP64 oracle, against single-case launches, and graph replays
against the eager result."""
import numpy as np
import pytest

import oracle
from gpu_common import make_plan, rel_l2, to_device, valid_mask
from workloads import configs

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-3}


def _small_cases():
    return configs.batched_cases(n_cases=6, seed=11, p_range=(200, 3000), n_range=(160, 600), o_range=(3, 70),
                                 dtau=1.0 / 64.0)


_data = {}


def _case_data(cases):
    key = id(cases)
    if key not in _data:
        out = []
        for c in cases:
            rho, u, pp = c.data()
            p_ref, ts, nt = oracle.forward(c.surface, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0, rho, u, pp)
            out.append((rho, u, pp, p_ref, nt))
        _data[key] = out
    return _data[key]


CASES = _small_cases()


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_batch_forward_adjoint_vs_oracle_and_single(mode):
    import torch

    import paper_2312_16263_amd as fwh
    data = _case_data(CASES)
    print(f"[batch] mode={mode} cases=" + ", ".join(f"{c.n_panels}x{c.n_obs}x{c.n_tau}" for c in CASES), flush=True)
    plans = [make_plan(c, mode) for c in CASES]
    inputs = [to_device(d[:3]) for d in data]
    batch = fwh.Batch(plans, inputs, item_units=2e5)
    info = batch.info()
    print(f"    items={info['items']} grid={info['grid']} units={info['units']:.3e}", flush=True)
    p_b = [t.clone() for t in batch.forward()]
    for i, (c, d) in enumerate(zip(CASES, data)):
        p_ref, nt = d[3], d[4]
        m = valid_mask(nt, p_ref.shape[1])
        err = rel_l2(p_b[i].double().cpu().numpy(), p_ref, m)
        single = plans[i].forward(*inputs[i])
        err_s = rel_l2(p_b[i].double().cpu().numpy(), single.double().cpu().numpy(), m)
        print(f"    case {i} {c.name}: rel L2 vs oracle {err:.3e}, vs single-case launch {err_s:.3e}", flush=True)
        assert err <= TOL[mode], err
        assert err_s <= 1e-6, err_s
        assert np.all(p_b[i].cpu().numpy()[m == 0] == 0.0)
    # adjoint: identical kernels per case, so bitwise equal to single-case launches
    for po, gp in zip(batch.p_out, batch.grad_p):
        torch.mul(po, 2.0, out=gp)
    g_b = [tuple(x.clone() for x in g) for g in batch.adjoint()]
    torch.cuda.synchronize()
    for i in range(len(CASES)):
        g_s = plans[i].adjoint(*inputs[i], batch.grad_p[i])
        for a, b in zip(g_b[i], g_s):
            assert torch.equal(a, b)
    # and the gradient against the oracle's
    for i, (c, d) in enumerate(zip(CASES, data)):
        gbar = batch.grad_p[i].double().cpu().numpy()
        g_ref = oracle.adjoint(c.surface, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0, *[a.astype(np.float64) for a in d[:3]],
                               gbar)
        for gv, gr in zip(g_b[i], g_ref):
            err = rel_l2(gv.double().cpu().numpy(), gr)
            assert err <= 1e-5, (i, err)


def test_batch_graph_replays_match_eager():
    import torch

    import paper_2312_16263_amd as fwh
    data = _case_data(CASES)
    plans = [make_plan(c, "bf16") for c in CASES]
    inputs = [to_device(d[:3]) for d in data]
    batch = fwh.Batch(plans, inputs, item_units=2e5)
    batch.step()
    torch.cuda.synchronize()
    ref_p = [t.clone() for t in batch.p_out]
    ref_g = [tuple(x.clone() for x in g) for g in batch.grads]
    graph = batch.capture()
    for rep in range(3):
        # the program's own eager work between replays
        for t in batch.p_out:
            t.fill_(float("nan"))
        for g in batch.grads:
            for x in g:
                x.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(batch.p_out, ref_p):
            assert torch.equal(a, b), f"replay {rep}: forward differs"
        for g, r in zip(batch.grads, ref_g):
            for a, b in zip(g, r):
                assert torch.equal(a, b), f"replay {rep}: gradient differs"
        print(f"    replay {rep} matches the eager step", flush=True)


def test_batch_autotune_keeps_results(tmp_path):
    """The per-class tile tuner (rows per block and work per item for each class
    of case sizes, then the persistent grid) leaves the results within the
    oracle tolerance, and a cached choice is reused as it was made."""
    import torch

    import paper_2312_16263_amd as fwh
    data = _case_data(CASES)
    plans = [make_plan(c, "f32") for c in CASES]
    inputs = [to_device(d[:3]) for d in data]
    batch = fwh.Batch(plans, inputs)
    res = fwh.autotune(batch, candidates=[(4, 1e5), (2, 1e6), (4, 1e7)], bpc_candidates=(1, 2), reps=2,
                       cache_path=str(tmp_path / "tune.json"))
    for key, v in res["classes"].items():
        print(f"    class {key} ({v['cases']} cases): {v['table']} -> {v['choice']}", flush=True)
    print(f"    grid {res['grid_table']} -> {res['blocks_per_cu']} blocks/CU", flush=True)
    p = [t.clone() for t in batch.forward()]
    torch.cuda.synchronize()
    for i, d in enumerate(data):
        m = valid_mask(d[4], d[3].shape[1])
        assert rel_l2(p[i].double().cpu().numpy(), d[3], m) <= TOL["f32"]
    # cached choices are reused
    res2 = fwh.autotune(batch, cache_path=str(tmp_path / "tune.json"))
    assert res2["blocks_per_cu"] == res["blocks_per_cu"]
    assert {k: v["choice"] for k, v in res2["classes"].items()} == {k: v["choice"] for k, v in res["classes"].items()}


@pytest.mark.parametrize("rows", [2, 3])
def test_batch_rows_per_block(rows):
    """Shorter k blocks of the matrix-core batched gather (2 or 3 rows of 61
    samples) against the oracle."""
    import torch

    import paper_2312_16263_amd as fwh
    data = _case_data(CASES)
    plans = [make_plan(c, "f32", gather="mfma") for c in CASES]
    inputs = [to_device(d[:3]) for d in data]
    batch = fwh.Batch(plans, inputs, item_units=3e5)
    assert batch.gather == "mfma"
    for i in range(len(CASES)):
        batch.tune_case(i, None, rows, bind=False)
    batch.bind()
    p = [t.clone() for t in batch.forward()]
    torch.cuda.synchronize()
    for i, d in enumerate(data):
        m = valid_mask(d[4], d[3].shape[1])
        err = rel_l2(p[i].double().cpu().numpy(), d[3], m)
        print(f"    rows={rows} case {i}: rel L2 vs oracle {err:.3e}", flush=True)
        assert err <= TOL["f32"], err


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_batch_blocks_per_cu_same_results(mode):
    """The persistent gather's grid (1 to 4 resident blocks per CU) only changes
    which block takes which work item: the outputs are bit-identical."""
    import torch

    import paper_2312_16263_amd as fwh
    data = _case_data(CASES)
    plans = [make_plan(c, mode) for c in CASES]
    inputs = [to_device(d[:3]) for d in data]
    batch = fwh.Batch(plans, inputs)
    ref = None
    for bpc in (2, 1, 3, 4):
        print(f"[batch grid] mode={mode} blocks_per_cu={bpc}", flush=True)
        batch.tune(1e6, bpc)
        p = [t.clone() for t in batch.forward()]
        torch.cuda.synchronize()
        if ref is None:
            ref = p
            for i, d in enumerate(data):
                m = valid_mask(d[4], d[3].shape[1])
                assert rel_l2(p[i].double().cpu().numpy(), d[3], m) <= TOL[mode]
        else:
            for a, b in zip(p, ref):
                assert torch.equal(a, b), bpc
