"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs, element by element, at sizes the oracle finishes in seconds:
several tiles, ragged panel counts, ragged sample counts, the minimum record
length, a single panel and observer.  Tolerances (relative L2 over all valid
observer samples): plain FP64 form 1e-11; FP32 form 1e-5; BF16 coefficient
storage 2e-3; adjoints 1e-11 (FP64) and 1e-5 (FP32 arithmetic, both FP32 and
BF16 modes: the adjoint stores no BF16).  Gradients come back in the dtype of
the surface data, so with FP32 data the FP64 form is held to FP32 rounding
(1e-7)."""
import math

import numpy as np
import pytest

from gpu_common import make_plan, oracle_adjoint, oracle_forward, rel_l2, to_device, valid_mask
from workloads import configs, surfaces

pytestmark = pytest.mark.gpu

TOL_FWD = {"f64": 1e-11, "f32": 1e-5, "bf16": 2e-3}
TOL_ADJ = {"f64": 1e-11, "f32": 1e-5, "bf16": 1e-5}


def _cases():
    out = {}
    out["mono"] = configs.Case("mono", surfaces.sphere(1.0, 16, 32), surfaces.observer_circle(8, 50.0), 0.3, 5.0,
                               1 / 128, 256, kind="monopole")
    x = np.array([[7.0, -3.0, 1.0], [-20.0, 2.0, 0.5], [0.0, 12.0, -4.0], [3.0, 3.0, 3.0], [-5.0, -9.0, 0.0],
                  [40.0, 0.0, 0.0], [0.1, -6.0, 2.0]])
    out["dip_ragged"] = configs.Case("dip_ragged", surfaces.sphere(1.0, 12, 24), x, 0.5, 10.0, 1 / 100, 500,
                                     tau0=0.37, kind="dipole")
    foil = surfaces.extruded_contour(surfaces.joukowski_contour(100), 5, 1.0 / 9.0)
    out["foil_bb"] = configs.Case("foil_bb", foil, surfaces.observer_circle(9, 10.0, center=(0.5, 0, 0)), 0.17, 5.5,
                                  configs.AIRFOIL_DTAU, 333, kind="broadband", seed=5, data_dtype=np.float32)
    one = surfaces.sphere(1.0, 4, 8).subset([5])
    out["min_one"] = configs.Case("min_one", one, np.array([[3.0, 1.0, 0.5]]), 0.4, 30.0, 0.05, 4, kind="monopole")
    s65 = surfaces.sphere(1.0, 8, 16).subset(np.arange(3, 68))
    out["ragged65"] = configs.Case("ragged65", s65, surfaces.observer_circle(3, 4.0), 0.2, -12.0, 0.2, 5,
                                   kind="dipole", omega=3.0)
    return out


CASES = _cases()
_cache = {}


def _data(name):
    if name not in _cache:
        c = CASES[name]
        rho, u, pp = c.data()
        p_ref, ts_ref, nt_ref = oracle_forward(c, rho, u, pp)
        _cache[name] = (rho, u, pp, p_ref, ts_ref, nt_ref)
    return _cache[name]


@pytest.mark.parametrize("mode", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", list(CASES))
def test_forward_parity(name, mode):
    import torch
    c = CASES[name]
    rho, u, pp, p_ref, ts_ref, nt_ref = _data(name)
    print(f"[forward parity] case={name} mode={mode} P={c.n_panels} O={c.n_obs} N={c.n_tau}", flush=True)
    plan = make_plan(c, mode)
    assert np.array_equal(plan.window.n_t, nt_ref)
    np.testing.assert_allclose(plan.window.t_start, ts_ref, rtol=1e-15, atol=0)
    assert plan.window.n_t_max == p_ref.shape[1]
    d = to_device((rho, u, pp))
    out = plan.forward(*d)
    torch.cuda.synchronize()
    p = out.double().cpu().numpy()
    m = valid_mask(nt_ref, p.shape[1])
    assert np.all(p[m == 0] == 0.0)
    err = rel_l2(p, p_ref, m)
    print(f"    rel L2 vs oracle = {err:.3e} (tol {TOL_FWD[mode]:.0e})", flush=True)
    assert err <= TOL_FWD[mode], err


@pytest.mark.parametrize("mode", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", ["mono", "dip_ragged", "foil_bb", "min_one", "ragged65"])
def test_adjoint_parity(name, mode):
    import torch
    c = CASES[name]
    rho, u, pp, p_ref, ts_ref, nt_ref = _data(name)
    print(f"[adjoint parity] case={name} mode={mode}", flush=True)
    gbar = 2.0 * p_ref
    g_ref = oracle_adjoint(c, rho, u, pp, gbar)
    plan = make_plan(c, mode)
    d = to_device((rho, u, pp))
    gb = torch.from_numpy(gbar).to(plan.out_dtype).cuda()
    g = plan.adjoint(*d, gb)
    torch.cuda.synchronize()
    tol = max(TOL_ADJ[mode], 1e-7 if rho.dtype == np.float32 else 0.0)
    for name_v, gv, gr in zip(("rho", "u", "p"), g, g_ref):
        err = rel_l2(gv.double().cpu().numpy(), gr)
        print(f"    d/d{name_v}: rel L2 vs oracle = {err:.3e} (tol {tol:.0e})", flush=True)
        assert err <= tol, (name_v, err)


def test_forward_padding_and_determinism():
    import torch
    c = CASES["dip_ragged"]
    rho, u, pp, p_ref, _, nt_ref = _data("dip_ragged")
    plan = make_plan(c, "f32")
    d = to_device((rho, u, pp))
    out = torch.full((c.n_obs, plan.window.n_t_max), float("nan"), dtype=torch.float32, device="cuda")
    a = plan.forward(*d, out=out).clone()
    b = plan.forward(*d).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    m = valid_mask(nt_ref, a.shape[1])
    assert np.all(a.cpu().numpy()[m == 0] == 0.0)
    ga = plan.adjoint(*d, 2 * a)
    gb = plan.adjoint(*d, 2 * a)
    for x, y in zip(ga, gb):
        assert torch.equal(x, y)


def test_adjoint_ignores_padding_of_grad():
    import torch
    c = CASES["mono"]
    rho, u, pp, p_ref, _, nt_ref = _data("mono")
    plan = make_plan(c, "f32")
    d = to_device((rho, u, pp))
    g = torch.from_numpy(2 * p_ref).float().cuda()
    g2 = g.clone()
    m = torch.from_numpy(valid_mask(nt_ref, g.shape[1])).cuda() == 0
    g2[m] = 1e30
    a = plan.adjoint(*d, g)
    b = plan.adjoint(*d, g2)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_window_error_is_reported():
    import paper_2312_16263_amd as fwh
    s = surfaces.sphere(30.0, 4, 8)           # delay spread much longer than the record
    with pytest.raises(fwh.FwhError) as ei:
        fwh.Plan(s.y, s.normal, s.dS, np.array([[100.0, 0, 0]]), 0.5, 0.0, 0.01, 0.0, 16, mode="f32")
    assert ei.value.code == fwh.FWH_EWINDOW


@pytest.mark.parametrize("gather", ["mfma", "lds", "direct", "stream"])
@pytest.mark.parametrize("mode", ["f32", "bf16"])
@pytest.mark.parametrize("name", ["dip_ragged", "foil_bb", "ragged65"])
def test_gather_variants(name, mode, gather):
    """Each forward gather kernel (matrix-core combine, LDS-staged windows,
    direct loads, whole-row streaming for at most 8 observers), chosen through
    fwh_plan_tune, against the oracle; the streaming one refuses 9 observers."""
    import paper_2312_16263_amd as fwh
    if gather == "stream" and CASES[name].n_obs > 8:
        with pytest.raises(fwh.FwhError) as ei:
            make_plan(CASES[name], mode, gather=gather)
        assert ei.value.code == fwh.FWH_EINVAL
        return
    import torch
    c = CASES[name]
    rho, u, pp, p_ref, _, nt_ref = _data(name)
    plan = make_plan(c, mode, gather=gather)
    assert plan.info()[0] == gather
    out = plan.forward(*to_device((rho, u, pp)))
    torch.cuda.synchronize()
    p = out.double().cpu().numpy()
    err = rel_l2(p, p_ref, valid_mask(nt_ref, p.shape[1]))
    print(f"    {name} {gather} gather {mode}: rel L2 vs oracle = {err:.3e}", flush=True)
    assert err <= TOL_FWD[mode], err


@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_autograd_function(mode):
    """fwh_apply under torch.autograd: J = sum p'^2, J.backward() runs the
    transposed gather and source adjoint; the gradients equal fwh_adjoint with
    dJ/dp' = 2 p' (same kernels, bit for bit) and the oracle's gradient."""
    import torch

    import paper_2312_16263_amd as fwh
    c = CASES["dip_ragged"]
    rho, u, pp, p_ref, _, _ = _data("dip_ragged")
    plan = make_plan(c, mode)
    d = [t.requires_grad_(True) for t in to_device((rho, u, pp))]
    p = fwh.fwh_apply(plan, *d)
    J = (p * p).sum()
    J.backward()
    torch.cuda.synchronize()
    g_direct = plan.adjoint(*[t.detach() for t in d], 2.0 * p.detach())
    for t, gd in zip(d, g_direct):
        assert torch.equal(t.grad, gd)
    g_ref = oracle_adjoint(c, rho, u, pp, 2.0 * p.detach().double().cpu().numpy())
    for t, gr in zip(d, g_ref):
        err = rel_l2(t.grad.double().cpu().numpy(), gr)
        print(f"    autograd {mode}: rel L2 vs oracle = {err:.3e}", flush=True)
        assert err <= TOL_ADJ[mode], err


@pytest.mark.parametrize("mode", ["f64", "f32"])
@pytest.mark.parametrize("seg_len", [16, 64, 256])
def test_post_rms_and_welch(mode, seg_len):
    """fwh_post (RMS directivity, Welch PSD with the spanwise correction)
    on the plan's own forward result against the post-processing oracle on the
    same signal, element by element; seg_len 256 exceeds some windows of the
    small case and must be rejected."""
    import torch

    import paper_2312_16263_amd as fwh
    from oracle import post
    c = CASES["foil_bb"]
    rho, u, pp, _, _, nt_ref = _data("foil_bb")
    plan = make_plan(c, mode)
    p = plan.forward(*to_device((rho, u, pp)))
    if seg_len > int(nt_ref.min()):
        with pytest.raises(fwh.FwhError) as ei:
            plan.post(p, seg_len)
        assert ei.value.code == fwh.FWH_ESIZE
        return
    psd, rms = plan.post(p, seg_len, span_ratio=650.0 / 50.8)
    torch.cuda.synchronize()
    pn = p.double().cpu().numpy()
    ref_psd = post.welch_all(pn, nt_ref, c.dtau, seg_len, 650.0 / 50.8)
    ref_rms = post.rms(pn, nt_ref)
    e_psd = rel_l2(psd.double().cpu().numpy(), ref_psd)
    e_rms = rel_l2(rms.double().cpu().numpy(), ref_rms)
    print(f"    post {mode} L={seg_len}: PSD rel L2 {e_psd:.3e}, RMS rel L2 {e_rms:.3e}", flush=True)
    assert e_psd <= 1e-5, e_psd
    assert e_rms <= 1e-6, e_rms


@pytest.mark.parametrize("gather", ["mfma", "lds", "direct", "stream"])
@pytest.mark.parametrize("splits", [130, 131, 7])
def test_many_panel_splits(gather, splits):
    """Many panel splits, including an empty last one: 16641 panels in 130
    splits of ceil(16641/130) = 129 panels leave split 130 without panels (its
    partial signal must be zeros); 131 splits of 128 panels; 7 uneven splits.
    Both forward gathers against the oracle on a short record with few observers."""
    import torch
    P = 16641
    c = configs.Case("split_sphere", surfaces.sphere(1.0, 129, 129), surfaces.observer_circle(5, 40.0, start_deg=11.0),
                     0.2, 7.0, 1.0 / 64.0, 128, kind="dipole")
    assert c.n_panels == P
    rho, u, pp = c.data()
    p_ref, _, nt_ref = oracle_forward(c, rho, u, pp)
    plan = make_plan(c, "f32", gather=gather, splits=splits)
    assert plan.info() == (gather, splits)
    out = plan.forward(*to_device((rho, u, pp)))
    torch.cuda.synchronize()
    p = out.double().cpu().numpy()
    err = rel_l2(p, p_ref, valid_mask(nt_ref, p.shape[1]))
    chunk = -(-P // splits)
    print(f"    {gather} gather, {splits} splits of {chunk} panels (last {P - (splits - 1) * chunk}): "
          f"rel L2 vs oracle = {err:.3e}", flush=True)
    assert err <= TOL_FWD["f32"], err
