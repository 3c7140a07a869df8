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


def test_fullsize_adjoint_central_differences():
    """dJ/d(rho, u_i, p') of J = sum p'^2 at the full size, on 64 seeded entries:
    central differences of J evaluated with the plain FP64 GPU forward (J is
    quadratic in p' and quartic in rho, u; h = 1e-4) against the FP64 and the
    FP32 adjoint through the C ABI."""
    import torch
    st = _setup()
    c = st["case"]
    rho, u, pp = st["data"]
    d = to_device((rho, u, pp))
    plan64 = make_plan(c, "f64")
    plan32 = make_plan(c, "f32")

    def J():
        p = plan64.forward(*d)
        return float((p * p).sum().item())

    p64 = plan64.forward(*d)
    g64 = plan64.adjoint(*d, 2.0 * p64)
    g32 = plan32.adjoint(*d, (2.0 * p64).float())
    rng = np.random.default_rng(2312)
    h = 1e-4
    fd, a64, a32 = [], [], []
    for e in range(64):
        v = int(rng.integers(0, 5))           # 0 rho, 1..3 u_i, 2 + ... p'
        n = int(rng.integers(0, c.n_tau))
        pnl = int(rng.integers(0, c.n_panels))
        if v == 0:
            x, idx, gi = d[0], (n, pnl), 0
        elif v <= 3:
            x, idx, gi = d[1], (v - 1, n, pnl), 1
        else:
            x, idx, gi = d[2], (n, pnl), 2
        x0 = x[idx].item()
        x[idx] = x0 + h
        jp = J()
        x[idx] = x0 - h
        jm = J()
        x[idx] = x0
        fd.append((jp - jm) / (2 * h))
        a64.append(g64[gi][idx].item())
        a32.append(g32[gi][idx].item())
    torch.cuda.synchronize()
    fd, a64, a32 = np.array(fd), np.array(a64), np.array(a32)
    e64 = np.linalg.norm(a64 - fd) / np.linalg.norm(fd)
    e32 = np.linalg.norm(a32 - fd) / np.linalg.norm(fd)
    print(f"    64 entries, |dJ| rms {np.sqrt(np.mean(fd * fd)):.3e}: rel L2 FP64 adjoint vs FD {e64:.3e}, "
          f"FP32 adjoint vs FD {e32:.3e}", flush=True)
    assert e64 <= 1e-6, e64
    assert e32 <= 1e-4, e32


def test_fullsize_post_sampled():
    """fwh_post at the full size (segments of 1024 samples, several per
    observer) on the FP32 forward result, against the oracle's RMS and Welch
    PSD of the oracle's own signals on the sampled observers."""
    import torch

    from oracle import post
    st = _setup()
    c = st["case"]
    plan = make_plan(c, "f32")
    p = plan.forward(*to_device(st["data"]))
    psd, rms = plan.post(p, 1024)
    torch.cuda.synchronize()
    nt = st["nt"][SAMPLED]
    ref_psd = post.welch_all(st["p_ref"], nt, c.dtau, 1024)
    ref_rms = post.rms(st["p_ref"], nt)
    e_psd = rel_l2(psd.double().cpu().numpy()[SAMPLED], ref_psd)
    e_rms = rel_l2(rms.double().cpu().numpy()[SAMPLED], ref_rms)
    print(f"    PSD rel L2 {e_psd:.3e}, RMS rel L2 {e_rms:.3e}", flush=True)
    assert e_psd <= 1e-5, e_psd
    assert e_rms <= 1e-5, e_rms


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_fullsize_eight_observers_streaming(mode):
    """The HBM-bound point of the benchmark: the same sphere and data with 8
    observers every 45 deg, where the streaming forward gather runs (every
    coefficient read once per panel split), against the oracle on all 8
    observers."""
    import torch
    st = _setup()
    c8 = configs.dipole_sphere(n_obs=8)
    rho, u, pp = st["data"]
    if "p8" not in st:
        p_ref, ts, nt = oracle.forward(c8.surface, c8.x_obs, c8.mach, c8.aoa_deg, c8.dtau, c8.tau0, rho, u, pp)
        st.update(p8=p_ref, nt8=nt)
        print("[fullsize 8 observers] oracle forward done", flush=True)
    plan = make_plan(c8, mode)
    assert plan.info()[0] == "stream", plan.info()
    assert np.array_equal(plan.window.n_t, st["nt8"])
    out = plan.forward(*to_device(st["data"]))
    torch.cuda.synchronize()
    p = out.double().cpu().numpy()
    ref = st["p8"]
    w = min(p.shape[1], ref.shape[1])
    err = rel_l2(p[:, :w], ref[:, :w], valid_mask(st["nt8"], w))
    print(f"    {mode} streaming gather {plan.info()}: rel L2 vs oracle, all 8 observers = {err:.3e}", flush=True)
    assert err <= TOL_FWD[mode], err
