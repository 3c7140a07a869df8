"""The chunked FP32/BF16 source stage and its adjoint against the FP64 oracle at
record lengths around every change of the chunk geometry: the padded length
NS (N = 52, 53), the first interior chunk of the source stage (N = 146, 147)
and of its adjoint (N = 144, 145), two interior chunks (N = 209, 211), the
minimum N = 4 and a longer record.  A ragged panel count (97, not a multiple
of the 32 panels of a block), both input dtypes.  Element-wise relative L2 over
the valid samples, tolerances as in the main parity tests."""
import numpy as np
import pytest

from gpu_common import make_plan, oracle_adjoint, oracle_forward, rel_l2, to_device, valid_mask
from workloads import configs, surfaces

pytestmark = pytest.mark.gpu

N_VALUES = [4, 52, 53, 144, 145, 146, 147, 209, 211, 300]
TOL = {"f32": 1e-5, "bf16": 2e-3}


def _case(n, dtype):
    surf = surfaces.sphere(1.0, 8, 16).subset(np.arange(5, 102))
    return configs.Case(f"chunks_N{n}", surf, surfaces.observer_circle(3, 10.0), 0.3, 7.0, 0.5, n,
                        tau0=0.1, kind="monopole", omega=1.0, data_dtype=dtype)


_cache = {}


def _data(n, dtype):
    key = (n, dtype)
    if key not in _cache:
        c = _case(n, dtype)
        rho, u, pp = c.data()
        p_ref, _, nt_ref = oracle_forward(c, rho, u, pp)
        _cache[key] = (c, rho, u, pp, p_ref, nt_ref)
    return _cache[key]


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["in_f32", "in_f64"])
@pytest.mark.parametrize("n", N_VALUES)
def test_chunked_source_forward(n, dtype):
    import torch
    c, rho, u, pp, p_ref, nt_ref = _data(n, dtype)
    print(f"[source chunks] N={n} in={np.dtype(dtype).name} P={c.n_panels}", flush=True)
    d = to_device((rho, u, pp))
    for mode in ("f32", "bf16"):
        plan = make_plan(c, mode)
        p = plan.forward(*d)
        torch.cuda.synchronize()
        m = valid_mask(nt_ref, p.shape[1])
        err = rel_l2(p.double().cpu().numpy(), p_ref, m)
        print(f"    forward {mode}: rel L2 vs oracle {err:.3e}", flush=True)
        assert err <= TOL[mode], (mode, err)


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["in_f32", "in_f64"])
@pytest.mark.parametrize("n", N_VALUES)
def test_chunked_source_adjoint(n, dtype):
    import torch
    c, rho, u, pp, p_ref, nt_ref = _data(n, dtype)
    gbar = 2.0 * p_ref
    g_ref = oracle_adjoint(c, rho, u, pp, gbar)
    plan = make_plan(c, "f32")
    d = to_device((rho, u, pp))
    g = plan.adjoint(*d, torch.from_numpy(gbar).float().cuda())
    torch.cuda.synchronize()
    for name, gv, gr in zip(("rho", "u", "p"), g, g_ref):
        err = rel_l2(gv.double().cpu().numpy(), gr)
        print(f"    N={n} d/d{name}: rel L2 vs oracle {err:.3e}", flush=True)
        assert err <= 1e-5, (name, err)
