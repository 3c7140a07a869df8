"""Helpers shared by the GPU tests: run the HIP path through the binding and
the FP64 oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import math

import numpy as np

import oracle


def rel_l2(a, b, mask=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if mask is not None:
        a = a * mask
        b = b * mask
    den = math.sqrt(float(np.sum(b * b)))
    return math.sqrt(float(np.sum((a - b) ** 2))) / (den if den > 0 else 1.0)


def valid_mask(n_t, width):
    return (np.arange(width)[None, :] < np.asarray(n_t)[:, None]).astype(np.float64)


def make_plan(case, mode, **kw):
    import paper_2312_16263_amd as fwh
    s = case.surface
    return fwh.Plan(s.y, s.normal, s.dS, case.x_obs, case.mach, case.aoa_deg, case.dtau, case.tau0, case.n_tau,
                    mode=mode, **kw)


def to_device(arrs, dtype=None):
    import torch
    out = []
    for a in arrs:
        t = torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(dtype)
        out.append(t.cuda())
    return out


def oracle_forward(case, rho, u, pp, obs_idx=None, nt_stride=None):
    return oracle.forward(case.surface, case.x_obs, case.mach, case.aoa_deg, case.dtau, case.tau0,
                          rho.astype(np.float64), u.astype(np.float64), pp.astype(np.float64), obs_idx=obs_idx,
                          nt_stride=nt_stride)


def oracle_adjoint(case, rho, u, pp, gbar):
    return oracle.adjoint(case.surface, case.x_obs, case.mach, case.aoa_deg, case.dtau, case.tau0,
                          rho.astype(np.float64), u.astype(np.float64), pp.astype(np.float64), gbar)
