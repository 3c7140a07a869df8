"""Seeded broadband surface data (input generation only).

Each (panel, variable) series is an independent zero-mean Gaussian process with
power spectrum |X(f)|^2 ~ f^(-5/3) above the lowest resolved frequency
1/(N dtau), no DC, scaled to the requested RMS.  It stands in for the turbulent
IDDES surface data of the paper's 30P30N case (Sec. IV C), which is not
available.  Panels are generated in fixed blocks, each seeded from
(seed, block index), so the data do not depend on how blocks are scheduled.
"""
from __future__ import annotations

import math

import numpy as np

BLOCK = 4096


def series_block(seed: int, block: int, n_series: int, n_tau: int, rms: float) -> np.ndarray:
    """[n_series, n_tau] float64 series for one block."""
    rng = np.random.default_rng([seed, block])
    nf = n_tau // 2 + 1
    f = np.arange(nf, dtype=np.float64)
    amp = np.zeros(nf)
    amp[1:] = f[1:] ** (-5.0 / 6.0)
    spec = (rng.standard_normal((n_series, nf)) + 1j * rng.standard_normal((n_series, nf))) * amp[None, :]
    x = np.fft.irfft(spec, n=n_tau, axis=1)
    x -= x.mean(axis=1, keepdims=True)
    x *= rms / np.sqrt(np.mean(x * x, axis=1, keepdims=True))
    return x


def surface_data(P: int, n_tau: int, aoa_deg: float, seed: int, rms: float = 0.01, dtype=np.float32):
    """rho [N,P] = 1 + rho', u [3,N,P] = U0 + u', p' [N,P] (time-major), each
    perturbation an independent broadband series with the given RMS."""
    a = math.radians(aoa_deg)
    U = (math.cos(a), math.sin(a), 0.0)
    rho = np.empty((n_tau, P), dtype=dtype)
    u = np.empty((3, n_tau, P), dtype=dtype)
    pp = np.empty((n_tau, P), dtype=dtype)
    for b0 in range(0, P, BLOCK):
        b1 = min(P, b0 + BLOCK)
        x = series_block(seed, b0 // BLOCK, 5 * (b1 - b0), n_tau, rms).reshape(5, b1 - b0, n_tau)
        rho[:, b0:b1] = (1.0 + x[0]).T
        for i in range(3):
            u[i, :, b0:b1] = (U[i] + x[1 + i]).T
        pp[:, b0:b1] = x[4].T
    return rho, u, pp


def surface_data_torch(P: int, n_tau: int, aoa_deg: float, seed: int, rms: float = 0.01, device="cuda",
                       block: int = 8192):
    """Device-side version of `surface_data` (same spectrum, RMS and layout;
    torch's generator, so a different realisation): FP32 tensors rho [N,P],
    u [3,N,P], p' [N,P].  Blocks of panels are seeded from (seed, block)."""
    import torch
    a = math.radians(aoa_deg)
    U = (math.cos(a), math.sin(a), 0.0)
    rho = torch.empty((n_tau, P), dtype=torch.float32, device=device)
    u = torch.empty((3, n_tau, P), dtype=torch.float32, device=device)
    pp = torch.empty((n_tau, P), dtype=torch.float32, device=device)
    nf = n_tau // 2 + 1
    f = torch.arange(nf, dtype=torch.float64, device=device)
    amp = torch.zeros(nf, dtype=torch.float64, device=device)
    amp[1:] = f[1:] ** (-5.0 / 6.0)
    g = torch.Generator(device=device)
    for b0 in range(0, P, block):
        b1 = min(P, b0 + block)
        g.manual_seed(int(seed) * 1000003 + b0 // block)
        m = 5 * (b1 - b0)
        re = torch.randn((m, nf), generator=g, dtype=torch.float64, device=device)
        im = torch.randn((m, nf), generator=g, dtype=torch.float64, device=device)
        x = torch.fft.irfft(torch.complex(re, im) * amp, n=n_tau, dim=1)
        x -= x.mean(dim=1, keepdim=True)
        x *= rms / torch.sqrt(torch.mean(x * x, dim=1, keepdim=True))
        x = x.reshape(5, b1 - b0, n_tau)
        rho[:, b0:b1] = (1.0 + x[0]).T.float()
        for i in range(3):
            u[i, :, b0:b1] = (U[i] + x[1 + i]).T.float()
        pp[:, b0:b1] = x[4].T.float()
    return rho, u, pp
