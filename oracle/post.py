"""FP64 CPU oracle of the post-processing of the observer signals.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by the tests and
the benchmark, never by the product path; it shares no code with the GPU
library.

* RMS pressure per observer (the directivity plots of Sec. IV A and IV B):
  sqrt of the mean of p'^2 over the observer's N_t samples.
* Welch power spectral density (Sec. IV C): the signal is cut into segments
  of L samples with 50 % overlap, each multiplied by a Hanning window, the
  squared magnitudes of their discrete Fourier transforms are averaged and
  scaled to a one-sided density; Eq. (PSD_corr) then adds the spanwise
  correction 10 log10(b_exp / b_m), i.e. multiplies the density by
  b_exp / b_m.

Readings (the paper gives neither): the window is the periodic Hann window
w_n = (1 - cos(2 pi n / L)) / 2 (the usual choice for spectral estimation);
segments are not detrended (p' is already a fluctuation); the density is
one-sided, PSD_f = c_f |X_f|^2 / (f_s sum_n w_n^2), c_f = 2 except at f = 0
and f = f_s / 2 (c_f = 1), f_s = 1 / dt, averaged over the
floor((N_t - L) / (L / 2)) + 1 segments starting at multiples of L / 2.
Pinned by tests/test_oracle_post.py against scipy.signal.welch with the same
settings, Parseval's identity and a pure tone.
"""
from __future__ import annotations

import numpy as np


def rms(p: np.ndarray, n_t: np.ndarray) -> np.ndarray:
    """RMS of each observer's first n_t[o] samples of p [O][>= max n_t]."""
    out = np.empty(p.shape[0])
    for o in range(p.shape[0]):
        x = np.asarray(p[o, : int(n_t[o])], dtype=np.float64)
        out[o] = np.sqrt(np.mean(x * x))
    return out


def hann(L: int) -> np.ndarray:
    n = np.arange(L, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / L)


def welch(x: np.ndarray, dt: float, L: int, span_ratio: float = 1.0) -> np.ndarray:
    """One-sided Welch density of one signal x (FP64), L // 2 + 1 frequencies."""
    x = np.asarray(x, dtype=np.float64)
    if L < 2 or L % 2 or x.size < L:
        raise ValueError("need an even segment length L <= len(x)")
    w = hann(L)
    hop = L // 2
    nseg = (x.size - L) // hop + 1
    acc = np.zeros(L // 2 + 1)
    for s in range(nseg):
        seg = x[s * hop: s * hop + L] * w
        # DFT X_f = sum_n seg_n exp(-2 pi i f n / L), f = 0 .. L/2 (numpy's real FFT is that sum)
        X = np.fft.rfft(seg)
        acc += (X.real * X.real + X.imag * X.imag)
    c = np.full(L // 2 + 1, 2.0)
    c[0] = 1.0
    c[-1] = 1.0
    fs = 1.0 / dt
    return span_ratio * c * acc / nseg / (fs * np.sum(w * w))


def welch_all(p: np.ndarray, n_t: np.ndarray, dt: float, L: int, span_ratio: float = 1.0) -> np.ndarray:
    """welch() of every observer's valid samples: [O][L // 2 + 1]."""
    return np.stack([welch(p[o, : int(n_t[o])], dt, L, span_ratio) for o in range(p.shape[0])])


def frequencies(dt: float, L: int) -> np.ndarray:
    return np.arange(L // 2 + 1) / (L * dt)
