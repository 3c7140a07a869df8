"""Pins of the post-processing oracle (RMS directivity and Welch PSD with the
spanwise correction of Eq. (PSD_corr)): scipy.signal.welch with the same
settings, Parseval's identity, a pure tone, the RMS of a sine."""
import numpy as np
import pytest
from scipy import signal

from oracle import post


@pytest.mark.parametrize("L", [16, 64, 256])
@pytest.mark.parametrize("n", [256, 1000, 1537])
def test_welch_matches_scipy(L, n):
    rng = np.random.default_rng(L * 7 + n)
    x = rng.standard_normal(n)
    dt = 1.2642e-3
    f, ref = signal.welch(x, fs=1.0 / dt, window="hann", nperseg=L, noverlap=L // 2, detrend=False,
                          return_onesided=True, scaling="density", average="mean")
    got = post.welch(x, dt, L)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=0)
    np.testing.assert_allclose(post.frequencies(dt, L), f, rtol=1e-14)


def test_span_correction_is_additive_in_db():
    x = np.random.default_rng(3).standard_normal(512)
    a = post.welch(x, 0.01, 64)
    b = post.welch(x, 0.01, 64, span_ratio=650.0 / 50.8)
    np.testing.assert_allclose(10 * np.log10(b) - 10 * np.log10(a), 10 * np.log10(650.0 / 50.8), rtol=1e-12)


def test_parseval_single_segment_rectangular_power():
    # one segment (n = L): sum_f PSD_f df equals the windowed mean power sum (w x)^2 / sum w^2
    rng = np.random.default_rng(5)
    L, dt = 128, 0.5
    x = rng.standard_normal(L)
    psd = post.welch(x, dt, L)
    w = post.hann(L)
    df = 1.0 / (L * dt)
    np.testing.assert_allclose(np.sum(psd) * df, np.sum((w * x) ** 2) / np.sum(w * w), rtol=1e-12)


def test_pure_tone_peak_and_power():
    # a sine on a bin centre: the density integrates to its mean power A^2 / 2 (Hann leakage is confined
    # to the neighbouring bins), and the peak sits on the tone's bin
    L, dt, A = 256, 1e-3, 3.0
    k = 20
    n = np.arange(4096)
    x = A * np.sin(2 * np.pi * k * n / L)
    psd = post.welch(x, dt, L)
    df = 1.0 / (L * dt)
    assert int(np.argmax(psd)) == k
    np.testing.assert_allclose(np.sum(psd) * df, A * A / 2, rtol=1e-10)


def test_rms():
    n = np.arange(1000)
    p = np.stack([2.0 * np.sin(2 * np.pi * n / 100), np.ones(1000)])
    r = post.rms(p, np.array([1000, 10]))
    np.testing.assert_allclose(r, [2.0 / np.sqrt(2.0), 1.0], rtol=1e-12)
