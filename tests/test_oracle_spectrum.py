"""Pins of the oracle's energy spectrum and enstrophy (Sec. IV) by Parseval's
identity and single-mode closed forms."""
import numpy as np

from oracle import diagnostics
import workloads


def test_parseval():
    _, bx, by = workloads.noisy_rest(32, 32, 0.01, seed=4)
    Ek, _ = diagnostics.spectrum(bx, by, nbins=40)      # 40 > 16 sqrt(2): every mode binned
    assert abs(Ek.sum() - 0.5 * (bx ** 2 + by ** 2).sum() / 32 ** 2) < 1e-16


def test_single_mode():
    n, m, A = 64, 5, 0.02
    y = np.arange(n)
    bx = np.repeat((A * np.sin(2 * np.pi * m * y / n))[:, None], n, axis=1)
    Ek, Z = diagnostics.spectrum(bx, np.zeros_like(bx), nbins=20)
    expect = np.zeros(20)
    expect[m] = A * A / 4
    np.testing.assert_allclose(Ek, expect, atol=1e-18)
    assert abs(Z - A * A * (2 * np.pi * m / n) ** 2 / 4) < 1e-15


def test_enstrophy_equals_mean_square_vorticity():
    """Z = 1/2 <|w|^2> with w = curl beta computed spectrally, by Parseval."""
    _, bx, by = workloads.noisy_rest(24, 24, 0.01, seed=8)
    n = 24
    k = np.fft.fftfreq(n, 1.0 / n)
    KY, KX = np.meshgrid(k, k, indexing="ij")
    w = np.fft.ifft2(1j * 2 * np.pi / n * (KX * np.fft.fft2(by) - KY * np.fft.fft2(bx)))
    _, Z = diagnostics.spectrum(bx, by, nbins=4)
    assert abs(Z - 0.5 * (np.abs(w) ** 2).mean()) < 1e-15
