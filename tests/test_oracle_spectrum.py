"""Pins of the oracle's energy spectrum and enstrophy (Sec. IV) by Parseval's
identity and single-mode closed forms, and of the driven-band velocity filter
(Sec. V) by plane-wave closed forms and consistency with the spectrum."""
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


def test_band_filter_removes_exactly_the_driven_modes():
    """A field of three plane waves, one inside the band [5.5, 8.5]: the filter
    returns the other two exactly (closed form), and the mean speed is that of
    the remaining field."""
    n = 32
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep_x = 0.01 * np.sin(2 * np.pi * 2 * y / n)              # |k| = 2
    keep_y = 0.02 * np.cos(2 * np.pi * (3 * x + 1 * y) / n)    # |k| = sqrt(10)
    band = 0.03 * np.cos(2 * np.pi * (5 * x + 4 * y) / n + 0.3)   # |k| = sqrt(41) = 6.4
    fx, fy, speed = diagnostics.filtered_velocity(keep_x + band, keep_y - 2 * band, 5.5, 8.5)
    assert np.abs(fx - keep_x).max() < 1e-15
    assert np.abs(fy - keep_y).max() < 1e-15
    assert abs(speed - np.mean(np.hypot(keep_x, keep_y))) < 1e-15


def test_band_filter_beyond_the_lattice_is_identity_and_consistent_with_spectrum():
    g = np.random.Generator(np.random.Philox(5))
    bx, by = 0.01 * g.standard_normal((2, 16, 16))
    fx, fy, _ = diagnostics.filtered_velocity(bx, by, 100.0, 200.0)
    assert np.abs(fx - bx).max() < 1e-16 and np.abs(fy - by).max() < 1e-16
    # removing the shells |k| in [2.5, 4.5] removes spectrum bins 3 and 4 only
    fx, fy, _ = diagnostics.filtered_velocity(bx, by, 2.5, 4.5)
    E0, _ = diagnostics.spectrum(bx, by, 12)
    E1, _ = diagnostics.spectrum(fx, fy, 12)
    want = E0.copy()
    want[3:5] = 0.0
    assert np.abs(E1 - want).max() < 1e-18


def test_spectrum_average_special_cases():
    """Constant samples have zero error; the estimate is homogeneous of degree
    one and independent of the sample order; two samples m(1 +- d) give
    (m/2)(sqrt(d (2 + d)) + sqrt(d (2 - d))), the root taken of the magnitude."""
    m = np.array([1.0, 0.5, 2e-3])
    mean, err = diagnostics.spectrum_average(np.tile(m, (5, 1)))
    assert np.array_equal(mean, m) and np.all(err == 0)
    d = 0.1
    S = np.stack([m * (1 + d), m * (1 - d)])
    mean, err = diagnostics.spectrum_average(S)
    assert np.abs(mean - m).max() < 1e-16
    want = 0.5 * m * (np.sqrt(d * (2 + d)) + np.sqrt(d * (2 - d)))
    assert np.abs(err - want).max() < 1e-15
    g = np.random.Generator(np.random.Philox(1))
    R = g.random((7, 4))
    _, e1 = diagnostics.spectrum_average(R)
    _, e2 = diagnostics.spectrum_average(3.0 * R[::-1])
    assert np.abs(e2 - 3.0 * e1).max() < 1e-14


def _r2(n):
    """Representations of n as a sum of two squares of integers (signs and
    order counted), by Jacobi's two-square theorem: 4 (d_1(n) - d_3(n)),
    d_r the number of divisors congruent to r mod 4; r2(0) = 1."""
    if n == 0:
        return 1
    d = [q for q in range(1, n + 1) if n % q == 0]
    return 4 * (sum(1 for q in d if q % 4 == 1) - sum(1 for q in d if q % 4 == 3))


def test_shell_modes_by_the_two_square_theorem():
    """A shell b inside the lattice's wave-number box holds the k with
    (b - 1/2)^2 < |k|^2 < (b + 1/2)^2, i.e. |k|^2 = b^2 - b + 1 .. b^2 + b
    (ties are impossible: |k|^2 is an integer), so its count is a sum of r2."""
    for nx, ny in ((64, 64), (64, 32), (31, 33)):
        nb = (min(nx, ny) - 1) // 2           # shells with b + 1/2 inside the box
        got = diagnostics.shell_modes(nx, ny, nb)
        expect = [1] + [sum(_r2(m) for m in range(b * b - b + 1, b * b + b + 1))
                        for b in range(1, nb)]
        np.testing.assert_array_equal(got, expect)
    np.testing.assert_array_equal(diagnostics.shell_modes(64, 64, 5), [1, 8, 12, 16, 32])


def test_shell_modes_count_every_wave_vector_once():
    for nx, ny in ((16, 16), (16, 4), (5, 7), (1, 1), (2, 1), (1, 9)):
        nb = int(np.ceil(np.hypot(nx / 2, ny / 2))) + 2
        c = diagnostics.shell_modes(nx, ny, nb)
        assert c.sum() == nx * ny and c[-1] == 0
    # fewer bins: the higher shells are left out, the lower ones unchanged
    np.testing.assert_array_equal(diagnostics.shell_modes(16, 16, 4),
                                  diagnostics.shell_modes(16, 16, 20)[:4])


def test_angular_average_of_a_point_impulse_is_flat():
    """beta_x = nx ny delta(x) has beta_hat = 1 at every k, so each shell sum
    of the spectrum is 1/2 times the shell's number of wave vectors: the
    angular average (Sec. IV) is 1/2 in every shell."""
    nx, ny = 32, 16
    bx = np.zeros((ny, nx))
    bx[0, 0] = nx * ny
    Ek, _ = diagnostics.spectrum(bx, np.zeros_like(bx), 20)
    c = diagnostics.shell_modes(nx, ny, 20)
    np.testing.assert_allclose(Ek[c > 0] / c[c > 0], 0.5, rtol=1e-14)
    assert np.all(Ek[c == 0] == 0)
