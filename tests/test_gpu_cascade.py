"""Qualitative check of the inertial range of Sec. V on the paper's own
configuration (not a parity test: the trajectories are chaotic beyond a short
horizon, and the paper prints no numbers for its spectra).

Configuration (Sec. V): a periodic N x N x 1 lattice of side N alpha = 40.96
(N = 1024, alpha = 0.04), time step 0.05 (cfl = 0.05 / alpha = 1.25),
eta/s = 0.01 (relaxation time 5 (eta/s) / T, one step at T = 1), started at
rest, driven in the whole band k_f <= |k| < k_max with k_f = 6 in the
physical wave number 2 pi n / (N alpha), i.e. mode number n_f = 39.11, up
to the largest axis mode N/2.  The amplitude 1.3e-3 gives the filtered mean
speed of about 0.015 that the paper tunes its forcing to.  The spectrum is
averaged over the second to fourth quarter of 8000 steps (400 time units,
the paper's longest run).

The quantity compared with the -5/3 law is the paper's spectral energy
density, half the squared velocity amplitude averaged over the directions of
k (Sec. IV): the shell sum of the library's spectrum divided by the shell's
number of wave vectors.
"""
import numpy as np
import pytest

import paper_2101_06187_amd as rl

from gpu_helpers import dev, say

pytestmark = pytest.mark.gpu

SIDE = 40.96          # N alpha, the same for every lattice of the paper's series
DT = 0.05
K_F = 6.0             # physical wave number where the driven band starts


def _run(n, amplitude, steps, every=36, seed=1):
    alpha = SIDE / n
    n_f = K_F * SIDE / (2 * np.pi)
    lat = rl.Lattice(n, n, 1.0, storage="F64", cfl=DT / alpha,
                     forcing=rl.Forcing(amplitude, n_f, n / 2 - 0.5, seed))
    lat.set_relaxation("eta_s")
    lat.set_state(dev(np.ones((n, n))), dev(np.zeros((n, n))), dev(np.zeros((n, n))))
    lat.set_graph_chunk(every)
    spectra = []
    while lat.steps < steps:
        lat.step(every)
        if lat.steps >= steps // 4:
            spectra.append(lat.spectrum(n // 2)[0])
    assert lat.check() == rl.OK
    _, _, speed = lat.filtered_velocity(n_f, float("inf"))
    lat.close()
    mean = np.mean(spectra, axis=0)
    avg = mean / np.maximum(rl.shell_modes(n, n, n // 2), 1)
    return speed, mean, avg, int(n_f)


def _slope(y, lo, hi):
    k = np.arange(lo, hi + 1)
    return float(np.polyfit(np.log(k), np.log(y[lo:hi + 1]), 1)[0])


@pytest.fixture(scope="module")
def paper_run():
    return _run(1024, 1.3e-3, 8000)


def test_inertial_range_slope_on_the_paper_configuration(paper_run):
    speed, shell_sum, avg, n_f = paper_run
    # the inertial range 0 < k < k_f: shells 4 .. 38 (shell 39 holds driven modes)
    s_avg, s_sum = _slope(avg, 4, n_f - 1), _slope(shell_sum, 4, n_f - 1)
    say("filtered speed", speed, "slope of the angular average", s_avg, "of the shell sum", s_sum)
    assert 0.010 <= speed <= 0.025
    assert abs(s_avg - (-5.0 / 3.0)) <= 0.2
    # the energy of the inertial range falls with k: no pile-up below the band
    assert avg[4] > avg[n_f // 2] > avg[n_f - 1]


def test_undriven_shells_are_fed_quadratically():
    """The driven band is exactly k >= k_f, so the shells below it receive
    energy only through the quadratic terms of the dynamics: doubling the
    amplitude multiplies the filtered speed by 4 (a force leaking into the
    undriven shells would add a part linear in the amplitude)."""
    s1, _, a1, n_f = _run(512, 1e-3, 4000)
    s2, _, a2, _ = _run(512, 2e-3, 4000)
    say("filtered speeds", s1, s2, "ratio", s2 / s1)
    assert 3.6 <= s2 / s1 <= 4.4
    assert abs(_slope(a1, 4, n_f - 1) - _slope(a2, 4, n_f - 1)) <= 0.1


def test_finer_lattices_of_the_same_volume_conform_better(paper_run):
    """Sec. V's constant-volume series (N alpha = 40.96 with N = 256, 512,
    1024, the same driven band from k_f = 6): the inertial-range slope of the
    angular average comes closer to -5/3 as the lattice is refined.  The
    amplitudes keep each lattice stable (the slope does not depend on them,
    see the quadratic-feeding test)."""
    slopes = {}
    for n, amplitude in ((256, 1e-2), (512, 4e-3)):
        _, _, avg, n_f = _run(n, amplitude, 8000)
        slopes[n] = _slope(avg, 4, n_f - 1)
    _, _, avg, n_f = paper_run
    slopes[1024] = _slope(avg, 4, n_f - 1)
    say("slopes of the angular average by N", slopes)
    dev = {n: abs(s + 5.0 / 3.0) for n, s in slopes.items()}
    assert dev[1024] < dev[512] < dev[256]
