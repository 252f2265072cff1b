"""Pins of the oracle's Anderson-Witting collision (Sec. III A) and of whole-step
invariants: per-site conservation of T^{0 mu}, the rest state, global
conservation without forcing."""
import numpy as np
import pytest

from oracle import rlbm, diagnostics
import workloads


@pytest.mark.parametrize("which", ["sph26", "circ8"])
def test_collision_conserves_energy_momentum_per_site(which, request):
    """Landau frame + AW rate: sum_q w_q v_q^mu (F_c - F_s) = 0 at every site."""
    st = request.getfixturevalue(which)
    Fs = workloads.random_populations(st.v, 6, 6, seed=21, spread=0.4,
                                      z_mirror=(st.D == 3))
    T, _ = rlbm.moments(Fs, st)
    eps, u = rlbm.landau(T)
    beta = u[1:] / u[0]
    Feq = rlbm.equilibrium(eps, beta, st)
    Fc = rlbm.collide(Fs, Feq, beta, 0.7, st)
    Tc, _ = rlbm.moments(Fc, st)
    assert np.abs(Tc[0] - T[0]).max() < 1e-14


def test_plain_bgk_does_not_conserve(sph26):
    """Negative control: relaxing with the constant rate 1/tau instead of the
    Anderson-Witting rate violates momentum conservation visibly."""
    Fs = workloads.random_populations(sph26.v, 6, 6, seed=21, spread=0.4)
    T, _ = rlbm.moments(Fs, sph26)
    eps, u = rlbm.landau(T)
    beta = u[1:] / u[0]
    Feq = rlbm.equilibrium(eps, beta, sph26)
    Fc = Fs - (Fs - Feq) / 0.7
    Tc, _ = rlbm.moments(Fc, sph26)
    assert np.abs(Tc[0] - T[0]).max() > 1e-6


def test_rest_state_unchanged(sph26):
    F = rlbm.set_state(np.ones((6, 7)), np.zeros((6, 7)), np.zeros((6, 7)), sph26)
    F2 = rlbm.run(F, sph26, 0.51, 10)
    assert np.abs(F2 - 1.0).max() < 2e-15


def test_global_conservation_unforced(sph26):
    e, bx, by = workloads.noisy_rest(24, 24, 0.02, seed=1)
    F = rlbm.set_state(e, bx, by, sph26)
    c0 = diagnostics.conserved(F, sph26)
    F = rlbm.run(F, sph26, 0.55, 120, cfl=0.8)
    c1 = diagnostics.conserved(F, sph26)
    assert abs(c1[0] - c0[0]) < 1e-13 * c0[0]
    assert np.abs(c1[1:] - c0[1:]).max() < 1e-13 * c0[0]


def test_global_conservation_unforced_circ8(circ8):
    e, bx, by = workloads.noisy_rest(16, 16, 0.02, seed=4)
    F = rlbm.set_state(e, bx, by, circ8)
    c0 = diagnostics.conserved(F, circ8)
    F = rlbm.run(F, circ8, 0.6, 60)
    c1 = diagnostics.conserved(F, circ8)
    assert np.abs(c1 - c0).max() < 1e-13 * c0[0]


def test_unstable_state_is_flagged(sph26):
    e, bx, by = workloads.noisy_rest(4, 4, 0.0, seed=0)
    F = rlbm.set_state(e, bx, by, sph26)
    F = -F                                    # negative energy density everywhere
    with pytest.raises(FloatingPointError):
        rlbm.step(F, sph26, 0.6)
