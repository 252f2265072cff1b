"""Pins of the oracle's projected force term (Sec. III C, App. B) and of the
stirring-force field (Sec. V).

The injection rates are derived here from the kinetic equation itself, not
from the paper's projection: with df/dt = -F_i d f/dp^i, integration by parts
gives
    d T^{0 mu}/dt = F_i N^{i mu}  (energy: F.N, momentum: F N^0),
    d T^{ij}/dt   = F_i N^j + F_j N^i - F_k N3^{kij}
where N are number-weighted moments (measure d^3p, no p^0 weight).  Under the
closure f = exp(-p) A(v) the ratio of number- to energy-weighted moments is
Gamma(D)/Gamma(D+1) = 1/D (1/3 on the sphere, 1/2 on the circle).
"""
import json
import os

import numpy as np
import pytest

from oracle import rlbm, forcing
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _state(st, seed):
    F = workloads.random_populations(st.v, 5, 5, seed=seed, spread=0.4,
                                     z_mirror=(st.D == 3))
    T, R = rlbm.moments(F, st)
    g = np.random.Generator(np.random.Philox(seed + 100))
    fx = g.standard_normal((5, 5))
    fy = g.standard_normal((5, 5))
    return F, T, R, fx, fy


@pytest.mark.parametrize("which", ["sph26", "circ8"])
def test_injection_rates_match_kinetic_equation(which, request):
    st = request.getfixturevalue(which)
    d = st.D
    F, T, R, fx, fy = _state(st, 3)
    dt = 0.8
    dF = rlbm.force_source(T, R, fx, fy, dt, st)
    dT, _ = rlbm.moments(dF, st)
    ratio = 1.0 / d
    N0 = ratio * T[0, 0]
    N = ratio * T[0, 1:]
    Fv = np.zeros((d, 5, 5))
    Fv[0], Fv[1] = fx, fy
    np.testing.assert_allclose(dT[0, 0], dt * (Fv * N).sum(0), atol=1e-14)
    for i in range(d):
        np.testing.assert_allclose(dT[0, 1 + i], dt * Fv[i] * N0, atol=1e-14)
    # second moment: the l = 2 projection carries it exactly
    N3 = ratio * R
    for i in range(d):
        for j in range(d):
            expect = dt * (Fv[i] * N[j] + Fv[j] * N[i]
                           - np.einsum("kyx,kyx->yx", Fv, N3[:, i, j]))
            np.testing.assert_allclose(dT[1 + i, 1 + j], expect, atol=1e-14)


def test_force_matches_printed_final_form(sph26):
    """The printed final form of Sec. III C (coefficients 3/12, 1/2, 5/4, 5/2)
    must equal the oracle's route through the App. B coefficients."""
    gold = json.load(open(os.path.join(GOLDEN, "force_term.json")))["final_form"]
    F, T, R, fx, fy = _state(sph26, 7)
    dt = 1.0
    dF = rlbm.force_source(T, R, fx, fy, dt, sph26)
    V0 = 2 * T[0, 0]
    V1 = 2 * T[0, 1:]
    V3 = 2 * R
    Fv = np.stack([fx, fy, np.zeros_like(fx)])
    for q in range(26):
        v = sph26.v[q]
        Fdotv = v[0] * fx + v[1] * fy
        term1 = (Fv * V1).sum(0)
        term2 = Fdotv * V0
        term3 = np.einsum("iyx,j,k,ijkyx->yx", Fv, v, v, V3)
        term4 = Fdotv * np.einsum("k,kyx->yx", v, V1)
        proj = (gold["c1"] * term1 + gold["c2"] * term2 + gold["c3"] * term3
                + gold["c4"] * term4)
        np.testing.assert_allclose(dF[q], -dt * proj, atol=1e-14)


def test_printed_coefficients_reassemble(sph26):
    """App. B's a2 is traceless and, with a0 and a1, reassembles to the final
    form: 5/12 - 1/6 = 3/12 (the F.V1 term)."""
    c = json.load(open(os.path.join(GOLDEN, "force_term.json")))["coefficients"]
    assert abs(c["a2_FV3"] + c["a2_F_iV1_j"] + 3 * c["a2_delta_FV1"]) < 1e-15
    final = json.load(open(os.path.join(GOLDEN, "force_term.json")))["final_form"]
    assert abs(c["a0_FV1"] + c["a2_delta_FV1"] - final["c1"]) < 1e-15


def test_force_zero_when_unforced(sph26):
    F, T, R, fx, fy = _state(sph26, 1)
    dF = rlbm.force_source(T, R, 0 * fx, 0 * fy, 1.0, sph26)
    assert np.abs(dF).max() == 0.0


# --------------------------- stirring-force field ---------------------------


def _annulus_half_count(k_lo, k_hi):
    n = 0
    K = int(k_hi) + 1
    for kx in range(-K, K + 1):
        for ky in range(-K, K + 1):
            if k_lo ** 2 <= kx * kx + ky * ky <= k_hi ** 2:
                n += 1
    return n // 2


@pytest.mark.parametrize("shell", [(4, 6), (8, 12), (2, 4), (32, 40), (1, 1)])
def test_mode_count_is_half_the_annulus(shell):
    km = forcing.modes(256, 256, *shell)
    assert len(km) == _annulus_half_count(*shell)
    assert len({tuple(k) for k in km}) == len(km)
    assert all(k[1] > 0 or k[0] > 0 for k in km)


def test_force_field_matches_inverse_fft():
    nx, ny, A = 48, 40, 3e-3
    km = forcing.modes(nx, ny, 3.0, 7.5)
    r, th, ph = forcing.mode_draws(len(km), seed=2, step=5, realization=1)
    fx, fy = forcing.force_field(nx, ny, A, 3.0, 7.5, 2, 5, 1)
    for comp, f in ((np.cos(th), fx), (np.sin(th), fy)):
        S = np.zeros((ny, nx), dtype=complex)
        for (kx, ky), rm, cm, pm in zip(km, r, comp, ph):
            c = 0.5 * A * rm * cm * np.exp(1j * pm)
            S[ky % ny, kx % nx] += c
            S[(-ky) % ny, (-kx) % nx] += np.conj(c)
        f_fft = np.fft.ifft2(S).real * nx * ny
        np.testing.assert_allclose(f, f_fft, atol=1e-13 * A * len(km))


def test_force_field_zero_average_and_redrawn():
    fx, fy = forcing.force_field(32, 32, 1.0, 2, 4, 9, 0)
    assert abs(fx.sum()) < 1e-11 and abs(fy.sum()) < 1e-11
    gx, _ = forcing.force_field(32, 32, 1.0, 2, 4, 9, 1)
    assert np.abs(fx - gx).max() > 1e-3


def test_nyquist_shell_rejected():
    with pytest.raises(ValueError):
        forcing.modes(16, 16, 6, 8)


def test_force_at_points_equals_field():
    fx, fy = forcing.force_field(40, 36, 2e-3, 3, 6, 4, 11, 2)
    ys, xs = np.meshgrid(np.arange(36), np.arange(40), indexing="ij")
    gx, gy = forcing.force_at(40, 36, 2e-3, 3, 6, 4, 11, xs, ys, 2)
    assert np.abs(gx - fx).max() < 1e-17 and np.abs(gy - fy).max() < 1e-17
