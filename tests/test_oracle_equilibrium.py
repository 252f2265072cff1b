"""Pins of the oracle's equilibrium (Sec. III A/B) and Landau solve (Sec. III A/B).

* moments of F_eq equal the ideal massless-fluid tensor (P = eps/D) exactly;
* F_eq equals the second-order angular projection of the actual Juettner
  distribution, computed by brute-force numerical quadrature on the sphere;
* the Landau solve inverts T_eq and agrees with an independent scalar
  root-finding route on arbitrary (non-equilibrium) tensors.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import rlbm
import workloads


def _rand_fields(n, seed, vmax=0.5):
    g = np.random.Generator(np.random.Philox(seed))
    eps = 0.5 + g.random((n, n))
    ang = 2 * np.pi * g.random((n, n))
    mag = vmax * g.random((n, n))
    return eps, mag * np.cos(ang), mag * np.sin(ang)


@pytest.mark.parametrize("which", ["sph26", "circ8"])
def test_equilibrium_moments_closed_form(which, request):
    st = request.getfixturevalue(which)
    d = st.D
    eps, bx, by = _rand_fields(5, 11)
    beta = np.zeros((d, 5, 5))
    beta[0], beta[1] = bx, by
    Feq = rlbm.equilibrium(eps, beta, st)
    T, _ = rlbm.moments(Feq, st)
    gamma = 1 / np.sqrt(1 - bx ** 2 - by ** 2)
    u = np.concatenate([gamma[None], gamma[None] * beta])
    g = np.diag([-1.0] + [1.0] * d)
    expect = ((d + 1) / d * eps)[None, None] * u[:, None] * u[None] \
        + (eps / d)[None, None] * g[:, :, None, None]
    np.testing.assert_allclose(T, expect, atol=2e-15 * 4, rtol=0)
    # massless: the tensor is traceless, T^mu_mu = 0
    trace = -T[0, 0] + sum(T[i, i] for i in range(1, d + 1))
    assert np.abs(trace).max() < 1e-14


def _sphere_grid(n_mu=48, n_phi=96):
    mu, wmu = np.polynomial.legendre.leggauss(n_mu)
    phi = 2 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    MU, PHI = np.meshgrid(mu, phi, indexing="ij")
    s = np.sqrt(1 - MU ** 2)
    v = np.stack([s * np.cos(PHI), s * np.sin(PHI), MU], axis=-1).reshape(-1, 3)
    w = (np.repeat(wmu[:, None], n_phi, axis=1) / 2.0 / n_phi).reshape(-1)
    return v, w


def test_equilibrium_is_projection_of_juettner(sph26):
    """Energy-weighted Juettner distribution, integrated over |p| in closed form:
    (1/3!) int dp p^3 exp(-p gamma (1 - beta.v) / T) = (T / (gamma (1 - beta.v)))^4,
    which at rest is the energy density eps = T^4 of the lattice normalisation.
    Its projection on P0, P1, P2 with the orthogonality weights of App. A,
    evaluated by numerical quadrature on the sphere, must be the oracle's F_eq.
    """
    vg, wg = _sphere_grid()
    P2g = vg[:, :, None] * vg[:, None, :] - np.eye(3)[None] / 3
    rng = np.random.Generator(np.random.Philox(5))
    for _ in range(6):
        eps = 0.5 + rng.random()
        b = 0.3 * (2 * rng.random(2) - 1)
        beta3 = np.array([b[0], b[1], 0.0])
        gamma = 1 / np.sqrt(1 - b @ b)
        FJ = eps / (gamma * (1 - vg @ beta3)) ** 4
        c0 = (wg * FJ).sum()
        c1 = 3 * (wg[:, None] * FJ[:, None] * vg).sum(0)
        c2 = 7.5 * (wg[:, None, None] * FJ[:, None, None] * P2g).sum(0)
        vq = sph26.v
        P2q = vq[:, :, None] * vq[:, None, :] - np.eye(3)[None] / 3
        proj = c0 + vq @ c1 + np.einsum("qij,ij->q", P2q, c2)
        beta = np.zeros((3, 1, 1))
        beta[0], beta[1] = b[0], b[1]
        Feq = rlbm.equilibrium(np.full((1, 1), eps), beta, sph26)[:, 0, 0]
        np.testing.assert_allclose(Feq, proj, rtol=0, atol=1e-12)


def test_landau_inverts_equilibrium(sph26):
    eps, bx, by = _rand_fields(6, 3, vmax=0.9)
    F = rlbm.set_state(eps, bx, by, sph26)
    T, _ = rlbm.moments(F, sph26)
    e2, u = rlbm.landau(T)
    np.testing.assert_allclose(e2, eps, rtol=1e-13)
    np.testing.assert_allclose(u[1] / u[0], bx, atol=1e-13)
    np.testing.assert_allclose(u[2] / u[0], by, atol=1e-13)
    assert np.abs(u[3]).max() < 1e-14


def test_landau_matches_scalar_root(sph26):
    """Independent route: for T^{0z} = T^{iz} = 0 the Landau condition reduces to
    (eps I + Pi) beta = J and eps = E - J.beta, i.e. the root of
    g(eps) = eps - E + J^T (eps I + Pi)^-1 J on eps > 0 (Pi = spatial 2x2 block).
    """
    F = workloads.random_populations(sph26.v, 4, 4, seed=9, spread=0.6)
    T, _ = rlbm.moments(F, sph26)
    eps, u = rlbm.landau(T)
    for j in range(4):
        for i in range(4):
            E = T[0, 0, j, i]
            J = T[0, 1:3, j, i]
            Pi = T[1:3, 1:3, j, i]

            def g(e):
                return e - E + J @ np.linalg.solve(e * np.eye(2) + Pi, J)

            e_root = brentq(g, 1e-6 * E, E, xtol=1e-16, rtol=1e-15)
            b_root = np.linalg.solve(e_root * np.eye(2) + Pi, J)
            assert abs(e_root - eps[j, i]) < 1e-13 * E
            np.testing.assert_allclose(u[1:3, j, i] / u[0, j, i], b_root, atol=1e-13)
