"""Pin of the whole oracle step by the exact linear theory of a shear wave.

Around the rest state (eps = 1, beta = 0) the step is linear in small
deviations.  Built here from first principles, independently of the oracle:
  * streaming of a Fourier mode exp(i k y) by linear interpolation of the pull
    source y - cfl v_y multiplies population q by
        S_q(k) = sum_m tent(m + cfl v_q^y) exp(i k m);
  * at linear order the Landau frame gives d eps = dE and (eps + P) beta = J,
    i.e. d beta = (3/4) dJ, and the equilibrium (Sec. III B) becomes
    dF_eq,q = dE + 3 dJ . v_q = sum_r w_r (1 + 3 v_q . v_r) dF_r;
  * the Anderson-Witting rate gamma (1 - beta.v)/tau is 1/tau at this order.
So one step is M = (I - (I - P) / tau) S(k).  The shear wave decays with the
eigenvalue of M of largest modulus in the x-momentum sector.  The paper's
viscosity (Sec. III A: eta = tau_R (eps + P) / 5, kinematic tau_R / 5) with the
usual lattice correction tau - 1/2, plus the numerical diffusion of linear
interpolation, must be the small-k limit of that eigenvalue.
"""
import numpy as np
import pytest

from oracle import rlbm, diagnostics
import workloads


def _tent(d):
    return np.maximum(0.0, 1.0 - np.abs(d))


def shear_eigenvalue(st, tau, k, cfl=1.0):
    Q = st.Q
    m = np.arange(-2, 3)
    S = np.array([(_tent(m + cfl * st.v[q, 1]) * np.exp(1j * k * m)).sum()
                  for q in range(Q)])
    P = st.w[None, :] * (1 + 3 * st.v @ st.v.T)
    M = (np.eye(Q) - (np.eye(Q) - P) / tau) @ np.diag(S)
    lam, vec = np.linalg.eig(M)
    jx = np.abs((st.w * st.v[:, 0]) @ vec)         # x-momentum content
    sector = jx > 1e-8 * jx.max()
    return lam[sector][np.argmax(np.abs(lam[sector]))]


@pytest.mark.parametrize("tau", [1.0, 0.6])
def test_viscosity_small_k_limit(sph26, tau):
    n = 1024
    k = 2 * np.pi / n
    lam = shear_eigenvalue(sph26, tau, k)
    nu_measured = -np.log(np.abs(lam)) / k ** 2
    delta = np.abs(sph26.v[:, 1])
    nu_interp = 1.5 * (sph26.w * sph26.v[:, 0] ** 2 * delta * (1 - delta)).sum()
    nu_theory = (tau - 0.5) / 5 + nu_interp
    assert abs(nu_measured / nu_theory - 1) < 2e-3


def test_shear_wave_decay_matches_linear_theory(sph26):
    n, tau = 64, 1.0
    lam = abs(shear_eigenvalue(sph26, tau, 2 * np.pi / n))
    e, bx, by = workloads.shear_wave(n, 0.01)
    F = rlbm.set_state(e, bx, by, sph26)
    F = rlbm.run(F, sph26, tau, 100)
    a0 = np.abs(np.fft.rfft(diagnostics.fields(F, sph26)[1][:, 0])[1])
    F = rlbm.run(F, sph26, tau, 200)
    a1 = np.abs(np.fft.rfft(diagnostics.fields(F, sph26)[1][:, 0])[1])
    rate = (a1 / a0) ** (1 / 200)
    assert abs(rate / lam - 1) < 1e-6
    # an x-uniform flow stays x-uniform; beta_y appears only at second order in
    # the amplitude (non-uniform viscous heating changes the pressure)
    eps, ux, uy, _ = diagnostics.fields(F, sph26)
    assert np.abs(ux - ux[:, :1]).max() < 1e-15
    assert np.abs(uy - uy[:, :1]).max() < 1e-15
    assert np.abs(uy).max() < 1e-2 * 0.01 ** 2


@pytest.mark.parametrize("cfl", [0.8, 1.25])
def test_shear_wave_decay_matches_linear_theory_other_cfl(sph26, cfl):
    """The same check with the pull displacement below one node and above it
    (sources up to two nodes upstream)."""
    n, tau = 32, 0.8
    lam = abs(shear_eigenvalue(sph26, tau, 2 * np.pi / n, cfl))
    e, bx, by = workloads.shear_wave(n, 0.01)
    F = rlbm.set_state(e, bx, by, sph26)
    F = rlbm.run(F, sph26, tau, 60, cfl=cfl)
    a0 = np.abs(np.fft.rfft(diagnostics.fields(F, sph26, cfl)[1][:, 0])[1])
    F = rlbm.run(F, sph26, tau, 120, cfl=cfl)
    a1 = np.abs(np.fft.rfft(diagnostics.fields(F, sph26, cfl)[1][:, 0])[1])
    rate = (a1 / a0) ** (1 / 120)
    assert abs(rate / lam - 1) < 1e-6
