"""Pins of the oracle's constant-eta/s relaxation time (Sec. III A:
tau_R = 5 (eta/s) / T, massless gas eps ~ T^4, so tau(eps) = tau eps^(-1/4)).

A spatially uniform state at rest whose populations deviate from equilibrium
without changing E and J keeps its Landau frame (eps = E, beta = 0), streams
into itself, and relaxes with the Anderson-Witting rate 1/tau(eps) exactly:
the deviation is multiplied by 1 - 1/tau(eps) in one step.  At eps = 16 the
local relaxation time is half the reference one, at eps = 1/16 twice it."""
import numpy as np
import pytest

from oracle import diagnostics, rlbm
import workloads


def _hot_uniform_state(st, eps0, seed=3, ny=4, nx=5):
    """F_eq(eps0, 0) plus a deviation with zero energy and momentum moments
    (projected out with the quadrature), the same at every site."""
    g = np.random.Generator(np.random.Philox(seed))
    d = 0.05 * eps0 * (2.0 * g.random(st.Q) - 1.0)
    # z-mirror symmetric deviation, as every state of the one-layer lattice
    for q in range(st.Q):
        if st.D == 3 and st.v[q, 2] < 0:
            m = np.flatnonzero(np.all(np.isclose(st.v, st.v[q] * [1, 1, -1]), axis=1))[0]
            d[q] = d[m]
    # remove the components along 1, v_x, v_y, v_z (w-weighted least squares)
    basis = np.concatenate([np.ones((st.Q, 1)), st.v[:, :st.D]], axis=1)   # (Q, 1+D)
    Wm = np.diag(st.w)
    coef = np.linalg.solve(basis.T @ Wm @ basis, basis.T @ Wm @ d)
    d = d - basis @ coef
    Feq = rlbm.set_state(np.full((ny, nx), eps0), np.zeros((ny, nx)), np.zeros((ny, nx)), st)
    return Feq, Feq + d[:, None, None]


@pytest.mark.parametrize("eps0,scale", [(16.0, 2.0), (1.0 / 16.0, 0.5), (1.0, 1.0)])
@pytest.mark.parametrize("which", ["sph26", "circ8"])
def test_uniform_relaxation_factor(which, eps0, scale, request):
    st = request.getfixturevalue(which)
    tau = 0.8
    Feq, F = _hot_uniform_state(st, eps0)
    for eta_s, rate in ((False, 1.0 / tau), (True, scale / tau)):
        F1 = rlbm.step(F, st, tau, eta_s=eta_s)
        ratio = (F1 - Feq) / (F - Feq)
        mask = np.abs(F - Feq) > 1e-4 * eps0
        assert mask.sum() > st.Q            # a real deviation on most planes
        assert np.abs(ratio[mask] - (1.0 - rate)).max() < 1e-11, (eta_s, eps0)


def test_eta_s_step_conserves_energy_momentum(sph26):
    """Per-site relaxation times keep the Anderson-Witting step conservative."""
    F = workloads.random_populations(sph26.v, 12, 10, seed=8, spread=0.3)
    F = F * np.linspace(0.5, 3.0, 10)[None, None, :]     # energy varies across x
    c0 = diagnostics.conserved(F, sph26)
    F3 = rlbm.run(F, sph26, 0.7, 3, eta_s=True)
    c3 = diagnostics.conserved(F3, sph26)
    assert np.abs(c3 - c0).max() < 1e-13 * c0[0]


def test_eta_s_differs_from_constant_tau_where_eps_differs(sph26):
    """Negative control: on a state with eps != 1 the two modes differ."""
    F = workloads.random_populations(sph26.v, 6, 6, seed=2, spread=0.3) * 2.0
    a = rlbm.step(F, sph26, 0.7, eta_s=False)
    b = rlbm.step(F, sph26, 0.7, eta_s=True)
    assert np.abs(a - b).max() > 1e-3
