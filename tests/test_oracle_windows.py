"""The windowed oracle evaluations that the full-size GPU parity tests use
(test infrastructure): one step on a 3x3 window, two steps on a 5x5 window,
against the oracle run on the whole lattice.  A site pulls only from its 3x3
neighbourhood when cfl <= 1, so both must agree exactly at the window centre."""
import numpy as np
import pytest

from oracle import rlbm as orlbm
from oracle import stencil as ostencil
import workloads

from gpu_helpers import gather_patches, oracle_step_at, oracle_two_steps_at

SPH = ostencil.sph26()


@pytest.mark.parametrize("cfl", [1.0, 0.85])
def test_windows_match_whole_lattice(cfl):
    import torch
    nx, ny = 13, 11
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=31, spread=0.3)
    force = dict(amplitude=3e-3, k_lo=1.0, k_hi=2.5, seed=4)
    tau = 0.6
    xs = np.array([0, 6, 12, 3, 12])
    ys = np.array([0, 5, 10, 10, 0])
    F1 = orlbm.run(F0, SPH, tau, 1, cfl=cfl, force=force)
    F2 = orlbm.run(F0, SPH, tau, 2, cfl=cfl, force=force)
    Ft = torch.from_numpy(F0)
    one = oracle_step_at(gather_patches(Ft, xs, ys), SPH, tau, cfl, force=force, step_index=0,
                         sites=(xs, ys), nxy=(nx, ny))
    two = oracle_two_steps_at(gather_patches(Ft, xs, ys, radius=2), SPH, tau, cfl, force, 0,
                              (xs, ys), (nx, ny))
    assert np.abs(one - F1[:, ys, xs]).max() < 1e-14
    assert np.abs(two - F2[:, ys, xs]).max() < 1e-14
