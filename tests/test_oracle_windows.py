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


def test_field_window_strip_matches_whole_lattice():
    """The stored field references (tests/golden/make_field_windows.py):
    windows of radius N + 1 side by side in one periodic strip, advanced N
    forced steps, give the fields of the whole-lattice oracle run at their
    centres."""
    import importlib.util
    import os
    from oracle import diagnostics as odiag
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location(
        "make_field_windows", os.path.join(here, "golden", "make_field_windows.py"))
    mfw = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mfw)
    wl = workloads.Workload("small", 40, 0.57, 3, "noise", 0.01, 5, (2e-3, 3.0, 6.0, 9))
    xs, ys = [0, 39, 17, 5], [0, 39, 22, 31]
    steps = 3
    got = mfw.window_fields(wl, xs, ys, steps)
    e, bx, by = workloads.initial_fields(wl)
    force = dict(amplitude=2e-3, k_lo=3.0, k_hi=6.0, seed=9)
    F = orlbm.run(orlbm.set_state(e, bx, by, SPH), SPH, wl.tau, steps, force=force)
    eps, gx, gy, T6 = odiag.fields(F, SPH, 1.0)
    want = {"eps": eps, "beta_x": gx, "beta_y": gy}
    for i, name in enumerate(("T00", "T0x", "T0y", "Txx", "Txy", "Tyy")):
        want[name] = T6[i]
    for name, arr in want.items():
        assert np.abs(np.asarray(got[name]) - arr[ys, xs]).max() < 1e-14, name
