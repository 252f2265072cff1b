"""GPU parity for 1 < cfl <= 2 (sources up to two nodes upstream; the paper's
finest grid, spacing 0.04 with dt = 0.05, has cfl = 1.25) against the oracle,
through the C ABI.  Tile kernel form only."""
import numpy as np
import pytest

import paper_2101_06187_amd as rl
from oracle import diagnostics as odiag
from oracle import rlbm as orlbm
from oracle import stencil as ostencil
import workloads

from gpu_helpers import (dev, field_errors, fold, gpu_fields, host, lib_to_oracle,
                         oracle_to_lib, rel, say, unfold)

pytestmark = pytest.mark.gpu

SPH = ostencil.sph26()


@pytest.mark.parametrize("cfl", [1.25, 1.5, 1.9, 2.0])
@pytest.mark.parametrize("shape,forced", [((67, 9), False), ((40, 33), True), ((5, 3), False),
                                          ((3, 2), False)])
def test_cfl2_one_step_f64(cfl, shape, forced):
    nx, ny = shape
    say("cfl2 one step", cfl, shape, forced)
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=nx * 11 + ny, spread=0.3)
    force = dict(amplitude=3e-3, k_lo=1.0, k_hi=2.3, seed=5) if forced else None
    fr = rl.Forcing(3e-3, 1.0, 2.3, 5) if forced else None
    lat = rl.Lattice(nx, ny, 0.7, storage="F64", cfl=cfl, forcing=fr)
    assert lat.kernel()[0] == "tile"
    lat.set_populations(dev(oracle_to_lib(F0)))
    lat.step(2)
    F2 = lib_to_oracle(host(lat.populations()))
    F2o = orlbm.run(F0, SPH, 0.7, 2, cfl=cfl, force=force)
    err = rel(F2, F2o)
    say("populations err", err)
    assert err < 1e-13
    assert lat.check() == rl.OK


def test_cfl2_fields_and_reduced_storage():
    """Fields (stage (c) with the two-node stream) and FP32 / F16S storage
    on the 512 x 512 forced workload at cfl 1.25."""
    n, cfl = 512, 1.25
    e, bx, by = workloads.noisy_rest(n, n, 0.005, seed=1)
    force = dict(amplitude=1e-5, k_lo=4.0, k_hi=6.0, seed=2)
    Fo = orlbm.run(orlbm.set_state(e, bx, by, SPH), SPH, 0.55, 3, cfl=cfl, force=force)
    ref = odiag.fields(Fo, SPH, cfl)
    for storage, tol_eps, tol_beta in (("F64", 1e-12, 1e-12), ("F32", 1e-6, 2e-4),
                                       ("F16S", 5e-5, 2e-2)):
        lat = rl.Lattice(n, n, 0.55, storage=storage, cfl=cfl,
                         forcing=rl.Forcing(1e-5, 4.0, 6.0, 2))
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(3)
        errs = field_errors(gpu_fields(lat), ref)
        say("cfl 1.25 forced512", storage, errs)
        assert errs["eps"] < tol_eps
        assert errs["beta_x"] < tol_beta and errs["beta_y"] < tol_beta
        if storage == "F64":
            assert errs["T"] < 1e-12


def test_cfl2_shear_wave_decays_at_linear_theory_rate():
    """32 x 32 shear wave at cfl 1.25, tau 0.8: the decay rate over steps
    60-300 equals the discrete linear theory's shear eigenvalue."""
    from test_oracle_shear_wave import shear_eigenvalue
    n, tau, cfl = 32, 0.8, 1.25
    e, bx, by = workloads.shear_wave(n, 0.01)
    lat = rl.Lattice(n, n, tau, storage="F64", cfl=cfl)
    lat.set_state(dev(e), dev(bx), dev(by))
    c0 = lat.conserved()
    lat.step(60)
    a0 = np.abs(np.fft.rfft(host(lat.fields()[1])[:, 0])[1])
    lat.step(240)
    a1 = np.abs(np.fft.rfft(host(lat.fields()[1])[:, 0])[1])
    lam = abs(shear_eigenvalue(SPH, tau, 2 * np.pi / n, cfl))
    rate = (a1 / a0) ** (1 / 240)
    say("cfl 1.25 decay", rate, lam)
    assert abs(rate / lam - 1) < 1e-6
    c1 = lat.conserved()
    assert np.abs(c1 - c0).max() < 1e-13 * c0[0]


def test_cfl2_march_form_rejected_and_folded_stencil():
    lat = rl.Lattice(64, 64, 0.7, storage="F32", cfl=1.25)
    for kind in ("march", "staged"):
        with pytest.raises(rl.RlbmError) as ex:
            lat.set_kernel(kind, 0)
        assert ex.value.code == rl.EUNSUPPORTED
    lat.set_kernel("tile", 2)
    nx, ny = 40, 24
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=5, spread=0.3)
    f = rl.Lattice(nx, ny, 0.7, stencil="SPH26_ZFOLD", storage="F64", cfl=1.6)
    f.set_populations(dev(fold(F0)))
    f.step(2)
    assert rel(unfold(host(f.populations())), orlbm.run(F0, SPH, 0.7, 2, cfl=1.6)) < 1e-13


def test_cfl2_ensemble_with_mixed_cfl():
    """Lattices with cfl 1.25 and 0.9 in one ensemble: each equals its own
    single-lattice run against the oracle."""
    sizes, taus, cfls = [(48, 40), (64, 32)], [0.6, 0.7], [1.25, 0.9]
    ens = rl.Ensemble(sizes, taus, storage="F64", cfl=cfls)
    F = []
    for r, (nx, ny) in enumerate(sizes):
        e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=r)
        ens.set_state(r, dev(e), dev(bx), dev(by))
        F.append(orlbm.set_state(e, bx, by, SPH))
    ens.step(3)
    for r in range(2):
        Fo = orlbm.run(F[r], SPH, taus[r], 3, cfl=cfls[r])
        assert rel(lib_to_oracle(host(ens.populations(r))), Fo) < 1e-13
