"""GPU parity of the constant-eta/s relaxation mode (Sec. III A:
tau_R = 5 (eta/s) / T, tau(eps) = tau eps^(-1/4)) against the oracle, through
the C ABI.  Tolerances as in the constant-tau parity tests."""
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


def _hot_random(nx, ny, seed):
    """Random non-equilibrium populations whose energy density varies from
    about 0.5 to 3 across the lattice (tau(eps) varies by a factor 1.6)."""
    F = workloads.random_populations(SPH.v, ny, nx, seed=seed, spread=0.3)
    return F * np.linspace(0.5, 3.0, nx)[None, None, :]


@pytest.mark.parametrize("shape", [(67, 9), (40, 33)])
@pytest.mark.parametrize("forced", [False, True])
@pytest.mark.parametrize("cfl", [1.0, 0.8])
def test_eta_s_one_step_f64(shape, forced, cfl):
    nx, ny = shape
    say("eta_s one step", shape, forced, cfl)
    F0 = _hot_random(nx, ny, seed=nx + 3 * ny)
    force = dict(amplitude=3e-3, k_lo=1.0, k_hi=2.3, seed=5) if forced else None
    fr = rl.Forcing(3e-3, 1.0, 2.3, 5) if forced else None
    lat = rl.Lattice(nx, ny, 0.75, storage="F64", cfl=cfl, forcing=fr)
    lat.set_relaxation("eta_s")
    lat.set_populations(dev(oracle_to_lib(F0)))
    lat.step(2)
    F2 = lib_to_oracle(host(lat.populations()))
    F2o = orlbm.run(F0, SPH, 0.75, 2, cfl=cfl, force=force, eta_s=True)
    err = rel(F2, F2o)
    say("populations err", err)
    assert err < 1e-13
    # and the constant-tau result is visibly different on this state
    F2c = orlbm.run(F0, SPH, 0.75, 2, cfl=cfl, force=force)
    assert rel(F2, F2c) > 1e-4


def test_eta_s_folded_stencil():
    nx, ny = 40, 24
    F0 = _hot_random(nx, ny, seed=12)
    lat = rl.Lattice(nx, ny, 0.7, stencil="SPH26_ZFOLD", storage="F64",
                     forcing=rl.Forcing(2e-3, 1.0, 3.0, 9))
    lat.set_relaxation("eta_s")
    lat.set_populations(dev(fold(F0)))
    lat.step(2)
    F2 = unfold(host(lat.populations()))
    F2o = orlbm.run(F0, SPH, 0.7, 2, force=dict(amplitude=2e-3, k_lo=1.0, k_hi=3.0, seed=9),
                    eta_s=True)
    assert rel(F2, F2o) < 1e-13


@pytest.mark.parametrize("storage", ["F32", "F16S"])
def test_eta_s_kernel_forms_bitwise(storage):
    nx, ny = 130, 37
    e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=4)
    e = e * np.linspace(0.7, 1.6, nx)[None, :]
    fr = rl.Forcing(1e-4, 2.0, 5.0, 3)
    ref = None
    forms = [("tile", 1), ("tile", 4), ("staged", 4), ("march", 0), ("march", 3),
             ("march2", 0), ("march2", 4)]
    if storage == "F16S":
        forms += [("march_pairs", 0), ("march_pairs", 3)]
    for kind, param in forms:
        lat = rl.Lattice(nx, ny, 0.56, storage=storage, forcing=fr)
        lat.set_relaxation("eta_s")
        lat.set_kernel(kind, param)
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(5)
        F = host(lat.populations())
        if ref is None:
            ref = F
        else:
            assert np.array_equal(F, ref), (kind, param)


def test_eta_s_forced512_short_horizon_f64():
    """512 x 512 forced workload with a hot half (eps 1 -> 2 across x) and the
    constant-eta/s mode: 3 steps, fields within 1e-12 of the oracle."""
    n = 512
    e, bx, by = workloads.noisy_rest(n, n, 0.005, seed=1)
    e = e * (1.0 + 0.5 * (1.0 + np.sin(2 * np.pi * np.arange(n) / n)))[None, :]
    lat = rl.Lattice(n, n, 0.55, storage="F64", forcing=rl.Forcing(1e-5, 4.0, 6.0, 2))
    lat.set_relaxation("eta_s")
    lat.set_state(dev(e), dev(bx), dev(by))
    lat.step(3)
    Fo = orlbm.run(orlbm.set_state(e, bx, by, SPH), SPH, 0.55, 3,
                   force=dict(amplitude=1e-5, k_lo=4.0, k_hi=6.0, seed=2), eta_s=True)
    errs = field_errors(gpu_fields(lat), odiag.fields(Fo, SPH, 1.0))
    say("eta_s forced512", errs)
    assert max(errs.values()) < 1e-12


def test_eta_s_checkpoint_and_ensemble():
    n = 48
    e, bx, by = workloads.noisy_rest(n, n, 0.01, seed=8)
    e = e * 1.5
    fr = rl.Forcing(1e-4, 2.0, 4.0, 12)
    a = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    a.set_relaxation("eta_s")
    a.set_state(dev(e), dev(bx), dev(by))
    a.step(4)
    blob = a.save()
    a.step(5)
    b = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    with pytest.raises(rl.RlbmError):
        b.load(blob)                       # constant-tau lattice: other configuration
    b.set_relaxation("eta_s")
    b.load(blob)
    b.step(5)
    assert np.array_equal(host(a.populations()), host(b.populations()))
    # the same lattice inside an ensemble (realization 0) evolves identically
    ens = rl.Ensemble([(n, n), (64, 32)], [0.6, 0.7], storage="F32",
                      forcings=[rl.Forcing(1e-4, 2.0, 4.0, 12), rl.Forcing(1e-4, 2.0, 4.0, 1)])
    ens.set_relaxation("eta_s")
    ens.set_state(0, dev(e), dev(bx), dev(by))
    e2, bx2, by2 = workloads.noisy_rest(32, 64, 0.01, seed=2)
    ens.set_state(1, dev(e2), dev(bx2), dev(by2))
    ens.step(9)
    c = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    c.set_relaxation("eta_s")
    c.set_state(dev(e), dev(bx), dev(by))
    c.step(9)
    assert np.array_equal(host(ens.populations(0)), host(c.populations()))
