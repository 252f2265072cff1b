"""GPU parity of the z-folded SPH26 path (17 stored populations) against the
FP64 oracle's full 26-direction step, through the C ABI.

The fold is exact on z-mirror-symmetric states, which every state of the
one-layer lattice is, so the oracle of the folded path is the unfolded oracle:
inputs are folded on the way in and results unfolded on the way out.
Tolerances are those of the unfolded parity tests (FP64: 1e-13 on the
populations after one step; fields 1e-12)."""
import numpy as np
import pytest

import paper_2101_06187_amd as rl
from oracle import diagnostics as odiag
from oracle import rlbm as orlbm
from oracle import stencil as ostencil
import workloads

from gpu_helpers import (dev, field_errors, fold, gather_patches, gpu_fields, host,
                         oracle_step_at, rel, sample_sites, say, unfold)

pytestmark = pytest.mark.gpu

SPH = ostencil.sph26()
FOLD = "SPH26_ZFOLD"


@pytest.mark.parametrize("shape", [(5, 3), (130, 5), (67, 9)])
@pytest.mark.parametrize("forced", [False, True])
@pytest.mark.parametrize("cfl", [1.0, 0.8])
def test_fold_one_step_random_populations_f64(shape, forced, cfl):
    nx, ny = shape
    say("fold one step", shape, forced, cfl)
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=nx * 5 + ny, spread=0.3)
    force = None
    if forced:
        if nx < 3 or ny < 3:
            pytest.skip("lattice too small for a k = 1 forcing mode")
        force = dict(amplitude=3e-3, k_lo=1.0, k_hi=1.0 if min(nx, ny) < 6 else 2.3, seed=5)
    fr = rl.Forcing(force["amplitude"], force["k_lo"], force["k_hi"], force["seed"]) if force else None
    lat = rl.Lattice(nx, ny, 0.62, stencil=FOLD, storage="F64", cfl=cfl, forcing=fr)
    lat.set_populations(dev(fold(F0)))
    lat.step(1)
    F1 = unfold(host(lat.populations()))
    F1o = orlbm.step(F0, SPH, 0.62, cfl, force, 0)
    err = rel(F1, F1o)
    say("populations err", err)
    assert err < 1e-13
    assert lat.check() == rl.OK


def test_fold_set_state_and_shear_wave():
    """Equilibrium initialisation, then 200 unforced steps of the 64 x 64
    shear wave: fields against the oracle."""
    n = 64
    e, bx, by = workloads.shear_wave(n, 0.01)
    lat = rl.Lattice(n, n, 1.0, stencil=FOLD, storage="F64")
    lat.set_state(dev(e), dev(bx), dev(by))
    F0o = orlbm.set_state(e, bx, by, SPH)
    assert rel(unfold(host(lat.populations())), F0o) < 1e-15
    c0 = lat.conserved()
    lat.step(200)
    Fo = orlbm.run(F0o, SPH, 1.0, 200)
    errs = field_errors(gpu_fields(lat), odiag.fields(Fo, SPH, 1.0))
    say("fold shear 200 steps", errs)
    assert max(errs.values()) < 1e-12
    co = odiag.conserved(Fo, SPH)
    c1 = lat.conserved()
    assert np.abs(c1 - co).max() < 1e-12 * co[0]
    assert abs(c1[0] - c0[0]) < 1e-13 * c0[0]


@pytest.mark.parametrize("storage,tol", [("F64", 1e-12), ("F32", 2e-4), ("F16S", 2e-2)])
def test_fold_forced512_short_horizon(storage, tol):
    """512 x 512 forced workload, 3 steps: the folded path against the oracle
    (F64) and against the unfolded path at the same storage (reduced forms:
    same rounding steps on the same values, so the two agree far inside the
    storage tolerance)."""
    n = 512
    e, bx, by = workloads.noisy_rest(n, n, 0.005, seed=1)
    fr = rl.Forcing(1e-5, 4.0, 6.0, 2)
    a = rl.Lattice(n, n, 0.55, stencil=FOLD, storage=storage, forcing=fr)
    b = rl.Lattice(n, n, 0.55, stencil="SPH26", storage=storage, forcing=fr)
    for lat in (a, b):
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(3)
    ga, gb = gpu_fields(a), gpu_fields(b)
    if storage == "F64":
        Fo = orlbm.run(orlbm.set_state(e, bx, by, SPH), SPH, 0.55, 3,
                       force=dict(amplitude=1e-5, k_lo=4.0, k_hi=6.0, seed=2))
        errs = field_errors(ga, odiag.fields(Fo, SPH, 1.0))
        say("fold forced512 F64 vs oracle", errs)
        assert max(errs.values()) < tol
        assert rel(unfold(host(a.populations())), Fo) < 1e-13
    errs = field_errors(ga, gb)
    say("fold vs unfolded", storage, errs)
    assert errs["eps"] < 1e-6 and errs["beta_x"] < tol and errs["beta_y"] < tol


@pytest.mark.parametrize("storage", ["F64", "F32", "F16S"])
def test_fold_kernel_forms_are_bitwise_equal(storage):
    nx, ny = 130, 37
    e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=4)
    fr = rl.Forcing(1e-4, 2.0, 5.0, 3)
    ref = None
    forms = [("tile", 1), ("tile", 4), ("staged", 4), ("march", 0), ("march", 3), ("march", 500),
             ("march2", 0), ("march2", 4)]
    if storage == "F16S":
        forms += [("march_pairs", 0), ("march_pairs", 3), ("march_pairs", 500)]
    for kind, param in forms:
        lat = rl.Lattice(nx, ny, 0.56, stencil=FOLD, storage=storage, forcing=fr)
        lat.set_kernel(kind, param)
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(5)
        F = host(lat.populations())
        if ref is None:
            ref = F
        else:
            assert np.array_equal(F, ref), (kind, param)


@pytest.mark.parametrize("kind", ["tile", "staged", "march"])
def test_fold_full_size_sampled_one_step(kind):
    """2048 x 2048 forced F32 workload, one step in the benchmark's launch
    configuration, checked at sampled sites against the oracle's stages."""
    import torch
    n, tau = 2048, 0.52
    force = dict(amplitude=1e-5, k_lo=8.0, k_hi=12.0, seed=2)
    e, bx, by = workloads.noisy_rest(n, n, 0.005, seed=1)
    lat = rl.Lattice(n, n, tau, stencil=FOLD, storage="F32",
                     forcing=rl.Forcing(1e-5, 8.0, 12.0, 2))
    lat.set_kernel(kind, 0 if kind == "march" else 4)
    lat.set_state(dev(e), dev(bx), dev(by))
    F0 = lat.populations()
    xs, ys = sample_sites(n, n, 64, seed=11)
    P = unfold(gather_patches(F0, xs, ys))
    del F0
    lat.step(1)
    F1 = lat.populations()
    got = unfold(host(F1[:, torch.as_tensor(ys, device="cuda:0"),
                         torch.as_tensor(xs, device="cuda:0")]))
    want = oracle_step_at(P, SPH, tau, 1.0, force, 0, (xs, ys), (n, n))
    err = float(np.abs(got - want).max())
    say("fold 2048 sampled", kind, err)
    assert err < 4e-6
    del F1
    torch.cuda.empty_cache()


def test_fold_ensemble_matches_unfolded():
    sizes = [(64, 64), (96, 40)]
    taus = [0.55, 0.7]
    frs = [rl.Forcing(1e-4, 2.0, 4.0, r) for r in range(2)]
    a = rl.Ensemble(sizes, taus, stencil=FOLD, storage="F64", forcings=frs)
    b = rl.Ensemble(sizes, taus, stencil="SPH26", storage="F64", forcings=frs)
    for r, (nx, ny) in enumerate(sizes):
        e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=r)
        for ens in (a, b):
            ens.set_state(r, dev(e), dev(bx), dev(by))
    a.step(4)
    b.step(4)
    for r in range(2):
        errs = field_errors(tuple(host(t) for t in a.fields(r)),
                            tuple(host(t) for t in b.fields(r)))
        say("fold ensemble", r, errs)
        assert max(errs.values()) < 1e-12
