"""GPU parity of the HIP RLBM step against the FP64 oracle, through the C ABI.

Tolerances (normwise, see gpu_helpers.field_errors):
  F64 storage  -- 1e-12 on every field and on the populations (both sides
                  FP64; differences come only from rounding order, FMA
                  contraction and the Newton vs eigen-solver Landau routes);
  F32 storage  -- FP32 arithmetic and storage: populations after one step from
                  identical inputs within 32 units in the last place of the
                  largest |F - 1| (tolerances.one_step_bound);
  F16S/BF16S   -- the same plus half a unit in the last place of the new
                  deviation F - 1 in FP16 / BF16 (the storage rounding).
"""
import numpy as np
import pytest

import paper_2101_06187_amd as rl
from oracle import diagnostics as odiag
from oracle import rlbm as orlbm
from oracle import stencil as ostencil
import workloads

from gpu_helpers import (dev, field_errors, gather_patches, gpu_fields, host, lib_to_oracle,
                         oracle_step_at, oracle_to_lib, oracle_two_steps_at, rel, sample_sites,
                         say)
from tolerances import one_step_bound

pytestmark = pytest.mark.gpu

SPH = ostencil.sph26()


def _oracle_fields(F_or, st, cfl=1.0):
    e, bx, by, T6 = odiag.fields(F_or, st, cfl)
    return e, bx, by, T6


@pytest.mark.parametrize("storage", ["F64", "F32"])
def test_set_state_matches_oracle_equilibrium(storage):
    say("set_state", storage)
    e, bx, by = workloads.noisy_rest(40, 70, 0.05, seed=3)
    lat = rl.Lattice(70, 40, 0.7, storage=storage)
    lat.set_state(dev(e), dev(bx), dev(by))
    F = lib_to_oracle(host(lat.populations()))
    Fo = orlbm.set_state(e, bx, by, SPH)
    tol = 1e-15 if storage == "F64" else 1e-7
    assert rel(F, Fo) < tol
    errs = field_errors(gpu_fields(lat), _oracle_fields(Fo, SPH))
    say(errs)
    assert max(errs.values()) < (1e-12 if storage == "F64" else 1e-6)


@pytest.mark.parametrize("shape", [(5, 3), (130, 5), (64, 9), (67, 2)])
@pytest.mark.parametrize("forced", [False, True])
@pytest.mark.parametrize("cfl", [1.0, 0.8])
def test_one_step_random_populations_f64(shape, forced, cfl):
    """Random (non-equilibrium, z-mirror-symmetric) populations on small and
    ragged lattices: one step, every population, against the oracle."""
    nx, ny = shape
    say("one step", shape, forced, cfl)
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=nx * 7 + ny, spread=0.3)
    force = dict(amplitude=3e-3, k_lo=1.0, k_hi=2.3, seed=5) if forced else None
    if forced and (nx < 6 or ny < 6):
        force = dict(amplitude=3e-3, k_lo=1.0, k_hi=1.0, seed=5)
        if nx < 3 or ny < 3:
            pytest.skip("lattice too small for a k = 1 forcing mode")
    fr = rl.Forcing(force["amplitude"], force["k_lo"], force["k_hi"], force["seed"]) if force else None
    lat = rl.Lattice(nx, ny, 0.62, storage="F64", cfl=cfl, forcing=fr)
    lat.set_populations(dev(oracle_to_lib(F0)))
    lat.step(1)
    F1 = lib_to_oracle(host(lat.populations()))
    F1o = orlbm.step(F0, SPH, 0.62, cfl, force, 0)
    err = rel(F1, F1o)
    say("populations err", err)
    assert err < 1e-13
    assert lat.check() == rl.OK


def test_shear_wave_parity_and_decay():
    """Shear-wave workload (64 x 64, tau 1, unforced): 200 steps compared
    field by field with the oracle; 1000 steps on the GPU must decay at the
    linear-theory rate and conserve T^{0 mu}."""
    n = 64
    e, bx, by = workloads.shear_wave(n, 0.01)
    lat = rl.Lattice(n, n, 1.0, storage="F64")
    lat.set_state(dev(e), dev(bx), dev(by))
    c0 = lat.conserved()
    lat.step(200)
    Fo = orlbm.run(orlbm.set_state(e, bx, by, SPH), SPH, 1.0, 200)
    errs = field_errors(gpu_fields(lat), _oracle_fields(Fo, SPH))
    say("shear 200 steps", errs)
    assert max(errs.values()) < 1e-12
    a200 = np.abs(np.fft.rfft(host(lat.fields()[1])[:, 0])[1])
    lat.step(800)
    a1000 = np.abs(np.fft.rfft(host(lat.fields()[1])[:, 0])[1])
    from test_oracle_shear_wave import shear_eigenvalue
    lam = abs(shear_eigenvalue(SPH, 1.0, 2 * np.pi / n))
    rate = (a1000 / a200) ** (1 / 800)
    say("decay rate", rate, "linear theory", lam)
    assert abs(rate / lam - 1) < 1e-6
    c1 = lat.conserved()
    say("conservation drift", c1 - c0)
    assert abs(c1[0] - c0[0]) < 1e-13 * c0[0]
    assert np.abs(c1[1:] - c0[1:]).max() < 1e-13 * c0[0]


def _forced512(storage, steps):
    n = 512
    e, bx, by = workloads.noisy_rest(n, n, 0.005, seed=1)
    fr = rl.Forcing(1e-5, 4.0, 6.0, 2)
    lat = rl.Lattice(n, n, 0.55, storage=storage, forcing=fr)
    lat.set_state(dev(e), dev(bx), dev(by))
    lat.step(steps)
    F = orlbm.set_state(e, bx, by, SPH)
    F = orlbm.run(F, SPH, 0.55, steps,
                  force=dict(amplitude=1e-5, k_lo=4.0, k_hi=6.0, seed=2))
    return lat, F


def test_forced512_short_horizon_f64():
    """512 x 512 forced workload (tau 0.55, shell [4, 6], A = 1e-5, seeds 1/2):
    3 steps, all fields within 1e-12 of the oracle."""
    lat, Fo = _forced512("F64", 3)
    errs = field_errors(gpu_fields(lat), _oracle_fields(Fo, SPH))
    say("forced512 F64", errs)
    assert max(errs.values()) < 1e-12
    assert rel(lib_to_oracle(host(lat.populations())), Fo) < 1e-13


@pytest.mark.parametrize("storage,tol_eps,tol_beta",
                         [("F32", 1e-6, 2e-4), ("F16S", 5e-5, 2e-2), ("BF16S", 5e-4, 1e-1)])
def test_forced512_short_horizon_reduced_storage(storage, tol_eps, tol_beta):
    """The same workload with reduced population storage: stated field error."""
    lat, Fo = _forced512(storage, 3)
    errs = field_errors(gpu_fields(lat), _oracle_fields(Fo, SPH))
    say("forced512", storage, errs)
    assert errs["eps"] < tol_eps
    assert errs["beta_x"] < tol_beta and errs["beta_y"] < tol_beta


@pytest.mark.parametrize("storage,n,shell,amp,tau,form", [
    ("F32", 2048, (8.0, 12.0), 1e-5, 0.52, None),
    ("F16S", 2048, (8.0, 12.0), 1e-5, 0.52, None),
    ("BF16S", 2048, (8.0, 12.0), 1e-5, 0.52, None),
    ("BF16S", 2048, (8.0, 12.0), 1e-5, 0.52, ("march_pairs", 0)),
    ("F32", 8192, (32.0, 40.0), 2e-6, 0.505, None),
    ("F16S", 8192, (32.0, 40.0), 2e-6, 0.505, None),
    ("F16S", 8192, (32.0, 40.0), 2e-6, 0.505, ("march_pairs", 0)),
])
def test_full_size_sampled_one_step(storage, n, shell, amp, tau, form):
    """Full-size workloads in the benchmark's launch configurations (the
    library's default form, and the paired form the benchmark's autotuner
    picks for 16-bit storage at 8192^2): after a few steps, one more step is
    checked at sampled sites (incl. the four corners) against the oracle
    applied to the 3x3 neighbourhood."""
    import torch
    say("full size", storage, n, form)
    sigma, seed = (0.005, 1) if n == 2048 else (0.002, 3)
    e, bx, by = workloads.noisy_rest(n, n, sigma, seed)
    fr = rl.Forcing(amp, shell[0], shell[1], 2)
    lat = rl.Lattice(n, n, tau, storage=storage, forcing=fr)
    if form is not None:
        lat.set_kernel(*form)
    lat.set_graph_chunk(8)
    lat.set_state(dev(e), dev(bx), dev(by))
    del e, bx, by
    lat.step(8)
    xs, ys = sample_sites(n, n, 48, seed=n)
    F_before = lat.populations()
    P = gather_patches(F_before, xs, ys)
    del F_before
    torch.cuda.empty_cache()
    lat.step(1)
    F_after = lat.populations()
    got = host(F_after[:, torch.as_tensor(ys, device="cuda:0"), torch.as_tensor(xs, device="cuda:0")])
    del F_after
    torch.cuda.empty_cache()
    P_or = lib_to_oracle(P.reshape(P.shape[0], -1)).reshape(P.shape)
    want = oracle_step_at(P_or, SPH, tau, 1.0,
                          force=dict(amplitude=amp, k_lo=shell[0], k_hi=shell[1], seed=2),
                          step_index=8, sites=(xs, ys), nxy=(n, n))
    got_or = lib_to_oracle(got)
    d = np.abs(got_or - want)
    scale = max(np.abs(want - 1.0).max(), np.abs(P_or - 1.0).max())
    bound = one_step_bound(storage, want - 1.0, scale)
    say("max |dF|", d.max(), "max bound", bound.max(), "worst ratio", (d / bound).max())
    assert np.all(d <= bound)
    assert lat.check() == rl.OK
    lat.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,shell,amp,tau,seg", [
    (2048, (8.0, 12.0), 1e-5, 0.52, 12),
    (8192, (32.0, 40.0), 2e-6, 0.505, 16),
])
def test_full_size_sampled_two_step_form(n, shell, amp, tau, seg):
    """The two-step form at full size with FP32 storage, as the benchmark's
    autotuner runs it: after 8 steps (4 launches), one more launch is checked
    at sampled sites (incl. the four corners) against two oracle steps on the
    5x5 neighbourhood.  Bound: twice the one-step bound."""
    import torch
    say("full size two-step", n, seg)
    sigma, seed = (0.005, 1) if n == 2048 else (0.002, 3)
    e, bx, by = workloads.noisy_rest(n, n, sigma, seed)
    fr = rl.Forcing(amp, shell[0], shell[1], 2)
    lat = rl.Lattice(n, n, tau, storage="F32", forcing=fr)
    lat.set_kernel("march2", seg)
    lat.set_graph_chunk(8)
    lat.set_state(dev(e), dev(bx), dev(by))
    del e, bx, by
    lat.step(8)
    assert lat.kernel() == ("march2", seg)
    xs, ys = sample_sites(n, n, 48, seed=n + 1)
    F_before = lat.populations()
    P = gather_patches(F_before, xs, ys, radius=2)
    del F_before
    torch.cuda.empty_cache()
    lat.step(2)
    F_after = lat.populations()
    got = host(F_after[:, torch.as_tensor(ys, device="cuda:0"), torch.as_tensor(xs, device="cuda:0")])
    del F_after
    torch.cuda.empty_cache()
    P_or = lib_to_oracle(P.reshape(P.shape[0], -1)).reshape(P.shape)
    want = oracle_two_steps_at(P_or, SPH, tau, 1.0,
                               dict(amplitude=amp, k_lo=shell[0], k_hi=shell[1], seed=2),
                               8, (xs, ys), (n, n))
    d = np.abs(lib_to_oracle(got) - want)
    scale = max(np.abs(want - 1.0).max(), np.abs(P_or - 1.0).max())
    bound = one_step_bound("F32", want - 1.0, scale, steps=2)
    say("max |dF|", d.max(), "bound", bound.max())
    assert np.all(d <= bound)
    assert lat.check() == rl.OK
    lat.close()


@pytest.mark.parametrize("storage", ["F64", "F32", "F16S", "BF16S"])
@pytest.mark.parametrize("shape", [(96, 104), (130, 37)])
def test_kernel_form_and_shape_do_not_change_results(storage, shape):
    """Per-site arithmetic is independent of the kernel form (tile / row
    marching / two-step row marching) and of the launch shape (tile height,
    segment length): bitwise, also on a ragged lattice whose last strip is 2
    columns wide, over 5 steps (two pairs and one single step for the
    two-step form)."""
    nx, ny = shape
    e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=4)
    fr = rl.Forcing(1e-4, 2.0, 5.0, 3)
    ref = None
    for kind, param in [("tile", 1), ("tile", 2), ("tile", 4), ("tile", 8), ("staged", 4),
                        ("march", 0), ("march", 1), ("march", 3), ("march", 16), ("march", 500),
                        ("march2", 0), ("march2", 1), ("march2", 3), ("march2", 16),
                        ("march2", 500)]:
        lat = rl.Lattice(nx, ny, 0.56, storage=storage, forcing=fr)
        lat.set_kernel(kind, param)
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(5)
        F = host(lat.populations())
        if ref is None:
            ref = F
        else:
            assert np.array_equal(F, ref), (kind, param)


@pytest.mark.parametrize("kind", ["tile", "staged", "march", "march2"])
def test_both_kernel_forms_match_oracle(kind):
    """Random populations on a ragged lattice, forced, cfl < 1, both forms."""
    nx, ny = 67, 13
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=77, spread=0.3)
    force = dict(amplitude=3e-3, k_lo=1.0, k_hi=3.0, seed=8)
    lat = rl.Lattice(nx, ny, 0.6, storage="F64", cfl=0.9,
                     forcing=rl.Forcing(3e-3, 1.0, 3.0, 8))
    lat.set_kernel(kind, 2 if kind == "tile" else 4)
    lat.set_populations(dev(oracle_to_lib(F0)))
    lat.step(2)
    F2 = lib_to_oracle(host(lat.populations()))
    F2o = orlbm.run(F0, SPH, 0.6, 2, cfl=0.9, force=force)
    assert rel(F2, F2o) < 1e-13


def test_graph_replay_matches_direct_launches():
    """Captured-graph stepping equals direct launches bitwise, replay after
    replay, with eager work and synchronisations in between."""
    import torch
    n = 128
    e, bx, by = workloads.noisy_rest(n, n, 0.01, seed=6)
    fr = rl.Forcing(1e-4, 3.0, 6.0, 9)
    a = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    b = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    for lat in (a, b):
        lat.set_state(dev(e), dev(bx), dev(by))
    b.set_graph_chunk(4)
    for rep in range(4):
        a.step(8)
        b.step(8)          # two graph replays
        junk = torch.randn(1000, device="cuda:0").sum()   # eager work in between
        torch.cuda.synchronize()
        assert np.array_equal(host(a.populations()), host(b.populations())), rep
        assert a.steps == b.steps == 8 * (rep + 1)
    del junk


@pytest.mark.parametrize("chunk", [4, 5])
def test_two_step_form_graph_replay_and_checkpoint(chunk):
    """The two-step form through captured graphs of even and odd step
    counts, and a checkpoint taken between pairs, against one-step launches
    of the tile form: bitwise."""
    import torch
    n = 96
    e, bx, by = workloads.noisy_rest(n, n, 0.01, seed=6)
    fr = rl.Forcing(1e-4, 3.0, 6.0, 9)
    a = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    b = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    a.set_kernel("tile", 4)
    b.set_kernel("march2", 0)
    for lat in (a, b):
        lat.set_state(dev(e), dev(bx), dev(by))
    b.set_graph_chunk(chunk)
    for rep in range(3):
        a.step(2 * chunk + 1)
        b.step(2 * chunk + 1)      # two graph replays and one single step
        junk = torch.randn(1000, device="cuda:0").sum()
        torch.cuda.synchronize()
        assert np.array_equal(host(a.populations()), host(b.populations())), rep
    blob = b.save()
    b.step(7)
    c = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    c.set_kernel("march2", 3)
    c.load(blob)
    c.step(7)
    a.step(7)
    assert np.array_equal(host(c.populations()), host(b.populations()))
    assert np.array_equal(host(a.populations()), host(b.populations()))
    assert b.check() == rl.OK
    del junk


def test_full_ensemble_in_benchmark_configuration():
    """The 256-lattice ensemble workload (sides 64/128/256, tau in [0.51, 0.8],
    FP32, forcing shell [2, 4] with counter word r) in the form the
    benchmark's autotuner picks for it (two-step, 8-row segments): after 4
    steps, realizations of every side against the oracle, every population
    (4 x the one-step FP32 bound)."""
    import torch
    spec = workloads.ensemble()
    sizes = [(n, n) for n, _ in spec]
    taus = [t for _, t in spec]
    frs = [rl.Forcing(1e-5, 2.0, 4.0, r) for r in range(len(spec))]
    ens = rl.Ensemble(sizes, taus, storage="F32", forcings=frs)
    inits = []
    for r, (n, _) in enumerate(spec):
        e, bx, by = workloads.noisy_rest(n, n, 0.005, seed=r)
        inits.append((e, bx, by))
        ens.set_state(r, dev(e), dev(bx), dev(by))
    ens.set_kernel("march2", 8)
    ens.set_graph_chunk(2)
    ens.step(4)
    assert ens.check() == rl.OK
    picked = {}
    for r, (n, _) in enumerate(spec):           # the first realization of each side, and the last
        picked.setdefault(n, r)
    for r in sorted(set(picked.values()) | {len(spec) - 1}):
        n, tau = spec[r]
        F0r = orlbm.set_state(*inits[r], SPH)
        F = orlbm.run(F0r, SPH, tau, 4,
                      force=dict(amplitude=1e-5, k_lo=2.0, k_hi=4.0, seed=r), realization=r)
        got = lib_to_oracle(host(ens.populations(r)))
        d = float(np.abs(got - F).max())
        # four steps from the rounded initial state: 4 x the one-step bound at
        # the initial scale, plus the FP32 rounding of that state
        scale = max(np.abs(F - 1.0).max(), np.abs(F0r - 1.0).max())
        bound = one_step_bound("F32", F - 1.0, scale, steps=5).max()
        say("ensemble", r, n, tau, "max |dF|", d, "bound", bound)
        assert d <= bound
    ens.close()
    torch.cuda.empty_cache()


def test_two_step_form_default_segment():
    """Parameter 0 of the two-step form is a 12-row segment (its measured best
    on lattices much larger than the caches), also on a lattice shorter than
    that, which then runs as one segment per strip."""
    for ny in (64, 8):
        lat = rl.Lattice(256, ny, 0.6, storage="F32")
        lat.set_kernel("march2", 0)
        assert lat.kernel() == ("march2", 12)
        lat.close()


def test_autotune_keeps_results_bitwise():
    """The autotuner (lattice and ensemble) tries every form while stepping;
    the state after it equals plain tile-form stepping by the same count."""
    n = 160
    e, bx, by = workloads.noisy_rest(n, n, 0.01, seed=3)
    fr = rl.Forcing(1e-4, 2.0, 5.0, 4)
    lat = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    lat.set_state(dev(e), dev(bx), dev(by))
    form = lat.autotune(3)
    say("autotuned", form, "after", lat.steps, "steps")
    assert form[0] in rl.KERNELS
    ref = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    ref.set_kernel("tile", 4)
    ref.set_state(dev(e), dev(bx), dev(by))
    ref.step(lat.steps)
    lat.step(5)
    ref.step(5)
    assert np.array_equal(host(lat.populations()), host(ref.populations()))
    sizes = [(64, 64), (96, 40)]
    frs = [rl.Forcing(1e-4, 2.0, 4.0, r) for r in range(2)]
    ens = rl.Ensemble(sizes, [0.6, 0.7], storage="F32", forcings=frs)
    singles = [rl.Lattice(nx, ny, t, storage="F32", forcing=rl.Forcing(1e-4, 2.0, 4.0, 0))
               for (nx, ny), t in zip(sizes, [0.6, 0.7])]
    for r, (nx, ny) in enumerate(sizes):
        e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=r)
        ens.set_state(r, dev(e), dev(bx), dev(by))
        if r == 0:
            singles[0].set_state(dev(e), dev(bx), dev(by))
    form = ens.autotune(3)
    say("ensemble autotuned", form, "after", ens.steps, "steps")
    singles[0].step(ens.steps)
    assert np.array_equal(host(ens.populations(0)), host(singles[0].populations()))


def test_checkpoint_resume_is_bitwise():
    n = 64
    e, bx, by = workloads.noisy_rest(n, n, 0.01, seed=8)
    fr = rl.Forcing(1e-4, 2.0, 4.0, 12)
    a = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    a.set_state(dev(e), dev(bx), dev(by))
    a.step(7)
    blob = a.save()
    a.step(9)
    b = rl.Lattice(n, n, 0.6, storage="F32", forcing=fr)
    b.load(blob)
    assert b.steps == 7
    b.step(9)
    assert np.array_equal(host(a.populations()), host(b.populations()))
    c = rl.Lattice(n, n, 0.61, storage="F32", forcing=fr)
    with pytest.raises(rl.RlbmError):
        c.load(blob)


@pytest.mark.parametrize("storage,first,second", [
    ("F32", ("march2", 4), ("tile", 4)),
    ("F32", ("tile", 1), ("march2", 3)),
    ("F16S", ("march2", 4), ("march_pairs", 3)),
    ("BF16S", ("march_pairs", 0), ("march", 2)),
])
def test_checkpoint_resume_across_kernel_forms(storage, first, second):
    """A checkpoint taken by one kernel form after an odd number of steps (the
    two-step form ends with a one-step launch) and resumed by another equals
    uninterrupted stepping bitwise: the state, the step count, the buffer
    parity and the force-table ring carry over between forms."""
    nx, ny = 130, 37
    e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=21)
    fr = rl.Forcing(1e-4, 2.0, 5.0, 14)
    ref = rl.Lattice(nx, ny, 0.58, storage=storage, forcing=fr)
    ref.set_kernel("tile", 4)
    ref.set_state(dev(e), dev(bx), dev(by))
    ref.step(16)
    a = rl.Lattice(nx, ny, 0.58, storage=storage, forcing=fr)
    a.set_kernel(*first)
    a.set_state(dev(e), dev(bx), dev(by))
    a.step(7)
    blob = a.save()
    a.close()
    b = rl.Lattice(nx, ny, 0.58, storage=storage, forcing=fr)
    b.set_kernel(*second)
    b.load(blob)
    assert b.steps == 7
    b.step(9)
    assert np.array_equal(host(b.populations()), host(ref.populations()))


def test_conserved_matches_oracle():
    e, bx, by = workloads.noisy_rest(48, 80, 0.02, seed=2)
    lat = rl.Lattice(80, 48, 0.7, storage="F64")
    lat.set_state(dev(e), dev(bx), dev(by))
    lat.step(3)
    Fo = orlbm.run(orlbm.set_state(e, bx, by, SPH), SPH, 0.7, 3)
    c = lat.conserved()
    co = odiag.conserved(Fo, SPH)
    assert np.abs(c - co).max() < 1e-12 * co[0]


@pytest.mark.parametrize("n", [64, 256])
def test_spectrum_matches_oracle(n):
    e, bx, by = workloads.noisy_rest(n, n, 0.01, seed=5)
    lat = rl.Lattice(n, n, 0.6, storage="F64", forcing=rl.Forcing(1e-4, 2, 4, 1))
    lat.set_state(dev(e), dev(bx), dev(by))
    lat.step(2)
    nb = n
    Ek, Z = lat.spectrum(nb)
    _, gx, gy, _ = gpu_fields(lat)
    Eo, Zo = odiag.spectrum(gx, gy, nb)
    say("spectrum", rel(Ek, Eo), abs(Z - Zo) / Zo)
    assert rel(Ek, Eo) < 1e-12
    assert abs(Z - Zo) < 1e-12 * Zo


@pytest.mark.parametrize("n,band", [(64, (3.5, 6.5)), (256, (6.0, float("inf"))),
                                    (128, (0.0, 0.5)), (64, (100.0, 200.0))])
def test_filtered_velocity_matches_oracle(n, band):
    """Driven-band filter (Sec. V): the GPU fields with the band removed and
    their mean speed against the oracle's filter of the same fields."""
    e, bx, by = workloads.noisy_rest(n, n, 0.01, seed=7)
    lat = rl.Lattice(n, n, 0.6, storage="F64", forcing=rl.Forcing(1e-4, 4, 6, 3))
    lat.set_state(dev(e), dev(bx), dev(by))
    lat.step(2)
    _, gx, gy, _ = gpu_fields(lat)
    fx, fy, speed = lat.filtered_velocity(*band)
    ox, oy, ospeed = odiag.filtered_velocity(gx, gy, *band)
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    say("filter", n, band, np.abs(host(fx) - ox).max() / scale, abs(speed - ospeed) / ospeed)
    assert np.abs(host(fx) - ox).max() < 1e-12 * scale
    assert np.abs(host(fy) - oy).max() < 1e-12 * scale
    assert abs(speed - ospeed) < 1e-12 * ospeed


def test_spectrum_rejects_non_power_of_two():
    lat = rl.Lattice(48, 48, 0.6)
    with pytest.raises(rl.RlbmError) as ex:
        lat.spectrum(10)
    assert ex.value.code == rl.EUNSUPPORTED
    with pytest.raises(rl.RlbmError) as ex:
        lat.filtered_velocity(2.0, 4.0)
    assert ex.value.code == rl.EUNSUPPORTED


def test_unstable_state_is_flagged():
    """Condition forced from the host: a lattice whose populations carry a
    negative energy density; every kernel exits normally, the flag trips."""
    n = 16
    F = -np.ones((26, n, n))
    lat = rl.Lattice(n, n, 0.6, storage="F64")
    lat.set_populations(dev(F))
    assert lat.check() == rl.OK
    lat.step(1)
    assert lat.check() == rl.EUNSTABLE


@pytest.mark.parametrize("storage", ["F64", "F32", "F16S", "BF16S"])
def test_circ8_kernel_forms_are_bitwise_equal(storage):
    """The 8-direction stencil through every kernel form (ragged 130 x 37
    lattice: a 2-column last strip, segments that do not divide 37)."""
    nx, ny = 130, 37
    e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=9)
    fr = rl.Forcing(1e-4, 2.0, 5.0, 6)
    forms = [("tile", 1), ("tile", 4), ("staged", 4), ("march", 0), ("march", 3),
             ("march2", 0), ("march2", 5)]
    if storage in ("F16S", "BF16S"):
        forms += [("march_pairs", 0), ("march_pairs", 3)]
    ref = None
    for kind, param in forms:
        lat = rl.Lattice(nx, ny, 0.6, stencil="CIRC8", storage=storage, forcing=fr)
        lat.set_kernel(kind, param)
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(7)
        assert lat.check() == rl.OK
        F = host(lat.populations())
        lat.close()
        if ref is None:
            ref = F
        else:
            assert np.array_equal(F, ref), (kind, param)


def test_circ8_parity():
    st = ostencil.circ8()
    F0 = workloads.random_populations(st.v, 20, 36, seed=3, spread=0.3, z_mirror=False)
    lat = rl.Lattice(36, 20, 0.66, stencil="CIRC8", storage="F64",
                     forcing=rl.Forcing(2e-3, 1.0, 3.0, 4))
    lat.set_populations(dev(oracle_to_lib(F0, "CIRC8")))
    lat.step(2)
    F2 = lib_to_oracle(host(lat.populations()), "CIRC8")
    F2o = orlbm.run(F0, st, 0.66, 2, force=dict(amplitude=2e-3, k_lo=1.0, k_hi=3.0, seed=4))
    assert rel(F2, F2o) < 1e-13


@pytest.mark.parametrize("kind", ["auto", "staged", "march2"])
def test_ensemble_matches_oracle(kind):
    """Independent lattices of different sizes and tau in one persistent
    launch per step (or per pair of steps); realization r draws its force
    with counter word r."""
    sizes = [(64, 64), (128, 64), (64, 128), (96, 40)]
    taus = [0.55, 0.7, 0.61, 0.8]
    frs = [rl.Forcing(1e-4, 2.0, 4.0, r) for r in range(4)]
    ens = rl.Ensemble(sizes, taus, storage="F64", forcings=frs)
    if kind != "auto":
        ens.set_kernel(kind, 4 if kind == "staged" else 5)
    inits = []
    for r, (nx, ny) in enumerate(sizes):
        e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=r)
        inits.append((e, bx, by))
        ens.set_state(r, dev(e), dev(bx), dev(by))
    ens.step(3)
    for r, (nx, ny) in enumerate(sizes):
        F = orlbm.set_state(*inits[r], SPH)
        F = orlbm.run(F, SPH, taus[r], 3,
                      force=dict(amplitude=1e-4, k_lo=2.0, k_hi=4.0, seed=r), realization=r)
        got = lib_to_oracle(host(ens.populations(r)))
        say("ensemble", r, rel(got, F))
        assert rel(got, F) < 1e-13
    assert ens.check() == rl.OK


@pytest.mark.parametrize("storage", ["F16S", "BF16S"])
@pytest.mark.parametrize("shape,cfl,forced", [((96, 104), 1.0, True), ((130, 37), 1.0, True),
                                              ((38, 9), 0.9, True), ((200, 66), 0.9, False),
                                              ((256, 20), 1.0, True), ((2, 33), 0.9, False),
                                              ((4, 5), 1.0, False), ((124, 7), 1.0, True),
                                              ((126, 2), 1.0, False), ((248, 12), 0.9, True),
                                              ((250, 6), 1.0, True)])
def test_paired_form_is_bitwise_equal_to_tile_form(storage, shape, cfl, forced):
    """The paired marching form (two columns per lane, 128-column strips) on
    ragged lattices -- the last strip 2 to 126 columns wide, a single strip
    narrower than the wavefront's lanes, lattices of 2 and 4 columns or of 2
    rows, one or two whole strips -- equals the tile form bit for bit
    over 5 steps, for several segment lengths."""
    nx, ny = shape
    e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=nx + ny)
    # the driven shell 2 <= |k| <= 5, narrowed to stay below the Nyquist wave
    # number of the smallest lattices
    fr = rl.Forcing(1e-4, 2.0, min(5.0, min(nx, ny) // 2 - 1), 3) if forced else None

    def run(kind, param):
        lat = rl.Lattice(nx, ny, 0.56, storage=storage, cfl=cfl, forcing=fr)
        lat.set_kernel(kind, param)
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(5)
        assert lat.kernel() == (kind, param) or param == 0
        assert lat.check() == rl.OK
        return host(lat.populations())

    ref = run("tile", 4)
    # segment lengths of every remainder mod 3 (the row loop is unrolled three times)
    for param in (0, 1, 2, 3, 4, 16, 500):
        assert np.array_equal(run("march_pairs", param), ref), param


@pytest.mark.parametrize("nx", [3, 37, 129])
def test_paired_form_rejected_for_odd_nx(nx):
    """A pair of columns never straddles the periodic wrap: odd nx is refused
    (EUNSUPPORTED), and the autotuner passes over the form."""
    lat = rl.Lattice(nx, 8, 0.6, storage="F16S")
    with pytest.raises(rl.RlbmError) as ex:
        lat.set_kernel("march_pairs", 0)
    assert ex.value.code == rl.EUNSUPPORTED
    kind, _ = lat.autotune(2)
    assert kind != "march_pairs"


def test_paired_form_rejected_for_32_and_64_bit_storage():
    for storage in ("F64", "F32"):
        lat = rl.Lattice(64, 64, 0.7, storage=storage)
        with pytest.raises(rl.RlbmError) as ex:
            lat.set_kernel("march_pairs", 0)
        assert ex.value.code == rl.EUNSUPPORTED


def test_paired_form_in_an_ensemble():
    """16-bit ensemble of uneven lattices in the paired form equals the tile form."""
    sizes = [(64, 64), (130, 64), (64, 128), (96, 40)]
    taus = [0.55, 0.7, 0.61, 0.8]
    frs = [rl.Forcing(1e-4, 2.0, 4.0, r) for r in range(4)]
    out = []
    for kind, param in (("tile", 4), ("march_pairs", 5)):
        ens = rl.Ensemble(sizes, taus, storage="F16S", forcings=frs)
        ens.set_kernel(kind, param)
        for r, (nx, ny) in enumerate(sizes):
            e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=r)
            ens.set_state(r, dev(e), dev(bx), dev(by))
        ens.step(3)
        out.append([host(ens.populations(r)) for r in range(len(sizes))])
        assert ens.check() == rl.OK
    for a, b in zip(*out):
        assert np.array_equal(a, b)
