"""The stirring-force term of the reduced-precision forms against the oracle.

The FP32 and 16-bit storage forms build the force field with FP32 arithmetic
(force table per row, synthesis across each row); these tests isolate that
part of the step and compare it with the FP64 oracle (Sec. III C force term,
App. B projection, Sec. V forcing recipe) at bounds that a wrong force would
exceed by orders of magnitude (``tolerances.py``; the CPU test
``test_tolerance_sensitivity.py`` shows it for a 20 % error).

  * Rest-state probe.  At eps = 1, beta = 0 every population is 1: streaming
    moves uniform planes, the Landau frame is the rest frame and the
    collision leaves F = F_eq = 1, so the stored deviation F - 1 after one
    forced step is the force increment itself, dt F . v_q.  Checked at sampled
    sites of the full-size workloads (2048^2, shell [8, 12]; 8192^2, shell
    [32, 40], 41 table rows) in every storage form and in the kernel forms the
    benchmark runs, relative to the largest increment (FP32), or at the
    storage rounding of the increment itself (F16S, BF16S).
  * Strong forcing.  Random non-equilibrium populations on a 128^2 lattice
    driven on the shell [32, 40] (905 modes, |kx| up to 40) at amplitude 3e-3,
    so the force term is a large part of the update: one step (two for the
    two-step form) against the oracle, every population.
"""
import numpy as np
import pytest

import paper_2101_06187_amd as rl
from oracle import rlbm as orlbm
from oracle import stencil as ostencil
import workloads

from gpu_helpers import (dev, host, lib_to_oracle, oracle_step_at, oracle_to_lib,
                         oracle_two_steps_at, say)
from tolerances import one_step_bound, rest_force_bound

pytestmark = pytest.mark.gpu

SPH = ostencil.sph26()

C3 = dict(n=2048, shell=(8.0, 12.0), amp=1e-5, tau=0.52)
C5 = dict(n=8192, shell=(32.0, 40.0), amp=2e-6, tau=0.505)


def probe_sites(n, count, seed):
    """Random sites plus the columns where the cosine recurrence across a row
    is least accurate (x near 0 and near n / 2) and the four corners."""
    g = np.random.Generator(np.random.Philox(seed))
    xs = list(g.integers(0, n, count))
    ys = list(g.integers(0, n, count))
    for x in (0, 1, 2, n // 2 - 1, n // 2, n // 2 + 1, n - 1):
        xs.append(x)
        ys.append(int(g.integers(0, n)))
    xs += [0, n - 1, 0, n - 1]
    ys += [0, 0, n - 1, n - 1]
    return np.array(xs), np.array(ys)


def sample(F_dev, xs, ys):
    import torch
    t = F_dev[:, torch.as_tensor(ys, device="cuda:0"), torch.as_tensor(xs, device="cuda:0")]
    return host(t)


@pytest.mark.parametrize("cfg,storage,form", [
    (C3, "F32", None), (C3, "F32", ("march2", 18)), (C3, "F16S", None),
    (C3, "F16S", ("march_pairs", 0)), (C3, "BF16S", None), (C3, "BF16S", ("march_pairs", 0)),
    (C3, "F32", ("tile", 4)),
    (C5, "F32", None), (C5, "F32", ("march2", 24)), (C5, "F16S", ("march_pairs", 0)),
    (C5, "F16S", None), (C5, "BF16S", None),
])
def test_rest_state_force_probe(cfg, storage, form):
    import torch
    n, (klo, khi), amp, tau = cfg["n"], cfg["shell"], cfg["amp"], cfg["tau"]
    steps = 2 if form is not None and form[0] == "march2" else 1
    say("rest probe", n, storage, form, "steps", steps)
    fr = rl.Forcing(amp, klo, khi, 2)
    lat = rl.Lattice(n, n, tau, storage=storage, forcing=fr)
    if form is not None:
        lat.set_kernel(*form)
    one = torch.ones((n, n), dtype=torch.float64, device="cuda:0")
    zero = torch.zeros_like(one)
    lat.set_state(one, zero, zero)
    del one, zero
    lat.step(steps)
    assert lat.check() == rl.OK
    xs, ys = probe_sites(n, 200, seed=n + 7)
    F = lat.populations()
    got = lib_to_oracle(sample(F, xs, ys)) - 1.0
    del F
    lat.close()
    torch.cuda.empty_cache()
    force = dict(amplitude=amp, k_lo=klo, k_hi=khi, seed=2)
    w = 2 * steps + 1
    ones = np.ones((26, len(xs), w, w))
    if steps == 1:
        want = oracle_step_at(ones, SPH, tau, 1.0, force=force, step_index=0,
                              sites=(xs, ys), nxy=(n, n))
    else:
        want = oracle_two_steps_at(ones, SPH, tau, 1.0, force, 0, (xs, ys), (n, n))
    want -= 1.0
    d = np.abs(got - want)
    bound = rest_force_bound(storage, want)
    say("max |dF - dF_oracle|", d.max(), "max |dF|", np.abs(want).max(),
        "rel", d.max() / np.abs(want).max(), "worst bound ratio", (d / bound).max())
    assert np.all(d <= bound)


@pytest.mark.parametrize("storage,form", [
    ("F32", ("tile", 4)), ("F32", ("march", 0)), ("F32", ("march2", 6)), ("F32", ("staged", 4)),
    ("F16S", ("tile", 4)), ("F16S", ("march_pairs", 0)), ("F16S", ("march", 0)),
    ("BF16S", ("tile", 4)), ("BF16S", ("march_pairs", 0)),
])
def test_strong_forcing_one_step(storage, form):
    n, tau, amp = 128, 0.56, 3e-3
    force = dict(amplitude=amp, k_lo=32.0, k_hi=40.0, seed=11)
    steps = 2 if form[0] == "march2" else 1
    say("strong forcing", storage, form, "steps", steps)
    F0 = workloads.random_populations(SPH.v, n, n, seed=31, spread=0.3)
    lat = rl.Lattice(n, n, tau, storage=storage,
                     forcing=rl.Forcing(amp, force["k_lo"], force["k_hi"], force["seed"]))
    lat.set_kernel(*form)
    lat.set_populations(dev(oracle_to_lib(F0)))
    F0s = lib_to_oracle(host(lat.populations()))        # the stored (rounded) inputs
    lat.step(steps)
    assert lat.check() == rl.OK
    got = lib_to_oracle(host(lat.populations()))
    want = orlbm.run(F0s, SPH, tau, steps, force=force)
    # the force increment is a large part of the update here
    dforce = want - orlbm.run(F0s, SPH, tau, steps)
    scale = max(np.abs(want - 1.0).max(), np.abs(F0s - 1.0).max())
    bound = one_step_bound(storage, want - 1.0, scale, steps)
    d = np.abs(got - want)
    say("max |dF|", d.max(), "max force increment", np.abs(dforce).max(),
        "worst bound ratio", (d / bound).max())
    # a 20 % error of the force term would exceed the bound at most populations
    assert np.mean(0.2 * np.abs(dforce) > bound) > 0.5
    assert np.all(d <= bound)
