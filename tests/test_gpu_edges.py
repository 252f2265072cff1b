"""Edge cases of the GPU path against the oracle or against exact expectations:
zero steps, the rest state, the largest lattice side the ABI accepts, the
narrowest lattices of the two-step form (and its refusal below three rows), fast
flows (many Newton passes in the Landau solve), tau close to 1/2, a forcing
shell that holds no lattice mode, a one-lattice ensemble."""
import numpy as np
import pytest

import paper_2101_06187_amd as rl
from oracle import diagnostics as odiag
from oracle import rlbm as orlbm
from oracle import stencil as ostencil
import workloads

from gpu_helpers import dev, field_errors, gpu_fields, host, lib_to_oracle, oracle_to_lib, rel, say

pytestmark = pytest.mark.gpu

SPH = ostencil.sph26()


@pytest.mark.parametrize("kind", ["tile", "staged", "march", "march2"])
def test_zero_steps_change_nothing(kind):
    e, bx, by = workloads.noisy_rest(40, 70, 0.01, seed=1)
    lat = rl.Lattice(70, 40, 0.6, storage="F32", forcing=rl.Forcing(1e-4, 2, 4, 1))
    lat.set_kernel(kind, {"tile": 2, "staged": 4}.get(kind, 0))
    lat.set_state(dev(e), dev(bx), dev(by))
    F0 = host(lat.populations())
    lat.step(0)
    assert lat.steps == 0
    assert np.array_equal(host(lat.populations()), F0)


@pytest.mark.parametrize("storage", ["F64", "F32", "F16S"])
def test_rest_state_stays_stationary(storage):
    """eps = 1, beta = 0 everywhere, unforced: every population stays at its
    equilibrium value to rounding (the equilibrium of eps = 1 is 1 up to the
    last bit of A0), and beta stays exactly zero (plus and minus members of
    every class remain equal, so the momentum sums cancel exactly)."""
    n = 48
    lat = rl.Lattice(n, n, 0.51, storage=storage)
    one, zero = np.ones((n, n)), np.zeros((n, n))
    lat.set_state(dev(one), dev(zero), dev(zero))
    F0 = host(lat.populations())
    lat.step(25)
    F1 = host(lat.populations())
    say("rest drift", storage, np.abs(F1 - F0).max())
    assert np.abs(F1 - F0).max() <= 1e-15
    _, ux, uy, _ = gpu_fields(lat)
    assert np.abs(ux).max() == 0.0 and np.abs(uy).max() == 0.0


@pytest.mark.parametrize("shape", [(65536, 2), (2, 65536), (65536, 3)])
def test_longest_side_one_step(shape):
    """The largest side the ABI accepts (65536), against a side of 2 or 3:
    random populations, one step of every form, against the oracle."""
    nx, ny = shape
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=nx + ny, spread=0.3)
    F1o = orlbm.step(F0, SPH, 0.7, 0.9)
    for kind in ("tile", "staged", "march"):
        lat = rl.Lattice(nx, ny, 0.7, storage="F64", cfl=0.9)
        lat.set_kernel(kind, {"tile": 2, "staged": 4}.get(kind, 0))
        lat.set_populations(dev(oracle_to_lib(F0)))
        lat.step(1)
        err = rel(lib_to_oracle(host(lat.populations())), F1o)
        say("longest side", shape, kind, err)
        assert err < 1e-13
        lat.close()


@pytest.mark.parametrize("storage", ["F16S", "BF16S"])
@pytest.mark.parametrize("shape", [(65536, 2), (2, 65536), (65536, 3)])
def test_longest_side_paired_form(storage, shape):
    """The paired 16-bit form on the largest side the ABI accepts (512
    strips of 128 columns, or one strip of 2 columns over 65536 rows), three
    steps from random populations, bit for bit equal to the tile form; forced
    where the short side leaves a mode below its Nyquist wave number."""
    nx, ny = shape
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=nx + 3 * ny, spread=0.05)
    fr = rl.Forcing(3e-3, 1.0, 1.2, 7) if min(nx, ny) >= 3 else None
    out = []
    for kind, param in (("tile", 2), ("march_pairs", 0)):
        lat = rl.Lattice(nx, ny, 0.7, storage=storage, forcing=fr)
        lat.set_kernel(kind, param)
        lat.set_populations(dev(oracle_to_lib(F0)))
        lat.step(3)
        assert lat.check() == rl.OK
        out.append(host(lat.populations()))
        lat.close()
    say("longest side, paired", storage, shape)
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("shape,forced", [((65536, 3), False), ((130, 3), True), ((70, 4), False),
                                          ((2, 4099), False), ((3, 67), True)])
def test_two_step_form_narrow_lattices(shape, forced):
    """The two-step form on the fewest rows it accepts (its input window
    reaches two rows past a segment on either side, wrapped by one period)
    and on lattices narrower than a strip (every lane's column wrapped).
    Two steps of random populations, one segment, one-row and ragged
    segments, against the oracle."""
    nx, ny = shape
    force = dict(amplitude=3e-3, k_lo=1.0, k_hi=1.4, seed=5) if forced else None
    fr = rl.Forcing(force["amplitude"], force["k_lo"], force["k_hi"], force["seed"]) if forced else None
    F0 = workloads.random_populations(SPH.v, ny, nx, seed=nx + 3 * ny, spread=0.3)
    F2o = orlbm.run(F0, SPH, 0.7, 2, cfl=0.9, force=force)
    for param in (0, 1, 2):
        say("two-step narrow", shape, forced, param)
        lat = rl.Lattice(nx, ny, 0.7, storage="F64", cfl=0.9, forcing=fr)
        lat.set_kernel("march2", param)
        lat.set_populations(dev(oracle_to_lib(F0)))
        lat.step(2)
        err = rel(lib_to_oracle(host(lat.populations())), F2o)
        say("err", err)
        assert err < 1e-13
        assert lat.check() == rl.OK
        lat.close()


@pytest.mark.parametrize("shape,param", [((62 * 8, 40), 4), ((62 * 8 + 3, 37), 3),
                                         ((62 * 5, 24), 3), ((62 * 3 - 1, 50), 5),
                                         ((62 * 2, 9), 2), ((62, 17), 0), ((62 * 9 + 1, 12), 1)])
def test_two_step_form_strip_groups(shape, param):
    """The two-step form's blocks of g adjacent strips x 8 / g segments (g =
    4, 2 or 1, chosen from the padding of strips and segments): lattices of
    1 to 10 strips, ragged last strips and segment counts that do not divide
    into the block, FP32 with forcing, 6 steps (three launches) bitwise equal
    to the tile form; then an ensemble of such lattices at once."""
    nx, ny = shape
    e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=nx + ny)
    fr = rl.Forcing(1e-4, 1.0, min(4.0, ny // 2 - 1), 9)

    def run(kind, p):
        lat = rl.Lattice(nx, ny, 0.57, storage="F32", forcing=fr)
        lat.set_kernel(kind, p)
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(6)
        assert lat.check() == rl.OK
        out = host(lat.populations())
        lat.close()
        return out

    assert np.array_equal(run("march2", param), run("tile", 4)), (shape, param)


def test_two_step_form_strip_groups_in_an_ensemble():
    sizes = [(62 * 8, 40), (124, 9), (62 * 3 - 1, 50), (64, 64), (200, 30)]
    taus = [0.55, 0.6, 0.7, 0.8, 0.65]
    frs = [rl.Forcing(1e-4, 1.0, 3.0, r) for r in range(len(sizes))]
    out = []
    for kind, param in (("tile", 4), ("march2", 3), ("march2", 0)):
        ens = rl.Ensemble(sizes, taus, storage="F32", forcings=frs)
        ens.set_kernel(kind, param)
        for r, (nx, ny) in enumerate(sizes):
            e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=r)
            ens.set_state(r, dev(e), dev(bx), dev(by))
        ens.step(4)
        assert ens.check() == rl.OK
        out.append([host(ens.populations(r)) for r in range(len(sizes))])
        ens.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)


def test_two_step_form_refused_below_three_rows():
    """ny = 2 is below what the two-step form reads: EUNSUPPORTED from the
    lattice and the ensemble; the autotuner leaves it out and keeps a form
    whose results equal the tile form's."""
    nx, ny = 130, 2
    lat = rl.Lattice(nx, ny, 0.7, storage="F32")
    with pytest.raises(rl.RlbmError) as ex:
        lat.set_kernel("march2", 0)
    assert ex.value.code == rl.EUNSUPPORTED
    ens = rl.Ensemble([(64, 8), (64, 2)], [0.6, 0.7], storage="F32")
    with pytest.raises(rl.RlbmError) as ex:
        ens.set_kernel("march2", 0)
    assert ex.value.code == rl.EUNSUPPORTED
    ens.close()
    e, bx, by = workloads.noisy_rest(ny, nx, 0.01, seed=2)
    lat.set_state(dev(e), dev(bx), dev(by))
    kind, param = lat.autotune(4)
    say("autotuned on ny = 2", kind, param, lat.steps)
    assert kind != "march2"
    ref = rl.Lattice(nx, ny, 0.7, storage="F32")
    ref.set_kernel("tile", 1)
    ref.set_state(dev(e), dev(bx), dev(by))
    ref.step(lat.steps)
    lat.step(3)
    ref.step(3)
    assert np.array_equal(host(lat.populations()), host(ref.populations()))
    assert lat.check() == rl.OK


def test_fast_flow_landau():
    """Populations with a strong one-sided momentum (|beta| up to ~0.5): the
    Landau solve takes several Newton passes; one step against the oracle."""
    nx, ny = 40, 24
    F = workloads.random_populations(SPH.v, ny, nx, seed=9, spread=0.1)
    boost = 1.0 + 1.2 * SPH.v[:, 0]              # more energy moving along +x
    F = F * boost[:, None, None]
    _, bx, by, _ = odiag.fields(F, SPH, 1.0)
    say("max |beta| of the input", np.hypot(bx, by).max())
    assert np.hypot(bx, by).max() > 0.3
    F1o = orlbm.run(F, SPH, 0.8, 2)
    lat = rl.Lattice(nx, ny, 0.8, storage="F64")
    lat.set_populations(dev(oracle_to_lib(F)))
    lat.step(2)
    assert rel(lib_to_oracle(host(lat.populations())), F1o) < 1e-13
    assert lat.check() == rl.OK


def test_tau_close_to_half():
    """tau = 0.5001 (viscosity nearly zero, over-relaxation omega ~ 2): 5 steps
    of the forced 128^2 workload against the oracle."""
    n, tau = 128, 0.5001
    e, bx, by = workloads.noisy_rest(n, n, 0.002, seed=4)
    force = dict(amplitude=1e-5, k_lo=2.0, k_hi=4.0, seed=3)
    lat = rl.Lattice(n, n, tau, storage="F64", forcing=rl.Forcing(1e-5, 2.0, 4.0, 3))
    lat.set_state(dev(e), dev(bx), dev(by))
    lat.step(5)
    Fo = orlbm.run(orlbm.set_state(e, bx, by, SPH), SPH, tau, 5, force=force)
    errs = field_errors(gpu_fields(lat), odiag.fields(Fo, SPH, 1.0))
    say("tau 0.5001", errs)
    assert max(errs.values()) < 1e-12


def test_forcing_shell_without_modes_is_unforced():
    """The shell 1.1 <= |k| <= 1.2 holds no integer wave vector: the lattice
    evolves exactly as an unforced one."""
    assert len(rl.forcing_modes(64, 64, rl.Forcing(1e-3, 1.1, 1.2, 5))) == 0
    e, bx, by = workloads.noisy_rest(64, 64, 0.01, seed=2)
    a = rl.Lattice(64, 64, 0.6, storage="F32", forcing=rl.Forcing(1e-3, 1.1, 1.2, 5))
    b = rl.Lattice(64, 64, 0.6, storage="F32")
    for lat in (a, b):
        lat.set_state(dev(e), dev(bx), dev(by))
        lat.step(6)
    assert np.array_equal(host(a.populations()), host(b.populations()))


def test_one_lattice_ensemble_equals_lattice():
    e, bx, by = workloads.noisy_rest(72, 56, 0.01, seed=6)
    fr = rl.Forcing(1e-4, 2.0, 4.0, 0)
    ens = rl.Ensemble([(56, 72)], [0.62], storage="F32", forcings=[fr])
    lat = rl.Lattice(56, 72, 0.62, storage="F32", forcing=fr)
    ens.set_state(0, dev(e), dev(bx), dev(by))
    lat.set_state(dev(e), dev(bx), dev(by))
    ens.step(7)
    lat.step(7)
    assert np.array_equal(host(ens.populations(0)), host(lat.populations()))


def _z_symmetrize(F):
    """Copy every population with v_z > 0 onto its z mirror (library order)."""
    v, _ = rl.stencil_info("SPH26")
    for q in range(len(v)):
        if v[q, 2] < 0:
            m = int(np.argmin(np.abs(v - v[q] * np.array([1.0, 1.0, -1.0])).max(axis=1)))
            F[q] = F[m]


def test_set_populations_rejects_states_without_z_mirror_symmetry():
    """The 26-direction step assumes F(a, b, c) = F(a, b, -c) (one-layer
    lattice).  Input that breaks it in one value is refused with EINVAL and
    leaves the stored state as it was; the folded and 8-direction stencils
    take any input.  Only the library's own check reads the input."""
    n = 24
    F = workloads.random_populations(SPH.v, n, n, seed=5, spread=0.2)
    lat = rl.Lattice(n, n, 0.6, storage="F64")
    lat.set_populations(dev(oracle_to_lib(F)))
    before = host(lat.populations())
    v, _ = rl.stencil_info("SPH26")
    q = int(np.flatnonzero(v[:, 2] < 0)[3])
    bad = oracle_to_lib(F).copy()
    bad[q, 7, 11] += 1e-12
    with pytest.raises(rl.RlbmError) as ex:
        lat.set_populations(dev(bad))
    assert ex.value.code == rl.EINVAL
    assert np.array_equal(host(lat.populations()), before)
    bad[q, 7, 11] = np.nan
    with pytest.raises(rl.RlbmError):
        lat.set_populations(dev(bad))
    lat.step(1)
    assert lat.check() == rl.OK
    # other stencils: no symmetry to check
    for name in ("SPH26_ZFOLD", "CIRC8"):
        L = rl.Lattice(n, n, 0.6, stencil=name, storage="F64")
        G = 1.0 + 0.1 * np.random.default_rng(3).standard_normal((L.Q, n, n))
        L.set_populations(dev(G))
        assert np.array_equal(host(L.populations()), G)


def test_stream_copy_probe():
    """The library's streaming copy moves the bytes exactly and reports a
    positive time; misuse is refused."""
    import torch
    a = torch.randn(1 << 22, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    ms = rl.stream_copy(a, b, reps=3)
    assert ms > 0
    assert torch.equal(a, b)
    with pytest.raises(ValueError):
        rl.stream_copy(a, b[:-1])
    with pytest.raises(rl.RlbmError):
        rl.stream_copy(a, a)


def _bf16_rne(d32):
    """FP32 -> BF16 bits, round to nearest even (finite inputs)."""
    u = d32.view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


@pytest.mark.parametrize("storage", ["F32", "F16S", "BF16S"])
def test_storage_rounding_is_round_to_nearest_even(storage):
    """Populations written into the reduced storage forms are rounded to
    nearest even: the stored deviation F - 1 equals numpy's rounding of the
    FP32 deviation, bit for bit, including exact ties of both parities."""
    nx, ny = 64, 8
    Q = rl.Lattice(nx, ny, 0.7, storage=storage).Q
    rng = np.random.default_rng(21)
    F = 1.0 + rng.uniform(-0.3, 0.3, size=(Q, ny, nx))
    ties = np.array([0x3C008000, 0x3C018000, 0xBC008000, 0xBC018000, 0x3A7F8000,
                     0x00000000, 0x80000000], dtype=np.uint32).view(np.float32)
    F.reshape(-1)[:ties.size] = 1.0 + ties.astype(np.float64)
    h16 = np.array([0x3C00 + 0x0400, 0x1001], dtype=np.uint16).view(np.float16)
    F.reshape(-1)[ties.size:ties.size + 2] = 1.0 + h16.astype(np.float64) + np.array([2.0 ** -22, -2.0 ** -22])
    _z_symmetrize(F)          # the ties sit in population 0, which has v_z = 0
    lat = rl.Lattice(nx, ny, 0.7, storage=storage)
    lat.set_populations(dev(F))
    got = host(lat.populations())
    d32 = (F - 1.0).astype(np.float32)
    if storage == "F32":
        want = d32.astype(np.float64) + 1.0
    elif storage == "F16S":
        want = d32.astype(np.float16).astype(np.float64) + 1.0
    else:
        want = (_bf16_rne(d32).astype(np.uint32) << 16).view(np.float32).astype(np.float64) + 1.0
    assert np.array_equal(got, want)
    # one step of an unforced lattice keeps every stored value on the storage grid
    lat.step(1)
    d = (host(lat.populations()) - 1.0).astype(np.float32)
    if storage == "F16S":
        assert np.array_equal(d.astype(np.float16).astype(np.float32), d)
    elif storage == "BF16S":
        assert np.all((d.view(np.uint32) & 0xFFFF) == 0)
