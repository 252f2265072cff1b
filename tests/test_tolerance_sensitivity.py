"""The reduced-precision bounds of the GPU force tests can see a wrong force.

CPU only: the oracle's step with a deliberately wrong force term (amplitude
20 % too large; the third-moment or the current term of the App. B projection
20 % too large; the x component of the force with the wrong sign) is compared
with the correct oracle step under exactly the bounds that
``test_gpu_force_precision.py`` applies to the GPU result.  Each mistake must
exceed the bound of every storage form.
"""
import numpy as np
import pytest

from oracle import forcing as oforcing
from oracle import rlbm as orlbm
from oracle import stencil as ostencil
import workloads

from tolerances import half_ulp, one_step_bound, rest_force_bound, ulp32

SPH = ostencil.sph26()
STORAGES = ("F32", "F16S", "BF16S")


def _step(F, tau, force, step_index=0, scale_amp=1.0, scale_R=1.0, scale_J=1.0, flip_x=False):
    """The oracle's step (stream, moments, Landau, equilibrium, collide, force)
    with optional mistakes planted in the force term."""
    Fs = orlbm.stream(F, SPH, 1.0)
    T, R = orlbm.moments(Fs, SPH)
    eps, u = orlbm.landau(T)
    beta = u[1:] / u[0]
    Fn = orlbm.collide(Fs, orlbm.equilibrium(eps, beta, SPH), beta, tau, SPH)
    ny, nx = F.shape[1:]
    fx, fy = oforcing.force_field(nx, ny, force["amplitude"] * scale_amp, force["k_lo"],
                                  force["k_hi"], force["seed"], step_index)
    if flip_x:
        fx = -fx
    Tm = T.copy()
    Tm[0, 1:] *= scale_J
    return Fn + orlbm.force_source(Tm, R * scale_R, fx, fy, 1.0, SPH)


MISTAKES = {
    "amplitude x 1.2": dict(scale_amp=1.2),
    "third moment x 1.2": dict(scale_R=1.2),
    "current x 1.2": dict(scale_J=1.2),
    "force x sign": dict(flip_x=True),
}


@pytest.fixture(scope="module")
def strong():
    """The strong-forcing case of the GPU test on a smaller lattice with the
    same shell structure relative to its size (96^2, shell [24, 30])."""
    n, tau = 96, 0.56
    force = dict(amplitude=3e-3, k_lo=24.0, k_hi=30.0, seed=11)
    F0 = workloads.random_populations(SPH.v, n, n, seed=31, spread=0.3)
    want = _step(F0, tau, force)
    # the plain oracle step agrees with this re-assembled one
    assert np.abs(want - orlbm.step(F0, SPH, tau, 1.0, force, 0)).max() < 1e-14
    return F0, tau, force, want


@pytest.mark.parametrize("mistake", sorted(MISTAKES))
@pytest.mark.parametrize("storage", STORAGES)
def test_strong_forcing_bound_sees_a_wrong_force(strong, storage, mistake):
    F0, tau, force, want = strong
    wrong = _step(F0, tau, force, **MISTAKES[mistake])
    scale = max(np.abs(want - 1.0).max(), np.abs(F0 - 1.0).max())
    bound = one_step_bound(storage, want - 1.0, scale)
    frac = np.mean(np.abs(wrong - want) > bound)
    # one value past the bound fails the GPU test; require many
    assert frac > 0.02, (storage, mistake, frac)


@pytest.mark.parametrize("n,shell,amp", [(2048, (8.0, 12.0), 1e-5), (8192, (32.0, 40.0), 2e-6)])
@pytest.mark.parametrize("storage", STORAGES)
def test_rest_probe_bound_sees_a_wrong_force(n, shell, amp, storage):
    """At rest the stored deviation is dt F . v_q; a 20 % amplitude error or a
    flipped component exceeds the rest-probe bound at most sampled values."""
    g = np.random.Generator(np.random.Philox(5))
    xs, ys = g.integers(0, n, 64), g.integers(0, n, 64)
    fx, fy = oforcing.force_at(n, n, amp, shell[0], shell[1], 2, 0, xs, ys)
    v = SPH.v
    want = fx[None] * v[:, :1] + fy[None] * v[:, 1:2]          # (Q, S): dt = 1
    bound = rest_force_bound(storage, want)
    for wrong in (1.2 * want, -fx[None] * v[:, :1] + fy[None] * v[:, 1:2]):
        assert np.mean(np.abs(wrong - want) > bound) > 0.5


def test_rest_probe_value_is_the_force_projection():
    """The oracle's full step from the rest state leaves F - 1 = dt F . v_q
    (the closed form the rest probe relies on)."""
    n, tau = 16, 0.6
    force = dict(amplitude=1e-3, k_lo=2.0, k_hi=4.0, seed=3)
    F = np.ones((26, n, n))
    got = orlbm.step(F, SPH, tau, 1.0, force, 0) - 1.0
    fx, fy = oforcing.force_field(n, n, force["amplitude"], force["k_lo"], force["k_hi"],
                                  force["seed"], 0)
    want = fx[None] * SPH.v[:, 0, None, None] + fy[None] * SPH.v[:, 1, None, None]
    assert np.abs(got - want).max() < 1e-15


def test_storage_spacings():
    """half_ulp / ulp32 against numpy's own FP16 and FP32 spacings, and the
    BF16 spacing against its definition (8 significant bits)."""
    v = np.array([1e-7, 3e-5, 6.1e-5, 1e-3, 0.3, 0.999])
    assert np.allclose(half_ulp("F16S", v), 0.5 * np.spacing(v.astype(np.float16)).astype(float))
    assert np.allclose(ulp32(v), np.spacing(v.astype(np.float32)).astype(float))
    assert np.allclose(half_ulp("BF16S", np.array([1.0, 0.3])), [2.0 ** -8, 2.0 ** -10])
