"""Long-horizon statistics of the forced 512 x 512 workload, every storage form
against the FP64 form.

Beyond a short horizon the trajectories of different precisions are compared
by statistics, not step by step: the time-averaged shell energy spectrum and
enstrophy (Sec. IV) over the workload's full 20000 steps, sampled every 500
steps after a spin-up, with the error estimate of the paper's appendix on the
minimum simulation time (the sample average of sqrt|<E>^2 - E_i^2|).  Every
form must stay stable over the whole run.
"""
import numpy as np
import pytest

import paper_2101_06187_amd as rl
import workloads

from gpu_helpers import dev, say

pytestmark = pytest.mark.gpu

NBINS = 32
SPIN_UP, EVERY, STEPS = 4000, 500, 20000


def _run(storage):
    wl = workloads.WORKLOADS["forced512"]
    A, klo, khi, seed = wl.forcing
    lat = rl.Lattice(wl.n, wl.n, wl.tau, storage=storage, forcing=rl.Forcing(A, klo, khi, seed))
    e, bx, by = workloads.initial_fields(wl)
    lat.set_state(dev(e), dev(bx), dev(by))
    lat.set_graph_chunk(EVERY)
    lat.step(SPIN_UP)
    spectra, enstrophy = [], []
    while lat.steps < STEPS:
        lat.step(EVERY)
        Ek, Z = lat.spectrum(NBINS)
        spectra.append(Ek)
        enstrophy.append(Z)
    assert lat.steps == STEPS
    assert lat.check() == rl.OK, storage
    lat.close()
    spectra = np.array(spectra)
    mean, err = rl.spectrum_average(spectra)
    return mean, err, spectra.sum(axis=1), np.array(enstrophy)


def _se(x):
    """Standard error of the mean of a sample series."""
    return float(np.std(x, ddof=1) / np.sqrt(len(x)))


def test_time_averaged_spectrum_and_enstrophy_match_f64():
    ref_mean, ref_err, ref_E, ref_Z = _run("F64")
    assert ref_mean.sum() > 0.0
    band = ref_mean > 1e-3 * ref_mean.max()            # bins that hold the energy
    for storage, rel_tol in (("F32", 1e-4), ("F16S", 1e-3), ("BF16S", 1e-2)):
        mean, err, E, Z = _run(storage)
        d = np.abs(mean - ref_mean)
        dE, dZ = abs(E.mean() - ref_E.mean()), abs(Z.mean() - ref_Z.mean())
        say(storage, "max |dE(k)|/err in band", float((d[band] / (err[band] + ref_err[band])).max()),
            "total energy", E.mean(), ref_E.mean(), "rel", dE / ref_E.mean(), "se", _se(E), _se(ref_E),
            "enstrophy rel", dZ / ref_Z.mean(), "se", _se(Z), _se(ref_Z))
        # every energy-holding shell within the paper's error estimate
        assert np.all(d[band] <= err[band] + ref_err[band])
        # time-averaged total energy and enstrophy within three standard errors of
        # the means, plus the relative precision of the stored deviation
        assert dE <= 3 * (_se(E) + _se(ref_E)) + rel_tol * ref_E.mean()
        assert dZ <= 3 * (_se(Z) + _se(ref_Z)) + rel_tol * ref_Z.mean()


def test_kernel_forms_stay_bitwise_equal_over_a_long_run():
    """The 512^2 forced workload over 3000 steps in every kernel form, with
    graph replay: the forms compute the same bits at every site and step, so
    the chaotic trajectories stay identical (FP32 and F16S storage)."""
    wl = workloads.WORKLOADS["forced512"]
    A, klo, khi, seed = wl.forcing
    e, bx, by = workloads.initial_fields(wl)
    for storage, forms in (("F32", [("tile", 4), ("tile", 1), ("staged", 4), ("march", 2), ("march2", 8)]),
                           ("F16S", [("tile", 4), ("march", 2), ("march_pairs", 2), ("march2", 8)])):
        ref = None
        for kind, param in forms:
            lat = rl.Lattice(wl.n, wl.n, wl.tau, storage=storage, forcing=rl.Forcing(A, klo, khi, seed))
            lat.set_kernel(kind, param)
            lat.set_state(dev(e), dev(bx), dev(by))
            lat.set_graph_chunk(50)
            lat.step(3000)
            assert lat.check() == rl.OK
            F = lat.populations().cpu().numpy()
            lat.close()
            if ref is None:
                ref = F
            else:
                say(storage, kind, param, "max |dF| vs", forms[0], float(np.abs(F - ref).max()))
                assert np.array_equal(F, ref), (storage, kind, param)
