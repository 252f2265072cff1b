"""The allocation-free spectrum entry point (rlbm_spectrum_static) against
rlbm_spectrum with caller scratch, through the C ABI: two calls in a row,
the second on a smaller lattice, bit for bit; the size limit is refused
before any device work."""
import ctypes

import numpy as np
import pytest

import paper_2101_06187_amd as rl
import workloads

from gpu_helpers import dev, say

pytestmark = pytest.mark.gpu


def _lattice(n, seed):
    e, bx, by = workloads.noisy_rest(n, n, 0.01, seed=seed)
    lat = rl.Lattice(n, n, 0.6, storage="F64", forcing=rl.Forcing(1e-4, 2.0, 5.0, seed))
    lat.set_state(dev(e), dev(bx), dev(by))
    lat.step(3)
    return lat


def test_static_spectrum_equals_caller_scratch_spectrum():
    for n, seed in ((1024, 4), (128, 5)):          # the second call: a smaller lattice
        lat = _lattice(n, seed)
        nb = n // 2
        Ek_s, Z_s = lat.spectrum_static(nb)
        Ek, Z = lat.spectrum(nb)
        say("static spectrum", n, float(np.abs(Ek_s - Ek).max()), abs(Z_s - Z))
        assert np.array_equal(Ek_s, Ek)
        assert Z_s == Z
        assert Ek.sum() > 0
        lat.close()


def test_static_spectrum_refuses_lattices_beyond_its_scratch():
    lat = rl.Lattice(2048, 1024, 0.6, storage="F32")
    with pytest.raises(rl.RlbmError) as ex:
        lat.spectrum_static(16)
    assert ex.value.code == rl.ENOSPACE
    Ek = np.zeros(4)
    assert rl.lib().rlbm_spectrum_static(lat._ctx, Ek.ctypes.data_as(ctypes.c_void_p), 0, None) == rl.EINVAL
    lat.close()
