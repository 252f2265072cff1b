"""CPU-only checks of the C ABI: the library loads, exports every function the
header declares, and its host logic (stencil table, forcing modes, workspace
size, argument validation) agrees with the oracle.  No device work is done."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2101_06187_amd as rl
from oracle import forcing as oforcing
from oracle import stencil as ostencil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "rlbm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(rlbm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = rl.lib()
    names = header_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    assert sorted(n for n, _, _ in rl.SIGNATURES) == names


def test_status_strings():
    L = rl.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.rlbm_status_string(code)
    assert L.rlbm_status_string(-99) == b"unknown status"


@pytest.mark.parametrize("name", ["SPH26", "CIRC8"])
def test_stencil_table_matches_oracle(name):
    v, w = rl.stencil_info(name)
    st = ostencil.by_name(name)
    assert v.shape == st.v.shape
    used = set()
    for q in range(len(v)):
        d = np.abs(st.v - v[q]).max(axis=1)
        j = int(np.argmin(d))
        assert d[j] < 1e-15 and j not in used
        used.add(j)
        assert abs(w[q] - st.w[j]) < 1e-17


def test_stencil_classes_are_antipodal():
    """The library stores each class's +u members then their antipodes."""
    v, _ = rl.stencil_info("SPH26")
    # classes as laid out in the library: sizes of (plus, minus) groups
    layout = [(1, 1), (1, 1), (2, 0), (1, 1), (1, 1), (2, 2), (2, 2), (2, 2), (2, 2)]
    q = 0
    for npl, nmi in layout:
        for i in range(nmi):
            assert np.allclose(v[q + i], -v[q + npl + i], atol=1e-15)
        q += npl + nmi
    assert q == 26


def test_zfold_table_is_the_mirror_sum_of_sph26():
    """The folded table: one representative (v_z >= 0) per z-mirror pair of
    the oracle's SPH26 set, at the pair's summed weight; angular averages of
    every mirror-even monomial up to degree 7 agree with the full set."""
    v, w = rl.stencil_info("SPH26_ZFOLD")
    st = ostencil.sph26()
    assert v.shape == (17, 3) and np.all(v[:, 2] >= 0)
    covered = []
    for q in range(17):
        for sz in (1.0, -1.0):
            d = np.abs(st.v - v[q] * np.array([1.0, 1.0, sz])).max(axis=1)
            assert d.min() < 1e-15
            covered.append(int(np.argmin(d)))
    mirror_pairs = {covered[2 * q]: covered[2 * q + 1] for q in range(17)}
    assert set(covered) == set(range(26))
    for q in range(17):
        j, k = covered[2 * q], covered[2 * q + 1]
        want = st.w[j] if j == k else st.w[j] + st.w[k]
        assert abs(w[q] - want) < 1e-17
    assert len(mirror_pairs) == 17
    for a in range(8):
        for b in range(8 - a):
            for c in range(0, 8 - a - b, 2):
                full = np.sum(st.w * st.v[:, 0] ** a * st.v[:, 1] ** b * st.v[:, 2] ** c)
                fold = np.sum(w * v[:, 0] ** a * v[:, 1] ** b * v[:, 2] ** c)
                assert abs(full - fold) < 1e-15, (a, b, c)


@pytest.mark.parametrize("n,shell", [(512, (4, 6)), (2048, (8, 12)), (64, (2, 4)),
                                     (8192, (32, 40)), (48, (3.0, 7.5)), (100, (1, 1.5))])
def test_forcing_modes_match_oracle(n, shell):
    f = rl.Forcing(1e-5, shell[0], shell[1], 2)
    got = rl.forcing_modes(n, n + 2, f)
    want = oforcing.modes(n, n + 2, *shell)
    assert np.array_equal(got, want)


def test_forcing_modes_nyquist_rejected():
    with pytest.raises(rl.RlbmError) as e:
        rl.forcing_modes(16, 16, rl.Forcing(1.0, 6, 8, 0))
    assert e.value.code == rl.EINVAL


@pytest.mark.parametrize("storage,s", [("F64", 8), ("F32", 4), ("F16S", 2), ("BF16S", 2)])
def test_workspace_bytes(storage, s):
    b = rl.workspace_bytes(512, 512, "SPH26", storage, rl.Forcing(1e-5, 4, 6, 2))
    assert 2 * 26 * 512 * 512 * s <= b <= 2 * 26 * 512 * 512 * s + (1 << 20)


def test_zfold_workspace_is_17_of_26():
    a = rl.workspace_bytes(512, 512, "SPH26", "F32")
    b = rl.workspace_bytes(512, 512, "SPH26_ZFOLD", "F32")
    assert 2 * 17 * 512 * 512 * 4 <= b < a
    assert b - 2 * 17 * 512 * 512 * 4 == a - 2 * 26 * 512 * 512 * 4


def _init(**kw):
    L = rl.lib()
    args = dict(nx=64, ny=64, cfl=1.0, tau=0.6, stencil=0, storage=0, ws=256, ws_bytes=1 << 30)
    args.update(kw)
    lat = rl._Lattice(args["nx"], args["ny"], args["cfl"])
    ctx = ctypes.c_void_p()
    return L.rlbm_init(ctypes.byref(ctx), ctypes.byref(lat), args["tau"], args["stencil"], None,
                       args["storage"], ctypes.c_void_p(args["ws"]) if args["ws"] else None,
                       args["ws_bytes"], None)


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(tau=0.3), dict(cfl=0.0), dict(cfl=2.5),
                                dict(nx=1), dict(ny=0), dict(stencil=7), dict(storage=9),
                                dict(ws=0), dict(ws=257)])
def test_init_rejects_invalid_arguments(kw):
    assert _init(**kw) == rl.EINVAL


def test_init_rejects_small_workspace():
    assert _init(ws_bytes=1024) == rl.ENOSPACE


def test_null_context_calls_fail_cleanly():
    L = rl.lib()
    assert L.rlbm_step(None, 1) == rl.EINVAL
    assert L.rlbm_fields(None, None, None, None, None) == rl.EINVAL
    assert L.rlbm_set_relaxation(None, 1) == rl.EINVAL
    assert L.rlbm_batch_set_relaxation(None, 1) == rl.EINVAL
    L.rlbm_destroy(None)
    L.rlbm_batch_destroy(None)


def test_spectrum_average_matches_oracle():
    from oracle import diagnostics
    g = np.random.Generator(np.random.Philox(9))
    S = g.random((11, 17)) * np.geomspace(1.0, 1e-6, 17)
    mean, err = rl.spectrum_average(S)
    om, oe = diagnostics.spectrum_average(S)
    assert np.abs(mean - om).max() <= 1e-15 * np.abs(om).max()
    assert np.abs(err - oe).max() <= 1e-14 * np.abs(oe).max()
    with pytest.raises(rl.RlbmError):
        rl.spectrum_average(np.zeros((0, 3)))


def test_shell_modes_match_oracle():
    from oracle import diagnostics
    for nx, ny, nb in ((64, 64, 50), (64, 64, 7), (16, 4, 14), (5, 7, 8), (1, 1, 3), (2, 1, 4),
                       (128, 32, 100), (1, 9, 6), (256, 2, 130), (1024, 1024, 724)):
        np.testing.assert_array_equal(rl.shell_modes(nx, ny, nb),
                                      diagnostics.shell_modes(nx, ny, nb), err_msg=f"{nx}x{ny}")
    assert rl.shell_modes(8192, 8192, 5794).sum() == 8192 * 8192   # corner |k| = 5792.6
    L = rl.lib()
    out = np.zeros(4, dtype=np.int64)
    for args in ((0, 4, 4), (4, 0, 4), (4, 4, 0)):
        assert L.rlbm_shell_modes(*args, out.ctypes.data_as(rl._P)) == rl.EINVAL
    assert L.rlbm_shell_modes(4, 4, 4, None) == rl.EINVAL
