"""Brute-force pins of the oracle's streaming (Sec. III B, linear interpolation)
and moment sums (Sec. III A) on tiny lattices, with explicit Python loops and a
different formulation of the interpolant (tent functions over all nodes)."""
import numpy as np
import pytest

from oracle import rlbm
import workloads


def _tent(d):
    return max(0.0, 1.0 - abs(d))


def brute_stream(F, v, cfl):
    Q, ny, nx = F.shape
    out = np.zeros_like(F)
    for q in range(Q):
        for y in range(ny):
            for x in range(nx):
                px = x - cfl * v[q, 0]
                py = y - cfl * v[q, 1]
                acc = 0.0
                # every node of the periodic lattice, at its nearest image
                for yy in range(ny):
                    for xx in range(nx):
                        dx = (xx - px + nx / 2) % nx - nx / 2
                        dy = (yy - py + ny / 2) % ny - ny / 2
                        acc += _tent(dx) * _tent(dy) * F[q, yy, xx]
                out[q, y, x] = acc
    return out


@pytest.mark.parametrize("shape", [(3, 3), (3, 5), (4, 4), (6, 5)])
@pytest.mark.parametrize("cfl", [1.0, 0.7, 0.35, 1.25, 1.6, 2.0])
def test_stream_brute_force(sph26, shape, cfl):
    ny, nx = shape
    F = workloads.random_populations(sph26.v, ny, nx, seed=ny * 10 + nx)
    np.testing.assert_allclose(rlbm.stream(F, sph26, cfl), brute_stream(F, sph26.v, cfl),
                               atol=4e-15, rtol=0)


def test_stream_circ8_brute_force(circ8):
    F = workloads.random_populations(circ8.v, 4, 5, seed=4, z_mirror=False)
    np.testing.assert_allclose(rlbm.stream(F, circ8, 0.8), brute_stream(F, circ8.v, 0.8),
                               atol=4e-15, rtol=0)


def test_stream_conserves_plane_sums(sph26):
    F = workloads.random_populations(sph26.v, 8, 8, seed=1)
    Fs = rlbm.stream(F, sph26, 0.9)
    np.testing.assert_allclose(Fs.sum(axis=(1, 2)), F.sum(axis=(1, 2)), rtol=1e-15)


def test_axis_directions_shift_exactly_at_unit_cfl(sph26):
    F = workloads.random_populations(sph26.v, 5, 7, seed=2)
    Fs = rlbm.stream(F, sph26, 1.0)
    for q in range(26):
        vx, vy, vz = sph26.v[q]
        if abs(abs(vx) - 1) < 1e-12:
            assert np.array_equal(Fs[q], np.roll(F[q], int(round(vx)), axis=1))
        if abs(abs(vy) - 1) < 1e-12:
            assert np.array_equal(Fs[q], np.roll(F[q], int(round(vy)), axis=0))
        if abs(abs(vz) - 1) < 1e-12:
            assert np.array_equal(Fs[q], F[q])


def test_moments_brute_force(sph26):
    F = workloads.random_populations(sph26.v, 3, 4, seed=3, z_mirror=False)
    T, R = rlbm.moments(F, sph26)
    for y in range(3):
        for x in range(4):
            Tb = np.zeros((4, 4))
            Rb = np.zeros((3, 3, 3))
            for q in range(26):
                p = [1.0, *sph26.v[q]]
                for a in range(4):
                    for b in range(4):
                        Tb[a, b] += sph26.w[q] * F[q, y, x] * p[a] * p[b]
                for i in range(3):
                    for j in range(3):
                        for k in range(3):
                            Rb[i, j, k] += (sph26.w[q] * F[q, y, x] * sph26.v[q, i]
                                            * sph26.v[q, j] * sph26.v[q, k])
            np.testing.assert_allclose(T[:, :, y, x], Tb, atol=1e-15)
            np.testing.assert_allclose(R[:, :, :, y, x], Rb, atol=1e-15)
