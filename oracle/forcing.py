"""Stirring force of the oracle (test infrastructure; see ``oracle/__init__``).

The paper (Sec. V, simulation method) drives the flow with a force applied in
Fourier space: every wave vector of the discrete spectral lattice inside the
driven range gets a random magnitude up to a maximum |F| and a random direction
in the plane; the spectral field is transformed to configuration space and
enters the force term of Sec. III C.  The force is zero-averaged (Sec. III C).

Readings where the paper is silent (all listed in the design notes):
  * driven range = integer wave vectors (kx, ky) with k_lo <= |k| <= k_hi,
    restricted to the half plane ky > 0 or (ky == 0 and kx > 0), so that the
    configuration-space field is real; there is no k = 0 mode, which makes the
    force zero-averaged exactly;
  * modes are numbered m = 0, 1, ... in lexicographic (ky, kx) order;
  * per mode, Philox4x32-10 with key (seed low 32 bits, seed high 32 bits) and
    counter (m, step, realization, 0) gives words x0, x1, x2: magnitude
    r = u(x0) in (0, 1), in-plane direction theta = 2 pi u(x1) and phase
    phi = 2 pi u(x2), with u(x) = (x + 1/2) 2^-32; the force is redrawn every
    time step;
  * F(x, y) = A * sum_m r_m (cos theta_m, sin theta_m)
                   * cos(2 pi (kx x / nx + ky y / ny) + phi_m).
"""
import numpy as np

from .philox import philox4x32_10, uniform_open01


def modes(nx, ny, k_lo, k_hi):
    """Integer wave vectors of the driven shell, half plane, (ky, kx) order.

    Every mode must lie strictly below the Nyquist wave number of its axis
    (|kx| < nx/2, ky < ny/2); a shell that reaches it is rejected.
    """
    out = []
    kmax = int(np.floor(k_hi)) + 1
    for ky in range(0, kmax + 1):
        for kx in range(-kmax, kmax + 1):
            if ky == 0 and kx <= 0:
                continue
            k2 = kx * kx + ky * ky
            if k2 < k_lo * k_lo or k2 > k_hi * k_hi:
                continue
            if 2 * abs(kx) >= nx or 2 * ky >= ny:
                raise ValueError("forcing shell reaches the Nyquist wave number")
            out.append((kx, ky))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def mode_draws(n_modes, seed, step, realization=0):
    """(r, theta, phi) for every mode of one time step (reading above)."""
    m = np.arange(n_modes, dtype=np.uint64)
    x0, x1, x2, _ = philox4x32_10(m, step, realization, 0,
                                  seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    r = uniform_open01(x0)
    theta = 2.0 * np.pi * uniform_open01(x1)
    phi = 2.0 * np.pi * uniform_open01(x2)
    return r, theta, phi


def force_field(nx, ny, amplitude, k_lo, k_hi, seed, step, realization=0):
    """Configuration-space force (Fx, Fy), each (ny, nx), by direct summation."""
    km = modes(nx, ny, k_lo, k_hi)
    fx = np.zeros((ny, nx))
    fy = np.zeros((ny, nx))
    if amplitude == 0.0 or len(km) == 0:
        return fx, fy
    r, theta, phi = mode_draws(len(km), seed, step, realization)
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for (kx, ky), rm, th, ph in zip(km, r, theta, phi):
        c = np.cos(2.0 * np.pi * (kx * x / nx + ky * y / ny) + ph)
        fx += amplitude * rm * np.cos(th) * c
        fy += amplitude * rm * np.sin(th) * c
    return fx, fy


def force_at(nx, ny, amplitude, k_lo, k_hi, seed, step, xs, ys, realization=0):
    """The same force evaluated only at the points (xs, ys), by direct summation
    (for sampled checks on lattices too large for ``force_field``)."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    fx = np.zeros(xs.shape)
    fy = np.zeros(xs.shape)
    km = modes(nx, ny, k_lo, k_hi)
    if amplitude == 0.0 or len(km) == 0:
        return fx, fy
    r, theta, phi = mode_draws(len(km), seed, step, realization)
    for (kx, ky), rm, th, ph in zip(km, r, theta, phi):
        c = np.cos(2.0 * np.pi * (kx * xs / nx + ky * ys / ny) + ph)
        fx += amplitude * rm * np.cos(th) * c
        fy += amplitude * rm * np.sin(th) * c
    return fx, fy
