"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: only random draws, the
standard initial fields of the workloads and the table of workload shapes.
Both the oracle and the HIP library consume these arrays; neither side's
computation lives here.

Workloads (2D periodic lattices, populations initialised at equilibrium):
  shear64     64 x 64, tau 1.0, unforced; eps = 1, beta_x = 0.01 sin(2 pi y/64),
              beta_y = 0; 1000 steps (shear-wave decay, conservation).
  forced512   512 x 512, tau 0.55; eps = 1, beta ~ N(0, 0.005^2) per component
              (seed 1); force shell |k| in [4, 6], amplitude 1e-5, seed 2;
              FP64 and FP32 populations; 20000 steps.
  forced2048  2048 x 2048, tau 0.52; same initial recipe; shell [8, 12],
              amplitude 1e-5, seed 2; FP32 vs FP16/BF16 populations.
  ensemble    256 independent lattices, side drawn uniformly from
              {64, 128, 256}, tau uniform in [0.51, 0.8] (both from
              Generator(Philox(0)) in realization order); eps = 1,
              beta ~ N(0, 0.005^2) with seed r; shell [2, 4], amplitude 1e-5,
              force seed r; FP32 populations; 10000 steps.
  forced8192  8192 x 8192, tau 0.505; eps = 1, beta ~ N(0, 0.002^2) (seed 3);
              shell [32, 40], amplitude 2e-6, force seed 2; FP32 populations.
The paper's own runs (N = 128 ... 1024, driven shell from k_f = 6) are forced
2D periodic turbulence of the same kind; no dataset is involved.
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                      # square lattice side
    tau: float
    steps: int
    init: str                   # "shear" or "noise"
    sigma: float = 0.0          # noise standard deviation of each beta component
    init_seed: int = 0
    forcing: Optional[Tuple[float, float, float, int]] = None  # (A, k_lo, k_hi, seed)
    storages: Tuple[str, ...] = ("F64",)
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "shear64": Workload("shear64", 64, 1.0, 1000, "shear", storages=("F64",)),
    "forced512": Workload("forced512", 512, 0.55, 20000, "noise", 0.005, 1,
                          (1e-5, 4.0, 6.0, 2), ("F64", "F32")),
    "forced2048": Workload("forced2048", 2048, 0.52, 50000, "noise", 0.005, 1,
                           (1e-5, 8.0, 12.0, 2), ("F32", "F16S", "BF16S")),
    "forced8192": Workload("forced8192", 8192, 0.505, 100000, "noise", 0.002, 3,
                           (2e-6, 32.0, 40.0, 2), ("F32", "F16S")),
}


def shear_wave(n, amplitude=0.01):
    """eps = 1, beta_x = amplitude sin(2 pi y / n), beta_y = 0; arrays (n, n)."""
    y = np.arange(n, dtype=np.float64)
    bx = np.repeat((amplitude * np.sin(2.0 * np.pi * y / n))[:, None], n, axis=1)
    return np.ones((n, n)), bx, np.zeros((n, n))


def noisy_rest(ny, nx, sigma, seed):
    """eps = 1 and Gaussian beta, drawn beta_x first then beta_y."""
    g = np.random.Generator(np.random.Philox(seed))
    bx = sigma * g.standard_normal((ny, nx))
    by = sigma * g.standard_normal((ny, nx))
    return np.ones((ny, nx)), bx, by


def initial_fields(wl: Workload, ny=None, nx=None):
    ny = wl.n if ny is None else ny
    nx = wl.n if nx is None else nx
    if wl.init == "shear":
        return shear_wave(nx)
    return noisy_rest(ny, nx, wl.sigma, wl.init_seed)


def ensemble(n_real=256, seed=0, sides=(64, 128, 256), tau_range=(0.51, 0.8)):
    """Per-realization lattice side and tau for the ensemble workload."""
    g = np.random.Generator(np.random.Philox(seed))
    out = []
    for r in range(n_real):
        side = int(sides[g.integers(0, len(sides))])
        tau = float(g.uniform(*tau_range))
        out.append((side, tau))
    return out


def random_populations(v, ny, nx, seed, spread=0.2, z_mirror=True):
    """Random positive populations (Q, ny, nx) around 1, for brute-force tests.

    ``v`` is the (Q, 3) direction table of whichever side uses the array.  With
    ``z_mirror`` the value of direction (a, b, c) equals that of (a, b, -c), the
    symmetry every state of the 2D model has.
    """
    g = np.random.Generator(np.random.Philox(seed))
    Q = v.shape[0]
    F = 1.0 + spread * (2.0 * g.random((Q, ny, nx)) - 1.0)
    if z_mirror:
        for q in range(Q):
            if v[q, 2] < 0:
                mirror = np.flatnonzero(np.all(np.isclose(
                    v, [v[q, 0], v[q, 1], -v[q, 2]], atol=1e-12), axis=1))[0]
                F[q] = F[mirror]
    return F
