"""Write field_windows.json: the oracle's macroscopic fields after a fixed
number of steps of the 2048^2 and 8192^2 forced workloads, at sampled sites.

    python tests/golden/make_field_windows.py

Calls only ``oracle/`` (and the seeded input generators of ``workloads/``).
With cfl <= 1 a site after N steps depends only on the (2N + 1)^2 window of
the initial state around it, and its fields (the Landau frame of the streamed
populations, as the library's fields call returns them) on the
(2N + 3)^2 window.  Each window is initialised from the workload's initial
fields (F = F_eq, Sec. III C step (a)) and advanced N steps with the oracle's
stages, the force evaluated at the window's true lattice coordinates (Sec. V
forcing, redrawn every step); the windows sit side by side in one periodic
strip, and whatever leaks across a window edge travels one site per step,
so the centres stay exact.

The stored values are the expected fields for the GPU field-error checks
(tests/test_gpu_field_errors.py) and the field errors the benchmark reports.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import diagnostics as odiag   # noqa: E402
from oracle import forcing as oforcing    # noqa: E402
from oracle import rlbm as orlbm          # noqa: E402
from oracle import stencil as ostencil    # noqa: E402
import workloads                          # noqa: E402

STEPS = 8
SITES = 24
FIELDS = ("eps", "beta_x", "beta_y", "T00", "T0x", "T0y", "Txx", "Txy", "Tyy")


def sites(n, count, seed):
    g = np.random.Generator(np.random.Philox(seed))
    xs = [int(v) for v in g.integers(0, n, count - 4)] + [0, n - 1, 0, n // 2]
    ys = [int(v) for v in g.integers(0, n, count - 4)] + [0, n - 1, n - 1, n // 2]
    return xs, ys


def window_fields(wl, xs, ys, steps):
    st = ostencil.sph26()
    n = wl.n
    R = steps + 1
    w = 2 * R + 1
    e, bx, by = workloads.initial_fields(wl)
    d = np.arange(-R, R + 1)
    Y = np.concatenate([np.repeat(((y + d) % n)[:, None], w, axis=1) for y in ys], axis=1)
    X = np.concatenate([np.repeat(((x + d) % n)[None, :], w, axis=0) for x in xs], axis=1)
    F = orlbm.set_state(e[Y, X], bx[Y, X], by[Y, X], st)
    del e, bx, by
    A, klo, khi, seed = wl.forcing
    for s in range(steps):
        Fs = orlbm.stream(F, st, 1.0)
        T, R3 = orlbm.moments(Fs, st)
        eps, u = orlbm.landau(T)
        beta = u[1:] / u[0]
        Fn = orlbm.collide(Fs, orlbm.equilibrium(eps, beta, st), beta, wl.tau, st)
        fx, fy = oforcing.force_at(n, n, A, klo, khi, seed, s, X.ravel(), Y.ravel())
        F = Fn + orlbm.force_source(T, R3, fx.reshape(X.shape), fy.reshape(X.shape), 1.0, st)
    eps, bx, by, T6 = odiag.fields(F, st, 1.0)
    centre = R + w * np.arange(len(xs))
    out = {"eps": eps[R, centre], "beta_x": bx[R, centre], "beta_y": by[R, centre]}
    for i, name in enumerate(FIELDS[3:]):
        out[name] = T6[i, R, centre]
    return {k: [float(v) for v in vals] for k, vals in out.items()}


def main():
    data = {"_source": "oracle/ (FP64 NumPy), windows of the initial state advanced "
                       f"{STEPS} steps; fields as the library's fields call defines them "
                       "(stage (c) of the next step: stream, T^{mu nu}, Landau frame)",
            "steps": STEPS, "workloads": {}}
    for name, seed in (("forced2048", 2048), ("forced8192", 8192)):
        wl = workloads.WORKLOADS[name]
        xs, ys = sites(wl.n, SITES, seed)
        data["workloads"][name] = {"x": xs, "y": ys, "fields": window_fields(wl, xs, ys, STEPS)}
        print(name, "done", flush=True)
    with open(os.path.join(HERE, "field_windows.json"), "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
