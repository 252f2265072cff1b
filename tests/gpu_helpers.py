"""Shared helpers of the GPU parity tests: direction-order mapping between the
library and the oracle, host/device conversion, error norms, sampled one-step
oracle evaluation on large lattices."""
import sys

import numpy as np

import paper_2101_06187_amd as rl
from oracle import forcing as oforcing
from oracle import rlbm as orlbm
from oracle import stencil as ostencil


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch():
    import torch as t
    return t


def perm(name="SPH26"):
    """perm[q_lib] = index of the same direction in the oracle's table."""
    v, _ = rl.stencil_info(name)
    st = ostencil.by_name(name)
    p = np.array([int(np.argmin(np.abs(st.v - v[q]).max(axis=1))) for q in range(len(v))])
    assert len(set(p)) == len(p)
    return p


def lib_to_oracle(F_lib, name="SPH26"):
    p = perm(name)
    out = np.empty_like(F_lib)
    out[p] = F_lib
    return out


def oracle_to_lib(F_or, name="SPH26"):
    return np.ascontiguousarray(F_or[perm(name)])


def dev(a):
    return torch().from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def host(t):
    return t.detach().to("cpu").numpy()


def rel(a, b):
    """Normwise relative error max|a - b| / max|b|."""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def field_errors(gpu, ref):
    """Per-field normwise errors.  beta is a vector field: both components are
    normalised by the largest |beta| component; the T planes by max T^00."""
    ge, gx, gy, gT = gpu
    re, rx, ry, rT = ref
    vmax = max(np.abs(rx).max(), np.abs(ry).max(), 1e-300)
    tmax = np.abs(rT[0]).max()
    return {
        "eps": rel(ge, re),
        "beta_x": float(np.abs(gx - rx).max() / vmax),
        "beta_y": float(np.abs(gy - ry).max() / vmax),
        "T": float(np.abs(gT - rT).max() / tmax),
    }


def gpu_fields(lat):
    return tuple(host(t) for t in lat.fields())


def sample_sites(nx, ny, n, seed):
    g = np.random.Generator(np.random.Philox(seed))
    xs = list(g.integers(0, nx, n)) + [0, nx - 1, 0, nx - 1, nx // 2]
    ys = list(g.integers(0, ny, n)) + [0, 0, ny - 1, ny - 1, ny // 2]
    return np.array(xs), np.array(ys)


def gather_patches(F_dev, xs, ys, radius=1):
    """(Q, S, w, w) FP64 patches, w = 2 radius + 1, of a device population
    tensor around sites (periodic)."""
    t = torch()
    Q, ny, nx = F_dev.shape
    dx = t.arange(-radius, radius + 1, device=F_dev.device)
    X = (t.as_tensor(xs, device=F_dev.device)[:, None] + dx[None, :]) % nx    # (S, 3)
    Y = (t.as_tensor(ys, device=F_dev.device)[:, None] + dx[None, :]) % ny
    P = F_dev[:, Y[:, :, None], X[:, None, :]]                                 # (Q, S, 3, 3)
    return host(P)


def oracle_step_at(patches, st, tau, cfl, force=None, step_index=0, sites=None, nxy=None,
                   realization=0):
    """Oracle one-step result at the centre of each 3x3 patch (oracle order).

    The centre of a 3x3 window depends only on the window (cfl <= 1), so the
    oracle's stages applied to the window give the exact update there.
    """
    Q, S = patches.shape[:2]
    out = np.empty((Q, S))
    fxs = fys = None
    if force is not None and force["amplitude"] != 0.0:
        nx, ny = nxy
        fxs, fys = oforcing.force_at(nx, ny, force["amplitude"], force["k_lo"], force["k_hi"],
                                     force["seed"], step_index, sites[0], sites[1], realization)
    for s in range(S):
        F = patches[:, s]
        Fs = orlbm.stream(F, st, cfl)
        T, R = orlbm.moments(Fs, st)
        eps, u = orlbm.landau(T)
        beta = u[1:] / u[0]
        Feq = orlbm.equilibrium(eps, beta, st)
        Fn = orlbm.collide(Fs, Feq, beta, tau, st)
        if fxs is not None:
            fx = np.full((3, 3), fxs[s])
            fy = np.full((3, 3), fys[s])
            Fn = Fn + orlbm.force_source(T, R, fx, fy, cfl, st)
        out[:, s] = Fn[:, 1, 1]
    return out


def oracle_two_steps_at(patches, st, tau, cfl, force, step_index, sites, nxy, realization=0):
    """Oracle result of two steps at the centre of each 5x5 patch (oracle
    order): one step on the whole window is exact on its inner 3x3 (a site
    pulls from its 3x3 neighbourhood, cfl <= 1), a second step on that 3x3 is
    exact at its centre.  The force is evaluated at every site of each window,
    at steps step_index and step_index + 1."""
    Q, S = patches.shape[:2]
    xs, ys = (np.asarray(v) for v in sites)
    nx, ny = nxy
    F = patches                                                 # (Q, S, w, w)
    for k in (0, 1):
        w = F.shape[2]
        r = w // 2
        d = np.arange(-r, r + 1)
        X = (xs[:, None, None] + d[None, None, :]) % nx         # (S, 1, w)
        Y = (ys[:, None, None] + d[None, :, None]) % ny         # (S, w, 1)
        X, Y = np.broadcast_arrays(X, Y)
        fx = fy = None
        if force is not None and force["amplitude"] != 0.0:
            fx, fy = oforcing.force_at(nx, ny, force["amplitude"], force["k_lo"], force["k_hi"],
                                       force["seed"], step_index + k, X.ravel(), Y.ravel(),
                                       realization)
            fx, fy = fx.reshape(S, w, w), fy.reshape(S, w, w)
        out = np.empty((Q, S, w - 2, w - 2))
        for s in range(S):
            Fs = orlbm.stream(F[:, s], st, cfl)
            T, R = orlbm.moments(Fs, st)
            eps, u = orlbm.landau(T)
            beta = u[1:] / u[0]
            Feq = orlbm.equilibrium(eps, beta, st)
            Fn = orlbm.collide(Fs, Feq, beta, tau, st)
            if fx is not None:
                Fn = Fn + orlbm.force_source(T, R, fx[s], fy[s], cfl, st)
            out[:, s] = Fn[:, 1:-1, 1:-1]
        F = out
    return F[:, :, 0, 0]


def fold_maps():
    """For each direction of the library's z-folded SPH26 table: the oracle
    (SPH26) index of the same direction and of its z mirror."""
    v, _ = rl.stencil_info("SPH26_ZFOLD")
    st = ostencil.sph26()
    up = np.array([int(np.argmin(np.abs(st.v - v[q]).max(axis=1))) for q in range(len(v))])
    mv = v * np.array([1.0, 1.0, -1.0])
    dn = np.array([int(np.argmin(np.abs(st.v - mv[q]).max(axis=1))) for q in range(len(v))])
    assert sorted(set(up) | set(dn)) == list(range(26))
    return up, dn


def fold(F_or):
    """Oracle SPH26 populations (z-mirror symmetric) -> folded library order."""
    up, dn = fold_maps()
    assert np.array_equal(F_or[up], F_or[dn])
    return np.ascontiguousarray(F_or[up])


def unfold(F_lib):
    """Folded library populations -> oracle SPH26 order (mirror pairs equal)."""
    up, dn = fold_maps()
    out = np.empty((26,) + F_lib.shape[1:], dtype=F_lib.dtype)
    out[up] = F_lib
    out[dn] = F_lib
    return out
