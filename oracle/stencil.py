"""Momentum stencils for the oracle (test infrastructure; see ``oracle/__init__``).

SPH26 -- the paper's "spherical D3Q27" momentum set (Sec. V, model set-up;
Sec. III B says the set comes from quadrature of the angular polynomials of
App. A, is spherical and off-lattice).  The paper prints neither vectors nor
weights.  Reading taken here: the 26 non-zero directions of the 3x3x3 cube,
normalised to unit length, with the weights of the 26-point Lebedev rule on the
sphere (faces 1/21, edges 4/105, corners 9/280), which integrates every
polynomial of degree <= 7 exactly under the angular average used throughout the
paper.  The 27th (zero) momentum cannot carry a massless particle, so its
weight is 0 and it is not stored.  Exactness is pinned by brute force in
``tests/test_oracle_stencil.py`` (no library routine involved).

CIRC8 -- the 2+1 dimensional analogue: 8 unit directions in the plane at angles
2 pi q / 8, weight 1/8 each, exact for circle averages of degree <= 7.  Used
with the two-dimensional ideal-gas closure P = eps/2.  Not the paper's stencil;
it exists so that the 2D ideal-gas closed forms can be checked as well.

``D`` is the dimension of the angular average (3 for the sphere, 2 for the
circle); the equation of state of a massless gas is then P = eps / D.
"""
from dataclasses import dataclass
import itertools

import numpy as np


@dataclass(frozen=True)
class Stencil:
    name: str
    v: np.ndarray      # (Q, 3) unit vectors; v[:, 2] is the out-of-plane component
    w: np.ndarray      # (Q,) quadrature weights, sum 1
    D: int             # angular dimension of the quadrature

    @property
    def Q(self):
        return self.v.shape[0]


def sph26() -> Stencil:
    """Spherical 26-direction set with Lebedev degree-7 weights (reading of Sec. V)."""
    cube = np.array([c for c in itertools.product((-1, 0, 1), repeat=3)
                     if c != (0, 0, 0)], dtype=np.float64)
    v = cube / np.sqrt((cube ** 2).sum(axis=1))[:, None]
    nonzero = (cube != 0).sum(axis=1)
    w = np.empty(len(cube))
    w[nonzero == 1] = 1.0 / 21.0
    w[nonzero == 2] = 4.0 / 105.0
    w[nonzero == 3] = 9.0 / 280.0
    return Stencil("SPH26", v, w, 3)


def circ8() -> Stencil:
    """Eight in-plane unit directions, equal weights (2+1-D analogue)."""
    ang = 2.0 * np.pi * np.arange(8) / 8.0
    v = np.stack([np.cos(ang), np.sin(ang), np.zeros(8)], axis=1)
    w = np.full(8, 1.0 / 8.0)
    return Stencil("CIRC8", v, w, 2)


def by_name(name: str) -> Stencil:
    return {"SPH26": sph26, "CIRC8": circ8}[name.upper()]()
