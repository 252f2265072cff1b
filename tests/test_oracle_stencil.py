"""Pins of the oracle's momentum stencils against sphere/circle mathematics and
the relations the paper prints (App. A, App. B).  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dfact(n):
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


def sphere_moment(a, b, c):
    """<x^a y^b z^c> over the unit sphere, closed form (double factorials)."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    return _dfact(a - 1) * _dfact(b - 1) * _dfact(c - 1) / _dfact(a + b + c + 1)


def circle_moment(a, b):
    """<cos^a sin^b> over the unit circle, closed form."""
    if a % 2 or b % 2:
        return 0.0
    return _dfact(a - 1) * _dfact(b - 1) / _dfact(a + b)


def test_sph26_basic(sph26):
    assert sph26.Q == 26
    np.testing.assert_allclose(np.linalg.norm(sph26.v, axis=1), 1.0, atol=1e-15)
    assert abs(sph26.w.sum() - 1.0) < 1e-15
    # antipodal pairs carry equal weight
    for q in range(26):
        p = np.flatnonzero(np.all(np.abs(sph26.v + sph26.v[q]) < 1e-12, axis=1))
        assert len(p) == 1 and sph26.w[p[0]] == sph26.w[q]


@pytest.mark.parametrize("degree", range(0, 8))
def test_sph26_exact_through_degree_7(sph26, degree):
    v, w = sph26.v, sph26.w
    for a in range(degree + 1):
        for b in range(degree + 1 - a):
            c = degree - a - b
            q = (w * v[:, 0] ** a * v[:, 1] ** b * v[:, 2] ** c).sum()
            assert abs(q - sphere_moment(a, b, c)) < 1e-15, (a, b, c)


def test_sph26_not_exact_at_degree_8(sph26):
    """Negative control: the rule has degree exactly 7."""
    v, w = sph26.v, sph26.w
    q = (w * v[:, 0] ** 8).sum()
    assert abs(q - sphere_moment(8, 0, 0)) > 1e-3


@pytest.mark.parametrize("degree", range(0, 8))
def test_circ8_exact_through_degree_7(circ8, degree):
    v, w = circ8.v, circ8.w
    for a in range(degree + 1):
        b = degree - a
        q = (w * v[:, 0] ** a * v[:, 1] ** b).sum()
        assert abs(q - circle_moment(a, b)) < 1e-15, (a, b)


def _delta_product(pairs, idx, values):
    out = 1.0
    for p, r in pairs:
        out *= 1.0 if values[idx.index(p)] == values[idx.index(r)] else 0.0
    return out


def _polys(v):
    P0 = np.ones(len(v))
    P1 = v
    P2 = v[:, :, None] * v[:, None, :] - np.eye(3)[None] / 3.0
    return P0, P1, P2


def test_printed_angular_relations_hold_on_sph26(sph26):
    """App. A orthogonality and App. B angular integrals, as printed."""
    rel = json.load(open(os.path.join(GOLDEN, "appendix_angular.json")))["relations"]
    v, w = sph26.v, sph26.w
    P0, P1, P2 = _polys(v)
    for r in rel:
        idx = r["indices"]
        for values in itertools.product(range(3), repeat=len(idx)):
            if r["lhs"] == "P0 P0":
                lhs = (w * P0 * P0).sum()
            elif r["lhs"] == "P1_i P1_j":
                lhs = (w * P1[:, values[0]] * P1[:, values[1]]).sum()
            elif r["lhs"] == "P2_ij P2_lm":
                lhs = (w * P2[:, values[0], values[1]] * P2[:, values[2], values[3]]).sum()
            elif r["lhs"] == "v_i v_j":
                lhs = (w * v[:, values[0]] * v[:, values[1]]).sum()
            elif r["lhs"] == "v_i v_j v_l v_m":
                lhs = (w * v[:, values[0]] * v[:, values[1]] * v[:, values[2]]
                       * v[:, values[3]]).sum()
            else:
                raise AssertionError(r["lhs"])
            rhs = sum(c * _delta_product(pairs, idx, values) for c, pairs in r["terms"])
            assert abs(lhs - rhs) < 1e-15, (r["cite"], values, lhs, rhs)
