"""Pin of the oracle's Philox4x32-10 against the published known-answer vectors."""
import json
import os

import numpy as np

from oracle.philox import philox4x32_10, uniform_open01

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_known_answer_vectors():
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))["vectors"]
    for vec in kat:
        c = [int(x, 16) for x in vec["ctr"]]
        k = [int(x, 16) for x in vec["key"]]
        out = philox4x32_10(*c, *k)
        assert [int(x) for x in out] == [int(x, 16) for x in vec["out"]]


def test_vectorised_matches_scalar():
    m = np.arange(50, dtype=np.uint64)
    vec = philox4x32_10(m, 7, 3, 0, 0x1234, 0x5678)
    for i in range(50):
        sc = philox4x32_10(i, 7, 3, 0, 0x1234, 0x5678)
        assert all(int(vec[j][i]) == int(sc[j]) for j in range(4))


def test_uniform_open_interval():
    u = uniform_open01(np.array([0, 0xFFFFFFFF], dtype=np.uint32))
    assert 0.0 < u[0] < u[1] < 1.0
    assert u[0] == 2.0 ** -33
