"""Per-field error of every storage form on the full-size workloads.

After 8 steps of the 2048^2 (shell [8, 12], tau 0.52) and 8192^2 (shell
[32, 40], tau 0.505) forced workloads from their seeded initial state, the
library's fields -- eps, beta and the six planes T^{00}, T^{0x}, T^{0y},
T^{xx}, T^{xy}, T^{yy} -- at 24 sampled sites are compared with the oracle's
fields at the same sites (``tests/golden/field_windows.json``, written by
``tests/golden/make_field_windows.py`` from oracle windows; Sec. III A/B
moments and Landau frame, Sec. III C step, Sec. V forcing).  Errors are
normwise per field, max |got - want| / max |want| over the sites, beta as a
vector (both components over the largest |beta| component).  The bound of
each storage form follows from its rounding: the reduced forms start from
the state rounded to their storage, and that rounding (relative to |F - 1|,
which is about three times |beta| here) carries into beta directly.
"""
import json
import os

import numpy as np
import pytest

import paper_2101_06187_amd as rl
import workloads

from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "field_windows.json")
FIELDS = ("eps", "beta", "T00", "T0x", "T0y", "Txx", "Txy", "Tyy")

# normwise bounds per storage form: (eps and the diagonal T planes, beta and
# the off-diagonal / momentum planes)
# the planes of the flow (beta, T^{0x}, T^{0y}, T^{xy}) are three orders of
# magnitude smaller than eps here, so their relative errors are larger.
# Measured on the GPU: F64 3e-15 / 8e-13, F32 1e-9 / 6e-7, F16S 1e-6 / 5e-4,
# BF16S 1.3e-5 / 4e-3; the bounds leave a factor of about ten.
BOUNDS = {"F64": (1e-13, 1e-11), "F32": (1e-8, 6e-6), "F16S": (1e-5, 5e-3), "BF16S": (1e-4, 4e-2)}


def field_errors_at(lat, xs, ys, want):
    """Normwise per-field errors of the library's fields at (xs, ys)."""
    import torch
    e, bx, by, T = lat.fields()
    iy = torch.as_tensor(ys, device="cuda:0")
    ix = torch.as_tensor(xs, device="cuda:0")
    got = {"eps": host(e[iy, ix]), "beta_x": host(bx[iy, ix]), "beta_y": host(by[iy, ix])}
    for i, name in enumerate(("T00", "T0x", "T0y", "Txx", "Txy", "Tyy")):
        got[name] = host(T[i][iy, ix])
    del e, bx, by, T
    out = {}
    for name in ("eps", "T00", "T0x", "T0y", "Txx", "Txy", "Tyy"):
        w = np.asarray(want[name])
        out[name] = float(np.abs(got[name] - w).max() / np.abs(w).max())
    wx, wy = np.asarray(want["beta_x"]), np.asarray(want["beta_y"])
    vmax = max(np.abs(wx).max(), np.abs(wy).max())
    out["beta"] = float(max(np.abs(got["beta_x"] - wx).max(), np.abs(got["beta_y"] - wy).max()) / vmax)
    return out


@pytest.mark.parametrize("name", ["forced2048", "forced8192"])
@pytest.mark.parametrize("storage,form", [("F64", None), ("F32", None), ("F32", ("march2", 16)),
                                          ("F16S", ("march_pairs", 0)), ("BF16S", None)])
def test_fields_after_eight_steps(name, storage, form):
    import torch
    gold = json.load(open(GOLDEN))
    steps = gold["steps"]
    case = gold["workloads"][name]
    wl = workloads.WORKLOADS[name]
    A, klo, khi, seed = wl.forcing
    say("fields", name, storage, form)
    lat = rl.Lattice(wl.n, wl.n, wl.tau, storage=storage, forcing=rl.Forcing(A, klo, khi, seed))
    if form is not None:
        lat.set_kernel(*form)
    e, bx, by = workloads.initial_fields(wl)
    lat.set_state(dev(e), dev(bx), dev(by))
    del e, bx, by
    lat.step(steps)
    assert lat.check() == rl.OK
    errs = field_errors_at(lat, case["x"], case["y"], case["fields"])
    lat.close()
    torch.cuda.empty_cache()
    say({k: f"{v:.2e}" for k, v in errs.items()})
    b_diag, b_flow = BOUNDS[storage]
    for k in ("eps", "T00", "Txx", "Tyy"):
        assert errs[k] < b_diag, (k, errs[k])
    for k in ("beta", "T0x", "T0y", "Txy"):
        assert errs[k] < b_flow, (k, errs[k])
