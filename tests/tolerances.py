"""Error bounds of the reduced-precision storage forms against the oracle.

Shared by the GPU parity tests and by the CPU tests that show the bounds are
tight enough to see a wrong force term (``test_tolerance_sensitivity.py``).

Every storage form but F64 computes in FP32 and stores the deviation F - 1
(the rest equilibrium at eps = 1 has F_q = 1 for every q):
  * F32   -- the deviation in FP32 (24 significant bits);
  * F16S  -- in FP16 (11 significant bits, subnormal below 2^-14);
  * BF16S -- in BF16 (8 significant bits, FP32's exponent range).
One step from the same stored inputs then differs from the FP64 oracle by the
FP32 arithmetic of the step -- a few units in the last place of the largest
deviation it handles -- plus, for the 16-bit forms, the rounding of the new
deviation to the storage type (half a unit in its last place).
"""
import numpy as np

# FP32 arithmetic of one step, in units in the last place of the largest
# |F - 1| of the sample.  Measured on the GPU: 2-9 units (the most with a
# strong force on 41 table rows).
F32_ULPS = 16

# The force increment alone (the rest-state probe: at eps = 1, beta = 0 every
# other part of the step is exact): its FP32 synthesis error relative to the
# largest increment of the sample.  Measured on the GPU: 1.8e-7 (2048^2) and
# 2.7e-7 (8192^2, 41 table rows).
REST_F32_REL = 4e-6


def ulp32(scale):
    """Spacing of FP32 numbers at |scale| (2^-23 relative, 2^-149 at 0)."""
    a = np.abs(np.asarray(scale, dtype=np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
    return 2.0 ** (e - 23)


def half_ulp(storage, v):
    """Half the spacing of the storage type at |v| (elementwise, FP64)."""
    a = np.abs(np.asarray(v, dtype=np.float64))
    if storage == "F64":
        return np.zeros_like(a)
    if storage == "F32":
        return 0.5 * ulp32(a)
    if storage == "F16S":
        e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))   # subnormals: spacing 2^-24
        return 0.5 * 2.0 ** (e - 10)
    if storage == "BF16S":
        e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
        return 0.5 * 2.0 ** (e - 7)
    raise ValueError(storage)


def one_step_bound(storage, want_dev, scale=None, steps=1):
    """Elementwise bound on |got - want| for the populations after `steps`
    steps from identical stored inputs.  want_dev = want - 1 (the oracle's new
    deviation); scale = the largest |F - 1| the step handles (default: the
    largest |want_dev|)."""
    want_dev = np.asarray(want_dev, dtype=np.float64)
    if scale is None:
        scale = np.abs(want_dev).max()
    f32 = steps * F32_ULPS * ulp32(scale)
    if storage == "F32":
        return np.full(want_dev.shape, f32)
    # the FP32 result, then rounded once to the storage type; a two-step
    # launch rounds the intermediate row as a one-step launch stores it
    return steps * half_ulp(storage, np.abs(want_dev) + f32) + f32


def rest_force_bound(storage, want_dev):
    """Bound on |got - want| for the rest-state probe: the stored deviation is
    the force increment, computed in FP32 and rounded to the storage type."""
    want_dev = np.asarray(want_dev, dtype=np.float64)
    f32 = REST_F32_REL * np.abs(want_dev).max()
    if storage == "F32":
        return np.full(want_dev.shape, f32)
    return half_ulp(storage, np.abs(want_dev) + f32) + f32
