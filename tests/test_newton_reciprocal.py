"""The cone kernels' Newton reciprocal along a voxel column, emulated in float32.

Where den changes by at most 2.5e-4 of itself per voxel step, the kernels start
from a hardware reciprocal (within 1 ulp) at the segment's first voxel and then
take r <- r + r (1 - den r) (two fused multiply-adds) at each further voxel.
One Newton step from a start that is off by e relatively lands off by about
e^2, and the start is off by the step's change in den plus the previous error.
This checks that the relative error stays at float32 rounding over 16-voxel
segments at the plan's largest allowed change and with the worst start.
"""
import numpy as np

F32 = np.float32


def fma32(a, b, c):
    # float32 fused multiply-add: exact product and sum in float64, one rounding
    return F32(np.float64(a) * np.float64(b) + np.float64(c))


def newton_walk(den0, dden, r0, n):
    r, out = r0, [r0]
    for z in range(1, n):
        den = fma32(F32(z), dden, den0)
        r = fma32(r, fma32(-den, r, F32(1.0)), r)
        out.append(r)
    return np.array(out, np.float64)


def test_error_stays_at_rounding_at_the_threshold():
    rng = np.random.Generator(np.random.PCG64(11))
    worst = 0.0
    for _ in range(2000):
        den0 = F32(rng.uniform(0.3, 2.0))
        dden = F32(rng.choice([-1.0, 1.0]) * 2.5e-4 * float(den0) * rng.uniform(0.5, 1.0))
        exact0 = 1.0 / np.float64(den0)
        r0 = F32(exact0) * F32(1.0 + rng.choice([-1.0, 0.0, 1.0]) * 2.0 ** -23)   # within 1 ulp
        got = newton_walk(den0, dden, r0, 16)
        dens = np.array([fma32(F32(z), dden, den0) for z in range(16)], np.float64)
        worst = max(worst, float(np.max(np.abs(got * dens - 1.0))))
    assert worst < 3.0e-7, worst


def test_error_grows_past_the_threshold():
    """The same walk at 40x the allowed change in den: the error is no longer at
    rounding (the plan takes the plain reciprocal there)."""
    den0 = F32(0.5)
    dden = F32(1e-2 * 0.5)
    got = newton_walk(den0, dden, F32(1.0 / 0.5), 16)
    dens = np.array([fma32(F32(z), dden, den0) for z in range(16)], np.float64)
    assert float(np.max(np.abs(got * dens - 1.0))) > 1e-5
