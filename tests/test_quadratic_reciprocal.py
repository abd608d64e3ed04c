"""The cone kernels' reciprocal along a voxel segment, emulated in float32.

Where den changes by at most 5e-4 of itself per voxel step, the kernels form
den at a segment's middle zc (z = 7.5 of a 16-voxel segment, 3.5 of an 8-voxel
column), take its hardware reciprocal (within 1 ulp), refine it by one Newton
step, and evaluate 1/den at voxel z as the quadratic Taylor polynomial
r0 + r1 t + r2 t^2 in t = z - zc, with r1 = -r0^2 dden and r2 = -r1 r0 dden (two
fused multiply-adds per voxel).  The polynomial's remainder is
(t dden / den)^3 / (1 + t dden / den) of 1/den, below (7.5 x 5e-4)^3 = 5.3e-8
over a 16-voxel segment.  This checks that the relative error stays at float32
rounding at the plan's largest allowed change and with the worst start, for
both segment lengths, and that it does not at 40x that change (where the plan
takes a reciprocal per voxel).
"""
import numpy as np
import pytest

F32 = np.float32


def fma32(a, b, c):
    # float32 fused multiply-add: exact product and sum in float64, one rounding
    return F32(np.float64(a) * np.float64(b) + np.float64(c))


def mul32(a, b):
    return F32(np.float64(a) * np.float64(b))


def quadratic_walk(den0, dden, ulps, n):
    zc = F32(0.5 * (n - 1))
    dc = fma32(zc, dden, den0)                                   # den at the middle
    r_start = F32(1.0 / np.float64(dc)) * F32(1.0 + ulps * 2.0 ** -23)   # hardware reciprocal, within 1 ulp
    r0 = fma32(r_start, fma32(-dc, r_start, F32(1.0)), r_start)   # one Newton step
    r1 = mul32(mul32(-r0, r0), dden)
    r2 = mul32(mul32(-r1, r0), dden)
    out = []
    for z in range(n):
        t = F32(z) - zc
        out.append(fma32(t, r1, fma32(mul32(t, t), r2, r0)))
    return np.array(out, np.float64)


def rel_error(den0, dden, ulps, n=16):
    got = quadratic_walk(den0, dden, ulps, n)
    dens = np.float64(den0) + np.arange(n) * np.float64(dden)   # the exact den of each voxel
    return float(np.max(np.abs(got * dens - 1.0)))


@pytest.mark.parametrize("n", [16, 8])
def test_error_stays_at_rounding_at_the_threshold(n):
    rng = np.random.Generator(np.random.PCG64(11))
    worst = 0.0
    for _ in range(2000):
        den0 = F32(rng.uniform(0.3, 2.0))
        dden = F32(rng.choice([-1.0, 1.0]) * 5e-4 * float(den0) * rng.uniform(0.5, 1.0))
        worst = max(worst, rel_error(den0, dden, rng.choice([-1.0, 0.0, 1.0]), n))
    assert worst < 3.0e-7, worst


def test_error_grows_past_the_threshold():
    """At 40x the allowed change in den the cubic remainder is far above rounding."""
    den0 = F32(0.5)
    assert rel_error(den0, F32(2e-2 * 0.5), 0.0) > 1e-5


def test_expanding_about_the_first_voxel_would_not_hold_at_the_threshold():
    """The same polynomial about a segment's first voxel reaches 15 steps: at the
    5e-4 threshold its remainder, (15 x 5e-4)^3 = 4.2e-7, is above rounding."""
    den0, dden = F32(0.5), F32(5e-4 * 0.5)
    r0 = F32(1.0 / np.float64(den0))
    r1 = mul32(mul32(-r0, r0), dden)
    r2 = mul32(mul32(-r1, r0), dden)
    got = fma32(F32(15), r1, fma32(F32(225), r2, r0))
    assert abs(float(got) * (0.5 + 15 * float(dden)) - 1.0) > 3.0e-7
