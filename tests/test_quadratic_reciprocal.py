"""The cone kernels' reciprocal along a voxel segment, emulated in float32.

Where den changes by at most 2.5e-4 of itself per voxel step, the kernels take
the hardware reciprocal of den at a segment's first voxel (within 1 ulp), refine
it by one Newton step, and evaluate 1/den at voxel z as the quadratic Taylor
polynomial r0 + r1 z + r2 z^2, with r1 = -r0^2 dden and r2 = -r1 r0 dden (two
fused multiply-adds per voxel).  The polynomial's remainder is
(z dden / den)^3 / (1 + z dden / den) of 1/den, below (15 x 2.5e-4)^3 = 5.3e-8
over a 16-voxel segment.  This checks that the relative error stays at float32
rounding at the plan's largest allowed change and with the worst start, and that
it does not at 40x that change (where the plan takes a reciprocal per voxel).
"""
import numpy as np

F32 = np.float32


def fma32(a, b, c):
    # float32 fused multiply-add: exact product and sum in float64, one rounding
    return F32(np.float64(a) * np.float64(b) + np.float64(c))


def mul32(a, b):
    return F32(np.float64(a) * np.float64(b))


def quadratic_walk(den0, dden, r_start, n):
    r0 = fma32(r_start, fma32(-den0, r_start, F32(1.0)), r_start)   # one Newton step
    r1 = mul32(mul32(-r0, r0), dden)
    r2 = mul32(mul32(-r1, r0), dden)
    out = [r0]
    for z in range(1, n):
        out.append(fma32(F32(z), r1, fma32(F32(z * z), r2, r0)))
    return np.array(out, np.float64)


def rel_error(den0, dden, r_start, n=16):
    got = quadratic_walk(den0, dden, r_start, n)
    dens = np.float64(den0) + np.arange(n) * np.float64(dden)   # the exact den of each voxel
    return float(np.max(np.abs(got * dens - 1.0)))


def test_error_stays_at_rounding_at_the_threshold():
    rng = np.random.Generator(np.random.PCG64(11))
    worst = 0.0
    for _ in range(2000):
        den0 = F32(rng.uniform(0.3, 2.0))
        dden = F32(rng.choice([-1.0, 1.0]) * 2.5e-4 * float(den0) * rng.uniform(0.5, 1.0))
        r_start = F32(1.0 / np.float64(den0)) * F32(1.0 + rng.choice([-1.0, 0.0, 1.0]) * 2.0 ** -23)   # within 1 ulp
        worst = max(worst, rel_error(den0, dden, r_start))
    assert worst < 3.0e-7, worst


def test_error_grows_past_the_threshold():
    """At 40x the allowed change in den the cubic remainder is far above rounding."""
    den0 = F32(0.5)
    assert rel_error(den0, F32(1e-2 * 0.5), F32(1.0 / 0.5)) > 1e-5
