"""GPU smooth Crofton weight (eq. 9) against the float64 oracle.

Closed-form orbits (circle, half circle, circle + arc, circle + line) are checked
on every entry of small Radon grids, the sinusoid on sampled entries (the
oracle's per-bin crossing search), the full 496-view sinusoid of the benchmark
workload on sampled entries of a few views, and the weight end to end: the
uniform ball off the mid-plane reconstructed exactly on circle + line with the
GPU weight.  M lies in [0, 1]; float32 storage rounds it by 6e-8, and the two
float64 crossing searches differ by rounding only, so the bar is 1e-6 absolute.

Where the plane is tangent to the orbit at every crossing, eq. 9 is 0/0 and
falls back to 1/n, and whether such a plane still counts as crossing a circle
is decided by rounding (M is then 1/2 on one side and 1 on the other).  On
exactly these entries the geometric factor c_geo of the filter is zero up to
rounding (below 1e-12 of its maximum, against at least 4% of it elsewhere on
these grids), so the weight never reaches the reconstruction there: M is
compared where |c_geo| > 1e-9 max |c_geo|, and M c_geo everywhere.
"""
import math

import numpy as np
import pytest

import synth
from oracle import crofton as C
from oracle import pipeline as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_M = 1e-6


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


def grid(n_theta=24, nu=40, nv=34, du=1.3):
    return synth.Grid(nu=nu, nv=nv, du=du, dv=du, n_theta=n_theta, n_s=synth.radon_bins(nu, nv), ds=du,
                      nx=16, ny=16, nz=12, vx=1.0, vy=1.0, vz=1.0)


ORBITS = {
    "circle": lambda: synth.circle_orbit(36, 750.0, 1200.0),
    "half-circle": lambda: synth.circle_orbit(40, 750.0, 1200.0, start=0.3, span=math.pi),
    "circle+arc": lambda: synth.circle_arc_orbit(12, 36, 750.0, 1200.0, 30.0),
    "circle+line": lambda: synth.circle_line_orbit(36, 11, 750.0, 1200.0, 200.0),
}


def cgeo(g, views, v):
    return O.c_geo(g, views, v)


def compare(M, ref, cg, scale=None):
    """max |M - ref| over the entries the filter uses, and max |(M - ref) c_geo| / max |c_geo|
    (scale: max |c_geo| of the whole view when only some of its entries are given)."""
    scale = np.abs(cg).max() if scale is None else scale
    used = np.abs(cg) > 1e-9 * scale
    return np.max(np.abs(M - ref)[used]), np.max(np.abs((M - ref) * cg)) / scale


def gpu_M(P, plan, views, **kw):
    M = torch.full((plan.n_views,) + plan.sino_shape, float("nan"), device="cuda")
    P.dc_crofton_weights(plan, views.meta["segments"], views.meta["sid"], M, **kw)
    return M


@pytest.mark.parametrize("name", list(ORBITS))
def test_closed_form_orbits_every_entry(P, name):
    g, views = grid(), ORBITS[name]()
    print("\n[gpu crofton]", name, flush=True)
    plan = P.Plan(g, views)
    M = gpu_M(P, plan, views).cpu().numpy().astype(np.float64)
    ref = np.stack([C.M_view_closed_form(views, g, v) for v in range(len(views))])
    cg = np.stack([cgeo(g, views, v) for v in range(len(views))])
    assert np.all(np.isfinite(M)) and M.min() >= 0.0 and M.max() <= 1.0
    d_used, d_all = compare(M, ref, cg)
    assert d_used <= TOL_M and d_all <= TOL_M, (d_used, d_all)


def test_one_half_on_a_full_circle(P):
    """On a full circle every plane through a source point meets the orbit twice
    with equal weight (Sec. 2.4), so M = 1/2 wherever the plane is not the orbit's."""
    g, views = grid(n_theta=16), synth.circle_orbit(36, 750.0, 1200.0)
    plan = P.Plan(g, views)
    M = gpu_M(P, plan, views).cpu().numpy()
    for v in (0, 7, 20):
        cg = O.c_geo(g, views, v)
        np.testing.assert_allclose(M[v][np.abs(cg) > 1e-9], 0.5, rtol=1e-7)


def test_sinusoid_sampled_entries(P):
    g = grid(n_theta=20, nu=36, nv=30, du=1.5)
    views = synth.sinusoid_orbit(24, 750.0, 1200.0, amp_mm=100.0, periods=2)
    plan = P.Plan(g, views)
    M = gpu_M(P, plan, views).cpu().numpy().astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(4))
    for v in (0, 5, 13, 23):
        bins = [(int(rng.integers(g.n_theta)), int(rng.integers(g.n_s))) for _ in range(12)] + [(0, g.n_s // 2)]
        ref = C.M_view(views, g, v, bins=bins)
        got = np.array([M[v, k, m] for k, m in bins])
        cg = cgeo(g, views, v)
        d_used, d_all = compare(got, ref, np.array([cg[k, m] for k, m in bins]), np.abs(cg).max())
        assert d_used <= TOL_M and d_all <= TOL_M, (v, got, ref)


def test_benchmark_sinusoid_sampled_entries(P):
    """The 496-view sinusoid and 360 x 725 Radon grid of the benchmark workload."""
    g, views = synth.config_geometry("C2")
    plan = P.Plan(g, views)
    M = torch.empty((plan.n_views,) + plan.sino_shape, device="cuda")
    sel = (0, 131, 400)
    for v in sel:
        P.dc_crofton_weights(plan, views.meta["segments"], views.meta["sid"], M, v0=v, nv=1)
    Mh = M.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(5))
    for v in sel:
        bins = [(int(rng.integers(g.n_theta)), int(rng.integers(g.n_s))) for _ in range(10)]
        ref = C.M_view(views, g, v, bins=bins)
        got = np.array([Mh[v, k, m] for k, m in bins], np.float64)
        cg = cgeo(g, views, v)
        scale = np.abs(cg).max()
        cgb = np.array([cg[k, m] for k, m in bins])
        used = np.abs(cgb) > 1e-9 * scale
        assert np.max(np.abs(got - ref)[used]) <= TOL_M, (v, got, ref)
        assert np.all(np.isfinite(Mh[v])) and Mh[v].min() >= 0.0 and Mh[v].max() <= 1.0 + 1e-6


def test_view_ranges_and_determinism(P):
    g, views = grid(), ORBITS["circle+arc"]()
    plan = P.Plan(g, views)
    full = gpu_M(P, plan, views)
    part = torch.full_like(full, -1.0)
    P.dc_crofton_weights(plan, views.meta["segments"], views.meta["sid"], part, v0=5, nv=20)
    assert torch.equal(part[5:25], full[5:25])
    assert bool((part[:5] == -1).all()) and bool((part[25:] == -1).all())
    assert torch.equal(gpu_M(P, plan, views), full)


def test_ball_off_midplane_exact_with_gpu_weight(P):
    """Circle + line satisfies Tuy's condition for a ball off the mid-plane: the
    reconstruction with the GPU weight matches the oracle's reconstruction with
    the oracle's weight, and is exact (mean 1 inside the ball)."""
    N = 112
    g = synth.Grid(nu=N, nv=N, du=1.2, dv=1.2, n_theta=120, n_s=synth.radon_bins(N, N), ds=1.2,
                   nx=24, ny=24, nz=12, vx=0.5, vy=0.5, vz=0.5, oz=9.0)
    views = synth.circle_line_orbit(90, 41, 100.0, 200.0, half_len=32.0)
    b = synth.ball([0.0, 0.0, 9.0], 6.0)
    gp = synth.project_ellipsoids(b, g, views).numpy()
    plan = P.Plan(g, views)
    M = gpu_M(P, plan, views)
    f = P.reconstruct(plan, M, g=torch.as_tensor(gp, dtype=torch.float32, device="cuda")).cpu().numpy()
    Mo = np.stack([C.M_view_closed_form(views, g, v) for v in range(len(views))])
    ref = O.reconstruct(gp.astype(np.float32).astype(np.float64), Mo, g, views)
    assert float(np.linalg.norm(f - ref) / np.linalg.norm(ref)) < 1e-5
    X, Y, Z = np.meshgrid(*(((np.arange(n) - (n - 1) / 2) * 0.5 + o) for n, o in ((g.nx, 0.0), (g.ny, 0.0),
                                                                                  (g.nz, 9.0))), indexing="ij")
    inside = (X ** 2 + Y ** 2 + (Z - 9.0) ** 2) < 3.0 ** 2
    assert abs(f.transpose(2, 1, 0)[inside].mean() - 1.0) < 5e-3


def test_argument_checks(P):
    g, views = grid(), ORBITS["circle+arc"]()
    plan = P.Plan(g, views)
    M = torch.empty((plan.n_views,) + plan.sino_shape, device="cuda")
    segs = views.meta["segments"]
    sid = views.meta["sid"]
    bad = [dict(segs[0]), dict(segs[1], start=segs[1]["start"] + 1)]          # gap between segments
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_crofton_weights(plan, bad, sid, M)
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_crofton_weights(plan, segs, sid, M, taper=0.0)
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_crofton_weights(plan, [dict(segs[0], closed=True), segs[1]], sid, M)   # closed arc
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_crofton_weights(plan, [segs[0], dict(segs[1], dlam=segs[1]["dlam"] * 0.9)], sid, M)  # not one turn
    with pytest.raises(ValueError):
        P.dc_crofton_weights(plan, [dict(segs[0], kind="samples"), segs[1]], sid, M)
    batched = P.Plan.batched(g, [views, views])
    Mb = torch.empty((batched.n_views,) + batched.sino_shape, device="cuda")
    with pytest.raises(P.DcError, match="DC_ENOTSUP"):
        P.dc_crofton_weights(batched, segs, sid, Mb)
    import ctypes
    L = P._lib.lib()
    arr = P.ops.make_segments(segs)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    sv = synth.sinusoid_orbit(24, 750.0, 1200.0)
    sp = P.Plan(grid(), sv)
    sarr = P.ops.make_segments(sv.meta["segments"])
    Ms = torch.empty((sp.n_views,) + sp.sino_shape, device="cuda")
    st = L.dc_crofton_weights(sp.handle, sarr, 1, 750.0, 2, 0.05, 0.01, 64, ctypes.c_void_p(Ms.data_ptr()), 0, 24,
                              ctypes.c_void_p(small.data_ptr()), 16, None)
    assert st == P._lib.DC_ESHAPE
    assert L.dc_crofton_workspace_bytes(arr, 2, 64) == 256          # no sinusoid: no sample table
