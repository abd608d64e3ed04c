"""GPU parity at the library's size limits: the longest sinogram row it accepts
(n_s = 4096, staged in LDS by the 2D kernels) and the deepest volume (nz = 1024,
64 slabs of 16 slices in the cone adjoint), and the single-view case, each
against the float64 oracle.  Sizes one above each limit are rejected on the
host before anything is enqueued.
"""
import numpy as np
import pytest

import synth
from oracle import pipeline as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def long_rows():
    # 1024^2 detector at 0.5 mm, 4096 bins at 0.2 mm (819 mm > the 724 mm diagonal)
    return (synth.Grid(nu=1024, nv=1024, du=0.5, dv=0.5, n_theta=16, n_s=4096, ds=0.2,
                       nx=8, ny=8, nz=8, vx=1.0, vy=1.0, vz=1.0),
            synth.sinusoid_orbit(2, 750.0, 1200.0))


def deep_volume(n_views=5):
    # 1024 slices of 0.3 mm on a 256^2 detector at 2 mm; 5 views = one full and one partial view group
    return (synth.Grid(nu=256, nv=256, du=2.0, dv=2.0, n_theta=20, n_s=synth.radon_bins(256, 256), ds=2.0,
                       nx=12, ny=12, nz=1024, vx=1.0, vy=1.0, vz=0.3),
            synth.sinusoid_orbit(n_views, 750.0, 1200.0))


def test_longest_sinogram_rows(P):
    g, views = long_rows()
    print("\n[gpu limits] n_s = 4096", g.as_dict(), flush=True)
    plan = P.Plan(g, views)
    V = len(views)
    x = synth.rand_array((V, g.nv, g.nu), 41, 0.0, 1.0)
    R = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_weight_radon(plan, dev(x), R)
    assert rel(host(R), O.weight_radon(x.astype(np.float64), g, views)) < TOL32
    H = synth.rand_array((V, g.n_theta, g.n_s), 42)
    gF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_detector_bp(plan, dev(H), gF)
    assert rel(host(gF), O.detector_bp(H.astype(np.float64), g)) < TOL32
    GH = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_detector_bp_adjoint(plan, dev(x), GH)
    assert rel(host(GH), O.detector_bp_adjoint(x.astype(np.float64), g)) < TOL32
    M = synth.rand_array((V, g.n_theta, g.n_s), 43, 0.0, 1.0)
    Hf = torch.empty_like(R)
    P.dc_filter(plan, dev(H), dev(M), Hf)
    ref = O.filter_stack(H.astype(np.float64), M.astype(np.float64), g, views)
    assert rel(host(Hf), ref) < TOL32


def test_deepest_volume(P):
    g, views = deep_volume()
    print("\n[gpu limits] nz = 1024", g.as_dict(), flush=True)
    plan = P.Plan(g, views)
    V = len(views)
    gF = synth.rand_array((V, g.nv, g.nu), 44)
    f = torch.empty((g.nz, g.ny, g.nx), device="cuda")
    P.dc_cone_bp(plan, dev(gF), f)
    assert rel(host(f), O.cone_bp(gF.astype(np.float64), g, views)) < TOL32
    Gf, fr = synth.rand_array((g.nz, g.ny, g.nx), 45), synth.rand_array((g.nz, g.ny, g.nx), 46)
    GgF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_cone_bp_adjoint(plan, dev(Gf), GgF, f_relu=dev(fr))
    ref = O.cone_bp_adjoint(Gf.astype(np.float64), g, views, relu_f=fr)
    assert rel(host(GgF), ref) < TOL32


def test_single_view_chain(P):
    g, views = deep_volume(1)
    plan = P.Plan(g, views)
    gp = synth.rand_array((1, g.nv, g.nu), 47, 0.0, 1.0)
    M = np.full((1, g.n_theta, g.n_s), 0.5, np.float32)
    f = P.reconstruct(plan, dev(M), g=dev(gp))
    ref = O.reconstruct(gp.astype(np.float64), M.astype(np.float64), g, views)
    assert rel(host(f), ref) < TOL32


def test_one_above_each_limit_is_rejected(P):
    import dataclasses
    g, views = long_rows()
    with pytest.raises(P.DcError, match="DC_ESHAPE"):
        P.Plan(dataclasses.replace(g, n_s=4097), views)
    g, views = deep_volume()
    with pytest.raises(P.DcError, match="DC_ESHAPE"):
        P.Plan(dataclasses.replace(g, nz=1025), views)


def test_smoothing_arguments_are_checked_on_the_host(P):
    """The smoothing calls reject bad sigma / radius before any launch."""
    g, v = synth.config_geometry("C1", n_views=4)
    plan = P.Plan(g, v)
    M = torch.zeros((4, g.n_theta, g.n_s), device="cuda")
    for sigma, radius, status in [(0.0, 5, "DC_EINVAL"), (2.0, 0, "DC_EINVAL"), (2.0, 256, "DC_EINVAL"),
                                  (2.0, g.n_s, "DC_ESHAPE")]:
        with pytest.raises(P.DcError, match=status):
            P.dc_smooth_weights(plan, M, M, sigma, radius)


def test_wide_shallow_volume_in_the_cone_adjoint(P):
    """An 8200 x 8192 x 1 volume: the cone adjoint's z-bricks (16 slices, 15 of
    them padding here) span more than 2^32 bytes, so brick offsets must be formed
    in 64 bits.  The slice sits 100 mm above the orbit plane, so rays cross it
    obliquely and few voxel centres share a detector cell.  Checked by the
    adjoint identity with the (oracle-tested) cone BP."""
    g = synth.Grid(nu=704, nv=128, du=1.0, dv=4.0, n_theta=8, n_s=synth.radon_bins(704, 128), ds=1.0,
                   nx=8200, ny=8192, nz=1, vx=0.05, vy=0.05, vz=0.5, oz=100.0)
    assert 16 * g.nx * g.ny * 4 > 2 ** 32
    views = synth.circle_orbit(3, 750.0, 1200.0)
    print("\n[gpu limits] 8200 x 8192 x 1", flush=True)
    plan = P.Plan(g, views)
    gen = torch.Generator(device="cuda").manual_seed(9)
    x = torch.randn((len(views), g.nv, g.nu), device="cuda", generator=gen)
    y = torch.randn((g.nz, g.ny, g.nx), device="cuda", generator=gen)
    Ax = torch.empty_like(y)
    Aty = torch.empty_like(x)
    P.dc_cone_bp(plan, x, Ax)
    P.dc_cone_bp_adjoint(plan, y, Aty)
    lhs = float((Ax.double() * y.double()).sum())
    rhs = float((x.double() * Aty.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * float(Ax.double().norm() * y.double().norm())
    assert float(Aty.abs().max()) > 0


def test_smoothing_on_a_long_angle_axis(P):
    """The mu pass stages n_theta + 2 radius rows of a column block in one
    workgroup's LDS: 1200 angles with the paper's radius 60 (1320 rows, above a
    64 KiB budget) against the oracle, and the first size past 160 KiB rejected."""
    import dataclasses
    from oracle import smooth as OS
    g = synth.Grid(nu=56, nv=48, du=1.0, dv=1.0, n_theta=1200, n_s=synth.radon_bins(56, 48), ds=1.0,   # 74 bins
                   nx=12, ny=12, nz=10, vx=1.0, vy=1.0, vz=1.0)
    v = synth.circle_orbit(2, 750.0, 1200.0)
    plan = P.Plan(g, v)
    rng = np.random.Generator(np.random.PCG64(4))
    M = rng.uniform(-1, 0, (2, g.n_theta, g.n_s)).astype(np.float32)
    Ms = torch.empty((2, g.n_theta, g.n_s), device="cuda")
    P.dc_smooth_weights(plan, dev(M), Ms, 20.0, 60)
    assert rel(host(Ms), OS.smooth_weights(M.astype(np.float64), 20.0, 60)) < 1e-5
    GM = torch.empty_like(Ms)
    P.dc_smooth_weights_adjoint(plan, dev(M), GM, 20.0, 60)
    assert rel(host(GM), OS.smooth_weights_adjoint(M.astype(np.float64), 20.0, 60)) < 1e-5
    # r + 1 + 16 (n_theta + 2 r + 4) floats must fit 40960: at 2433 angles radius 59
    # fits (40940) and radius 60 does not (40973)
    # at the bound itself the staged column block fills the LDS: a seeded nonzero
    # weight and its transpose against the oracle there
    big = P.Plan(dataclasses.replace(g, n_theta=2433), v)
    Mb = rng.uniform(-1, 0, (2, 2433, g.n_s)).astype(np.float32)
    Mbs = torch.empty((2, 2433, g.n_s), device="cuda")
    P.dc_smooth_weights(big, dev(Mb), Mbs, 20.0, 59)
    assert rel(host(Mbs), OS.smooth_weights(Mb.astype(np.float64), 20.0, 59)) < 1e-5
    GMb = torch.empty_like(Mbs)
    P.dc_smooth_weights_adjoint(big, dev(Mb), GMb, 20.0, 59)
    assert rel(host(GMb), OS.smooth_weights_adjoint(Mb.astype(np.float64), 20.0, 59)) < 1e-5
    with pytest.raises(P.DcError, match="DC_ENOTSUP"):
        P.dc_smooth_weights(big, Mbs, Mbs, 20.0, 60)


def test_detector_bp_on_bins_five_times_finer_than_pixels(P):
    """Bins of a fifth of the pixel pitch make the detector BP's LDS window 450
    intervals wide (the 512 cap is 128 KiB for 32 angles); such windows take the
    midpoint-local tap form, whose rounding does not grow with the window.  The
    detector BP and the weighted Radon's transpose (both interpolating), and the
    two splats, against the oracle at the float32 bar."""
    g = synth.Grid(nu=64, nv=48, du=1.0, dv=1.0, n_theta=24, n_s=400, ds=0.2,
                   nx=12, ny=12, nz=10, vx=1.0, vy=1.0, vz=1.0)
    views = synth.sinusoid_orbit(3, 750.0, 1200.0)
    plan = P.Plan(g, views)
    rng = np.random.Generator(np.random.PCG64(8))
    V = len(views)
    H = rng.uniform(-1, 1, (V, g.n_theta, g.n_s)).astype(np.float32)
    gF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_detector_bp(plan, dev(H), gF)
    e1 = rel(host(gF), O.detector_bp(H.astype(np.float64), g))
    Gg = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_weight_radon_adjoint(plan, dev(H), Gg)
    e2 = rel(host(Gg), O.weight_radon_adjoint(H.astype(np.float64), g, views))
    x = rng.uniform(-1, 1, (V, g.nv, g.nu)).astype(np.float32)
    R = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_weight_radon(plan, dev(x), R)
    e3 = rel(host(R), O.weight_radon(x.astype(np.float64), g, views))
    P.dc_detector_bp_adjoint(plan, dev(x), R)
    e4 = rel(host(R), O.detector_bp_adjoint(x.astype(np.float64), g))
    print("\n[gpu limits] ds = du/5: detector_bp %.2e, weight_radon_adjoint %.2e, weight_radon %.2e, "
          "detector_bp_adjoint %.2e" % (e1, e2, e3, e4), flush=True)
    assert max(e1, e2, e3, e4) < 1e-5
