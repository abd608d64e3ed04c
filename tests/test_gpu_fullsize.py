"""GPU parity at the full training workload, in the launch configuration the
benchmark times: one plan over all 496 views of the sinusoidal orbit, 512 x 512
detector, Radon 360 x 725, 256^3 volume, every stage called on the whole view
range.  The float64 oracle is evaluated on sampled views (2D stages and the
cone adjoint) or sampled voxels (cone BP); the full-size adjoint pairing and
run-to-run bit equality are checked on the GPU alone.
"""
import numpy as np
import pytest

import synth
from oracle import pipeline as O
from oracle import smooth as OS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
SAMPLE_VIEWS = [0, 247, 495]          # first, middle and last view (last view group)


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def c2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    grid, views = synth.config_geometry("C2")
    print("\n[gpu full-size] C2", grid.as_dict(), "views", len(views), flush=True)
    return P, grid, views, P.Plan(grid, views)


def urand(shape, seed, lo=-1.0, hi=1.0, dtype=torch.float32):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    return (torch.rand(shape, device="cuda", generator=gen, dtype=torch.float32) * (hi - lo) + lo).to(dtype)


def sub(views):
    return views.subset(np.array(SAMPLE_VIEWS))


def per_view(gpu, ref):
    return [rel(host(gpu[v]), ref[i]) for i, v in enumerate(SAMPLE_VIEWS)]


def test_full_weight_radon(c2):
    P, g, views, plan = c2
    V = len(views)
    x = urand((V, g.nv, g.nu), 21, 0.0, 1.0)
    R = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_weight_radon(plan, x, R)
    ref = O.weight_radon(host(x[SAMPLE_VIEWS]), g, sub(views))
    assert max(per_view(R, ref)) < TOL32
    R2 = torch.empty_like(R)
    P.dc_weight_radon(plan, x, R2)
    assert torch.equal(R, R2)          # fixed-point accumulation: bit-reproducible


@pytest.mark.parametrize("mode", ["analytic", "raw"])
def test_full_filter(c2, mode):
    P, g, views, plan = c2
    V = len(views)
    R, M = urand((V, g.n_theta, g.n_s), 22), urand((V, g.n_theta, g.n_s), 23, 0.0, 1.0)
    H = torch.empty_like(R)
    P.dc_filter(plan, R, M, H, mode=mode)
    ref = O.filter_stack(host(R[SAMPLE_VIEWS]), host(M[SAMPLE_VIEWS]), g, sub(views), mode)
    assert max(per_view(H, ref)) < TOL32


def test_full_filter_adjoint(c2):
    P, g, views, plan = c2
    V = len(views)
    GH, R, M = (urand((V, g.n_theta, g.n_s), s) for s in (24, 25, 26))
    GM, GR = torch.empty_like(GH), torch.empty_like(GH)
    P.dc_filter_adjoint(plan, GH, R, M, GM=GM, GR=GR)
    rGM, rGR = O.filter_stack_adjoint(host(GH[SAMPLE_VIEWS]), host(R[SAMPLE_VIEWS]), host(M[SAMPLE_VIEWS]), g,
                                      sub(views))
    assert max(per_view(GM, rGM)) < TOL32
    assert max(per_view(GR, rGR)) < TOL32


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_full_detector_bp(c2, store):
    P, g, views, plan = c2
    V = len(views)
    dt = torch.float32 if store == "f32" else torch.bfloat16
    H = urand((V, g.n_theta, g.n_s), 27, dtype=dt)
    gF = torch.empty((V, g.nv, g.nu), device="cuda", dtype=dt)
    P.dc_detector_bp(plan, H, gF)
    ref = O.detector_bp(host(H[SAMPLE_VIEWS]), g)
    # bf16 output: one rounding of each pixel (2^-9 relative) on top of float32
    assert max(per_view(gF, ref)) < (TOL32 if store == "f32" else 5e-3)


def test_full_detector_bp_adjoint(c2):
    P, g, views, plan = c2
    V = len(views)
    GgF = urand((V, g.nv, g.nu), 28)
    GH = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_detector_bp_adjoint(plan, GgF, GH)
    ref = O.detector_bp_adjoint(host(GgF[SAMPLE_VIEWS]), g)
    assert max(per_view(GH, ref)) < TOL32


def test_full_weight_radon_adjoint(c2):
    P, g, views, plan = c2
    V = len(views)
    GR = urand((V, g.n_theta, g.n_s), 29)
    Gg = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_weight_radon_adjoint(plan, GR, Gg)
    ref = O.weight_radon_adjoint(host(GR[SAMPLE_VIEWS]), g, sub(views))
    assert max(per_view(Gg, ref)) < TOL32


def _sample_voxels(g, n, seed):
    """n random voxel indices plus the 8 corners and the centre, as (iz, iy, ix)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.stack([rng.integers(0, m, n) for m in (g.nz, g.ny, g.nx)], axis=1)
    corners = np.array([[z, y, x] for z in (0, g.nz - 1) for y in (0, g.ny - 1) for x in (0, g.nx - 1)])
    centre = np.array([[g.nz // 2, g.ny // 2, g.nx // 2]])
    return np.concatenate([idx, corners, centre])


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_full_cone_bp(c2, store):
    P, g, views, plan = c2
    V = len(views)
    dt = torch.float32 if store == "f32" else torch.bfloat16
    gF = urand((V, g.nv, g.nu), 30, dtype=dt)
    f = torch.empty((g.nz, g.ny, g.nx), device="cuda")
    P.dc_cone_bp(plan, gF, f)
    idx = _sample_voxels(g, 3000, 31)
    pts = O.voxel_points(g)[idx[:, 0], idx[:, 1], idx[:, 2]]
    ref = O.cone_bp(host(gF), g, views, points=pts)
    got = host(f)[idx[:, 0], idx[:, 1], idx[:, 2]]
    # bf16 storage: the oracle gets the same bf16 values, so only float32
    # arithmetic separates the two
    assert rel(got, ref) < TOL32


def test_full_cone_bp_adjoint(c2):
    P, g, views, plan = c2
    V = len(views)
    Gf, fr = urand((g.nz, g.ny, g.nx), 32), urand((g.nz, g.ny, g.nx), 33)
    GgF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_cone_bp_adjoint(plan, Gf, GgF, f_relu=fr)
    ref = O.cone_bp_adjoint(host(Gf), g, sub(views), relu_f=host(fr))
    assert max(per_view(GgF, ref)) < TOL32
    GgF2 = torch.empty_like(GgF)
    P.dc_cone_bp_adjoint(plan, Gf, GgF2, f_relu=fr)
    assert torch.equal(GgF, GgF2)


def test_full_adjoint_pairings(c2):
    """<A x, y> = <x, A^T y> over all 496 views for the three linear stage pairs."""
    P, g, views, plan = c2
    V = len(views)

    def inner(a, b):
        return float((a.double() * b.double()).sum()), float(a.double().norm() * b.double().norm())

    pairs = []
    x, y = urand((V, g.nv, g.nu), 34), urand((g.nz, g.ny, g.nx), 35)
    Ax, Aty = torch.empty_like(y), torch.empty_like(x)
    P.dc_cone_bp(plan, x, Ax)
    P.dc_cone_bp_adjoint(plan, y, Aty)
    pairs.append((inner(Ax, y), inner(x, Aty)))
    del Ax, Aty
    x, y = urand((V, g.nv, g.nu), 36), urand((V, g.n_theta, g.n_s), 37)
    Ax, Aty = torch.empty_like(y), torch.empty_like(x)
    P.dc_weight_radon(plan, x, Ax)
    P.dc_weight_radon_adjoint(plan, y, Aty)
    pairs.append((inner(Ax, y), inner(x, Aty)))
    x, y = urand((V, g.n_theta, g.n_s), 38), urand((V, g.nv, g.nu), 39)
    Ax, Aty = torch.empty_like(y), torch.empty_like(x)
    P.dc_detector_bp(plan, x, Ax)
    P.dc_detector_bp_adjoint(plan, y, Aty)
    pairs.append((inner(Ax, y), inner(x, Aty)))
    for (lhs, n1), (rhs, n2) in pairs:
        assert abs(lhs - rhs) <= 1e-6 * max(n1, n2), (lhs, rhs, n1, n2)


def test_full_smooth_weights_paper_filter(c2):
    """The paper's Gaussian layer (sigma 20, 121 taps) over all 496 views."""
    P, g, views, plan = c2
    V = len(views)
    M = urand((V, g.n_theta, g.n_s), 40, -1.0, 0.0)
    Ms = torch.empty_like(M)
    P.dc_smooth_weights(plan, M, Ms, 20.0, 60)
    ref = OS.smooth_weights(host(M[SAMPLE_VIEWS]), 20.0, 60)
    assert max(per_view(Ms, ref)) < TOL32
    G = urand((V, g.n_theta, g.n_s), 41)
    GM = torch.empty_like(G)
    P.dc_smooth_weights_adjoint(plan, G, GM, 20.0, 60)
    ref = OS.smooth_weights_adjoint(host(G[SAMPLE_VIEWS]), 20.0, 60)
    assert max(per_view(GM, ref)) < TOL32
