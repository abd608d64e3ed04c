"""GPU parity at full size on a circular orbit: the benchmark's grid (512 x 512
detector, 256^3 volume) with the 248-view circle of the batched workload.  On
this orbit the detector's v axis stays along z, so the plan takes the
z-invariant forms of the cone backprojection and its transpose (one u and one
weight per voxel column and view), with the same staging and launch shapes as
the benchmark.  The float64 oracle is evaluated on sampled voxels (cone BP) and
sampled views (cone adjoint); the adjoint pairing is checked over all views.
"""
import numpy as np
import pytest

import synth
from oracle import pipeline as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
SAMPLE_VIEWS = [0, 123, 247]


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def circ():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    grid, _ = synth.config_geometry("C2", n_views=4)
    views = synth.circle_orbit(248, 750.0, 1200.0)
    print("\n[gpu full-size circle] C2 grid, 248-view circle", flush=True)
    return P, grid, views, P.Plan(grid, views)


def urand(shape, seed, lo=-1.0, hi=1.0, dtype=torch.float32):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    return (torch.rand(shape, device="cuda", generator=gen, dtype=torch.float32) * (hi - lo) + lo).to(dtype)


def _sample_voxels(g, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.stack([rng.integers(0, m, n) for m in (g.nz, g.ny, g.nx)], axis=1)
    corners = np.array([[z, y, x] for z in (0, g.nz - 1) for y in (0, g.ny - 1) for x in (0, g.nx - 1)])
    return np.concatenate([idx, corners, [[g.nz // 2, g.ny // 2, g.nx // 2]]])


def test_plan_geometry_is_z_invariant(circ):
    """The table the plan builds has no z-term in den or num_u on any view."""
    _, g, views, _ = circ
    assert np.all(views.ex[:, 2] == 0.0)
    assert np.all(np.cross(views.ex, views.ey)[:, 2] == 0.0)


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_circle_cone_bp(circ, store):
    P, g, views, plan = circ
    V = len(views)
    dt = torch.float32 if store == "f32" else torch.bfloat16
    gF = urand((V, g.nv, g.nu), 50, dtype=dt)
    f = torch.empty((g.nz, g.ny, g.nx), device="cuda")
    P.dc_cone_bp(plan, gF, f)
    idx = _sample_voxels(g, 2000, 51)
    pts = O.voxel_points(g)[idx[:, 0], idx[:, 1], idx[:, 2]]
    ref = O.cone_bp(host(gF), g, views, points=pts)
    assert rel(host(f)[idx[:, 0], idx[:, 1], idx[:, 2]], ref) < TOL32


def test_circle_cone_bp_adjoint(circ):
    P, g, views, plan = circ
    V = len(views)
    Gf, fr = urand((g.nz, g.ny, g.nx), 52), urand((g.nz, g.ny, g.nx), 53)
    GgF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_cone_bp_adjoint(plan, Gf, GgF, f_relu=fr)
    ref = O.cone_bp_adjoint(host(Gf), g, views.subset(np.array(SAMPLE_VIEWS)), relu_f=host(fr))
    assert max(rel(host(GgF[v]), ref[i]) for i, v in enumerate(SAMPLE_VIEWS)) < TOL32
    GgF2 = torch.empty_like(GgF)
    P.dc_cone_bp_adjoint(plan, Gf, GgF2, f_relu=fr)
    assert torch.equal(GgF, GgF2)


def test_circle_cone_adjoint_pairing(circ):
    P, g, views, plan = circ
    V = len(views)
    x, y = urand((V, g.nv, g.nu), 54), urand((g.nz, g.ny, g.nx), 55)
    Ax, Aty = torch.empty_like(y), torch.empty_like(x)
    P.dc_cone_bp(plan, x, Ax)
    P.dc_cone_bp_adjoint(plan, y, Aty)
    lhs, rhs = float((Ax.double() * y.double()).sum()), float((x.double() * Aty.double()).sum())
    scale = max(float(Ax.double().norm() * y.double().norm()), float(x.double().norm() * Aty.double().norm()))
    assert abs(lhs - rhs) <= 1e-6 * scale, (lhs, rhs, scale)
