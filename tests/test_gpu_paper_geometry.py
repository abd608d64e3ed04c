"""Every stage against the float64 oracle on the paper's own reconstruction
geometry (its Tables 1 and 2): a 128 x 512 x 512 volume of 0.25 mm voxels, 400
views of a non-square 620 x 480 detector with 0.616 mm pixels, the sinusoid with
a 20 degree tilt and frequency 5, and a Radon grid of 360 x 785.  Each stage runs
over all 400 views, as a reconstruction runs it; the oracle checks two views
(the first and one near the orbit's steepest tilt) for the 2D stages and the cone
FP, and 600 random voxels for the cone BP.  The cone FP's gradient is nonzero on
a random 0.5% of the voxels, so the oracle sums over those only.
"""
import numpy as np
import pytest

import synth
from oracle import pipeline as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VIEWS = [0, 217]
TOL32 = 1e-5


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def urand(shape, seed, lo=-1.0, hi=1.0):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    return torch.rand(shape, device="cuda", generator=gen) * (hi - lo) + lo


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    grid, views = synth.paper_geometry()
    print("\n[gpu paper geometry]", grid.as_dict(), "views", len(views), flush=True)
    return P, grid, views, P.Plan(grid, views)


def per_view(gpu, ref):
    return [rel(host(gpu[v]), ref[i]) for i, v in enumerate(VIEWS)]


@pytest.mark.timeout(600)
def test_weight_radon_and_detector_radon(setup):
    P, grid, views, plan = setup
    V = len(views)
    x = urand((V, grid.nv, grid.nu), 71, 0.0, 1.0)
    R = torch.empty((V, grid.n_theta, grid.n_s), device="cuda")
    P.dc_weight_radon(plan, x, R)
    e1 = per_view(R, O.weight_radon(host(x[VIEWS]), grid, views.subset(VIEWS)))
    P.dc_detector_bp_adjoint(plan, x, R)
    e2 = per_view(R, O.detector_bp_adjoint(host(x[VIEWS]), grid))
    print("[gpu paper geometry] weight_radon", e1, "detector_bp_adjoint", e2, flush=True)
    assert max(e1 + e2) < TOL32


@pytest.mark.timeout(600)
def test_detector_bp(setup):
    P, grid, views, plan = setup
    V = len(views)
    H = urand((V, grid.n_theta, grid.n_s), 72)
    gF = torch.empty((V, grid.nv, grid.nu), device="cuda")
    P.dc_detector_bp(plan, H, gF)
    e = per_view(gF, O.detector_bp(host(H[VIEWS]), grid))
    print("[gpu paper geometry] detector_bp", e, flush=True)
    assert max(e) < TOL32


@pytest.mark.timeout(600)
def test_cone_bp_at_sampled_voxels(setup):
    P, grid, views, plan = setup
    V = len(views)
    gF = urand((V, grid.nv, grid.nu), 73)
    f = torch.empty(plan.vol_shape, device="cuda")
    P.dc_cone_bp(plan, gF, f)
    rng = np.random.Generator(np.random.PCG64(74))
    idx = np.stack([rng.integers(0, n, 600) for n in (grid.nz, grid.ny, grid.nx)], axis=1)
    ref = O.cone_bp(host(gF), grid, views, points=O.voxel_centres(grid, idx))
    got = f.cpu().numpy()[idx[:, 0], idx[:, 1], idx[:, 2]]
    e = rel(got, ref)
    print("[gpu paper geometry] cone_bp at 600 voxels", e, flush=True)
    assert e < TOL32


@pytest.mark.timeout(600)
def test_cone_bp_adjoint_on_sampled_views(setup):
    P, grid, views, plan = setup
    V = len(views)
    rng = np.random.Generator(np.random.PCG64(75))
    flat = np.unique(rng.integers(0, grid.nx * grid.ny * grid.nz, int(0.005 * grid.nx * grid.ny * grid.nz)))
    iz, rem = np.divmod(flat, grid.nx * grid.ny)
    iy, ix = np.divmod(rem, grid.nx)
    idx = np.stack([iz, iy, ix], axis=1)
    sel = torch.as_tensor(flat, device="cuda")
    vals, frl = urand((len(flat),), 76), urand((len(flat),), 77)
    Gf = torch.zeros(grid.nx * grid.ny * grid.nz, device="cuda")
    fr = torch.zeros_like(Gf)
    Gf[sel], fr[sel] = vals, frl
    GgF = torch.empty((V, grid.nv, grid.nu), device="cuda")
    P.dc_cone_bp_adjoint(plan, Gf.view(plan.vol_shape), GgF, f_relu=fr.view(plan.vol_shape))
    ref = O.cone_bp_adjoint(host(vals), grid, views.subset(VIEWS), relu_f=host(frl), support=idx)
    e = per_view(GgF, ref)
    print("[gpu paper geometry] cone_bp_adjoint", e, flush=True)
    assert max(e) < TOL32
