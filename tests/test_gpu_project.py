"""GPU Siddon projector (data generation) against the oracle's Siddon: ragged and
C1 grids on sinusoid, circle+arc and random nearest-neighbour orbits, sampled
rays at the full C2 size, and batched plans reading each scan's own volume."""
import numpy as np
import pytest

import synth
from oracle import siddon as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-6   # float32 output of a float64 walk


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


def ragged():
    return synth.Grid(nu=70, nv=53, du=1.0, dv=1.1, n_theta=37, n_s=synth.radon_bins(70, 53), ds=1.0,
                      nx=41, ny=35, nz=27, vx=0.8, vy=0.8, vz=0.9, ox=0.4, oy=-0.3, oz=0.2)


CASES = {
    "ragged-sinusoid": lambda: (ragged(), synth.sinusoid_orbit(7, 750.0, 1200.0)),
    "ragged-circle+arc": lambda: (ragged(), synth.circle_arc_orbit(3, 4, 750.0, 1200.0, 30.0)),
    "C1-random-nn": lambda: (synth.config_geometry("C1")[0], synth.random_nn_orbit(6, 750.0, 1200.0, 10.0, 3)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_projector_matches_oracle_siddon(P, name):
    g, views = CASES[name]()
    rng = np.random.Generator(np.random.PCG64(1))
    vol = rng.uniform(0, 1, (g.nz, g.ny, g.nx)).astype(np.float32)
    plan = P.Plan(g, views)
    out = torch.empty((len(views), g.nv, g.nu), device="cuda")
    P.dc_project(plan, torch.as_tensor(vol, device="cuda"), out)
    ref = S.project(vol.astype(np.float64), g, views)
    assert rel(out.cpu().numpy(), ref) < TOL
    # a view range writes only its views
    out2 = torch.full_like(out, 7.0)
    P.dc_project(plan, torch.as_tensor(vol, device="cuda"), out2, v0=1, nv=2)
    assert torch.equal(out2[1:3], out[1:3]) and bool((out2[0] == 7.0).all())


def test_projector_full_size_sampled_rays(P):
    g, views = synth.config_geometry("C2")
    ell = synth.random_ellipsoids(20, g.nx * g.vx, 2)
    vol = synth.voxelize_torch(ell, g, device="cuda").float().contiguous()
    plan = P.Plan(g, views)
    out = torch.empty((len(views), g.nv, g.nu), device="cuda")
    P.dc_project(plan, vol, out)
    rng = np.random.Generator(np.random.PCG64(5))
    vh = vol.double().cpu().numpy()
    got, ref = [], []
    for v in (0, 247, 495):
        jj, ii = rng.integers(0, g.nv, 1500), rng.integers(0, g.nu, 1500)
        x = (ii - (g.nu - 1) / 2.0) * g.du
        y = (jj - (g.nv - 1) / 2.0) * g.dv
        p1 = views.det_center[v][None, :] + x[:, None] * views.ex[v] + y[:, None] * views.ey[v]
        p0 = np.broadcast_to(views.src[v], p1.shape)
        ref.append(S.project_rays(vh, g, p0, p1))
        got.append(out[v].cpu().numpy()[jj, ii])
    assert rel(np.concatenate(got), np.concatenate(ref)) < TOL


def test_batched_plan_projects_each_scan_with_its_volume(P):
    g = ragged()
    sets = [synth.sinusoid_orbit(5, 750.0, 1200.0), synth.random_nn_orbit(4, 750.0, 1200.0, 10.0, 1)]
    B = P.Plan.batched(g, sets)
    rng = np.random.Generator(np.random.PCG64(2))
    vols = torch.as_tensor(rng.uniform(0, 1, (2, g.nz, g.ny, g.nx)).astype(np.float32), device="cuda")
    out = torch.empty((B.n_views, g.nv, g.nu), device="cuda")
    P.dc_project(B, vols, out)
    f0 = B.first_view
    for s, v in enumerate(sets):
        one = torch.empty((len(v), g.nv, g.nu), device="cuda")
        P.dc_project(P.Plan(g, v), vols[s].clone(), one)
        assert torch.equal(out[f0[s]:f0[s + 1]], one), s
