"""Batched plans on the GPU: several scans with different orbits and view counts
share one grid and run every stage in one launch per kernel (the cone stages too:
the sinusoid, circle and circle+arc scans here take the quadratic, z-invariant
and plain forms, and each workgroup of the mixed launch takes its scan's).  Each result must
be bit-identical to the same scan run through its own single-scan plan (whose
parity with the oracle the other GPU tests establish), also for view ranges that
cross sample boundaries, and a training step captured in a HIP graph must
replay to the bits of the eager step.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def scans():
    grid = synth.Grid(nu=70, nv=53, du=1.0, dv=1.1, n_theta=37, n_s=synth.radon_bins(70, 53), ds=1.0,
                      nx=41, ny=35, nz=27, vx=0.8, vy=0.8, vz=0.9, ox=0.4, oy=-0.3, oz=0.2)
    return grid, [synth.sinusoid_orbit(7, 750.0, 1200.0), synth.circle_orbit(5, 750.0, 1200.0),
                  synth.circle_arc_orbit(4, 8, 750.0, 1200.0, 30.0)]


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    grid, sets = scans()
    batched = P.Plan.batched(grid, sets)
    singles = [P.Plan(grid, v) for v in sets]
    print("\n[gpu batched] samples", [len(v) for v in sets], "first", batched.first_view, flush=True)
    return P, grid, sets, batched, singles


def urand(shape, seed, lo=-1.0, hi=1.0):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    return torch.rand(shape, device="cuda", generator=gen) * (hi - lo) + lo


def split(x, plan):
    f = plan.first_view
    return [x[f[s]:f[s + 1]] for s in range(plan.n_samples)]


def test_plan_shapes(setup):
    P, grid, sets, B, singles = setup
    assert B.n_samples == 3 and B.n_views == sum(len(v) for v in sets)
    assert B.vol_shape == (3, grid.nz, grid.ny, grid.nx)
    assert singles[0].n_samples == 1 and singles[0].vol_shape == (grid.nz, grid.ny, grid.nx)


@pytest.mark.parametrize("stage", ["weight_radon", "filter", "detector_bp", "detector_bp_adjoint",
                                   "weight_radon_adjoint"])
def test_view_stages_match_single_plans(setup, stage):
    P, grid, sets, B, singles = setup
    V = B.n_views
    det, sino = (V,) + B.det_shape, (V,) + B.sino_shape
    if stage == "weight_radon":
        x, out, fn = urand(det, 1, 0, 1), torch.empty(sino, device="cuda"), P.dc_weight_radon
    elif stage == "filter":
        x, out = urand(sino, 2), torch.empty(sino, device="cuda")
        M = urand(sino, 3, 0, 1)
        fn = lambda plan, a, b: P.dc_filter(plan, a, M[plan_slice[plan]].clone(), b)  # noqa: E731
    elif stage == "detector_bp":
        x, out, fn = urand(sino, 4), torch.empty(det, device="cuda"), P.dc_detector_bp
    elif stage == "detector_bp_adjoint":
        x, out, fn = urand(det, 5), torch.empty(sino, device="cuda"), P.dc_detector_bp_adjoint
    else:
        x, out, fn = urand(sino, 6), torch.empty(det, device="cuda"), P.dc_weight_radon_adjoint
    f = B.first_view
    plan_slice = {B: slice(0, V)}
    for s, pl in enumerate(singles):
        plan_slice[pl] = slice(f[s], f[s + 1])
    fn(B, x, out)
    for s, pl in enumerate(singles):
        xs = x[f[s]:f[s + 1]].clone()
        os_ = torch.empty_like(out[f[s]:f[s + 1]])
        fn(pl, xs, os_)
        assert torch.equal(out[f[s]:f[s + 1]], os_), (stage, s)


@pytest.mark.parametrize("store", [torch.float32, torch.bfloat16])
def test_cone_stages_match_single_plans(setup, store):
    P, grid, sets, B, singles = setup
    V = B.n_views
    gF = urand((V,) + B.det_shape, 7).to(store)
    f = torch.full(B.vol_shape, 9.0, device="cuda")
    P.dc_cone_bp(B, gF, f, relu=True)
    Gf, fr = urand(B.vol_shape, 8), urand(B.vol_shape, 9)
    GgF = torch.empty((V,) + B.det_shape, device="cuda", dtype=store)
    P.dc_cone_bp_adjoint(B, Gf, GgF, f_relu=fr)
    for s, (pl, gs, Gs) in enumerate(zip(singles, split(gF, B), split(GgF, B))):
        fs = torch.empty(pl.vol_shape, device="cuda")
        P.dc_cone_bp(pl, gs.clone(), fs, relu=True)
        assert torch.equal(f[s], fs), s
        G1 = torch.empty_like(Gs)
        P.dc_cone_bp_adjoint(pl, Gf[s].clone(), G1, f_relu=fr[s].clone())
        assert torch.equal(Gs, G1), s


def test_ranges_across_sample_boundaries(setup):
    P, grid, sets, B, singles = setup
    V, f0 = B.n_views, B.first_view
    gF = urand((V,) + B.det_shape, 10)
    # views 3 .. first[2] + 2: the tail of sample 0, all of sample 1, the head of sample 2
    v0, v1 = 3, f0[2] + 2
    f = torch.full(B.vol_shape, 5.0, device="cuda")
    P.dc_cone_bp(B, gF, f, v0=v0, nv=v1 - v0)
    for s, (lo, hi) in enumerate([(v0, f0[1]), (f0[1], f0[2]), (f0[2], v1)]):
        pl = singles[s]
        ref = torch.empty(pl.vol_shape, device="cuda")
        P.dc_cone_bp(pl, gF[f0[s]:f0[s + 1]].clone(), ref, v0=lo - f0[s], nv=hi - lo)
        assert torch.equal(f[s], ref), s
    # accumulate the rest of sample 0: the whole sample's sum (to rounding order)
    P.dc_cone_bp(B, gF, f, accumulate=True, v0=0, nv=v0)
    full0 = torch.empty(singles[0].vol_shape, device="cuda")
    P.dc_cone_bp(singles[0], gF[:f0[1]].clone(), full0)
    assert float((f[0] - full0).abs().max()) <= 1e-5 * float(full0.abs().max())
    # an empty range writes the empty sum into the sample holding v0 only
    f2 = torch.full(B.vol_shape, 5.0, device="cuda")
    P.dc_cone_bp(B, gF, f2, v0=f0[1], nv=0)
    assert float(f2[1].abs().max()) == 0.0 and bool((f2[0] == 5.0).all()) and bool((f2[2] == 5.0).all())
    # the adjoint over a crossing range: only views in range are written
    Gf = urand(B.vol_shape, 11)
    GgF = torch.full((V,) + B.det_shape, 3.0, device="cuda")
    P.dc_cone_bp_adjoint(B, Gf, GgF, v0=v0, nv=v1 - v0)
    assert bool((GgF[:v0] == 3.0).all()) and bool((GgF[v1:] == 3.0).all())
    for s, (lo, hi) in enumerate([(v0, f0[1]), (f0[1], f0[2]), (f0[2], v1)]):
        pl = singles[s]
        G1 = torch.empty((pl.n_views,) + pl.det_shape, device="cuda")
        P.dc_cone_bp_adjoint(pl, Gf[s].clone(), G1, v0=lo - f0[s], nv=hi - lo)
        assert torch.equal(GgF[lo:hi], G1[lo - f0[s]:hi - f0[s]]), s


def test_batched_gradient_matches_single_plans(setup):
    P, grid, sets, B, singles = setup
    V, f0 = B.n_views, B.first_view
    g = urand((V,) + B.det_shape, 12, 0, 1)
    M = urand((V,) + B.sino_shape, 13, 0.3, 0.7)
    target = urand(B.vol_shape, 14, 0, 1e-3)
    Mt = M.clone().requires_grad_(True)
    f = P.reconstruct(B, Mt, g=g, relu=True)
    ((f - target) ** 2).sum().backward()
    for s, pl in enumerate(singles):
        Ms = M[f0[s]:f0[s + 1]].clone().requires_grad_(True)
        fs = P.reconstruct(pl, Ms, g=g[f0[s]:f0[s + 1]].clone(), relu=True)
        ((fs - target[s]) ** 2).sum().backward()
        assert torch.equal(f[s].detach(), fs.detach()), s
        assert torch.equal(Mt.grad[f0[s]:f0[s + 1]], Ms.grad), s


def test_graph_captured_training_step_replays_to_the_eager_bits(setup):
    """Stage calls enqueue kernels only, so a whole step can be captured; replays
    interleaved with eager work must reproduce the eager step exactly."""
    P, grid, sets, B, singles = setup
    V = B.n_views
    store = torch.bfloat16
    g = urand((V,) + B.det_shape, 15, 0, 1)
    target = urand(B.vol_shape, 16, 0, 1e-3)
    R = torch.empty((V,) + B.sino_shape, device="cuda")
    H = torch.empty((V,) + B.sino_shape, device="cuda", dtype=store)
    gF = torch.empty((V,) + B.det_shape, device="cuda", dtype=store)
    f = torch.empty(B.vol_shape, device="cuda")
    Gf = torch.empty_like(f)
    GgF = torch.empty_like(gF)
    GH = torch.empty_like(H)
    GM = torch.empty((V,) + B.sino_shape, device="cuda")
    M = torch.full((V,) + B.sino_shape, 0.5, device="cuda")

    def step():
        P.dc_weight_radon(B, g, R)
        P.dc_filter(B, R, M, H)
        P.dc_detector_bp(B, H, gF)
        P.dc_cone_bp(B, gF, f, relu=True)
        torch.mul(f - target, 2.0, out=Gf)
        P.dc_cone_bp_adjoint(B, Gf, GgF, f_relu=f)
        P.dc_detector_bp_adjoint(B, GgF, GH)
        P.dc_filter_adjoint(B, GH, R, M, GM=GM)

    step()
    torch.cuda.synchronize()
    eager_f, eager_GM = f.clone(), GM.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                                     # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for r in range(3):
        f.zero_()
        GM.zero_()
        R.fill_(1.0)                               # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(f, eager_f), r
        assert torch.equal(GM, eager_GM), r
