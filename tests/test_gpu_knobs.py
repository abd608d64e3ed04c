"""The plan's knobs and the autotuner on the GPU.

Every candidate value of every knob, against the float64 oracle at the float32
bar, on a ragged geometry and on the finer-detector geometries that force the
cone BP's staging classes; the knobs whose outputs do not depend on them (splat
angles and cone-FP tile width: integer sums; the detector BP's angle chunk: the
same sums in the same order) are also checked bit for bit.  Then
the autotuner: a timed search returns feasible knobs, the result file is read
back for the same geometry, DCFBP_KNOBS fixes the knobs without timing, and bad
values leave the plan unchanged.
"""
import os

import numpy as np
import pytest

import synth
from oracle import pipeline as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def ragged():
    return (synth.Grid(nu=70, nv=53, du=1.0, dv=1.1, n_theta=37, n_s=synth.radon_bins(70, 53), ds=1.0,
                       nx=41, ny=35, nz=27, vx=0.8, vy=0.8, vz=0.9, ox=0.4, oy=-0.3, oz=0.2),
            synth.sinusoid_orbit(7, 750.0, 1200.0))


def fine_detector(pitch):
    """A 23 x 19 x 13 volume under detectors of decreasing pitch: the cone BP's
    footprint per block grows, which moves it through its staging classes."""
    n = int(round(40 / pitch))
    return (synth.Grid(nu=n, nv=n, du=pitch, dv=pitch, n_theta=12, n_s=synth.radon_bins(n, n), ds=pitch,
                       nx=23, ny=19, nz=13, vx=1.0, vy=1.0, vz=1.0),
            synth.sinusoid_orbit(4, 750.0, 1200.0))


GEOMETRIES = {"ragged": ragged, "pitch-0.6": lambda: fine_detector(0.6), "pitch-0.3": lambda: fine_detector(0.3)}


@pytest.fixture(scope="module", params=list(GEOMETRIES))
def case(request, P):
    grid, views = GEOMETRIES[request.param]()
    print("\n[gpu knobs]", request.param, grid.as_dict(), flush=True)
    return request.param, grid, views, P.Plan(grid, views)


def test_splat_angles(P, case):
    name, g, views, plan = case
    V = len(views)
    x = synth.rand_array((V, g.nv, g.nu), 81, 0.0, 1.0)
    ref = O.weight_radon(x.astype(np.float64), g, views)
    base = None
    for kc in range(1, 9):
        plan.set_knobs(splat_angles=kc)
        R = torch.empty((V, g.n_theta, g.n_s), device="cuda")
        P.dc_weight_radon(plan, dev(x), R)
        assert rel(host(R), ref) < TOL32, kc
        base = R if base is None else base
        assert torch.equal(R, base), kc
    plan.set_knobs(splat_angles=0)


def test_detector_bp_tiles_and_angle_chunks(P, case):
    name, g, views, plan = case
    V = len(views)
    H = synth.rand_array((V, g.n_theta, g.n_s), 82)
    ref = O.detector_bp(H.astype(np.float64), g)
    for tx in (32, 64):
        first = None
        for kc in (16, 32, 64):
            plan.set_knobs(interp_tile_u=tx, interp_angles=kc)
            gF = torch.empty((V, g.nv, g.nu), device="cuda")
            P.dc_detector_bp(plan, dev(H), gF)
            assert rel(host(gF), ref) < TOL32, (tx, kc)
            # the angle chunking does not change the order of the sums
            first = gF if first is None else first
            assert torch.equal(gF, first), (tx, kc)
    plan.set_knobs(interp_tile_u=64, interp_angles=32)


def test_cone_blocks_and_tiles(P, case):
    name, g, views, plan = case
    V = len(views)
    gF = synth.rand_array((V, g.nv, g.nu), 83)
    ref = O.cone_bp(gF.astype(np.float64), g, views)
    outs = []
    for by in (16, 32):
        plan.set_knobs(bp_block_y=by)
        f = torch.empty((g.nz, g.ny, g.nx), device="cuda")
        P.dc_cone_bp(plan, dev(gF), f)
        assert rel(host(f), ref) < TOL32, by
        outs.append(f)
    # the same arithmetic per voxel, unless one block's footprint is too large to
    # stage (fine detectors) and its taps take the direct form with a reciprocal
    # per voxel: then the two agree to float32 rounding of the tap positions, which
    # on the 0.3 mm detector lie up to ~40 pixels from the column's anchor (one
    # ulp of 1/den moves them by ~4e-6 pixel), i.e. to the float32 bar
    assert rel(host(outs[0]), host(outs[1])) < TOL32
    Gf, fr = synth.rand_array((g.nz, g.ny, g.nx), 84), synth.rand_array((g.nz, g.ny, g.nx), 85)
    ref = O.cone_bp_adjoint(Gf.astype(np.float64), g, views, relu_f=fr)
    outs = []
    for ti in (16, 20, 24):
        plan.set_knobs(fp_tile_u=ti)
        GgF = torch.empty((V, g.nv, g.nu), device="cuda")
        P.dc_cone_bp_adjoint(plan, dev(Gf), GgF, f_relu=dev(fr))
        assert rel(host(GgF), ref) < TOL32, ti
        outs.append(GgF)
    assert all(torch.equal(o, outs[0]) for o in outs)
    plan.set_knobs(bp_block_y=32, fp_tile_u=20)


def test_bad_knobs_are_rejected_and_leave_the_plan_unchanged(P):
    g, views = ragged()
    plan = P.Plan(g, views)
    before = plan.knobs()
    for bad in ({"interp_tile_u": 48}, {"interp_angles": 8}, {"bp_block_y": 8}, {"fp_tile_u": 32},
                {"splat_angles": 9}):
        with pytest.raises(P.DcError, match="DC_EINVAL"):
            plan.set_knobs(**bad)
        assert plan.knobs() == before
    # 8 sinogram rows of 4096 bins do not fit a workgroup's LDS
    import dataclasses
    long = P.Plan(dataclasses.replace(g, n_s=4096, ds=0.2), views)
    with pytest.raises(P.DcError, match="DC_ENOTSUP"):
        long.set_knobs(splat_angles=8)
    x = synth.rand_array((len(views), g.nv, g.nu), 86, 0.0, 1.0)
    R = torch.empty((len(views), g.n_theta, 4096), device="cuda")
    P.dc_weight_radon(long, dev(x), R)          # still usable with its old knobs
    torch.cuda.synchronize()


def test_autotune_search_cache_and_environment(P, tmp_path, monkeypatch):
    g, views = ragged()
    plan = P.Plan(g, views)
    cache = str(tmp_path / "knobs.txt")
    monkeypatch.setenv("DCFBP_TUNE_CACHE", cache)
    monkeypatch.delenv("DCFBP_KNOBS", raising=False)
    r = plan.autotune()
    print("\n[gpu knobs] autotune:", r, flush=True)
    assert r["source"] == "timed"
    k = r["knobs"]
    assert 1 <= k["splat_angles"] <= 8 and k["interp_tile_u"] in (32, 64) and k["interp_angles"] in (16, 32, 64)
    assert k["bp_block_y"] in (16, 32) and k["fp_tile_u"] in (16, 20, 24)
    assert plan.knobs() == k and all(ms > 0 for ms in r["ms"].values())
    with open(cache) as fh:
        assert len(fh.read().split()) == 6
    # the same geometry on a new plan reads the file
    plan2 = P.Plan(g, views)
    r2 = plan2.autotune()
    assert r2["source"] == "cache" and r2["knobs"] == k
    # the environment wins, and the stages still match the oracle with its knobs
    monkeypatch.setenv("DCFBP_KNOBS", "splat=3,itile=32,iangles=16,bprows=16,fptile=24")
    r3 = plan2.autotune()
    assert r3["source"] == "environment"
    assert r3["knobs"] == {"splat_angles": 3, "interp_tile_u": 32, "interp_angles": 16, "bp_block_y": 16,
                           "fp_tile_u": 24}
    V = len(views)
    gp = synth.rand_array((V, g.nv, g.nu), 87, 0.0, 1.0)
    M = np.full((V, g.n_theta, g.n_s), 0.5, np.float32)
    f = P.reconstruct(plan2, dev(M), g=dev(gp))
    assert rel(host(f), O.reconstruct(gp.astype(np.float64), M.astype(np.float64), g, views)) < TOL32
    monkeypatch.setenv("DCFBP_KNOBS", "splat=3,nonsense=1")
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        plan2.autotune()
