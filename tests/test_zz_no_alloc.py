"""The allocation-free entry point dc_weight_radon_noalloc, called through the C
ABI: its output equals dc_weight_radon's bit for bit (same kernels, scratch in
the library's static device array instead of the plan's) and the oracle's at
the float32 bar, on consecutive calls whose second input is smaller (fewer
views, another plan, a view range), so a stale scale word from the first call
would show; sizes beyond the array are rejected on the host."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import pipeline as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


def _noalloc(P, plan, g, R, v0, nv):
    L = P._lib.lib()
    st = L.dc_weight_radon_noalloc(plan.handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(R.data_ptr()),
                                   P._lib.DC_F32, v0, nv, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _case(P, grid, views, seed, scale):
    V = len(views)
    x = synth.rand_array((V, grid.nv, grid.nu), seed, 0.0, scale)
    g = torch.as_tensor(x, device="cuda")
    plan = P.Plan(grid, views)
    return plan, g, x


def test_noalloc_weight_radon_matches_the_plan_scratch_form(P):
    big_grid, big_views = synth.config_geometry("C1", n_views=12)
    small_grid = synth.Grid(nu=40, nv=36, du=1.0, dv=1.0, n_theta=30, n_s=synth.radon_bins(40, 36), ds=1.0,
                            nx=16, ny=16, nz=12, vx=1.0, vy=1.0, vz=1.0)
    small_views = synth.sinusoid_orbit(5, 750.0, 1200.0)
    # first call: 12 views with values up to 1e3; second: 5 views of another plan
    # with values up to 1 (a stale, larger scale word would coarsen its quantum)
    for grid, views, seed, scale in ((big_grid, big_views, 71, 1e3), (small_grid, small_views, 72, 1.0)):
        plan, g, x = _case(P, grid, views, seed, scale)
        V = len(views)
        R1 = torch.full((V, grid.n_theta, grid.n_s), float("nan"), device="cuda")
        assert _noalloc(P, plan, g, R1, 0, V) == 0, P._lib.last_error()
        R2 = torch.empty_like(R1)
        P.dc_weight_radon(plan, g, R2)
        torch.cuda.synchronize()
        assert torch.equal(R1, R2)
        e = rel(R1.double().cpu().numpy(), O.weight_radon(x.astype(np.float64), grid, views))
        assert e < 1e-5, e
        print("\n[no-alloc] %d views: bit-identical, rel-L2 %.2e" % (V, e), flush=True)
    # a view range of the last plan: only views [1, 4) written, equal to the plan form
    R3 = torch.zeros_like(R1)
    assert _noalloc(P, plan, g, R3, 1, 3) == 0, P._lib.last_error()
    R4 = torch.zeros_like(R1)
    P.dc_weight_radon(plan, g, R4, v0=1, nv=3)
    torch.cuda.synchronize()
    assert torch.equal(R3, R4) and float(R3[0].abs().max()) == 0.0 and float(R3[4].abs().max()) == 0.0


def test_noalloc_weight_radon_rejects_more_views_than_its_scratch(P):
    g = synth.Grid(nu=8, nv=8, du=1.0, dv=1.0, n_theta=4, n_s=12, ds=1.0, nx=4, ny=4, nz=4,
                   vx=1.0, vy=1.0, vz=1.0)
    views = synth.circle_orbit(65537, 750.0, 1200.0)
    plan = P.Plan(g, views)
    x = torch.zeros((65537, 8, 8), device="cuda")
    R = torch.zeros((65537, 4, 12), device="cuda")
    assert _noalloc(P, plan, x, R, 0, 65537) == P._lib.DC_ESHAPE
    assert "65536" in P._lib.last_error()
    assert _noalloc(P, plan, x, R, 1, 65536) == 0
    torch.cuda.synchronize()
    assert float(R.abs().max()) == 0.0
