"""Fixed-point stages on inputs of high dynamic range, against the oracle.

The splat (dc_weight_radon, dc_detector_bp_adjoint) and the cone FP
(dc_cone_bp_adjoint) accumulate integer multiples of a unit tied to the largest
term: splat unit = max |term| over the view / splat_qmax; cone unit =
max |Gf| (D/U)^2_max(view) / cone_qmax (both from dc_plan_bounds).  Each term is
rounded once, so an output's absolute error is at most half a unit per rounded
term it sums:
  splat:   R(m) = a(m) - b(m) + b(m-1): at most 3 splat_max_terms terms,
  cone FP: A - B - C + E + (B - E)_left + (C - E)_below + E_diag: at most
           9 cone_max_terms terms,
times the stage's scale, plus the float32 rounding of the output.  These bounds
are asserted element by element on
  * magnitudes log-uniform over [1e-6, 1] with random signs, where the relative
    L2 error must also meet the float32 bar (the large outputs dominate it), and
  * one spike of 1e6 on a U[-1, 1] background, where outputs far below the
    spike's are accurate only to the spike's unit (the measured error is printed).
"""
import math

import numpy as np
import pytest

import synth
from oracle import pipeline as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    grid = synth.Grid(nu=70, nv=53, du=1.0, dv=1.1, n_theta=37, n_s=synth.radon_bins(70, 53), ds=1.0,
                      nx=41, ny=35, nz=27, vx=0.8, vy=0.8, vz=0.9, ox=0.4, oy=-0.3, oz=0.2)
    views = synth.sinusoid_orbit(7, 750.0, 1200.0)
    print("\n[gpu dynamic range]", grid.as_dict(), "views", len(views), flush=True)
    return P, grid, views, P.Plan(grid, views), P.plan_bounds(grid, views)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def log_uniform(shape, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    return (np.sign(r.uniform(-1, 1, shape)) * 10.0 ** r.uniform(-6, 0, shape)).astype(np.float32)


def spike(shape, seed, where):
    r = np.random.Generator(np.random.PCG64(seed))
    x = r.uniform(-1, 1, shape).astype(np.float32)
    x[where] = 1e6
    return x


def _check_splat(got, ref, terms, scale, b, name):
    """Per view: |got - ref| <= 1.5 splat_max_terms scale unit + output rounding."""
    worst = 0.0
    for v in range(ref.shape[0]):
        unit = float(np.abs(terms[v]).max()) / b["splat_qmax"]
        bound = 1.5 * b["splat_max_terms"] * scale * unit + 2.0 ** -23 * np.abs(ref[v])
        err = np.abs(got[v] - ref[v])
        assert np.all(err <= bound), (name, v, float((err / bound).max()))
        worst = max(worst, float((err / bound).max()))
    return worst


@pytest.mark.parametrize("kind", ["log-uniform", "spike"])
def test_splats_on_high_dynamic_range_inputs(setup, kind):
    P, g, views, plan, b = setup
    V = len(views)
    shape = (V, g.nv, g.nu)
    x = log_uniform(shape, 61) if kind == "log-uniform" else spike(shape, 62, (slice(None), 20, 31))
    # weighted Radon: the terms are w_cos g
    R = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_weight_radon(plan, dev(x), R)
    ref = O.weight_radon(x.astype(np.float64), g, views)
    wc = np.stack([O.w_cos(g, O.view_frame(views, v)[5]) for v in range(V)])
    r1 = _check_splat(host(R), ref, wc * x, g.du * g.dv / g.ds, b, "weight_radon")
    e1 = rel(host(R), ref)
    # detector Radon: the terms are GgF
    P.dc_detector_bp_adjoint(plan, dev(x), R)
    ref2 = O.detector_bp_adjoint(x.astype(np.float64), g)
    r2 = _check_splat(host(R), ref2, x, math.pi / g.n_theta, b, "detector_bp_adjoint")
    e2 = rel(host(R), ref2)
    msg = "[gpu dynamic range] splats, %s: rel-L2 %.2e / %.2e, max error / bound %.3f / %.3f" % (
        kind, e1, e2, r1, r2)
    if kind == "spike":
        # outputs the spike does not reach: error against their own size
        far = np.abs(ref2) < 1e-3 * np.abs(ref2).max()
        msg += ", detector Radon away from the spike: rel-L2 %.2e" % rel(host(R)[far], ref2[far])
    print(msg, flush=True)
    if kind == "log-uniform":
        assert max(e1, e2) < 1e-5


@pytest.mark.parametrize("kind", ["log-uniform", "spike"])
def test_cone_fp_on_high_dynamic_range_inputs(setup, kind):
    P, g, views, plan, b = setup
    V = len(views)
    shape = (g.nz, g.ny, g.nx)
    Gf = log_uniform(shape, 63) if kind == "log-uniform" else spike(shape, 64, (13, 17, 20))
    fr = np.random.Generator(np.random.PCG64(65)).uniform(-0.2, 1, shape).astype(np.float32)   # ReLU mask
    GgF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_cone_bp_adjoint(plan, dev(Gf), GgF, f_relu=dev(fr))
    got = host(GgF)
    ref = O.cone_bp_adjoint(Gf.astype(np.float64), g, views, relu_f=fr)
    gmax = float(np.abs(Gf * (fr > 0)).max())
    corners = np.array([[z, y, x] for z in (0, g.nz - 1) for y in (0, g.ny - 1) for x in (0, g.nx - 1)])
    worst = 0.0
    for v in range(V):
        _, _, U, D = O.project_points(O.voxel_centres(g, corners), g, views.subset([v]), 0)
        unit = gmax * float(((D / U) ** 2).max()) / b["cone_qmax"]
        bound = 4.5 * b["cone_max_terms"] * unit + 2.0 ** -23 * np.abs(ref[v])
        err = np.abs(got[v] - ref[v])
        assert np.all(err <= bound), (v, float((err / bound).max()))
        worst = max(worst, float((err / bound).max()))
    e = rel(got, ref)
    msg = "[gpu dynamic range] cone FP, %s: rel-L2 %.2e, max error / bound %.3f" % (kind, e, worst)
    if kind == "spike":
        far = np.abs(ref) < 1e-3 * np.abs(ref).max()
        msg += ", away from the spike: rel-L2 %.2e" % rel(got[far], ref[far])
    print(msg, flush=True)
    if kind == "log-uniform":
        assert e < 1e-5
