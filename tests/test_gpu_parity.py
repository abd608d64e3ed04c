"""GPU parity: every stage of the HIP library against the FP64 oracle.

Inputs are seeded float32 arrays (or exact ellipsoid projections); the oracle
gets the same float32 values in float64.  Bars (from the specification of this
library): relative L2 <= 1e-5 with float32 storage, <= 5e-3 with bf16 storage of
the filtered sinogram and detector images, gradients <= 1e-4.
"""
import math

import numpy as np
import pytest

import synth
from oracle import pipeline as O
from oracle import smooth as OS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_BF16 = 5e-3
TOL_GRAD = 1e-4


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def ragged_case():
    grid = synth.Grid(nu=70, nv=53, du=1.0, dv=1.1, n_theta=37, n_s=synth.radon_bins(70, 53), ds=1.0,
                      nx=41, ny=35, nz=27, vx=0.8, vy=0.8, vz=0.9, ox=0.4, oy=-0.3, oz=0.2)
    views = synth.sinusoid_orbit(7, 750.0, 1200.0)
    return grid, views


def rolled_circle_case():
    """A circle whose detector is rolled 7 degrees about its normal: den has no
    z-term but num_u does, so the cone stages must take their general form."""
    grid = synth.Grid(nu=46, nv=38, du=1.2, dv=1.2, n_theta=44, n_s=synth.radon_bins(46, 38), ds=1.2,
                      nx=28, ny=28, nz=26, vx=1.0, vy=1.0, vz=1.0)
    v = synth.circle_orbit(10, 750.0, 1200.0)
    c, s = math.cos(math.radians(7.0)), math.sin(math.radians(7.0))
    ex, ey = c * v.ex + s * v.ey, -s * v.ex + c * v.ey
    return grid, synth.Views(v.src, v.det_center, ex, ey, v.tangent, v.meta)


CASES = {
    "ragged": ragged_case,
    "rolled-circle": rolled_circle_case,
    # circle plus a line along z: every view keeps the v axis along z (z-invariant cone forms)
    "circle-line": lambda: (synth.Grid(nu=44, nv=40, du=1.2, dv=1.2, n_theta=40, n_s=synth.radon_bins(44, 40),
                                       ds=1.2, nx=26, ny=26, nz=30, vx=1.0, vy=1.0, vz=1.0),
                            synth.circle_line_orbit(8, 5, 750.0, 1200.0, 20.0)),
    "C1": lambda: synth.config_geometry("C1"),
    "arc": lambda: (synth.Grid(nu=48, nv=40, du=1.2, dv=1.2, n_theta=50, n_s=synth.radon_bins(48, 40), ds=1.2,
                               nx=30, ny=30, nz=30, vx=1.0, vy=1.0, vz=1.0),
                    synth.circle_arc_orbit(4, 8, 750.0, 1200.0, 30.0)),
    # the paper's fourth orbit (Sec. 4.4): random nearest-neighbour source positions
    "random-nn": lambda: (synth.Grid(nu=56, nv=44, du=1.1, dv=1.1, n_theta=41, n_s=synth.radon_bins(56, 44), ds=1.1,
                                     nx=28, ny=26, nz=24, vx=1.0, vy=1.0, vz=1.0),
                          synth.random_nn_orbit(9, 750.0, 1200.0, 10.0, 5)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, P):
    grid, views = CASES[request.param]()
    print("\n[gpu case]", request.param, grid.as_dict(), "views", len(views), flush=True)
    plan = P.Plan(grid, views)
    return request.param, grid, views, plan


def rnd(shape, seed, lo=-1.0, hi=1.0):
    return synth.rand_array(shape, seed, lo, hi)


# ------------------------------------------------------------ forward stages
def test_weight_radon(P, case):
    name, g, views, plan = case
    V = len(views)
    x = rnd((V, g.nv, g.nu), 1, 0.0, 1.0)
    R = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_weight_radon(plan, dev(x), R)
    ref = O.weight_radon(x.astype(np.float64), g, views)
    assert rel(host(R), ref) < TOL32


@pytest.mark.parametrize("mode", ["analytic", "raw"])
def test_filter(P, case, mode):
    name, g, views, plan = case
    V = len(views)
    R, M = rnd((V, g.n_theta, g.n_s), 2), rnd((V, g.n_theta, g.n_s), 3, 0.0, 1.0)
    H = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_filter(plan, dev(R), dev(M), H, mode=mode)
    ref = O.filter_stack(R.astype(np.float64), M.astype(np.float64), g, views, mode)
    assert rel(host(H), ref) < TOL32


def test_detector_bp(P, case):
    name, g, views, plan = case
    V = len(views)
    H = rnd((V, g.n_theta, g.n_s), 4)
    gF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_detector_bp(plan, dev(H), gF)
    assert rel(host(gF), O.detector_bp(H.astype(np.float64), g)) < TOL32


def test_cone_bp(P, case):
    name, g, views, plan = case
    V = len(views)
    gF = rnd((V, g.nv, g.nu), 5)
    f = torch.empty((g.nz, g.ny, g.nx), device="cuda")
    P.dc_cone_bp(plan, dev(gF), f)
    ref = O.cone_bp(gF.astype(np.float64), g, views)
    assert rel(host(f), ref) < TOL32
    # accumulate over two view ranges, then ReLU on the last call
    f2 = torch.empty_like(f)
    h = V // 2
    P.dc_cone_bp(plan, dev(gF), f2, v0=0, nv=h)
    P.dc_cone_bp(plan, dev(gF), f2, accumulate=True, relu=True, v0=h, nv=V - h)
    assert rel(host(f2), np.maximum(ref, 0)) < TOL32


# ------------------------------------------------------------ adjoint stages
def test_weight_radon_adjoint(P, case):
    name, g, views, plan = case
    V = len(views)
    GR = rnd((V, g.n_theta, g.n_s), 6)
    Gg = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_weight_radon_adjoint(plan, dev(GR), Gg)
    assert rel(host(Gg), O.weight_radon_adjoint(GR.astype(np.float64), g, views)) < TOL32


@pytest.mark.parametrize("mode", ["analytic", "raw"])
def test_filter_adjoint(P, case, mode):
    name, g, views, plan = case
    V = len(views)
    GH, R, M = rnd((V, g.n_theta, g.n_s), 7), rnd((V, g.n_theta, g.n_s), 8), rnd((V, g.n_theta, g.n_s), 9)
    GM = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    GR = torch.empty_like(GM)
    P.dc_filter_adjoint(plan, dev(GH), dev(R), dev(M), GM=GM, GR=GR, mode=mode)
    rGM, rGR = O.filter_stack_adjoint(GH.astype(np.float64), R.astype(np.float64), M.astype(np.float64), g,
                                      views, mode)
    assert rel(host(GM), rGM) < TOL32
    assert rel(host(GR), rGR) < TOL32
    # accumulate_GM adds to what is there
    P.dc_filter_adjoint(plan, dev(GH), dev(R), dev(M), GM=GM, mode=mode, accumulate_GM=True)
    assert rel(host(GM), 2 * rGM) < TOL32


def test_detector_bp_adjoint(P, case):
    name, g, views, plan = case
    V = len(views)
    GgF = rnd((V, g.nv, g.nu), 10)
    GH = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_detector_bp_adjoint(plan, dev(GgF), GH)
    assert rel(host(GH), O.detector_bp_adjoint(GgF.astype(np.float64), g)) < TOL32


def test_cone_bp_adjoint(P, case):
    name, g, views, plan = case
    V = len(views)
    Gf = rnd((g.nz, g.ny, g.nx), 11)
    fr = rnd((g.nz, g.ny, g.nx), 12)
    GgF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_cone_bp_adjoint(plan, dev(Gf), GgF)
    assert rel(host(GgF), O.cone_bp_adjoint(Gf.astype(np.float64), g, views)) < TOL32
    P.dc_cone_bp_adjoint(plan, dev(Gf), GgF, f_relu=dev(fr))
    assert rel(host(GgF), O.cone_bp_adjoint(Gf.astype(np.float64), g, views, relu_f=fr)) < TOL32


# ---------------------------------------------- Gaussian weight smoothing
def smooth_params(g):
    """The paper's sigma 20 / 121 taps where the angle grid allows it, else scaled down."""
    sigma = 20.0 if g.n_theta > 120 else g.n_theta / 8.0
    return sigma, min(60, int(3 * sigma), g.n_theta - 1, g.n_s - 1)


def test_smooth_weights_and_transpose(P, case):
    name, g, views, plan = case
    V = len(views)
    sigma, radius = smooth_params(g)
    M = rnd((V, g.n_theta, g.n_s), 20, -1.0, 0.0)
    Ms = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_smooth_weights(plan, dev(M), Ms, sigma, radius)
    assert rel(host(Ms), OS.smooth_weights(M.astype(np.float64), sigma, radius)) < TOL32
    G = rnd((V, g.n_theta, g.n_s), 21)
    GM = torch.empty_like(Ms)
    P.dc_smooth_weights_adjoint(plan, dev(G), GM, sigma, radius)
    assert rel(host(GM), OS.smooth_weights_adjoint(G.astype(np.float64), sigma, radius)) < TOL32
    # in place gives the same bits
    X = dev(M)
    P.dc_smooth_weights(plan, X, X, sigma, radius)
    assert torch.equal(X, Ms)
    Y = dev(G)
    P.dc_smooth_weights_adjoint(plan, Y, Y, sigma, radius)
    assert torch.equal(Y, GM)
    # adjoint identity on the GPU
    lhs = float((Ms.double() * dev(G).double()).sum())
    rhs = float((dev(M).double() * GM.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * float(Ms.double().norm() * dev(G).double().norm())


# ------------------------------------------------------ adjoint identities
def test_gpu_adjoint_identities(P, case):
    """<A x, y> = <x, A^T y> for the four stage pairs, evaluated on the GPU in float32."""
    name, g, views, plan = case
    V, K, S = len(views), g.n_theta, g.n_s
    r = torch.Generator(device="cuda").manual_seed(5)
    def N(*shape):
        return torch.randn(shape, device="cuda", generator=r)
    def inner(a, b):
        return float((a.double() * b.double()).sum()), float(a.double().norm() * b.double().norm())
    x, y = N(V, g.nv, g.nu), N(V, K, S)
    Ax, Aty = torch.empty_like(y), torch.empty_like(x)
    P.dc_weight_radon(plan, x, Ax); P.dc_weight_radon_adjoint(plan, y, Aty)
    pairs = [(inner(Ax, y), inner(x, Aty))]
    x, y = N(V, K, S), N(V, g.nv, g.nu)
    Ax, Aty = torch.empty_like(y), torch.empty_like(x)
    P.dc_detector_bp(plan, x, Ax); P.dc_detector_bp_adjoint(plan, y, Aty)
    pairs.append((inner(Ax, y), inner(x, Aty)))
    x, y = N(V, g.nv, g.nu), N(g.nz, g.ny, g.nx)
    Ax, Aty = torch.empty_like(y), torch.empty_like(x)
    P.dc_cone_bp(plan, x, Ax); P.dc_cone_bp_adjoint(plan, y, Aty)
    pairs.append((inner(Ax, y), inner(x, Aty)))
    R, M, GH = N(V, K, S), N(V, K, S), N(V, K, S)
    H, GM, GR = torch.empty_like(R), torch.empty_like(R), torch.empty_like(R)
    P.dc_filter(plan, R, M, H); P.dc_filter_adjoint(plan, GH, R, M, GM=GM, GR=GR)
    pairs.append((inner(H, GH), inner(M, GM)))
    pairs.append((inner(H, GH), inner(R, GR)))
    # float32 rounding is relative to |Ax| |y| (Cauchy-Schwarz), not to the
    # possibly cancelling inner product itself
    for (lhs, n1), (rhs, n2) in pairs:
        assert abs(lhs - rhs) <= 1e-6 * max(n1, n2), (lhs, rhs, n1, n2)


# ------------------------------------------------------------- end to end
def _projections(g, views, seed=1, n_ell=5):
    ell = synth.random_ellipsoids(n_ell, min(g.nx * g.vx, g.ny * g.vy, g.nz * g.vz), seed)
    return synth.project_ellipsoids(ell, g, views).numpy().astype(np.float32), ell


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_reconstruction_end_to_end(P, case, store):
    name, g, views, plan = case
    V = len(views)
    gp, _ = _projections(g, views)
    M = np.full((V, g.n_theta, g.n_s), 0.5, np.float32)
    dt = torch.float32 if store == "f32" else torch.bfloat16
    f = P.reconstruct(plan, dev(M), g=dev(gp), store_dtype=dt)
    ref = O.reconstruct(gp.astype(np.float64), M.astype(np.float64), g, views)
    assert rel(host(f), ref) < (TOL32 if store == "f32" else TOL_BF16)


@pytest.mark.parametrize("recompute_R", [False, True])
def test_gradient_wrt_M(P, case, recompute_R):
    """dL/dM against the oracle's chain of transposes; with recompute_R the
    backward rebuilds the Radon stack from g instead of keeping it."""
    name, g, views, plan = case
    V = len(views)
    gp, ell = _projections(g, views)
    rng = np.random.Generator(np.random.PCG64(3))
    M = rng.uniform(0.3, 0.7, (V, g.n_theta, g.n_s)).astype(np.float32)
    target = rng.uniform(0, 1e-3, (g.nz, g.ny, g.nx)).astype(np.float32)
    Mt = dev(M).requires_grad_(True)
    f = P.reconstruct(plan, Mt, g=dev(gp), recompute_R=recompute_R)
    loss = 0.5 * ((f - dev(target)) ** 2).sum()
    loss.backward()
    Gf = O.reconstruct(gp.astype(np.float64), M.astype(np.float64), g, views) - target
    ref = O.grad_M(gp.astype(np.float64), M.astype(np.float64), Gf, g, views)
    assert rel(host(Mt.grad), ref) < TOL_GRAD
    # the layer form gives the same bits
    M2 = dev(M).requires_grad_(True)
    f2 = P.DCFBP(plan, recompute_R=recompute_R).apply(dev(gp), M2)
    (0.5 * ((f2 - dev(target)) ** 2).sum()).backward()
    assert torch.equal(f2, f) and torch.equal(M2.grad, Mt.grad)


def test_gradient_wrt_M_through_the_smoothing_layer(P, case):
    """f = DC-FBP(g; G M) with the Gaussian layer G: dL/dM = G^T dL/dW at W = G M."""
    name, g, views, plan = case
    V = len(views)
    sigma, radius = smooth_params(g)
    gp, _ = _projections(g, views)
    rng = np.random.Generator(np.random.PCG64(5))
    M = rng.uniform(0.3, 0.7, (V, g.n_theta, g.n_s)).astype(np.float32)
    target = rng.uniform(0, 1e-3, (g.nz, g.ny, g.nx)).astype(np.float32)
    Mt = dev(M).requires_grad_(True)
    f = P.reconstruct(plan, Mt, g=dev(gp), smooth=(sigma, radius))
    (0.5 * ((f - dev(target)) ** 2).sum()).backward()
    W = OS.smooth_weights(M.astype(np.float64), sigma, radius)
    fo = O.reconstruct(gp.astype(np.float64), W, g, views)
    assert rel(host(f), fo) < TOL32
    ref = OS.smooth_weights_adjoint(O.grad_M(gp.astype(np.float64), W, fo - target, g, views), sigma, radius)
    assert rel(host(Mt.grad), ref) < TOL_GRAD


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_forward_backward_bit_reproducible(P, case, store):
    """Two runs of the whole chain (forward, ReLU, backward to dL/dM) give identical bits."""
    name, g, views, plan = case
    V = len(views)
    gp, _ = _projections(g, views)
    rng = np.random.Generator(np.random.PCG64(4))
    M = rng.uniform(0.3, 0.7, (V, g.n_theta, g.n_s)).astype(np.float32)
    target = rng.uniform(0, 1e-3, (g.nz, g.ny, g.nx)).astype(np.float32)
    dt = torch.float32 if store == "f32" else torch.bfloat16
    outs = []
    for _ in range(2):
        Mt = dev(M).requires_grad_(True)
        f = P.reconstruct(plan, Mt, g=dev(gp), store_dtype=dt, relu=True)
        ((f - dev(target)) ** 2).sum().backward()
        outs.append((f.detach().clone(), Mt.grad.clone()))
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])


def test_view_ranges_and_empty_range(P, case):
    name, g, views, plan = case
    V = len(views)
    x = dev(rnd((V, g.nv, g.nu), 13))
    full = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_weight_radon(plan, x, full)
    part = torch.full_like(full, 7.0)
    P.dc_weight_radon(plan, x, part, v0=0, nv=1)
    P.dc_weight_radon(plan, x, part, v0=1, nv=V - 1)
    # the splat accumulates in fixed point, so results are bit-reproducible
    assert torch.equal(part, full)
    untouched = torch.full_like(full, 3.0)
    P.dc_weight_radon(plan, x, untouched, v0=2, nv=0)
    assert bool((untouched == 3.0).all())
    f = torch.full((g.nz, g.ny, g.nx), 5.0, device="cuda")
    P.dc_cone_bp(plan, x, f, v0=0, nv=0)              # empty sum, overwrite -> zeros
    assert float(f.abs().max()) == 0.0


def test_c_side_argument_errors(P, case):
    import ctypes
    name, g, views, plan = case
    V = len(views)
    L = P._lib.lib()
    x = torch.zeros(V * g.nv * g.nu + 4, device="cuda")
    R = torch.zeros((V, g.n_theta, g.n_s), device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    mis = ctypes.c_void_p(x.data_ptr() + 4)
    assert L.dc_weight_radon(plan.handle, mis, ctypes.c_void_p(R.data_ptr()), 0, 0, V, s) == P._lib.DC_EALIGN
    ok = ctypes.c_void_p(x.data_ptr())
    assert L.dc_weight_radon(plan.handle, ok, ctypes.c_void_p(R.data_ptr()), 0, 1, V, s) == P._lib.DC_ESHAPE
    assert L.dc_weight_radon(plan.handle, ok, ctypes.c_void_p(R.data_ptr()), 9, 0, V, s) == P._lib.DC_EDTYPE
    assert L.dc_weight_radon(plan.handle, None, ctypes.c_void_p(R.data_ptr()), 0, 0, V, s) == P._lib.DC_EINVAL
    assert "range" in P._lib.last_error() or "null" in P._lib.last_error()
