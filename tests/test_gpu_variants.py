"""GPU parity for code paths that the ordinary test geometries never reach.

- Cone backprojection (eq. 11, A3d^T): a plan stages each view's detector
  footprint of a 16x32x8 voxel block in LDS, rows 64 or 128 pixels apart (the
  smallest pitch that holds the widest footprint over all blocks and views) and
  4, 8, 12 or 16 rows per thread of 512 (512 / pitch rows per pass, enough for
  the tallest footprint); wider or taller footprints take direct global taps.
  Ordinary geometries all fall in the first class (pitch 64, 4 rows).  Finer or
  anisotropic detectors here force each of the others, and `footprint_class`
  checks on the host that they do.
- Splat (the 2D Radon transform of eqs. 7, 8): when the sinogram rows are
  shorter than the detector diagonal, some pixels fall outside every bin, and
  the deposit takes its range-checked form.  The oracle drops those terms.
"""
import math

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


BLOCK = (16, 32, 8)   # voxels per backprojection workgroup along x, y, z
THREADS = 512         # threads per backprojection workgroup (one per x, y column)


def footprint_class(g, views):
    """(row pitch, staged rows per thread) for the widest and the tallest block
    footprint: the box [floor(min) - 1, floor(max) + 2] of the block's projected
    voxel centres on each axis, plus one pixel of slack per side."""
    pts = O.voxel_points(g)
    worst_w = worst_h = 0
    for v in range(len(views)):
        i, j, _, _ = O.project_points(pts, g, views, v)
        for z0 in range(0, g.nz, BLOCK[2]):
            for y0 in range(0, g.ny, BLOCK[1]):
                for x0 in range(0, g.nx, BLOCK[0]):
                    bi = i[z0:z0 + BLOCK[2], y0:y0 + BLOCK[1], x0:x0 + BLOCK[0]]
                    bj = j[z0:z0 + BLOCK[2], y0:y0 + BLOCK[1], x0:x0 + BLOCK[0]]
                    worst_w = max(worst_w, math.floor(bi.max()) - math.floor(bi.min()) + 5)
                    worst_h = max(worst_h, math.floor(bj.max()) - math.floor(bj.min()) + 5)
    pitch = next((p for p in (64, 128) if worst_w <= p), 0)
    if not pitch:
        return (0, 0)
    need = math.ceil(worst_h / (THREADS // pitch))
    stage = next((c for c in (4, 8, 12, 16) if need <= c), 0)
    return (pitch, stage) if stage else (0, 0)


def fine_detector(du, dv):
    """A 64 x 60 mm detector of du x dv pixels over a ragged 23x19x13 volume of 1 mm voxels."""
    nu = int(round(64 / du)) // 2 * 2 + 1
    nv = int(round(60 / dv)) // 2 * 2 + 1
    g = synth.Grid(nu=nu, nv=nv, du=du, dv=dv, n_theta=19, n_s=synth.radon_bins(nu, nv), ds=min(du, dv),
                   nx=23, ny=19, nz=13, vx=1.0, vy=1.0, vz=1.0, ox=0.3, oy=-0.2, oz=0.1)
    return g, synth.sinusoid_orbit(3, 750.0, 1200.0)


# (row pitch, staged rows per thread) -> detector pixel (du, dv) that forces it
STAGING = {(64, 4): (1.0, 0.6), (64, 8): (1.0, 0.5), (64, 12): (1.0, 0.2), (64, 16): (1.0, 0.15),
           (128, 4): (0.5, 1.5), (128, 8): (0.5, 1.0), (128, 12): (0.45, 0.4725), (128, 16): (0.3, 0.315),
           (0, 0): (0.2, 0.21)}


@pytest.mark.parametrize("cls", list(STAGING), ids=["pitch%d-rows%d" % c for c in STAGING])
@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_cone_bp_staging_classes(P, cls, store):
    g, views = fine_detector(*STAGING[cls])
    assert footprint_class(g, views) == cls
    b = P.plan_bounds(g, views)
    assert (b["bp_pitch"], b["bp_stage"]) == cls
    print("\n[gpu variants] cone_bp staging", cls, store, g.as_dict(), flush=True)
    plan = P.Plan(g, views)
    V = len(views)
    dt = torch.float32 if store == "f32" else torch.bfloat16
    gF = dev(synth.rand_array((V, g.nv, g.nu), 60 + cls[0] + cls[1]), dt)
    f = torch.empty((g.nz, g.ny, g.nx), device="cuda")
    P.dc_cone_bp(plan, gF, f)
    ref = O.cone_bp(host(gF), g, views)      # the oracle sees the same stored values
    assert rel(host(f), ref) < TOL32
    # accumulate over two view ranges, ReLU on the last
    f2 = torch.empty_like(f)
    P.dc_cone_bp(plan, gF, f2, v0=0, nv=1)
    P.dc_cone_bp(plan, gF, f2, accumulate=True, relu=True, v0=1, nv=V - 1)
    assert rel(host(f2), np.maximum(ref, 0)) < TOL32
    # adjoint pairing with the (staging-independent) transpose
    Gf = dev(synth.rand_array((g.nz, g.ny, g.nx), 70 + cls[0] + cls[1]))
    GgF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_cone_bp_adjoint(plan, Gf, GgF)
    x = gF.float()
    lhs = float((f.double() * Gf.double()).sum())
    rhs = float((x.double() * GgF.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * float(f.double().norm() * Gf.double().norm())


def narrow_sinogram():
    """Rows of 41 bins at the detector pitch on a 70x53 detector: the diagonal
    needs 88, so corner pixels on oblique angles land outside every bin."""
    g = synth.Grid(nu=70, nv=53, du=1.0, dv=1.1, n_theta=37, n_s=41, ds=1.0,
                   nx=21, ny=19, nz=13, vx=1.0, vy=1.0, vz=1.0)
    return g, synth.sinusoid_orbit(5, 750.0, 1200.0)


def test_narrow_sinogram_radon_pair(P):
    g, views = narrow_sinogram()
    assert g.n_s < synth.radon_bins(g.nu, g.nv)
    print("\n[gpu variants] narrow sinogram", g.as_dict(), flush=True)
    plan = P.Plan(g, views)
    V = len(views)
    x = synth.rand_array((V, g.nv, g.nu), 80, 0.0, 1.0)
    R = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_weight_radon(plan, dev(x), R)
    assert rel(host(R), O.weight_radon(x.astype(np.float64), g, views)) < TOL32
    Gg = torch.empty((V, g.nv, g.nu), device="cuda")
    GR = synth.rand_array((V, g.n_theta, g.n_s), 81)
    P.dc_weight_radon_adjoint(plan, dev(GR), Gg)
    assert rel(host(Gg), O.weight_radon_adjoint(GR.astype(np.float64), g, views)) < TOL32
    H = synth.rand_array((V, g.n_theta, g.n_s), 82)
    gF = torch.empty((V, g.nv, g.nu), device="cuda")
    P.dc_detector_bp(plan, dev(H), gF)
    assert rel(host(gF), O.detector_bp(H.astype(np.float64), g)) < TOL32
    GH = torch.empty((V, g.n_theta, g.n_s), device="cuda")
    P.dc_detector_bp_adjoint(plan, dev(x), GH)
    assert rel(host(GH), O.detector_bp_adjoint(x.astype(np.float64), g)) < TOL32
    # and the whole chain with its gradient
    M = synth.rand_array((V, g.n_theta, g.n_s), 83, 0.0, 1.0)
    f = P.reconstruct(P.Plan(g, views), dev(M), g=dev(x))
    assert rel(host(f), O.reconstruct(x.astype(np.float64), M.astype(np.float64), g, views)) < TOL32
