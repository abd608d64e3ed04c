"""GPU 3D SSIM (the structural loss term of eq. 13) against the float64 oracle:
value and gradient on small and ragged volumes, the value at the 256^3 training
size, bit-reproducibility, and host-side argument checks."""
import numpy as np
import pytest

import synth
from oracle import ssim as Q

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


def pair(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    y = rng.uniform(0, 1, shape)
    x = np.clip(y + rng.normal(0, 0.2, shape), 0, None)        # a noisy reconstruction of y
    return x.astype(np.float32), y.astype(np.float32)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("shape", [(24, 20, 22), (11, 13, 17), (19, 11, 11)])
def test_value_and_gradient(P, shape):
    x, y = pair(shape, 1)
    s, g = P.dc_ssim(dev(x), dev(y), 1.0, grad=True)
    ref = Q.ssim(x.astype(np.float64), y.astype(np.float64), 1.0)
    assert abs(float(s) - ref) <= 1e-5 * abs(ref)
    rg = Q.ssim_grad(x.astype(np.float64), y.astype(np.float64), 1.0)
    got = g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - rg) <= 1e-4 * np.linalg.norm(rg)
    s2, _ = P.dc_ssim(dev(x), dev(y), 1.0)
    assert torch.equal(s, s2)                     # same value without the gradient pass


def test_value_at_training_size_and_bit_reproducible(P):
    grid, _ = synth.config_geometry("C2", n_views=4)
    ell = synth.random_ellipsoids(20, grid.nx * grid.vx, 2)
    y = synth.voxelize_torch(ell, grid, device="cuda").float().contiguous()
    gen = torch.Generator(device="cuda").manual_seed(3)
    x = (y + 0.05 * torch.randn(y.shape, device="cuda", generator=gen)).clamp_min(0).contiguous()
    L = float(y.max())
    s, g = P.dc_ssim(x, y, L, grad=True)
    ref = Q.ssim(x.double().cpu().numpy(), y.double().cpu().numpy(), L, moments=Q.window_moments_separable)
    assert abs(float(s) - ref) <= 1e-5 * abs(ref)
    s2, g2 = P.dc_ssim(x, y, L, grad=True)
    assert torch.equal(s, s2) and torch.equal(g, g2)


def test_argument_checks(P):
    x = torch.zeros((10, 12, 12), device="cuda")
    with pytest.raises(P.DcError, match="DC_ESHAPE"):
        P.dc_ssim(x, x, 1.0)
    x = torch.zeros((12, 12, 12), device="cuda")
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_ssim(x, x, 0.0)
    L = P._lib.lib()
    out = torch.empty(1, device="cuda")
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    import ctypes
    st = L.dc_ssim(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 12, 12, 12, 1.0,
                   ctypes.c_void_p(out.data_ptr()), None, ctypes.c_void_p(small.data_ptr()), 64, None)
    assert st == P._lib.DC_ESHAPE
