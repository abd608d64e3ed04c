"""GPU Poisson noise (Philox4x64-10 + inversion / transformed rejection) against
the float64 oracle: counts bit-exact on line integrals spanning both branches
(lambda from 0.06 to 1e5), the noisy line integrals within one float32 rounding,
sub-ranges by element offset, in-place use, and sampled elements of a
full-size projection stack (496 x 512 x 512) with its standardised moments."""
import math

import numpy as np
import pytest

import synth
from oracle import noise as Nz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PHOTONS, MU = 1e5, 0.02


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


def line_integrals(n, seed):
    # lambda = 1e5 exp(-0.02 p) over p in [0, 720]: 0.06 .. 1e5 photons
    return synth.rand_array((n,), seed, 0.0, 720.0)


def test_counts_bit_exact_on_both_branches(P):
    p = line_integrals(12000, 1)
    pt = torch.as_tensor(p, device="cuda")
    out = torch.empty_like(pt)
    cnt = torch.empty(p.shape, dtype=torch.int64, device="cuda")
    P.dc_poisson_noise(pt, out, PHOTONS, MU, seed=77, counts=cnt)
    ref_out, ref_cnt = Nz.poisson_noise(p.astype(np.float64), PHOTONS, MU, 77)
    lam = PHOTONS * np.exp(-MU * p.astype(np.float64))
    assert (lam < 10).sum() > 500 and (lam >= 10).sum() > 500
    got = cnt.cpu().numpy()
    assert np.array_equal(got, ref_cnt), np.nonzero(got != ref_cnt)[0][:10]
    o = out.cpu().numpy()
    np.testing.assert_allclose(o, ref_out.astype(np.float32), rtol=2 ** -23, atol=0)


def test_offsets_in_place_and_determinism(P):
    p = line_integrals(5000, 2)
    pt = torch.as_tensor(p, device="cuda")
    full = P.dc_poisson_noise(pt, torch.empty_like(pt), PHOTONS, MU, seed=5)
    part = P.dc_poisson_noise(pt[1024:3072].clone(), torch.empty(2048, device="cuda"), PHOTONS, MU, seed=5, e0=1024)
    assert torch.equal(part, full[1024:3072])
    again = P.dc_poisson_noise(pt, torch.empty_like(pt), PHOTONS, MU, seed=5)
    assert torch.equal(again, full)
    other = P.dc_poisson_noise(pt, torch.empty_like(pt), PHOTONS, MU, seed=6)
    assert not torch.equal(other, full)
    x = pt.clone()
    P.dc_poisson_noise(x, x, PHOTONS, MU, seed=5)
    assert torch.equal(x, full)


def test_full_size_projection_stack(P):
    g, views = synth.config_geometry("C2")
    ell = synth.random_ellipsoids(20, g.nx * g.vx, 2)
    p = synth.project_ellipsoids(ell, g, views, device="cuda").float().contiguous()
    out = torch.empty_like(p)
    cnt = torch.empty(p.shape, dtype=torch.int64, device="cuda")
    P.dc_poisson_noise(p, out, PHOTONS, MU, seed=11, counts=cnt)
    flat_p, flat_c = p.reshape(-1), cnt.reshape(-1)
    rng = np.random.Generator(np.random.PCG64(3))
    idx = np.concatenate([rng.integers(0, flat_p.numel(), 1500), [0, flat_p.numel() - 1]])
    pv = flat_p[torch.as_tensor(idx, device="cuda")].double().cpu().numpy()
    ref = np.array([Nz.poisson_count(PHOTONS * math.exp(-MU * pv[i]), 11, int(e)) for i, e in enumerate(idx)])
    assert np.array_equal(flat_c[torch.as_tensor(idx, device="cuda")].cpu().numpy(), ref)
    lam = PHOTONS * torch.exp(-MU * p.double())
    z = (cnt.double() - lam) / lam.sqrt()
    assert abs(float(z.mean())) < 5 / math.sqrt(z.numel()) and abs(float(z.var()) - 1.0) < 0.01


def test_argument_checks(P):
    x = torch.zeros(16, device="cuda")
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_poisson_noise(x, x, 0.0, MU, seed=1)
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_poisson_noise(x, x, PHOTONS, -1.0, seed=1)
    with pytest.raises(P.DcError, match="DC_EALIGN"):
        P.dc_poisson_noise(x[1:9], torch.empty(8, device="cuda"), PHOTONS, MU, seed=1)
    with pytest.raises(ValueError):
        P.dc_poisson_noise(x, torch.empty(8, device="cuda"), PHOTONS, MU, seed=1)
