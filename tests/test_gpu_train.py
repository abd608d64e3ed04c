"""The paper's training recipe (Sec. 3.1, eq. 13) end to end on the GPU: RAW
weights initialised U[-1, 0], the Gaussian filter layer, MSE + gamma (1 - SSIM)
on normalised volumes, AdamW under a one-cycle schedule.  A short run on the
C1 workload must cut the loss by a large factor, and the SSIM term's gradient
must reach M (the loss with gamma > 0 differs from the MSE-only run)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    from paper_2410_14900_amd import train
    grid, views = synth.config_geometry("C1")
    ell = synth.random_ellipsoids(5, grid.nx * grid.vx, 1)
    g = synth.project_ellipsoids(ell, grid, views, device="cuda").float().contiguous()
    ref = synth.voxelize_torch(ell, grid, device="cuda").float().contiguous()
    return P, train, P.Plan(grid, views), g, ref


def test_training_cuts_the_loss(setup):
    P, train, plan, g, ref = setup
    M, losses = train.train_weights(plan, g, ref, steps=30, gamma=0.5, smooth=(20.0, 60))
    print("\n[gpu train] losses", ["%.4g" % x for x in losses[::5]], flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.1 * losses[0]
    assert M.shape == (plan.n_views,) + plan.sino_shape


def test_ssim_term_reaches_the_weights(setup):
    P, train, plan, g, ref = setup
    gen = torch.Generator(device="cuda").manual_seed(7)
    M0 = -torch.rand((plan.n_views,) + plan.sino_shape, device="cuda", generator=gen) * 1e-3
    grads = []
    for gamma in (0.0, 1.0):
        M = M0.clone().requires_grad_(True)
        f = P.reconstruct(plan, M, g=g, mode="raw", relu=True, smooth=(20.0, 60))
        train.paper_loss(f, ref, gamma).backward()
        grads.append(M.grad.clone())
    d = float((grads[1] - grads[0]).norm() / grads[0].norm())
    assert d > 1e-3
