"""The Adam/AdamW oracle against torch's own optimisers on the CPU (float64),
over several steps with changing gradients."""
import numpy as np
import pytest

from oracle import adam as A

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("wd", [0.0, 0.05])
def test_matches_torch_optimizers(wd):
    rng = np.random.Generator(np.random.PCG64(7))
    M0 = rng.uniform(-1, 0, 300)
    p = torch.tensor(M0, dtype=torch.float64, requires_grad=True)
    opt = (torch.optim.AdamW([p], lr=0.3, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd) if wd else
           torch.optim.Adam([p], lr=0.3, betas=(0.9, 0.999), eps=1e-8))
    M, m, v = M0.copy(), np.zeros(300), np.zeros(300)
    for t in range(1, 6):
        g = rng.normal(0, 1, 300) * (t % 3 + 0.1)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        M, m, v = A.adam_step(M, g, m, v, t, lr=0.3, weight_decay=wd)
        np.testing.assert_allclose(M, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_first_step_moves_each_weight_by_lr():
    # at t = 1 the bias-corrected ratio is g / (|g| + eps)
    g = np.array([2.0, -3.0, 1e-3, -5.0])
    M, m, v = A.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.1)
    np.testing.assert_allclose(M, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
