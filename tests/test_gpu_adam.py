"""GPU fused Adam/AdamW step against the float64 oracle over several steps, on a
length with a ragged tail (not a multiple of 4), and its argument checks."""
import numpy as np
import pytest

from oracle import adam as A

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_14900_amd as P
    return P


@pytest.mark.parametrize("wd", [0.0, 0.01])
def test_steps_match_oracle(P, wd):
    n = 1_000_003
    rng = np.random.Generator(np.random.PCG64(3))
    M0 = rng.uniform(-1, 0, n).astype(np.float32)
    M = torch.tensor(M0, device="cuda")
    m, v = torch.zeros_like(M), torch.zeros_like(M)
    t = torch.zeros(1, device="cuda")
    Mr, mr, vr = M0.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        g = (rng.normal(0, 1, n) * (0.1 if step % 2 else 10.0)).astype(np.float32)
        t.add_(1.0)
        P.dc_adam_step(M, torch.tensor(g, device="cuda"), m, v, t, 0.05, (0.9, 0.999), 1e-8, wd)
        Mr, mr, vr = A.adam_step(Mr, g.astype(np.float64), mr, vr, step, 0.05, weight_decay=wd)
        got = M.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - Mr)) <= 1e-6 * np.max(np.abs(Mr)), step
    assert np.linalg.norm(m.cpu().numpy() - mr) <= 1e-6 * np.linalg.norm(mr)
    assert np.linalg.norm(v.cpu().numpy() - vr) <= 1e-6 * np.linalg.norm(vr)


def test_argument_checks(P):
    x = torch.zeros(16, device="cuda")
    t = torch.ones(1, device="cuda")
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_adam_step(x, x.clone(), x.clone(), x.clone(), t, 0.1, (1.0, 0.999))
    with pytest.raises(P.DcError, match="DC_EINVAL"):
        P.dc_adam_step(x, x.clone(), x.clone(), x.clone(), t, 0.1, eps=0.0)
    with pytest.raises(P.DcError, match="DC_EALIGN"):
        y = torch.zeros(17, device="cuda")
        P.dc_adam_step(y[1:], y[1:].clone(), y[1:].clone(), y[1:].clone(), t, 0.1)
    with pytest.raises(ValueError):
        P.dc_adam_step(x, x.double(), x.clone(), x.clone(), t, 0.1)


def test_graph_replays_reproduce_eager_steps(P):
    """The step count lives on the device, so advancing it and updating M can be
    captured once and replayed: three replays give the three eager steps' bits."""
    n = 4099
    gen = torch.Generator(device="cuda").manual_seed(4)
    M0 = torch.rand(n, device="cuda", generator=gen)
    G = torch.randn(n, device="cuda", generator=gen)
    M, m, v, t = M0.clone(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"), torch.zeros(1, device="cuda")

    def reset():
        M.copy_(M0); m.zero_(); v.zero_(); t.zero_()

    def step():
        t.add_(1.0)
        P.dc_adam_step(M, G, m, v, t, 0.05, (0.9, 0.999), 1e-8, 0.01)

    eager = []
    for _ in range(3):
        step()
        eager.append(M.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                                  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    reset()
    torch.cuda.synchronize()
    for k in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(M, eager[k]), k
        G.mul_(1.0)                             # eager work between replays


def test_fused_optimizer_tracks_torch_adamw_under_one_cycle(P):
    """train.FusedAdamW under the one-cycle schedule (which also cycles beta1)
    against torch's AdamW with the same schedule, over ten steps."""
    from paper_2410_14900_amd import train
    gen = torch.Generator(device="cuda").manual_seed(8)
    M0 = -torch.rand(100_003, device="cuda", generator=gen)
    grads = [torch.randn(100_003, device="cuda", generator=gen) for _ in range(10)]
    runs = []
    for cls in (train.FusedAdamW, torch.optim.AdamW):
        p = M0.clone().requires_grad_(True)
        opt = cls([p], lr=0.1, weight_decay=0.01)
        sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=1.0, total_steps=10, div_factor=10.0,
                                                    final_div_factor=1.0)
        for gr in grads:
            p.grad = gr.clone()
            opt.step()
            sched.step()
        runs.append(p.detach().clone())
    err = float((runs[0] - runs[1]).abs().max() / runs[1].abs().max())
    assert err < 1e-5, err
