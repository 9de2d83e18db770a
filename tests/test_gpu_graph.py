"""Graph replay and determinism of the evaluation.

The whole evaluation is order independent: spreading sums in exact fixed point,
the fold, FFTs, mode stage and interpolation have fixed summation orders.  So
eager launches, HIP-graph replays and repeated calls must agree bit for bit.
"""
import numpy as np
import pytest

from paper_2305_15693_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,N,L,M", [(2, 50000, 223.6, 40), (3, 40000, 34.2, 10)])
def test_graph_replay_matches_eager_bitwise(gpu, d, N, L, M):
    import torch
    from paper_2305_15693_amd import fresco as F
    pos_np = I.positions(N, d, L, np.float32, seed=31 + d)
    w, s0 = I.stealthy_target(d, M, float(M))
    eager = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                      stream=torch.cuda.default_stream(gpu))
    side = torch.cuda.Stream(device=gpu)
    graphed = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                        stream=side)
    pos = torch.from_numpy(pos_np).to(gpu)
    loss_e, grad_e = eager.loss_grad(pos)
    grad_e = grad_e.clone()
    loss_dev = torch.zeros(1, dtype=torch.float64, device=gpu)
    grad = torch.empty_like(pos)
    torch.cuda.synchronize()
    for rep in range(4):
        graphed.loss_grad_async(pos, loss_dev, grad)
        side.synchronize()
        # unrelated device work and synchronisation between replays
        junk = (pos * 2.0).sum()
        torch.cuda.synchronize()
        assert float(loss_dev.item()) == loss_e, rep
        assert torch.equal(grad, grad_e), rep
        grad.fill_(float("nan"))
        torch.cuda.synchronize()
    # a second eager call reproduces the first one exactly
    loss_e2, grad_e2 = eager.loss_grad(pos)
    assert loss_e2 == loss_e
    assert torch.equal(grad_e2, grad_e)
    eager.close()
    graphed.close()
    del junk


def test_graph_replay_sees_new_positions(gpu):
    """A cached graph reads the position buffer at replay time."""
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 20000, 141.4, 30
    w, s0 = I.stealthy_target(d, M, float(M))
    side = torch.cuda.Stream(device=gpu)
    g = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                  stream=side)
    e = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                  stream=torch.cuda.default_stream(gpu))
    pos = torch.from_numpy(I.positions(N, d, L, np.float32, seed=5)).to(gpu)
    loss_dev = torch.zeros(1, dtype=torch.float64, device=gpu)
    grad = torch.empty_like(pos)
    torch.cuda.synchronize()
    g.loss_grad_async(pos, loss_dev, grad)
    side.synchronize()
    pos.copy_(torch.from_numpy(I.positions(N, d, L, np.float32, seed=6)).to(gpu))
    torch.cuda.synchronize()
    g.loss_grad_async(pos, loss_dev, grad)
    side.synchronize()
    loss_ref, grad_ref = e.loss_grad(pos)
    assert float(loss_dev.item()) == loss_ref
    assert torch.equal(grad, grad_ref)
    g.close()
    e.close()


def test_async_evaluation_inside_callers_graph_capture(gpu):
    """fresco_loss_grad_async called while the caller captures the context's
    stream (torch.cuda.graph) enqueues its launches into the caller's graph
    instead of starting a capture of its own; every replay of that graph, with
    unrelated eager work and synchronisation between replays, reproduces the
    eager evaluation bit for bit."""
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 20000, 141.4, 30
    w, s0 = I.stealthy_target(d, M, float(M))
    side = torch.cuda.Stream(device=gpu)
    g = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                  stream=side)
    e = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                  stream=torch.cuda.default_stream(gpu))
    pos = torch.from_numpy(I.positions(N, d, L, np.float32, seed=17)).to(gpu)
    loss_ref, grad_ref = e.loss_grad(pos)
    grad_ref = grad_ref.clone()
    loss_dev = torch.zeros(1, dtype=torch.float64, device=gpu)
    grad = torch.empty_like(pos)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        g.loss_grad_async(pos, loss_dev, grad)
    torch.cuda.synchronize()
    for rep in range(3):
        loss_dev.fill_(float("nan"))
        grad.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert float(loss_dev.item()) == loss_ref, rep
        assert torch.equal(grad, grad_ref), rep
        junk = (pos * 3.0).sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
    # outside the capture the context keeps its own graph cache working
    g.loss_grad_async(pos, loss_dev, grad)
    side.synchronize()
    assert float(loss_dev.item()) == loss_ref
    assert torch.equal(grad, grad_ref)
    del graph, junk
    g.close()
    e.close()
