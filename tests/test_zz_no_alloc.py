"""The allocation-free pair entry point (fresco_pair_energy_grad_noalloc) through
the C ABI, against the pair-context entry point it mirrors
(fresco_pair_energy_grad_async): the same kernels on the same cell geometry, so
energy and gradient agree bit for bit, and both against the FP64 oracle.  Two
calls in a row, the second on a smaller problem (the fixed scratch keeps the
first call's contents); from the second call on, no device memory is taken;
sizes beyond the scratch are rejected before any work."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_15693_amd import inputs as I

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("dtype,bar", [("f32", 1e-6), ("f64", 1e-12)])
def test_noalloc_pair_matches_pair_context(gpu, dtype, bar):
    import torch
    from paper_2305_15693_amd import fresco as F
    tdt = torch.float32 if dtype == "f32" else torch.float64
    ndt = np.float32 if dtype == "f32" else np.float64
    side = torch.cuda.Stream(device=gpu)
    # unit density in 3D (sigma = 0.5: 8 cells per unit volume), then a smaller 2D case
    cases = [(3, 60000, 60000 ** (1 / 3)), (2, 4000, 4000 ** 0.5)]
    for k, (d, N, L) in enumerate(cases):
        print(f"no-alloc pair call {k}: {dtype} d={d} N={N} L={L:.3f}", flush=True)
        pos_np = I.positions(N, d, L, ndt, seed=200 + k)
        pos = torch.from_numpy(pos_np).to(gpu)
        e_dev = torch.full((1,), float("nan"), dtype=torch.float64, device=gpu)
        grad = torch.full((N, d), float("nan"), dtype=tdt, device=gpu)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(gpu)[0]
        F.pair_energy_grad_noalloc(pos, e_dev, grad, L, sigma=0.5, stream=side)
        side.synchronize()
        free1 = torch.cuda.mem_get_info(gpu)[0]
        if k > 0:
            assert free1 == free0
        ref = F.PairContext(d, N, L, sigma=0.5, dtype=dtype, device=gpu, stream=side)
        e_ref = torch.zeros(1, dtype=torch.float64, device=gpu)
        g_ref = torch.empty_like(pos)
        ref.energy_grad_async(pos, e_ref, g_ref)
        side.synchronize()
        ref.close()
        e = float(e_dev.item())
        assert e == float(e_ref.item())
        assert torch.equal(grad, g_ref)
        eo, go = O.pair(pos_np.astype(np.float64), L, 0.5, cells=(N > 20000))
        print(f"  energy {e:.9e} (oracle {eo:.9e}), grad rel {_rel(grad.cpu().numpy(), go):.2e}",
              flush=True)
        assert abs(e - eo) <= bar * abs(eo)
        assert _rel(grad.cpu().numpy(), go) <= bar


def test_noalloc_pair_rejects_sizes_beyond_scratch(gpu):
    # 2e6 points at unit density in 3D need ~ 2e6 * 24 + 8 * 1.6e7 bytes of cell
    # list, beyond the 32 MiB scratch: ENOTSUP, outputs untouched
    import torch
    from paper_2305_15693_amd import fresco as F
    N, d = 2_000_000, 3
    L = N ** (1 / 3)
    pos = torch.rand(N, d, device=gpu) * L
    e_dev = torch.full((1,), -1.0, dtype=torch.float64, device=gpu)
    grad = torch.full((N, d), -1.0, device=gpu)
    with pytest.raises(F.FrescoError) as e:
        F.pair_energy_grad_noalloc(pos, e_dev, grad, L, sigma=0.5)
    assert e.value.code == F.ENOTSUP
    torch.cuda.synchronize()
    assert float(e_dev.item()) == -1.0
    assert bool((grad == -1.0).all())
