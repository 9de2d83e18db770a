"""The N = 1e9 2D workload (L = 31623, stealthy 0 < |n| <= 6000, tol 1e-5, FP32,
fine grid 24300^2 whose columns take the two-sub-column path) at full size.

The oracle cannot sum over 1.1e8 constrained modes for 1e9 points, so the
weights sit on 16 random constrained modes and their mirrors: the loss, S on
those modes and the gradient of 2048 sampled points are then exact direct sums
(rho by direct evaluation over all 1e9 points).  The gradient's sum rule
(translation invariance) is checked over all points.  Bar: 1e-4 at tol 1e-5.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_15693_amd import inputs as I

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_n1e9_sampled(gpu):
    import torch
    from paper_2305_15693_amd import fresco as F
    cfg = I.WORKLOADS["2d_n1e9_stealthy6000_f32"]
    d, N, L, M, kcut = cfg["d"], cfg["N"], cfg["L"], cfg["M"], cfg["kcut"]
    print("N = 1e9: generating positions", flush=True)
    pos = I.positions(N, d, L, np.float32, seed=cfg["seed"])
    # 16 random constrained modes (with their mirrors) carry weight 1
    rng = np.random.default_rng(cfg["seed"] + 1)
    P = 2 * M + 1
    w = np.zeros((P, P))
    picked = []
    while len(picked) < 16:
        n = rng.integers(-M, M + 1, 2)
        if 0 < n @ n <= kcut * kcut and w[n[0] + M, n[1] + M] == 0:
            w[n[0] + M, n[1] + M] = w[-n[0] + M, -n[1] + M] = 1.0
            picked.append(n)
    ctx = F.Context(d, N, L, M, w_cube=w, tol=cfg["tol"], dtype="f32", device=gpu)
    info = ctx.plan_info()
    print(f"plan: nf {info['nf']} col_split {info['col_split']} "
          f"device bytes {info['device_bytes'] / 2**30:.1f} GiB", flush=True)
    assert info["nf"] == [24300, 24300] and info["col_split"] == 2
    tpos = torch.from_numpy(pos).to(gpu)
    Sg = ctx.structure_factor(tpos)
    modes = np.array(picked + [-p for p in picked], dtype=np.int32)
    S_gpu = Sg[modes[:, 0] + M, modes[:, 1] + M].cpu().numpy().astype(np.float64)
    del Sg
    loss, grad = ctx.loss_grad(tpos)
    gsum = grad.double().sum(0).cpu().numpy()
    gabs = grad.double().abs().sum(0).cpu().numpy()
    gp = rng.choice(N, 2048, replace=False)
    g_gpu = grad[torch.from_numpy(gp).to(gpu)].cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    del grad, tpos
    ctx.close()
    print("oracle: rho on 16 modes over 1e9 points", flush=True)
    rho = O.rho_direct(pos, L, modes[:16])
    rho = np.concatenate([rho, np.conj(rho)])
    ones = np.ones(len(modes))
    r = O.loss_grad_from_rho(N, L, modes, ones, np.zeros(len(modes)), rho, pos[gp])
    print(f"N=1e9: S {rel(S_gpu, r['S']):.2e} loss {abs(loss - r['loss']) / r['loss']:.2e} "
          f"grad {rel(g_gpu, r['grad']):.2e} sum rule {np.abs(gsum / gabs).max():.2e}", flush=True)
    assert rel(S_gpu, r["S"]) < 1e-4
    assert abs(loss - r["loss"]) / r["loss"] < 1e-4
    assert rel(g_gpu, r["grad"]) < 1e-4
    assert np.abs(gsum / gabs).max() < 1e-4
