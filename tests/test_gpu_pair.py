"""Soft-core pair term on the GPU cell list (through the C ABI) against the FP64
oracle (brute force over all pairs, or the oracle's own cell list at large N).

U = (eps/alpha)(1 - r/sigma)^alpha for r < sigma, minimum image.  Bars: FP64
build 1e-12 (energy and normwise gradient), FP32 build 1e-6 (differences are
taken in FP64 from the FP32 coordinates, so only the final rounding to FP32
separates it from the oracle).
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


def _pair(gpu, d, N, L, dtype, sigma=0.5, alpha=2.0, eps=1.0):
    from paper_2305_15693_amd import fresco as F
    return F.PairContext(d, N, L, sigma=sigma, eps=eps, alpha=alpha, dtype=dtype, device=gpu)


def _t(gpu, a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(
        device=gpu, dtype=torch.float32 if dtype == "f32" else torch.float64)


CASES = [
    # d, N, L, dtype, alpha, bar
    (2, 3000, 54.8, "f64", 2.0, 1e-12),
    (3, 4000, 15.9, "f64", 2.5, 1e-12),
    (2, 3000, 54.8, "f32", 2.0, 1e-6),
    (3, 4000, 15.9, "f32", 2.0, 1e-6),
    (3, 500, (1.2, 6.0, 4.0), "f64", 2.0, 1e-12),  # two cells along x
]


@pytest.mark.parametrize("d,N,L,dtype,alpha,bar", CASES)
def test_pair_matches_brute_force(gpu, d, N, L, dtype, alpha, bar):
    print(f"pair d={d} N={N} L={L} {dtype} alpha={alpha}", flush=True)
    Lv = np.broadcast_to(np.asarray(L, float), (d,))
    pos_np = I.positions(N, d, Lv, np.float32 if dtype == "f32" else np.float64, seed=900 + d)
    # some coordinates outside the box: the minimum image must still find them
    pos_np[::7] += (Lv * np.array([1.0, -2.0, 3.0][:d])).astype(pos_np.dtype)
    pc = _pair(gpu, d, N, Lv, dtype, alpha=alpha)
    e, g = pc.energy_grad(_t(gpu, pos_np, dtype))
    g = g.cpu().numpy()
    e_ref, g_ref = O.pair(pos_np.astype(np.float64), Lv, 0.5, 1.0, alpha)
    assert e_ref > 0
    print(f"  energy {e:.12e} vs {e_ref:.12e}; grad rel {rel(g, g_ref):.3e}", flush=True)
    assert abs(e - e_ref) <= bar * e_ref
    assert rel(g, g_ref) < bar
    pc.close()


def test_pair_clustered_points_and_determinism(gpu):
    # many points per cell (a dense cluster) plus isolated ones; repeated calls
    # give bitwise identical results although atomics order the cell list
    import torch
    d, N, L = 3, 3000, 20.0
    rng = np.random.default_rng(5)
    pos_np = rng.uniform(0, L, (N, d))
    pos_np[:1500] = 7.0 + rng.uniform(0, 1.0, (1500, d))  # ~1500 points in ~1 unit^3
    pc = _pair(gpu, d, N, L, "f64")
    pos = _t(gpu, pos_np, "f64")
    e1, g1 = pc.energy_grad(pos)
    g1 = g1.clone()
    e2, g2 = pc.energy_grad(pos)
    torch.cuda.synchronize()
    assert e1 == e2 and torch.equal(g1, g2)
    e_ref, g_ref = O.pair(pos_np, L, 0.5)
    assert abs(e1 - e_ref) <= 1e-12 * e_ref
    assert rel(g1.cpu().numpy(), g_ref) < 1e-12
    assert np.abs(g1.cpu().numpy().sum(0)).max() < 1e-9 * np.abs(g_ref).sum()
    pc.close()


def test_pair_full_size_3d(gpu):
    # the packing workload: N = 1e7 at unit density in 3D, sigma = 0.5, against the
    # oracle's cell list over all points
    d, N = 3, 10_000_000
    L = N ** (1.0 / 3.0)
    print("pair full size 3D N=1e7 f32", flush=True)
    pos_np = I.positions(N, d, L, np.float32, seed=1003)
    pc = _pair(gpu, d, N, L, "f32")
    e, g = pc.energy_grad(_t(gpu, pos_np, "f32"))
    g = g.cpu().numpy()
    e_ref, g_ref = O.pair(pos_np.astype(np.float64), L, 0.5, cells=True)
    print(f"  energy {e:.10e} vs {e_ref:.10e}; grad rel {rel(g, g_ref):.3e}", flush=True)
    assert abs(e - e_ref) <= 1e-9 * e_ref
    assert rel(g, g_ref) < 1e-6
    pc.close()


def test_attached_pair_adds_to_loss_and_gradient(gpu):
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, M = 3, 20000, 8
    L = N ** (1.0 / 3.0)
    w, s0 = I.stealthy_target(d, M, M)
    pos = _t(gpu, I.positions(N, d, L, np.float64, seed=41), "f64")
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-12, dtype="f64", device=gpu)
    pc = _pair(gpu, d, N, L, "f64")
    l0, g0 = ctx.loss_grad(pos)
    g0 = g0.clone()
    e, ge = pc.energy_grad(pos)
    ctx.attach_pair(pc, 2.5)
    l1, g1 = ctx.loss_grad(pos)
    torch.cuda.synchronize()
    assert abs(l1 - (l0 + 2.5 * e)) <= 1e-12 * l1
    np.testing.assert_allclose(g1.cpu().numpy(), (g0 + 2.5 * ge).cpu().numpy(), rtol=1e-12,
                               atol=1e-12 * float(g0.abs().max()))
    ctx.attach_pair(None)
    l2, _ = ctx.loss_grad(pos)
    assert l2 == l0
    with pytest.raises(F.FrescoError):
        ctx.attach_pair(_pair(gpu, d, N + 1, L, "f64"))
    ctx.close()
    pc.close()


def test_lbfgs_with_pair_term_removes_overlaps(gpu):
    # the packing problem: minimising L_S + E drives the pair energy towards zero
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, M = 3, 4000, 5
    L = N ** (1.0 / 3.0)
    w, s0 = I.stealthy_target(d, M, M)
    pos = _t(gpu, I.positions(N, d, L, np.float32, seed=42), "f32")
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu)
    pc = _pair(gpu, d, N, L, "f32")
    e0, _ = pc.energy_grad(pos)
    ctx.attach_pair(pc, 1.0)
    l0, _ = ctx.loss_grad(pos)
    loss, nev = ctx.step(pos, 100)
    e1, _ = pc.energy_grad(pos)
    torch.cuda.synchronize()
    print(f"  total {l0:.4e} -> {loss:.4e}; pair energy {e0:.4e} -> {e1:.4e} ({nev} evals)",
          flush=True)
    assert loss < 0.2 * l0
    assert e1 < 0.2 * e0
    ctx.close()
    pc.close()
