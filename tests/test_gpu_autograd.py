"""The autograd wrappers and the backward of S through the C ABI, against the
FP64 oracle (derivative of S with respect to positions, Methods, "Analytical
gradients") and against finite differences.

Bars (normwise relative error): FP64 build at tol 1e-12: 1e-11; FP32 build at
tol 1e-6: 1e-5.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_15693_amd import inputs as I

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _ctx(gpu, d, N, L, M, kcut, tol, dtype, w=None, s0=None):
    from paper_2305_15693_amd import fresco as F
    if w is None:
        w, s0 = I.stealthy_target(d, M, kcut)
    return F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=tol, dtype=dtype, device=gpu)


def _t(gpu, a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(
        device=gpu, dtype=torch.float32 if dtype == "f32" else torch.float64)


@pytest.mark.parametrize("d,N,L,M,tol,dtype,bar", [
    (2, 1000, 31.6, 12, 1e-12, "f64", 1e-11),
    (3, 20000, 27.1, 8, 1e-6, "f32", 1e-5),
    (2, 3000, (40.0, 25.0), 10, 1e-6, "f32", 1e-5),
])
def test_sf_backward_matches_oracle(gpu, d, N, L, M, tol, dtype, bar):
    import torch
    print(f"sf_backward d={d} N={N} {dtype}", flush=True)
    Lv = np.broadcast_to(np.asarray(L, float), (d,))
    pos_np = I.positions(N, d, Lv, np.float32 if dtype == "f32" else np.float64, seed=500 + d)
    ctx = _ctx(gpu, d, N, Lv, M, M, tol, dtype)
    pos = _t(gpu, pos_np, dtype)
    rng = np.random.default_rng(600 + d)
    gS = rng.normal(size=ctx.cube_shape)
    S = ctx.structure_factor(pos)
    grad = ctx.structure_factor_backward(pos, _t(gpu, gS, dtype),
                                         token=ctx.sf_token()).cpu().numpy()
    torch.cuda.synchronize()
    ref = O.sf_vjp(pos_np.astype(np.float64), Lv, O.mode_vectors(d, M), gS.reshape(-1))
    e = rel(grad, ref)
    print(f"  rel err {e:.3e}", flush=True)
    assert e < bar
    # the same call without the preceding forward (state recomputed from pos)
    ctx2 = _ctx(gpu, d, N, Lv, M, M, tol, dtype)
    grad2 = ctx2.structure_factor_backward(pos, _t(gpu, gS, dtype)).cpu().numpy()
    np.testing.assert_array_equal(grad2, grad)
    ctx.close()
    ctx2.close()


def test_sf_backward_after_other_evaluations(gpu):
    # a loss evaluation at other positions in between must not leak into the
    # backward of the earlier forward
    import torch
    d, N, L, M = 2, 4000, 63.2, 16
    ctx = _ctx(gpu, d, N, L, M, M, 1e-6, "f32")
    p1 = _t(gpu, I.positions(N, d, L, np.float32, seed=1), "f32")
    p2 = _t(gpu, I.positions(N, d, L, np.float32, seed=2), "f32")
    gS = _t(gpu, np.random.default_rng(3).normal(size=ctx.cube_shape), "f32")
    import ctypes
    from paper_2305_15693_amd import fresco as F
    ctx.structure_factor(p1)
    g_ref = ctx.structure_factor_backward(p1, gS, token=ctx.sf_token()).clone()
    ctx.structure_factor(p1)
    tok = ctx.sf_token()
    ctx.loss_grad(p2)
    g = ctx.structure_factor_backward(p1, gS, token=tok)  # stale token: recomputed
    torch.cuda.synchronize()
    assert torch.equal(g, g_ref)
    # the C ABI refuses to reuse state that another evaluation replaced
    ctx.loss_grad(p2)
    st = F.lib().fresco_structure_factor_backward(ctx.handle, ctypes.c_void_p(p1.data_ptr()),
                                                  ctypes.c_void_p(gS.data_ptr()),
                                                  ctypes.c_void_p(g.data_ptr()), 1)
    assert st == F.EINVAL
    ctx.close()


def test_gradcheck_structure_factor_f64(gpu):
    # torch's numerical-vs-analytical Jacobian check of r -> S(n) on the whole cube
    import torch
    from paper_2305_15693_amd import autograd as A
    d, N, L, M = 2, 24, 6.0, 3
    ctx = _ctx(gpu, d, N, L, M, M, 1e-12, "f64")
    pos = _t(gpu, I.positions(N, d, L, np.float64, seed=9), "f64").requires_grad_(True)
    # eps = 1e-4: the differences then see transform noise of ~N 1e-12 / eps and a
    # truncation error of ~eps^2 |k|^3 N, both well inside atol
    ok = torch.autograd.gradcheck(lambda p: A.structure_factor(ctx, p), (pos,), eps=1e-4,
                                  atol=1e-5, rtol=1e-4)
    assert ok
    ctx.close()


@pytest.mark.parametrize("dtype,bar", [("f64", 1e-11), ("f32", 2e-5)])
def test_spectral_loss_through_S_equals_fused_gradient(gpu, dtype, bar):
    # A loss written in torch on S, differentiated through the backward of S, equals
    # the library's fused loss gradient (Eq. gradient), and LossFn's backward.
    import torch
    from paper_2305_15693_amd import autograd as A
    d, N, L, M = 2, 5000, 70.7, 20
    rng = np.random.default_rng(11)
    n = O.mode_vectors(d, M)
    kk = np.sqrt((n.astype(float) ** 2).sum(1)).reshape((2 * M + 1,) * d)
    w = ((kk > 0) & (kk <= M)).astype(float) * rng.uniform(0.5, 2.0, kk.shape)
    w = 0.5 * (w + w[::-1, ::-1])  # even weights: the loss counts n and -n alike
    s0 = np.where(w > 0, (kk / M) ** 2, 0.0)
    ctx = _ctx(gpu, d, N, L, M, M, 1e-12 if dtype == "f64" else 1e-6, dtype, w=w, s0=s0)
    pos_np = I.positions(N, d, L, np.float32 if dtype == "f32" else np.float64, seed=12)
    pos = _t(gpu, pos_np, dtype).requires_grad_(True)
    Wt, S0t = _t(gpu, w, dtype), _t(gpu, s0, dtype)
    S = A.structure_factor(ctx, pos)
    lt = (Wt.double() * (S.double() - S0t.double()) ** 2).sum()
    lt.backward()
    g_sf = pos.grad.detach().cpu().numpy()
    pos.grad = None
    lf = A.loss(ctx, pos)
    lf.backward()
    g_loss = pos.grad.detach().cpu().numpy()
    loss_ref, g_ref = ctx.loss_grad(pos.detach())
    torch.cuda.synchronize()
    assert float(lf) == loss_ref
    np.testing.assert_array_equal(g_loss, g_ref.cpu().numpy())
    assert abs(float(lt) - loss_ref) <= (1e-12 if dtype == "f64" else 1e-5) * loss_ref
    e = rel(g_sf, g_ref.cpu().numpy())
    print(f"  {dtype}: spectral-through-S vs fused gradient {e:.3e}", flush=True)
    assert e < bar
    ctx.close()


def test_composed_loss_matches_finite_differences(gpu):
    # Spectral loss plus the soft-core pair term in one backward (FP64 build),
    # against central differences with h = 1e-4 on 64 random coordinates: the
    # spectral part from the oracle's cancellation-free differences, the pair part
    # from differences of the oracle's cell-list energy.
    import torch
    from paper_2305_15693_amd import autograd as A
    from paper_2305_15693_amd import fresco as F
    d, N, M = 3, 20000, 10
    L = N ** (1.0 / 3.0)
    print("composed FD: 3D N=20000 f64", flush=True)
    pos_np = I.positions(N, d, L, np.float64, seed=77)
    ctx = _ctx(gpu, d, N, L, M, M, 1e-12, "f64")
    pctx = F.PairContext(d, N, L, sigma=0.5, eps=1.0, alpha=2.0, dtype="f64", device=gpu)
    pos = _t(gpu, pos_np, "f64").requires_grad_(True)
    total = A.loss(ctx, pos) + A.soft_core(pctx, pos)
    total.backward()
    g = pos.grad.detach().cpu().numpy()
    torch.cuda.synchronize()
    rng = np.random.default_rng(78)
    coords = np.stack([rng.integers(0, N, 64), rng.integers(0, d, 64)], 1)
    modes, W, S0 = O.constrained_set(d, M, *I.stealthy_target(d, M, M))
    h = 1e-4
    fd_s = O.finite_difference(pos_np, L, modes, W, S0, coords, h)
    fd_p = np.zeros(64)
    for c, (j, a) in enumerate(coords):
        pp, pm = pos_np.copy(), pos_np.copy()
        pp[j, a] += h
        pm[j, a] -= h
        fd_p[c] = (O.pair(pp, L, 0.5, cells=True)[0] - O.pair(pm, L, 0.5, cells=True)[0]) / (2 * h)
    fd = fd_s + fd_p
    got = g[coords[:, 0], coords[:, 1]]
    e = rel(got, fd)
    print(f"  autograd vs central differences on 64 coordinates: {e:.3e}", flush=True)
    assert e < 1e-6
    ctx.close()
    pctx.close()


def test_f32_composed_gradient_matches_oracle_sampled(gpu):
    # FP32 build, 3D, spectral + pair through one backward vs the FP64 oracle on
    # 128 sampled points (spectral: direct sums; pair: cell list, all points).
    import torch
    from paper_2305_15693_amd import autograd as A
    from paper_2305_15693_amd import fresco as F
    d, N, M = 3, 100000, 14
    L = N ** (1.0 / 3.0)
    print("composed f32: 3D N=1e5", flush=True)
    pos_np = I.positions(N, d, L, np.float32, seed=79)
    ctx = _ctx(gpu, d, N, L, M, M, 1e-6, "f32")
    pctx = F.PairContext(d, N, L, sigma=0.5, eps=1.0, alpha=2.0, dtype="f32", device=gpu)
    pos = _t(gpu, pos_np, "f32").requires_grad_(True)
    total = A.loss(ctx, pos) + A.soft_core(pctx, pos)
    total.backward()
    g = pos.grad.detach().cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    idx = np.random.default_rng(80).choice(N, 128, replace=False)
    modes, W, S0 = O.constrained_set(d, M, *I.stealthy_target(d, M, M))
    r = O.loss_grad(pos_np.astype(np.float64), L, modes, W, S0, grad_points=idx)
    e_p, g_p = O.pair(pos_np.astype(np.float64), L, 0.5, cells=True)
    ref = r["grad"] + g_p[idx]
    e = rel(g[idx], ref)
    print(f"  sampled gradient rel err {e:.3e}; loss {float(total):.6e} vs {r['loss'] + e_p:.6e}",
          flush=True)
    assert e < 1e-5
    assert abs(float(total) - (r["loss"] + e_p)) < 1e-5 * (r["loss"] + e_p)
    ctx.close()
    pctx.close()


def test_composed_loss_finite_differences_full_3d_shape(gpu):
    # The 3D workload's shape: N = 1e7 points at unit density (L = N^(1/3)),
    # modes |n| <= 60 (the 250^3 fine grid), soft core of diameter 0.5, FP64
    # build.  The stealthy weights sit on 96 random constrained modes (and their
    # mirrors) so that the oracle's direct sums stay affordable; grids, tiles and
    # launch shapes are those of the full problem.  Spectral loss + pair energy
    # through one backward, against central differences with h = 1e-4 on 64
    # random coordinates: the spectral part from the oracle's cancellation-free
    # differences, the pair part from the differences of each moved point's own
    # pairs (brute force over all points).
    import torch
    from paper_2305_15693_amd import autograd as A
    from paper_2305_15693_amd import fresco as F
    d, N, M = 3, 10_000_000, 60
    L = N ** (1.0 / 3.0)
    print("composed FD at the full 3D shape: N=1e7 M=60 f64", flush=True)
    pos_np = I.positions(N, d, L, np.float64, seed=1003)
    rng = np.random.default_rng(1004)
    w_full, _ = I.stealthy_target(d, M, float(M))
    idx = np.flatnonzero(w_full.ravel())
    w = np.zeros(w_full.size)
    w[rng.choice(idx, 96, replace=False)] = 1.0
    w = w.reshape(w_full.shape)
    w = np.maximum(w, w[::-1, ::-1, ::-1])
    ctx = F.Context(d, N, L, M, w_cube=w, tol=1e-12, dtype="f64", device=gpu)
    pctx = F.PairContext(d, N, L, sigma=0.5, eps=1.0, alpha=2.0, dtype="f64", device=gpu)
    assert ctx.plan_info()["nf"][:3] == [250, 250, 250]
    pos = _t(gpu, pos_np, "f64").requires_grad_(True)
    total = A.loss(ctx, pos) + A.soft_core(pctx, pos)
    total.backward()
    torch.cuda.synchronize()
    coords = np.stack([rng.integers(0, N, 64), rng.integers(0, d, 64)], 1)
    got = pos.grad.detach()[torch.from_numpy(coords[:, 0]).to(gpu),
                           torch.from_numpy(coords[:, 1]).to(gpu)].cpu().numpy()
    ctx.close()
    pctx.close()
    del pos, total
    modes, W, S0 = O.constrained_set(d, M, w, None)
    h = 1e-4
    fd_s = O.finite_difference(pos_np, L, modes, W, S0, coords, h)
    fd_p = O.pair_finite_difference(pos_np, L, coords, h, 0.5)
    fd = fd_s + fd_p
    e = rel(got, fd)
    print(f"  {len(modes)} modes, {int(np.count_nonzero(fd_p))} of 64 coordinates with pair terms; "
          f"autograd vs central differences: {e:.3e} (spectral part alone {rel(got - fd_p, fd_s):.3e})",
          flush=True)
    assert np.count_nonzero(fd_p) > 0
    assert e < 1e-6
