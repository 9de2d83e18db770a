"""L-BFGS on the GPU (fresco_step) against the textbook FP64 oracle L-BFGS.

The oracle run uses the direct-sum loss and gradient and the same options; in
the FP64 build the two trajectories agree to the accuracy of the transforms.
"""
import numpy as np
import pytest

from oracle import lbfgs as LB
from oracle import oracle as O
from paper_2305_15693_amd import inputs as I

pytestmark = pytest.mark.gpu


def _oracle_fg(N, d, L, modes, W, S0):
    def fg(x):
        r = O.loss_grad(x.reshape(N, d), L, modes, W, S0)
        return r["loss"], r["grad"].ravel()
    return fg


@pytest.mark.parametrize("d,N,L,M", [(2, 300, 17.3, 6), (3, 400, 7.4, 3)])
def test_lbfgs_trajectory_matches_oracle_fp64(gpu, d, N, L, M):
    import torch
    from paper_2305_15693_amd import fresco as F
    pos0 = I.positions(N, d, L, np.float64, seed=50 + d)
    w, s0 = I.stealthy_target(d, M, float(M))
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-12, dtype="f64", device=gpu,
                    stream=torch.cuda.Stream(device=gpu))
    max_step = ctx.default_max_step()
    modes, W, S0 = O.constrained_set(d, M, w, s0)
    ref = LB.run(_oracle_fg(N, d, L, modes, W, S0), pos0, 6, m=4, max_step=max_step)
    pos = torch.from_numpy(pos0.copy()).to(gpu)
    losses = []
    for k in range(1, 7):
        loss, nev = ctx.step(pos, 1, m=4, max_step=max_step)
        torch.cuda.synchronize()
        x = pos.cpu().numpy().ravel()
        err = np.linalg.norm(x - ref["xs"][k]) / np.linalg.norm(ref["xs"][k] - ref["xs"][0])
        print(k, loss, ref["fs"][k], err)
        assert abs(loss - ref["fs"][k]) <= 1e-9 * abs(ref["fs"][0]), k
        assert err < 1e-8, k
        losses.append(loss)
    assert all(b <= a for a, b in zip(losses, losses[1:]))
    ctx.close()


@pytest.mark.parametrize("m", [1, 2, 3, 5, 16])
def test_lbfgs_history_lengths_match_oracle_fp64(gpu, m):
    """History lengths other than 4 and 8 -- the shortest ones, odd ones and the
    largest, whose update kernels hold half-width packs -- follow the oracle over
    24 iterations:
    the ring fills and then drops its oldest pair every step, so the kept R^-1
    is extended and truncated many times."""
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 1024, 32.0, 16
    pos0 = I.positions(N, d, L, np.float64, seed=60 + m)
    w, s0 = I.stealthy_target(d, M, float(M))
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-12, dtype="f64", device=gpu,
                    stream=torch.cuda.Stream(device=gpu))
    ms = ctx.default_max_step()
    modes, W, S0 = O.constrained_set(d, M, w, s0)
    ref = LB.run(_oracle_fg(N, d, L, modes, W, S0), pos0, 24, m=m, max_step=ms)
    pos = torch.from_numpy(pos0.copy()).to(gpu)
    loss, nev = ctx.step(pos, 24, m=m, max_step=ms)
    x = pos.cpu().numpy().ravel()
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"] - pos0.ravel())
    print(f"m = {m}: loss {loss:.12e} (oracle {ref['f']:.12e}), evaluations {nev} "
          f"({ref['nevals']}), position error {err:.2e}", flush=True)
    assert nev == ref["nevals"]
    assert abs(loss - ref["f"]) <= 1e-9 * ref["fs"][0]
    assert err < 1e-7
    ctx.close()


def test_lbfgs_fp32_decreases_like_oracle(gpu):
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 4000, 63.2, 14
    pos0 = I.positions(N, d, L, np.float32, seed=61)
    w, s0 = I.stealthy_target(d, M, float(M))
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                    stream=torch.cuda.Stream(device=gpu))
    pos = torch.from_numpy(pos0.copy()).to(gpu)
    loss, nev = ctx.step(pos, 25)
    modes, W, S0 = O.constrained_set(d, M, w, s0)
    ref = LB.run(_oracle_fg(N, d, L, modes, W, S0), pos0.astype(np.float64), 25,
                 max_step=ctx.default_max_step())
    f0 = ref["fs"][0]
    print("gpu", loss, "oracle", ref["f"], "start", f0, "evals", nev, ref["nevals"])
    # the end point is a real decrease, of the same size as the FP64 run's
    assert loss < 0.2 * f0
    assert abs(loss - ref["f"]) < 0.05 * f0
    # and its loss is what the oracle computes at the returned positions (the
    # absolute error of S is set by the transform accuracy relative to the O(1)
    # scale of S, so it is measured against the starting loss)
    x = pos.cpu().numpy().astype(np.float64)
    assert abs(O.loss_grad(x, L, modes, W, S0, want_grad=False)["loss"] - loss) < 1e-10 * f0
    ctx.close()


def _f32_pair(gpu, streams, slack=None):
    import os
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 30000, 173.2, 30
    pos0 = I.positions(N, d, L, np.float32, seed=71)
    w, s0 = I.stealthy_target(d, M, float(M))
    ctxs = []
    for st in streams:
        if slack is not None:
            os.environ["FRESCO_SLACK"] = str(slack)
        try:
            ctxs.append(F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32",
                                  device=gpu, stream=st))
        finally:
            os.environ.pop("FRESCO_SLACK", None)
    return ctxs, pos0


def test_lbfgs_graph_eager_bitwise(gpu):
    """Graph replays and eager launches give the same trajectory bit for bit (the
    eager launches keep the cached tile order on the same trial steps)."""
    import torch
    (a, b), pos0 = _f32_pair(gpu, [torch.cuda.Stream(device=gpu), torch.cuda.default_stream(gpu)])
    assert a.plan_info()["slack"] == 2
    pa = torch.from_numpy(pos0.copy()).to(gpu)
    pb = torch.from_numpy(pos0.copy()).to(gpu)
    la, na = a.step(pa, 12)
    lb, nb = b.step(pb, 12)
    torch.cuda.synchronize()
    assert la == lb and na == nb
    assert torch.equal(pa, pb)
    # the loss of the last accepted trial step (its tile order possibly kept from
    # an earlier binning) against a plain evaluation at the returned positions
    lc, _ = a.loss_grad(pa)
    print(f"loss {la:.9e}, plain evaluation {lc:.9e}", flush=True)
    assert abs(lc - la) <= 1e-6 * abs(la)
    a.close()
    b.close()


def test_lbfgs_resume_bitwise_without_slack(gpu):
    """Without the cached tile order (slack 0) every trial step is binned: two
    calls of 6 iterations continue exactly like one call of 12, and the loss the
    update summed from the evaluation's partials is the one a plain evaluation
    at the returned positions gives (same partials, same order)."""
    import torch
    (a, b), pos0 = _f32_pair(gpu, [torch.cuda.Stream(device=gpu),
                                   torch.cuda.default_stream(gpu)], slack=0)
    assert a.plan_info()["slack"] == 0
    pa = torch.from_numpy(pos0.copy()).to(gpu)
    pb = torch.from_numpy(pos0.copy()).to(gpu)
    la, na = a.step(pa, 12)
    lb1, nb1 = b.step(pb, 6)
    lb2, nb2 = b.step(pb, 6)
    torch.cuda.synchronize()
    assert la == lb2
    assert torch.equal(pa, pb)
    assert na == nb1 + nb2 - 1  # the second call re-evaluates its starting point
    lc, _ = a.loss_grad(pa)
    assert lc == la
    a.close()
    b.close()


def test_lbfgs_cached_tile_order_follows_full_binning(gpu):
    """One chunk of 8 trial steps with the cached tile order (slack 2) against
    the same call binning every trial step (slack 0): the FP32 trajectories
    agree to the transform accuracy (later iterations of this non-convex
    minimisation amplify last-bit differences, so the comparison stops at the
    first chunk); a 40-iteration call converges like the binned one, and its
    returned loss is the oracle's at the returned positions."""
    import torch
    (a,), pos0 = _f32_pair(gpu, [torch.cuda.Stream(device=gpu)])
    (b,), _ = _f32_pair(gpu, [torch.cuda.Stream(device=gpu)], slack=0)
    f0, _ = a.loss_grad(torch.from_numpy(pos0.copy()).to(gpu))
    pa = torch.from_numpy(pos0.copy()).to(gpu)
    pb = torch.from_numpy(pos0.copy()).to(gpu)
    la, na = a.step(pa, 8)
    lb, nb = b.step(pb, 8)
    xa = pa.cpu().numpy().astype(np.float64)
    xb = pb.cpu().numpy().astype(np.float64)
    move = np.abs(xa - pos0).max()
    print(f"8 iterations: cached {la:.9e} ({na} evals), binned {lb:.9e} ({nb} evals), "
          f"largest move {move:.3f}, largest difference {np.abs(xa - xb).max():.2e}", flush=True)
    assert na == nb
    assert abs(la - lb) <= 1e-6 * abs(lb)
    assert np.abs(xa - xb).max() <= 1e-4 * move
    la, na = a.step(pa, 32)
    lb, nb = b.step(pb, 32)
    torch.cuda.synchronize()
    print(f"40 iterations: cached {la:.6e}, binned {lb:.6e}, start {f0:.6e}", flush=True)
    assert la < 1e-5 * f0 and lb < 1e-5 * f0
    d, N, L, M = 2, 30000, 173.2, 30
    w, s0 = I.stealthy_target(d, M, float(M))
    modes, W, S0 = O.constrained_set(d, M, w, s0)
    xa = pa.cpu().numpy().astype(np.float64)
    ref = O.loss_grad(xa, L, modes, W, S0, want_grad=False)["loss"]
    assert abs(ref - la) <= 1e-9 * f0
    a.close()
    b.close()


def test_lbfgs_cached_tile_order_matches_oracle_fp64(gpu):
    """One call of 24 iterations (three chunks of 8 trial steps, the tile order
    kept between binnings) follows the FP64 oracle's trajectory."""
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 1024, 32.0, 16
    pos0 = I.positions(N, d, L, np.float64, seed=54)
    w, s0 = I.stealthy_target(d, M, float(M))
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-12, dtype="f64", device=gpu,
                    stream=torch.cuda.Stream(device=gpu))
    assert ctx.plan_info()["slack"] == 2
    ms = ctx.default_max_step()
    modes, W, S0 = O.constrained_set(d, M, w, s0)
    ref = LB.run(_oracle_fg(N, d, L, modes, W, S0), pos0, 24, m=8, max_step=ms)
    pos = torch.from_numpy(pos0.copy()).to(gpu)
    loss, nev = ctx.step(pos, 24, max_step=ms)
    x = pos.cpu().numpy().ravel()
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"] - pos0.ravel())
    print(f"loss {loss:.12e} (oracle {ref['f']:.12e}), evaluations {nev} ({ref['nevals']}), "
          f"position error {err:.2e}", flush=True)
    assert nev == ref["nevals"]
    assert abs(loss - ref["f"]) <= 1e-9 * ref["fs"][0]
    assert err < 1e-7
    ctx.close()


@pytest.mark.parametrize("d,N,L,M,ranges", [(3, 8000, 20.0, 8, None), (2, 8000, 90.0, 20, "5")])
def test_lbfgs_fp64_reproducible(gpu, d, N, L, M, ranges):
    """The internal order is a stable sort by tile (or range of tiles): two
    contexts give the same FP64 trajectory bit for bit (every dot product is
    summed over the same order)."""
    import os
    import torch
    from paper_2305_15693_amd import fresco as F
    pos0 = I.positions(N, d, L, np.float64, seed=73)
    w, s0 = I.stealthy_target(d, M, float(M))
    out = []
    for _ in range(2):
        if ranges:
            os.environ["FRESCO_BIN_RANGES"] = ranges
        try:
            ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-12, dtype="f64", device=gpu,
                            stream=torch.cuda.Stream(device=gpu))
        finally:
            os.environ.pop("FRESCO_BIN_RANGES", None)
        if ranges:
            assert ctx.plan_info()["bin_ranges"] > 0
        p = torch.from_numpy(pos0.copy()).to(gpu)
        loss, nev = ctx.step(p, 10)
        torch.cuda.synchronize()
        out.append((loss, nev, p.cpu().numpy()))
        ctx.close()
    assert out[0][0] == out[1][0]
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])


def test_lbfgs_options_rejected(gpu):
    import torch
    from paper_2305_15693_amd import fresco as F
    ctx = F.Context(2, 100, 10.0, 3, k_cut=3.0, tol=1e-6, dtype="f32", device=gpu)
    pos = torch.rand(100, 2, device=gpu) * 10
    for kw in [dict(m=0), dict(m=17), dict(c1=1.5), dict(shrink=1.0), dict(max_step=-1.0)]:
        with pytest.raises(F.FrescoError) as e:
            ctx.step(pos, 3, **kw)
        assert e.value.code == F.EINVAL
    with pytest.raises(F.FrescoError):
        ctx.step(pos, -1)
    ctx.close()


def _fp64_case(gpu, wscale=1.0):
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 300, 17.3, 6
    pos0 = I.positions(N, d, L, np.float64, seed=52)
    w, s0 = I.stealthy_target(d, M, float(M))
    w = w * wscale
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-12, dtype="f64", device=gpu,
                    stream=torch.cuda.Stream(device=gpu))
    modes, W, S0 = O.constrained_set(d, M, w, s0)
    return ctx, pos0, _oracle_fg(N, d, L, modes, W, S0), (d, N, L, M)


def test_lbfgs_gtol_stop_counts_like_oracle(gpu):
    # gtol between the RMS gradients of the oracle's iterations 12 and 13 (5.4e-3
    # and 2.0e-3): both stop after 13 accepted iterations of a 500-iteration call
    # with the same number of evaluations; the replays issued after the stop are
    # bounded by two chunks (counted here through the per-stage launch counts)
    import torch
    ctx, pos0, fg, (d, N, L, M) = _fp64_case(gpu)
    gtol = 3.3e-3
    ms = ctx.default_max_step()
    ref = LB.run(fg, pos0, 500, m=8, max_step=ms, gtol=gtol)
    assert len(ref["xs"]) - 1 == 13
    pos = torch.from_numpy(pos0.copy()).to(gpu)
    ctx.set_timing(["interp"])
    loss, nev = ctx.step(pos, 500, max_step=ms, gtol=gtol)
    t = ctx.read_timing(reset=True)
    ctx.set_timing([])
    x = pos.cpu().numpy()
    print(f"gtol stop: evaluations {nev} (oracle {ref['nevals']}), executed {t['interp'][1]}, "
          f"loss {loss:.6e} (oracle {ref['f']:.6e})", flush=True)
    assert nev == ref["nevals"]
    assert abs(loss - ref["f"]) <= 1e-9 * ref["fs"][0]
    assert np.linalg.norm(x.ravel() - ref["x"]) <= 1e-7 * np.linalg.norm(ref["x"] - pos0.ravel())
    assert nev <= t["interp"][1] <= nev + 2 * 16  # two chunks of at most 16 trial steps
    ctx.close()


def test_lbfgs_line_search_failure_keeps_last_accepted_point(gpu):
    # weights scaled by 1e30 (the L-BFGS trajectory does not depend on the scale
    # of the loss): after 8 ordinary iterations and a reset of the history, a call
    # with a cap of one point spacing and no backtracking.  The gradient is so
    # large that the cap sets the steepest-descent step to a whole spacing, which
    # raises the loss (2.4e30 -> 1.5e31 in the oracle); the history is already
    # empty, so the second rejection ends the search: the call reports
    # ELINESEARCH, as the oracle raises, and leaves the positions at the last
    # accepted point, bit for bit
    import torch
    from paper_2305_15693_amd import fresco as F
    ctx, pos0, fg, (d, N, L, M) = _fp64_case(gpu, wscale=1e30)
    ms = ctx.default_max_step()
    ref = LB.run(fg, pos0, 8, m=8, max_step=ms)
    with pytest.raises(RuntimeError):
        LB.run(fg, ref["x"], 5, m=8, max_step=10 * ms, max_backtracks=0)
    pos = torch.from_numpy(pos0.copy()).to(gpu)
    loss8, _ = ctx.step(pos, 8, max_step=ms)
    torch.cuda.synchronize()
    keep = pos.clone()
    ctx.reset_history()  # first trial along -g with the large cap, as in the oracle run
    with pytest.raises(F.FrescoError) as e:
        ctx.step(pos, 5, max_step=10 * ms, max_backtracks=0)
    assert e.value.code == F.ELINESEARCH
    torch.cuda.synchronize()
    assert torch.equal(pos, keep)
    assert abs(loss8 - ref["f"]) <= 1e-9 * ref["fs"][0]
    # the context stays usable: an ordinary call continues from there
    loss, nev = ctx.step(pos, 2, max_step=ms)
    assert loss < loss8
    ctx.close()


def test_lbfgs_history_length_change_frees_buffers(gpu):
    # changing m reallocates the optimiser's vectors; the previous ones are freed,
    # so the context's device memory returns to the same size for the same m
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 20000, 141.4, 20
    w, s0 = I.stealthy_target(d, M, float(M))
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                    stream=torch.cuda.Stream(device=gpu))
    pos = torch.from_numpy(I.positions(N, d, L, np.float32, seed=88)).to(gpu)
    base = ctx.plan_info()["device_bytes"]
    sizes = []
    for m in (4, 12, 4, 12, 4):
        ctx.step(pos, 2, m=m)
        sizes.append(ctx.plan_info()["device_bytes"])
    print("device bytes", base, sizes, flush=True)
    assert sizes[0] == sizes[2] == sizes[4]
    assert sizes[1] == sizes[3]
    assert sizes[1] - sizes[0] == 2 * 8 * N * d * 4  # 8 more pairs of s and y
    ctx.close()


def test_device_memory_limit_reports_enomem(gpu):
    # FRESCO_DEVICE_MEMORY_LIMIT caps the context's device memory: creation below
    # what the plan needs fails with ENOMEM; a cap that fits the plan but not the
    # optimiser's buffers makes fresco_step fail with ENOMEM, releases what it had
    # allocated, and leaves the context usable for evaluations
    import os
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 20000, 141.4, 20
    w, s0 = I.stealthy_target(d, M, float(M))
    pos = torch.from_numpy(I.positions(N, d, L, np.float32, seed=89)).to(gpu)

    def make():
        return F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                         stream=torch.cuda.Stream(device=gpu))

    free = make()
    need = free.plan_info()["device_bytes"]
    ref_loss, ref_grad = free.loss_grad(pos)
    free.close()
    try:
        os.environ["FRESCO_DEVICE_MEMORY_LIMIT"] = str(need // 2)
        with pytest.raises(F.FrescoError) as e:
            make()
        assert e.value.code == F.ENOMEM
        os.environ["FRESCO_DEVICE_MEMORY_LIMIT"] = str(need + N * d * 4 * 3)
        ctx = make()
    finally:
        os.environ.pop("FRESCO_DEVICE_MEMORY_LIMIT", None)
    assert ctx.plan_info()["device_bytes"] == need
    with pytest.raises(F.FrescoError) as e:
        ctx.step(pos.clone(), 3)
    assert e.value.code == F.ENOMEM
    assert ctx.plan_info()["device_bytes"] == need
    loss, grad = ctx.loss_grad(pos)
    assert loss == ref_loss and torch.equal(grad, ref_grad)
    ctx.close()


def test_lbfgs_cached_tile_order_with_strengths_and_pair_fp64(gpu):
    """The kept tile order with polydisperse strengths (read through the kept
    permutation) and an attached soft-core pair term (which reads the trial
    points the record pass writes): one call of 24 iterations follows the FP64
    oracle L-BFGS on L_S + E."""
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, L, M = 2, 1024, 32.0, 16
    pos0 = I.positions(N, d, L, np.float64, seed=55)
    c = I.polydisperse_strengths(N, d, seed=56)
    w, s0 = I.stealthy_target(d, M, float(M))
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-12, dtype="f64", device=gpu,
                    stream=torch.cuda.Stream(device=gpu))
    assert ctx.plan_info()["slack"] == 2
    ctx.set_strengths(torch.from_numpy(c).to(gpu))
    sigma, eps, alpha, wp = 0.6, 1.0, 2.0, 3.0
    pc = F.PairContext(d, N, L, sigma=sigma, eps=eps, alpha=alpha, dtype="f64", device=gpu)
    ctx.attach_pair(pc, wp)
    ms = ctx.default_max_step()
    modes, W, S0 = O.constrained_set(d, M, w, s0)

    def fg(x):
        r = O.loss_grad_strengths(x.reshape(N, d), c, L, modes, W, S0)
        e, ge = O.pair(x.reshape(N, d), L, sigma, eps, alpha)
        return r["loss"] + wp * e, r["grad"].ravel() + wp * ge.ravel()

    ref = LB.run(fg, pos0, 24, m=8, max_step=ms)
    pos = torch.from_numpy(pos0.copy()).to(gpu)
    loss, nev = ctx.step(pos, 24, max_step=ms)
    x = pos.cpu().numpy().ravel()
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"] - pos0.ravel())
    print(f"loss {loss:.12e} (oracle {ref['f']:.12e}, start {ref['fs'][0]:.6e}), evaluations "
          f"{nev} ({ref['nevals']}), position error {err:.2e}", flush=True)
    assert nev == ref["nevals"]
    assert abs(loss - ref["f"]) <= 1e-9 * ref["fs"][0]
    assert err < 1e-7
    ctx.close()
    pc.close()
