"""Drivers over the optimiser: re-targeting a context (fresco_set_target),
warm-started sequences of targets (fresco_step_sequence; SI, movie encoding) and
cycles of minimisation and overlap removal (fresco_pair_replace_overlaps,
fresco_overlap_cycles; main text, quasicrystalline structures).

The overlap rule (a point is removed when a point of lower index lies closer
than the threshold, minimum image; replacements taken in index order) is
checked against a brute force over all pairs, bit for bit.
"""
import numpy as np
import pytest

from paper_2305_15693_amd import inputs as I

pytestmark = pytest.mark.gpu


def _overlaps_brute_force(pos, L, thr):
    """Indices i with some j < i closer than thr (minimum image), FP64."""
    p = pos.astype(np.float64)
    Lv = np.broadcast_to(np.asarray(L, np.float64), (p.shape[1],))
    out = []
    for i in range(1, len(p)):
        dv = p[i] - p[:i]
        dv -= Lv * np.rint(dv / Lv)
        if np.any(np.sum(dv * dv, 1) < thr * thr):
            out.append(i)
    return np.array(out, dtype=np.int64)


def _with_duplicates(N, d, L, dtype, seed, n_dup, n_near, thr):
    rng = np.random.default_rng(seed)
    pos = I.positions(N, d, L, dtype, seed=seed)
    src = rng.choice(N // 2, n_dup + n_near, replace=False)
    dst = N // 2 + rng.choice(N - N // 2, n_dup + n_near, replace=False)
    pos[dst[:n_dup]] = pos[src[:n_dup]]  # exact copies
    off = rng.normal(size=(n_near, d))
    off *= (0.3 * thr / np.linalg.norm(off, axis=1))[:, None]
    pos[dst[n_dup:]] = (pos[src[n_dup:]] + off).astype(dtype)  # closer than thr
    return pos


@pytest.mark.parametrize("d,N,dtype", [(2, 3000, "f32"), (3, 2500, "f64")])
def test_replace_overlaps_matches_brute_force(gpu, d, N, dtype):
    import torch
    from paper_2305_15693_amd import fresco as F
    ndt = np.float32 if dtype == "f32" else np.float64
    L = N ** (1.0 / d)
    thr = 1e-3
    pos_np = _with_duplicates(N, d, L, ndt, 70 + d, 40, 15, thr)
    flagged = _overlaps_brute_force(pos_np, L, thr)
    assert len(flagged) >= 50
    fresh_np = I.positions(200, d, L, ndt, seed=71 + d)
    pc = F.PairContext(d, N, L, sigma=thr, dtype=dtype, device=gpu)
    pos = torch.from_numpy(pos_np.copy()).to(gpu)
    fresh = torch.from_numpy(fresh_np).to(gpu)
    # too few fresh rows: refused, positions untouched
    with pytest.raises(F.FrescoError):
        pc.replace_overlaps(pos, thr, fresh[:10])
    assert np.array_equal(pos.cpu().numpy(), pos_np)
    n = pc.replace_overlaps(pos, thr, fresh)
    expect = pos_np.copy()
    expect[flagged] = fresh_np[:len(flagged)]
    print(f"{d}D {dtype}: {n} overlaps replaced (brute force {len(flagged)})", flush=True)
    assert n == len(flagged)
    assert np.array_equal(pos.cpu().numpy(), expect)
    # nothing left to replace
    assert pc.replace_overlaps(pos, thr, fresh[n:]) == 0
    pc.close()


def test_overlap_cycles_match_manual_cycles(gpu):
    # coincident points receive identical gradients and stay coincident under
    # the minimisation; the first cycle replaces them, the second finds none
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, M = 2, 3000, 12
    L = N ** 0.5
    thr = 1e-3
    pos_np = _with_duplicates(N, d, L, np.float32, 81, 30, 0, thr)
    fresh_np = I.positions(100, d, L, np.float32, seed=82)
    w, s0 = I.stealthy_target(d, M, float(M))
    fresh = torch.from_numpy(fresh_np).to(gpu)
    res = []
    for manual in (False, True):
        ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-6, dtype="f32", device=gpu,
                        stream=torch.cuda.Stream(device=gpu))
        pc = F.PairContext(d, N, L, sigma=thr, dtype="f32", device=gpu)
        pos = torch.from_numpy(pos_np.copy()).to(gpu)
        if manual:
            used, cyc, loss = 0, 0, None
            for _ in range(4):
                loss, _ = ctx.step(pos, 6)
                torch.cuda.synchronize()
                cyc += 1
                n = pc.replace_overlaps(pos, thr, fresh[used:])
                used += n
                if n == 0:
                    break
                ctx.reset_history()
            res.append((loss, cyc, used, pos.cpu().numpy()))
        else:
            loss, cyc, used = ctx.overlap_cycles(pc, pos, 6, 4, thr, fresh)
            res.append((loss, cyc, used, pos.cpu().numpy()))
        ctx.close()
        pc.close()
    print(f"overlap cycles: {res[0][1]} cycles, {res[0][2]} replaced, loss {res[0][0]:.6e}",
          flush=True)
    assert res[0][1] == 2 and res[0][2] == 30
    assert res[0][:3] == res[1][:3]
    assert np.array_equal(res[0][3], res[1][3])
    assert len(_overlaps_brute_force(res[0][3], L, thr)) == 0


def test_set_target_matches_a_new_context(gpu):
    # re-targeting in place and continuing equals a context created with the new
    # target from the same positions, bit for bit
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, M = 2, 20000, 20
    L = N ** 0.5
    wa, sa = I.power_law_target(d, M, 20.0, 2.0)
    wb, sb = I.power_law_target(d, M, 20.0, 4.0)
    pos0 = torch.from_numpy(I.positions(N, d, L, np.float32, seed=83)).to(gpu)
    a = F.Context(d, N, L, M, w_cube=wa, s0_cube=sa, relative=True, tol=1e-6, dtype="f32",
                  device=gpu, stream=torch.cuda.Stream(device=gpu))
    pa = pos0.clone()
    a.step(pa, 3)
    a.set_target(sb, wb, relative=True)
    # the re-targeted context evaluates the new loss (oracle, direct sums)
    from oracle import oracle as O
    modes, W, S0 = O.constrained_set(d, M, wb, sb, relative=True)
    xa = pa.cpu().numpy().astype(np.float64)
    ref = O.loss_grad(xa, L, modes, W, S0)
    l_new, g_new = a.loss_grad(pa)
    assert abs(l_new - ref["loss"]) <= 1e-5 * ref["loss"]
    assert np.linalg.norm(g_new.cpu().numpy() - ref["grad"]) <= 1e-5 * np.linalg.norm(ref["grad"])
    pb = pa.clone()
    la, na = a.step(pa, 5)
    b = F.Context(d, N, L, M, w_cube=wb, s0_cube=sb, relative=True, tol=1e-6, dtype="f32",
                  device=gpu, stream=torch.cuda.Stream(device=gpu))
    lb, nb = b.step(pb, 5)
    torch.cuda.synchronize()
    assert (la, na) == (lb, nb)
    assert torch.equal(pa, pb)
    assert a.plan_info()["n_constrained"] == b.plan_info()["n_constrained"]
    a.close()
    b.close()


def test_step_sequence_warm_starts(gpu):
    # stealthy frames whose cutoff grows from frame to frame: the driver equals
    # the manual loop of set_target + step bit for bit, and a frame started from
    # the previous frame reaches the gradient tolerance in fewer evaluations than
    # the same frame started from the Poisson points
    import torch
    from paper_2305_15693_amd import fresco as F
    d, N, M = 2, 8000, 12
    L = N ** 0.5
    ws = [I.stealthy_target(d, M, k)[0] for k in (9.0, 10.0, 11.0)]
    pos0 = torch.from_numpy(I.positions(N, d, L, np.float64, seed=84)).to(gpu)

    def ctx():
        return F.Context(d, N, L, M, w_cube=ws[0], tol=1e-12, dtype="f64", device=gpu,
                         stream=torch.cuda.Stream(device=gpu))

    c0 = ctx()
    g0 = c0.loss_grad(pos0)[1]
    gtol = 1e-3 * float(g0.pow(2).mean().sqrt())
    p = pos0.clone()
    losses, nevs, frames = c0.step_sequence(p, 400, w_cubes=ws, gtol=gtol)
    c0.close()
    c1 = ctx()
    q = pos0.clone()
    manual = []
    for t, w in enumerate(ws):
        c1.set_target(None, w)
        manual.append(c1.step(q, 400, gtol=gtol))
        assert torch.equal(frames[t], q)
    c1.close()
    assert [m[0] for m in manual] == losses and [m[1] for m in manual] == nevs
    assert torch.equal(p, frames[-1])
    cold = []
    for w in ws[1:]:
        c2 = ctx()
        c2.set_target(None, w)
        cold.append(c2.step(pos0.clone(), 400, gtol=gtol)[1])
        c2.close()
    print(f"warm-started frames: evaluations {nevs} (cold starts of frames 1.. {cold}), "
          f"losses {['%.3e' % x for x in losses]}", flush=True)
    assert all(nw < nc for nw, nc in zip(nevs[1:], cold))
