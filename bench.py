#!/usr/bin/env python3
"""Throughput of the FReSCo loss + gradient evaluation on one MI355X.

Headline workload (2D, N = 1e6 uniform random points, L = 1000, stealthy target
0 < |n| <= 300, nuFFT tolerance 1e-6, FP32): L-BFGS iterations of the plain
single-configuration path, as in the paper's minimisations.  A step is one
L-BFGS iteration (loss + gradient evaluations of its line search and the
optimiser update, all on the GPU, replayed from a captured HIP graph);
`value` is loss + gradient evaluations per second over the timed steps.
Inputs are resident in device memory before timing starts.

Prints one JSON line.  Besides the throughput it carries:
  plain_eval    stateless evaluations (fresco_loss_grad_async) per second on the
                same workload, points in the caller's random order;
  roofline      the dominant kernel, timed with HIP events on the library's
                stream: algorithmic bytes against the 8 TB/s HBM peak and
                algorithmic flops against the vector ALU peak (the bound is the
                larger fraction; the spreading and interpolation kernels are
                bound by vector-instruction issue), the measured VALU issue
                fraction, and whether the working set fits in the 256 MB
                Infinity Cache (the 2D workload's does);
  cpu_baseline  the FP64 direct-sum oracle timed on this host's cores on a
                bounded sample (all modes for a subset of the points), scaled
                to one full evaluation;
  stages_ms     average time of every stage of one evaluation;
  rocfft        the library's transforms (torch.fft.rfftn / irfftn, rocFFT on
                ROCm) timed on the same fine grid, as a comparison only, beside
                the time of this path's own FFT chain (pruned, with the fold and
                the mode stage inside);
  copy_gbs      a plain 1 GiB device copy timed on this GPU (the achievable
                streaming rate; the roofline also reports its fraction of it);
  fp64_context  plain evaluations per second of the same workload in the FP64
                build at tolerance 1e-12;
  secondary     the same measurements for the 3D workload (N = 1e7), plus the
                torch.autograd evaluation of spectral loss + soft-core pair
                term in one backward;
  batch         a ragged batch of 256 2D configurations: one batched launch vs
                a loop of the single-problem path, and batched L-BFGS steps.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "loss+grad evals/sec (N=1e6 2D, N=1e7 3D) + spread/interp HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
# Vector ALU peak without packed FP32 (this library's device code is built with
# packed FP32 off): 256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz.
# The 157.3 TFLOP/s datasheet FP32 figure needs packed FP32 (two lanes' worth
# per instruction); FP64 vector is 78.6 either way.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
ALU_PEAK_DATASHEET = {"f32": 157.3, "f64": 78.6}
# wave64 vector instructions the chip issues per second (1024 SIMDs, one every
# 4 cycles each)
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4
INFINITY_CACHE_MB = 256.0
DOM_REPS = 30  # launches of the dominant spread / interp kernel per timing bracket
def kernel_eval_flops(width):
    """Flops of the FP32 kernel values along one axis at one width: degree-9 per-cell
    polynomials in x, with mirrored cells (j and width - 1 - j) sharing one even and
    one odd part in y = x^2 (two 4-FMA chains and two combining FMAs per pair, four
    FMAs for the middle cell of an odd width) and y itself (one product)."""
    fmas = 10 * (width // 2) + 4 * (width % 2)
    return 2 * fmas + 1


def stage_flops(cfg, info):
    """Algorithmic flops per point of the spreading and interpolation kernels: the
    kernel values along each axis (with their derivatives for the interpolation, at
    width wi = w + 1; the derivative shares y = x^2 with the kernel) and the
    tensor-product contraction:
      spread:  d kernel evaluations + the w + w^2 (+ w^3) footprint products
      interp:  d (kernel + derivative) evaluations + 2 wi^d row FMAs
               + 3 wi^(d-1) (+ 4 wi in 3D)
    (FMA = 2 flops).  In FP64 the kernel values are exp and sqrt per cell, not
    polynomials; their flops are not counted (a lower bound)."""
    d, N = cfg["d"], cfg["N"]
    w = info["width"]
    wi = w + 1
    poly = cfg.get("dtype", "f32") == "f32"
    ev_s = kernel_eval_flops(w) if poly else 0
    ev_i = 2 * kernel_eval_flops(wi) - 1 if poly else 0
    sp = d * ev_s + sum(w ** k for k in range(1, d + 1))
    if d == 2:
        ip = d * ev_i + 2 * (2 * wi ** 2 + 3 * wi)
    else:
        ip = d * ev_i + 2 * (2 * wi ** 3 + 3 * wi ** 2 + 4 * wi)
    return {"spread": sp * N, "interp": ip * N, "per_point": {"spread": sp, "interp": ip}}


def stage_bytes(cfg, info, dtype_bytes):
    """Algorithmic HBM bytes of one launch of each stage (what the step must move)."""
    d, N = cfg["d"], cfg["N"]
    sp = sg = dtype_bytes
    cs = 2 * sg
    nf = info["nf"]
    M = info["kmax"]
    ngrid = 1
    for x in nf:
        ngrid *= x
    H0 = M[0] + 1
    P = [2 * m + 1 for m in M]
    nhalf = H0
    for a in range(1, d):
        nhalf *= P[a]
    rows = ngrid // nf[0]
    b = {}
    b["bin"] = 2 * N * d * sp + 4 * N
    b["spread"] = N * d * sp + ngrid * sg
    b["fold"] = 2 * ngrid * sg
    b["fft_rows_fwd"] = ngrid * sg + rows * H0 * cs
    # the gradient comes from one field (derivative interpolation), so the inverse
    # chain carries one array
    if d == 3:
        b["fft_cols_fwd"] = nf[2] * nf[1] * H0 * cs + nf[2] * P[1] * H0 * cs
        last_in = nf[2] * P[1] * H0 * cs
        b["fft_cols_inv"] = nf[2] * P[1] * H0 * cs + nf[2] * nf[1] * H0 * cs
    else:
        last_in = nf[1] * H0 * cs
    b["modes"] = last_in + 4 * nhalf * sg + last_in
    b["fft_rows_inv"] = rows * H0 * cs + ngrid * sg
    b["interp"] = ngrid * sg + 2 * N * d * sp
    return b


_STAGE_SOURCES = {
    "spread.hip": ("bin", "spread", "fold", "interp"),
    "fft.hip": ("fft_rows_fwd", "fft_cols_fwd", "modes", "fft_cols_inv", "fft_rows_inv"),
}


def stage_source_hash(stage):
    """sha256 of the sources that define a stage's kernel (with their headers)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2305_15693_amd", "csrc")
    main = [f for f, st in _STAGE_SOURCES.items() if stage in st]
    files = main + ["kernels.h", "common.h"] if main == ["spread.hip"] else \
        main + ["fft_lds.h", "fft.h", "common.h"]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, stage):
    """HBM bytes per launch of a stage's kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading), or None when there
    is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(stage)
    if not k or k.get("source_sha256") != stage_source_hash(stage):
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def measured_valu(workload, stage):
    """Wave64 vector instructions per launch of a stage's kernel from the committed
    counter summary (SQ_INSTS_VALU), or None when there is none or the kernel's
    sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(stage)
    if not k or k.get("source_sha256") != stage_source_hash(stage):
        return None
    return k["valu_insts"]


def copy_rate(dev):
    """GB/s of a plain 1 GiB device-to-device copy (bytes read + written)."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del src, dst
    torch.cuda.empty_cache()
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def rocfft_compare(nf, stages_ms, dev, reps=20):
    """torch.fft.rfftn / irfftn (rocFFT) on a real grid of the fine-grid shape,
    full and unpruned, against this path's FFT chain per evaluation."""
    import torch
    shape = tuple(reversed(nf))  # axis 0 fastest
    x = torch.randn(shape, dtype=torch.float32, device=dev)
    X = torch.fft.rfftn(x)
    y = torch.fft.irfftn(X, s=shape)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        X = torch.fft.rfftn(x)
    e[1].record()
    for _ in range(reps):
        y = torch.fft.irfftn(X, s=shape)
    e[2].record()
    torch.cuda.synchronize()
    chain = [k for k in stages_ms if k.startswith("fft_") or k == "modes"]
    del x, X, y
    torch.cuda.empty_cache()
    return {"grid": list(nf), "rfftn_ms": e[0].elapsed_time(e[1]) / reps,
            "irfftn_ms": e[1].elapsed_time(e[2]) / reps,
            "ours_fft_chain_ms": sum(stages_ms[k] for k in chain), "ours_stages": chain}


def roofline(name, cfg, info, kernel, avg_ms, alg_bytes):
    """Roofline of the dominant kernel: HBM (algorithmic bytes / 8 TB/s) and vector
    ALU (algorithmic flops / the non-packed FP32 or FP64 peak) fractions; the
    bound is the larger.  The measured VALU issue fraction (instructions from the
    committed counters over the chip's issue rate, against the same duration) is
    reported beside them.  The working set of the context (its device scratch,
    positions and gradient) is compared with the 256 MB Infinity Cache: below it,
    the bytes stream from that cache rather than from HBM."""
    dt = 4 if cfg["dtype"] == "f32" else 8
    gbs = alg_bytes / (avg_ms * 1e-3) / 1e9
    hbm = {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "algorithmic_bytes": alg_bytes, "traffic": measured_traffic(name, kernel)}
    fl = stage_flops(cfg, info)
    alu = None
    if kernel in ("spread", "interp"):
        tf = fl[kernel] / (avg_ms * 1e-3) / 1e12
        ds = ALU_PEAK_DATASHEET[cfg["dtype"]]
        alu = {"achieved": tf, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": tf / ALU_PEAK_TFLOPS, "flops_per_point": fl["per_point"][kernel],
               "peak_datasheet": ds, "frac_of_datasheet": tf / ds}
        vi = measured_valu(name, kernel)
        if vi is not None:
            alu["valu_insts_per_launch"] = vi
            alu["valu_issue_frac"] = vi / VALU_ISSUE_PER_S / (avg_ms * 1e-3)
    ws_mb = (info["device_bytes"] + 2 * cfg["N"] * cfg["d"] * dt) / 1e6
    out = {"kernel": kernel, "avg_ms": avg_ms, "hbm": hbm, "alu": alu,
           "working_set_mb": ws_mb, "infinity_cache_resident": ws_mb < INFINITY_CACHE_MB}
    main = alu if (alu is not None and alu["frac"] > hbm["frac"]) else hbm
    out.update(bound="alu" if main is alu else "hbm", achieved=main["achieved"],
               peak=main["peak"], unit=main["unit"], frac=main["frac"],
               traffic=hbm["traffic"])
    return out


def measure_fp64_context(name, steps, dev):
    """The same workload in the FP64 build (tolerance 1e-12, as the paper's FP64
    runs): plain evaluations per second, for precision context."""
    import numpy as np
    import torch

    from paper_2305_15693_amd import fresco as F
    from paper_2305_15693_amd import inputs as I

    cfg = I.WORKLOADS[name]
    d, N, L, M = cfg["d"], cfg["N"], cfg["L"], cfg["M"]
    w, s0 = I.stealthy_target(d, M, cfg["kcut"])
    stream = torch.cuda.Stream(device=dev)
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=1e-12, dtype="f64", device=dev,
                    stream=stream)
    pos = torch.from_numpy(I.positions(N, d, L, np.float64, seed=cfg["seed"])).to(dev)
    grad = torch.empty_like(pos)
    loss_dev = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(2):
        ctx.loss_grad_async(pos, loss_dev, grad)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        ctx.loss_grad_async(pos, loss_dev, grad)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out = {"workload": name.replace("_f32", "_f64"), "tol": 1e-12,
           "width": ctx.plan_info()["width"], "plain_evals_per_s": 1e3 / ms, "plain_ms": ms}
    ctx.close()
    del pos, grad
    torch.cuda.empty_cache()
    return out


def measure(name, steps, warmup, dev, lbfgs_steps):
    import numpy as np
    import torch

    from paper_2305_15693_amd import fresco as F
    from paper_2305_15693_amd import inputs as I

    cfg = I.WORKLOADS[name]
    d, N, L, M = cfg["d"], cfg["N"], cfg["L"], cfg["M"]
    dtype = cfg["dtype"]
    pos_np = I.positions(N, d, L, np.float32 if dtype == "f32" else np.float64, seed=cfg["seed"])
    w, s0 = I.stealthy_target(d, M, cfg["kcut"])
    # a dedicated stream: evaluations on it are replayed from captured HIP graphs
    stream = torch.cuda.Stream(device=dev)
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=cfg["tol"], dtype=dtype, device=dev,
                    stream=stream)
    info = ctx.plan_info()
    pos = torch.from_numpy(pos_np).to(dev)
    grad = torch.empty_like(pos)
    loss_dev = torch.zeros(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    # per-stage profile (untimed, eager launches): every stage bracketed with events
    ctx.set_timing(F.STAGES)
    for _ in range(3):
        ctx.loss_grad_async(pos, loss_dev, grad)
    ctx.read_timing(reset=True)
    for _ in range(5):
        ctx.loss_grad_async(pos, loss_dev, grad)
    prof = ctx.read_timing(reset=True)
    ctx.set_timing([])
    stages_ms = {k: v[0] / v[1] for k, v in prof.items()}
    sbytes = stage_bytes(cfg, info, 4 if dtype == "f32" else 8)
    single = [k for k in stages_ms if k in F.SINGLE_KERNEL_STAGES]
    dominant = max(single, key=lambda k: stages_ms[k])

    # stateless evaluations: graph replays of the whole evaluation
    for _ in range(warmup):
        ctx.loss_grad_async(pos, loss_dev, grad)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        ctx.loss_grad_async(pos, loss_dev, grad)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1)
    loss0 = float(loss_dev.item())

    # the dominant kernel, event-timed on the library's stream over as many
    # evaluations; the spread and interp kernels run DOM_REPS times back to back
    # inside each bracket, so that the time per launch is the kernel's own rather
    # than the bracket's launch overhead (it agrees with the kernel trace)
    ctx.set_timing([dominant], reps=DOM_REPS if dominant in ("spread", "interp") else 1)
    for _ in range(steps):
        ctx.loss_grad_async(pos, loss_dev, grad)
    dom = ctx.read_timing(reset=True)[dominant]
    ctx.set_timing([])
    dom_ms = dom[0] / dom[1]
    achieved = sbytes[dominant] / (dom_ms * 1e-3) / 1e9
    roof = roofline(name, cfg, info, dominant, dom_ms, sbytes[dominant])

    res = dict(workload=name, cfg=cfg, info=info, stages_ms=stages_ms,
               rocfft=rocfft_compare(info["nf"], stages_ms, dev),
               stage_gbs={k: sbytes[k] / (stages_ms[k] * 1e-3) / 1e9
                          for k in stages_ms if k in sbytes},
               plain_evals_per_s=steps / (ms_plain * 1e-3), plain_ms=ms_plain / steps,
               loss0=loss0, hbm_gbs=achieved, roofline=roof,
               pos_np=pos_np, w=w, s0=s0)

    if lbfgs_steps:
        # L-BFGS from the Poisson start: a few warm-up iterations on a copy (graph
        # capture, allocations), then the timed iterations from the start again
        warm = pos.clone()
        ctx.step(warm, max(1, warmup))
        ctx.reset_history()
        work = pos.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        loss, nev = ctx.step(work, lbfgs_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        res.update(lbfgs_ms=ms, lbfgs_wall_s=wall, lbfgs_evals=nev, lbfgs_iters=lbfgs_steps,
                   lbfgs_loss=loss, lbfgs_evals_per_s=nev / (ms * 1e-3))
        del warm, work
    ctx.close()
    del pos, grad
    torch.cuda.empty_cache()
    return res


def measure_autograd_pair(name, steps, dev):
    """3D packing workload through torch.autograd: spectral loss + soft-core pair
    term (sigma = 0.5, harmonic, weight 1) in one backward; also the pair pass alone."""
    import numpy as np
    import torch

    from paper_2305_15693_amd import autograd as A
    from paper_2305_15693_amd import fresco as F
    from paper_2305_15693_amd import inputs as I

    cfg = I.WORKLOADS[name]
    d, N, L, M = cfg["d"], cfg["N"], cfg["L"], cfg["M"]
    w, s0 = I.stealthy_target(d, M, cfg["kcut"])
    ctx = F.Context(d, N, L, M, w_cube=w, s0_cube=s0, tol=cfg["tol"], dtype=cfg["dtype"], device=dev)
    pctx = F.PairContext(d, N, L, sigma=cfg.get("sigma", 0.5), eps=1.0, alpha=2.0,
                         dtype=cfg["dtype"], device=dev)
    pos = torch.from_numpy(I.positions(N, d, L, np.float32, seed=cfg["seed"])).to(dev)
    pos.requires_grad_(True)

    def one():
        pos.grad = None
        total = A.loss(ctx, pos) + A.soft_core(pctx, pos)
        total.backward()
        return total

    for _ in range(2):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        total = one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    e_dev = torch.zeros((), dtype=torch.float64, device=dev)
    g = torch.empty_like(pos)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    pd = pos.detach()
    pctx.energy_grad_async(pd, e_dev, g)
    e0.record()
    for _ in range(steps):
        pctx.energy_grad_async(pd, e_dev, g)
    e1.record()
    torch.cuda.synchronize()
    pair_ms = e0.elapsed_time(e1) / steps
    out = {"autograd_evals_per_s": 1e3 / ms, "autograd_ms": ms, "pair_ms": pair_ms,
           "pair_energy": float(e_dev), "total_loss": float(total)}
    ctx.close()
    pctx.close()
    return out


def measure_batch(dev, steps):
    """Ragged batch of 256 2D configurations (N log-uniform in [1e3, 1e5], unit
    density, power-law targets |k| < 2 pi 20 / L, relative weights): one persistent
    batched launch per evaluation against a loop of the plain single-problem path
    over the same configurations, and batched L-BFGS iterations under graph replay."""
    import numpy as np
    import torch

    from paper_2305_15693_amd import fresco as F
    from paper_2305_15693_amd import inputs as I

    kcut, M = 20, 19
    cfgs = I.ragged_batch(nb=256, kcut=kcut, seed=1004)
    items, pos_l = [], []
    for c in cfgs:
        w, s0 = I.power_law_target(2, M, kcut, c["alpha"])
        items.append(dict(n=c["N"], box=c["L"], w_cube=w, s0_cube=s0, relative=True))
        pos_l.append(I.positions(c["N"], 2, c["L"], np.float32, seed=c["seed"]))
    stream = torch.cuda.Stream(device=dev)
    bc = F.BatchContext(2, M, items, tol=1e-6, dtype="f32", device=dev, stream=stream)
    pos = torch.from_numpy(np.concatenate(pos_l, 0)).to(dev)
    threads = bc.autotune(pos, reps=3)
    grad = torch.empty_like(pos)
    losses = torch.zeros(256, dtype=torch.float64, device=dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        bc.loss_grad_async(pos, losses, grad)
    e0.record(stream)
    for _ in range(steps):
        bc.loss_grad_async(pos, losses, grad)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1) / steps
    # loop of the plain path (each evaluation replayed from its captured graph)
    ctxs, views, grads, ldev = [], [], [], torch.zeros(256, dtype=torch.float64, device=dev)
    for b, c in enumerate(cfgs):
        w, s0 = I.power_law_target(2, M, kcut, c["alpha"])
        ctxs.append(F.Context(2, c["N"], c["L"], M, w_cube=w, s0_cube=s0, relative=True, tol=1e-6,
                              dtype="f32", device=dev, stream=stream))
        views.append(pos[bc.offsets[b]:bc.offsets[b + 1]])
        grads.append(torch.empty_like(views[-1]))
    for _ in range(2):
        for b in range(256):
            ctxs[b].loss_grad_async(views[b], ldev[b:b + 1], grads[b])
    torch.cuda.synchronize()
    reps = max(1, steps // 10)
    e0.record(stream)
    for _ in range(reps):
        for b in range(256):
            ctxs[b].loss_grad_async(views[b], ldev[b:b + 1], grads[b])
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1) / reps
    diff = float((ldev - losses).abs().max() / losses.abs().max())
    for cx in ctxs:
        cx.close()
    # batched L-BFGS iterations
    work = pos.clone()
    bc.step(work, 2, max_step=0.05)
    bc.reset_history()
    work.copy_(pos)
    torch.cuda.synchronize()
    e0.record(stream)
    loss, nev = bc.step(work, steps, max_step=0.05)
    e1.record(stream)
    torch.cuda.synchronize()
    it_ms = e0.elapsed_time(e1) / steps
    bc.close()
    return {"workload": "2d_ragged256_powerlaw_f32", "configs": 256, "points": int(pos.shape[0]),
            "autotuned_threads": threads, "batched_eval_ms": batch_ms, "loop_eval_ms": loop_ms,
            "speedup": loop_ms / batch_ms, "loss_max_rel_diff_batch_vs_loop": diff,
            "lbfgs_iter_ms": it_ms, "lbfgs_evals": nev, "lbfgs_iters": steps,
            "lbfgs_loss_start": float(losses.sum()), "lbfgs_loss_end": loss}


def cpu_baseline(res, rho_points=200000, grad_points=60000):
    """Oracle timed on a bounded sample of the same evaluation, scaled to one
    full evaluation.  Both of the oracle's sums are linear in the points: rho(k)
    over all constrained modes is timed on `rho_points` of the points and the
    gradient (all modes) on `grad_points` of them; each is scaled by N / sample."""
    import numpy as np

    from oracle import oracle as O

    cfg = res["cfg"]
    d, N, L, M = cfg["d"], cfg["N"], cfg["L"], cfg["M"]
    modes, W, S0 = O.constrained_set(d, M, res["w"], res["s0"])
    K = len(modes)
    rng = np.random.default_rng(0)
    pos = res["pos_np"]
    sub = pos[rng.choice(N, min(rho_points, N), replace=False)]
    t0 = time.perf_counter()
    O.loss_grad(sub, L, modes, W, S0, want_grad=False)
    t_rho = time.perf_counter() - t0
    gp = rng.choice(N, min(grad_points, N), replace=False)
    t0 = time.perf_counter()
    O.loss_grad(pos[:1], L, modes, W, S0, want_grad=False)
    t_one = time.perf_counter() - t0  # the rho pass of the call below (one point)
    t0 = time.perf_counter()
    O.loss_grad(pos[gp], L, modes, W, S0)
    t_grad = max(time.perf_counter() - t0 - t_rho * len(gp) / len(sub), 0.0)
    full = t_rho * (N / len(sub)) + t_grad * (N / len(gp))
    return {"value": 1.0 / full, "unit": "evals/s", "cores": O.threads(), "kind": "oracle",
            "sample": (f"rho over all {K} constrained modes for {len(sub)} of the {N} points "
                       f"({t_rho:.2f} s) and the gradient of {len(gp)} points over all modes "
                       f"({t_grad:.2f} s), each scaled by N / sample to one full evaluation "
                       f"({full:.0f} s); single-point call overhead {t_one * 1e3:.1f} ms")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed L-BFGS iterations")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="2d_n1e6_stealthy300_f32")
    ap.add_argument("--secondary", default="3d_n1e7_stealthy60_f32",
                    help="second workload measured the same way ('' to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the ragged-batch measurement")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-build context line")
    ap.add_argument("--plain", action="store_true",
                    help="a step is one loss + gradient evaluation (no optimiser), e.g. for "
                         "the N = 1e9 workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration in profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "the library runs on one GPU per process; no multi-GPU path exists", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        # a plain device copy of known size, for scaling the HBM byte counters of a
        # profiler run (FETCH_SIZE / WRITE_SIZE read for it vs 1 GiB moved each way)
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    if args.plain:
        r = measure(args.workload, args.steps, args.warmup, dev, 0)
        print(f"[bench] {args.workload}: plain {r['plain_evals_per_s']:.2f} evals/s",
              file=sys.stderr, flush=True)
    else:
        r = measure(args.workload, 50, args.warmup, dev, args.steps)
        print(f"[bench] {args.workload}: L-BFGS {r['lbfgs_evals_per_s']:.1f} evals/s, "
              f"plain {r['plain_evals_per_s']:.1f} evals/s", file=sys.stderr, flush=True)
    sec = None
    if args.secondary:
        s = measure(args.secondary, 10, 2, dev, max(5, args.steps // 10))
        print(f"[bench] {args.secondary}: L-BFGS {s['lbfgs_evals_per_s']:.1f} evals/s, "
              f"plain {s['plain_evals_per_s']:.1f} evals/s", file=sys.stderr, flush=True)
        sec = {"workload": s["workload"], "lbfgs_evals_per_s": s["lbfgs_evals_per_s"],
               "lbfgs_iters": s["lbfgs_iters"], "lbfgs_evals": s["lbfgs_evals"],
               "lbfgs_ms": s["lbfgs_ms"], "plain_evals_per_s": s["plain_evals_per_s"],
               "plain_ms": s["plain_ms"], "roofline": s["roofline"],
               "stages_ms": s["stages_ms"], "stage_gbs": s["stage_gbs"], "rocfft": s["rocfft"],
               "nf": s["info"]["nf"], "width": s["info"]["width"]}
        if s["cfg"]["d"] == 3:
            ag = measure_autograd_pair(args.secondary, 5, dev)
            print(f"[bench] {args.secondary} autograd (spectral + soft core): "
                  f"{ag['autograd_evals_per_s']:.1f} evals/s, pair pass {ag['pair_ms']:.3f} ms",
                  file=sys.stderr, flush=True)
            sec["autograd_with_pair"] = ag
    bat = None
    if not args.no_batch:
        bat = measure_batch(dev, 20)
        print(f"[bench] ragged batch: {bat['batched_eval_ms']:.3f} ms batched vs "
              f"{bat['loop_eval_ms']:.3f} ms loop ({bat['speedup']:.1f}x); L-BFGS iteration "
              f"{bat['lbfgs_iter_ms']:.3f} ms", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(r)
        print(f"[bench] cpu baseline: {cpu['value']:.3g} evals/s", file=sys.stderr, flush=True)
    cfg = r["cfg"]
    info = r["info"]
    f64 = None
    if not args.plain and not args.no_fp64:
        f64 = measure_fp64_context(args.workload, 10, dev)
        print(f"[bench] {f64['workload']} (FP64 build, tol 1e-12): plain "
              f"{f64['plain_evals_per_s']:.1f} evals/s", file=sys.stderr, flush=True)
    copy_gbs = copy_rate(dev)
    for rr in [r["roofline"]] + ([sec["roofline"]] if sec else []):
        rr["hbm"]["frac_of_copy"] = rr["hbm"]["achieved"] / copy_gbs
    out = {
        "metric": METRIC,
        "value": r["plain_evals_per_s"] if args.plain else r["lbfgs_evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["plain_ms"] if args.plain else r["lbfgs_ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg["dtype"] == "f32" else "f64",
        "data": "synthetic: i.i.d. uniform points, stealthy target",
        "config": {"workload": args.workload, "d": cfg["d"], "N": cfg["N"], "L": cfg["L"],
                   "kmax": cfg["M"], "k_cut": cfg["kcut"], "n_constrained": info["n_constrained"],
                   "tol": cfg["tol"], "nf": info["nf"], "width": info["width"],
                   "tiles": info["nbins"],
                   "step": ("one loss + gradient evaluation" if args.plain else
                            "one L-BFGS iteration (line-search evaluations + update)"),
                   "lbfgs_evals": r.get("lbfgs_evals"), "loss_start": r["loss0"],
                   "loss_end": r.get("lbfgs_loss")},
        "plain_eval": {"evals_per_s": r["plain_evals_per_s"], "ms": r["plain_ms"]},
        "roofline": r["roofline"],
        "cpu_baseline": cpu,
        "stages_ms": r["stages_ms"],
        "stage_gbs": r["stage_gbs"],
        "rocfft": r["rocfft"],
        "copy_gbs": copy_gbs,
        "fp64_context": f64,
        "secondary": sec,
        "batch": bat,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
