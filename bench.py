#!/usr/bin/env python3
"""Throughput of the FReSCo loss + gradient evaluation on one MI355X.

A step is one evaluation of the structure-factor loss and its gradient with
respect to every position (bin, spread, FFTs, mode stage, inverse FFTs,
interpolation, loss reduction), on synthetic uniform random points with the
stealthy target of the headline 2D workload (N = 1e6, L = 1000, 0 < |n| <= 300,
tolerance 1e-6).  Inputs are resident in device memory before timing starts.

Prints one JSON line.  Besides the throughput it carries:
  roofline      achieved algorithmic GB/s of the dominant kernel stage, timed
                with HIP events on the library's stream during the timed steps,
                against the 8 TB/s HBM peak;
  cpu_baseline  the FP64 direct-sum oracle timed on this host's cores on a
                bounded sample (all points, a subset of the modes and of the
                gradient points), scaled to one full evaluation;
  stages_ms     average time of every stage (separate untimed pass);
  secondary     the same measurement for the 3D workload (N = 1e7).
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


def measure(name, steps, warmup, dev):
    import numpy as np
    import torch

    from paper_2305_15693_amd import fresco as F
    from paper_2305_15693_amd import inputs as I

    cfg = I.WORKLOADS[name]
    d, N, L, M = cfg["d"], cfg["N"], cfg["L"], cfg["M"]
    dtype = cfg["dtype"]
    pos_np = I.positions(N, d, L, np.float32 if dtype == "f32" else np.float64, seed=cfg["seed"])
    w, s0 = I.stealthy_target(d, M, cfg["kcut"])
    # a dedicated stream: evaluations on it are replayed from a captured HIP graph
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
    nprof = 5
    for _ in range(nprof):
        ctx.loss_grad_async(pos, loss_dev, grad)
    prof = ctx.read_timing(reset=True)
    ctx.set_timing([])
    stages_ms = {k: v[0] / v[1] for k, v in prof.items()}
    sbytes = stage_bytes(cfg, info, 4 if dtype == "f32" else 8)
    # the roofline names one kernel: stages that are a single kernel launch
    single = [k for k in stages_ms if k in F.SINGLE_KERNEL_STAGES]
    dominant = max(single, key=lambda k: stages_ms[k])

    # timed region: graph replays of the whole evaluation
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
    ms_total = e0.elapsed_time(e1)
    loss = float(loss_dev.item())

    # the dominant kernel, event-timed on the library's stream over as many steps
    ctx.set_timing([dominant])
    for _ in range(steps):
        ctx.loss_grad_async(pos, loss_dev, grad)
    dom = ctx.read_timing(reset=True)[dominant]
    ctx.set_timing([])
    dom_ms = dom[0] / dom[1]
    achieved = sbytes[dominant] / (dom_ms * 1e-3) / 1e9
    res = dict(
        workload=name, cfg=cfg, info=info, ms_per_step=ms_total / steps,
        evals_per_s=steps / (ms_total * 1e-3), loss=loss, stages_ms=stages_ms,
        stage_gbs={k: sbytes[k] / (stages_ms[k] * 1e-3) / 1e9 for k in stages_ms if k in sbytes},
        roofline={"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                  "algorithmic_bytes": sbytes[dominant], "avg_ms": dom_ms},
        pos_np=pos_np, w=w, s0=s0)
    ctx.close()
    del pos, grad
    torch.cuda.empty_cache()
    return res


def cpu_baseline(res, budget_modes=256, grad_points=1024):
    """Oracle timed on a bounded sample of the same evaluation, scaled to one
    full evaluation (rho over all constrained modes for all points, then the
    gradient of every point over all modes)."""
    import numpy as np

    from oracle import oracle as O

    cfg = res["cfg"]
    d, N, L, M = cfg["d"], cfg["N"], cfg["L"], cfg["M"]
    modes, W, S0 = O.constrained_set(d, M, res["w"], res["s0"])
    K = len(modes)
    rng = np.random.default_rng(0)
    pick = rng.choice(K, min(budget_modes, K), replace=False)
    ms, Ws, S0s = modes[pick], W[pick], S0[pick]
    pos = res["pos_np"]
    t0 = time.perf_counter()
    O.loss_grad(pos, L, ms, Ws, S0s, want_grad=False)
    t_rho = time.perf_counter() - t0
    gp = rng.choice(N, grad_points, replace=False)
    t0 = time.perf_counter()
    O.loss_grad(pos, L, ms, Ws, S0s, grad_points=gp)
    t_both = time.perf_counter() - t0
    t_grad = max(t_both - t_rho, 0.0)
    full = t_rho * (K / len(pick)) + t_grad * (N / grad_points) * (K / len(pick))
    return {"value": 1.0 / full, "unit": "evals/s", "cores": O.threads(), "kind": "oracle",
            "sample": (f"all {N} points x {len(pick)} of {K} constrained modes for rho "
                       f"({t_rho:.2f} s), gradient of {grad_points} points over the same modes "
                       f"({t_grad:.2f} s); scaled linearly to the full evaluation "
                       f"({full:.1f} s)")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="2d_n1e6_stealthy300_f32")
    ap.add_argument("--secondary", default="3d_n1e7_stealthy60_f32",
                    help="second workload measured the same way ('' to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    main_res = measure(args.workload, args.steps, args.warmup, dev)
    print(f"[bench] {args.workload}: {main_res['evals_per_s']:.1f} evals/s", file=sys.stderr, flush=True)
    sec = None
    if args.secondary:
        s = measure(args.secondary, max(5, args.steps // 5), max(2, args.warmup // 2), dev)
        print(f"[bench] {args.secondary}: {s['evals_per_s']:.1f} evals/s", file=sys.stderr, flush=True)
        sec = {"workload": s["workload"], "evals_per_s": s["evals_per_s"],
               "ms_per_step": s["ms_per_step"], "roofline": s["roofline"],
               "stages_ms": s["stages_ms"], "stage_gbs": s["stage_gbs"], "loss": s["loss"],
               "nf": s["info"]["nf"], "width": s["info"]["width"]}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(main_res)
        print(f"[bench] cpu baseline: {cpu['value']:.3g} evals/s", file=sys.stderr, flush=True)
    cfg = main_res["cfg"]
    info = main_res["info"]
    out = {
        "metric": METRIC,
        "value": main_res["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg["dtype"] == "f32" else "f64",
        "data": "synthetic: i.i.d. uniform points, stealthy target",
        "config": {"workload": args.workload, "d": cfg["d"], "N": cfg["N"], "L": cfg["L"],
                   "kmax": cfg["M"], "k_cut": cfg["kcut"], "n_constrained": info["n_constrained"],
                   "tol": cfg["tol"], "nf": info["nf"], "width": info["width"],
                   "step": "one loss + gradient evaluation"},
        "roofline": main_res["roofline"],
        "cpu_baseline": cpu,
        "stages_ms": main_res["stages_ms"],
        "stage_gbs": main_res["stage_gbs"],
        "loss": main_res["loss"],
        "secondary": sec,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
