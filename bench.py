"""Benchmark: restored Mpixel/s of the EECMG cascade on one MI355X.

Workload (default): one 4096 x 4096 FP32 image (2000 shapes + 200 texture
patches), out-of-focus disk PSF of radius 6, N(0,1) noise, 9 levels
16 -> 4096, the paper's economic iteration counts as caps and the
discrepancy stopping rule (c = 1.1).  A step is one complete restore
(restriction, every level's smoother and transfer) of a device-resident
input into a device-resident output.

Prints one JSON line.  Besides the throughput it reports
  roofline:      the finest-level CGLS pass B kernel (dominant), algorithmic
                 HBM bytes per launch / its mean duration from HIP events on
                 the library's launch stream during the timed region;
  cpu_baseline:  the FP64 CPU oracle on a bounded sample of the same
                 workload (every level's initialisation, one iteration and
                 transfer timed at full size, scaled by the iteration counts
                 of the run).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VALU_PEAK_TFLOPS = 78.6   # non-packed FP32 FMA: 256 CU x 64 lanes x 2 flop x 2.4 GHz


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(p, stats):
    """Oracle (FP64, all host cores via OpenMP) timed on a bounded sample."""
    import oracle

    L = p.n_levels
    sizes = oracle.level_sizes(p.shape[0], p.shape[1], L)
    psfs = [None] * L
    psfs[L - 1] = p.psf
    for l in range(L - 2, -1, -1):
        psfs[l] = oracle.coarse_psf(psfs[l + 1], 0)
    gs = [None] * L
    gs[L - 1] = p.g_delta
    for l in range(L - 2, -1, -1):
        gs[l] = oracle.restrict(gs[l + 1], *sizes[l])
    total = 0.0
    rng = np.random.Generator(np.random.PCG64(1))
    for l in range(L):
        t0 = time.perf_counter()
        oracle.cgls(gs[l], psfs[l], cap=0)
        t_init = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.cgls(gs[l], psfs[l], cap=1, eps=0.0)
        t_one = time.perf_counter() - t0
        t_iter = max(t_one - t_init, 0.0)
        t_x = 0.0
        if l >= 2:
            (ha, wa), (hb, wb), (hc, wc) = sizes[l - 2], sizes[l - 1], sizes[l]
            uA = rng.uniform(0, 255, (ha, wa))
            uB = rng.uniform(0, 255, (hb, wb))
            t0 = time.perf_counter()
            ut = oracle.extrapolate(uA, uB)
            uc = oracle.prolong_quad(ut, hc, wc)
            us = oracle.local_smooth(uc)
            oracle.pm_step(us)
            t_x = time.perf_counter() - t0
        total += t_init + stats["iters"][l] * t_iter + t_x
    mpx = p.shape[0] * p.shape[1] / total / 1e6
    return {"value": mpx, "unit": "Mpixel/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "every level's CGLS init + one iteration + transfer at full 4096^2 size, scaled by the run's "
                      f"per-level iteration counts {stats['iters']}; estimated full restore {total:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", type=int, default=3, choices=[1, 2, 3])
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2311_03010_amd import eecmg, synth

    _log(f"bench: generating workload {args.workload}")
    p = synth.workload(args.workload)
    prec = p.precision
    H, W = p.shape
    g = torch.from_numpy(p.g_delta.astype(np.float64 if prec == "f64" else np.float32)).to("cuda:0")
    out = torch.empty_like(g)
    kw = dict(precision=prec, delta=p.delta, k=p.k)

    _log("bench: warmup")
    for _ in range(args.warmup):
        eecmg.restore_dev(g, p.psf, p.n_levels, out=out, **kw)
    torch.cuda.synchronize()

    fine_tiles = ((W + 63) // 64) * ((H + 31) // 32)
    eecmg.profile_reset()
    eecmg.profile_enable(True, min_blocks=fine_tiles)
    _log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        _, stats = eecmg.restore_dev(g, p.psf, p.n_levels, out=out, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eecmg.profile_enable(False)
    ms_step = dt / args.steps * 1e3
    value = H * W * args.steps / dt / 1e6

    # dominant kernel: finest-level CGLS pass B (r -= alpha q, s = H^T r, u += alpha p)
    # algorithmic HBM bytes per pixel: read r, u, write r, u, s = 5 x 4 B
    kern = {}
    for name, bpp in (("cg_pass_a", 12), ("cg_pass_b", 20)):
        n, ms, px = eecmg.profile_read(name)
        if n:
            avg_ms = ms / n
            px_launch = px / n
            kern[name] = {"launches": n, "avg_us": avg_ms * 1e3, "alg_bytes_per_px": bpp,
                          "gbs": bpp * px_launch / (avg_ms * 1e-3) / 1e9}
    rb = kern.get("cg_pass_b")
    roofline = None
    if rb:
        ach = rb["gbs"]
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_cg_b<float,6> (finest level)",
                    "avg_launch_us": round(rb["avg_us"], 2)}
    extra = {"kernels": kern, "iters_per_level": stats["iters"], "stop_reason": stats["reason"]}

    cpu = None
    if not args.no_cpu_baseline:
        _log("bench: cpu baseline (oracle sample)")
        cpu = cpu_baseline(p, stats)

    line = {"metric": "restored Mpixel/s (plain EECMG, 4096^2)" if args.workload == 3 else "restored Mpixel/s",
            "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if prec != "f64" else "f64", "data": "synthetic",
            "config": {"workload": p.name, "H": H, "W": W, "psf": "disk r=6" if args.workload == 3 else "gaussian",
                       "n_levels": p.n_levels, "precision": prec, "stop_rule": "discrepancy c=1.1",
                       "caps": "economic m_l rule", "form": "plain"},
            "roofline": roofline, "cpu_baseline": cpu, "detail": extra}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
