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
                 the library's launch stream during the timed region (launches
                 that found their level already stopped are excluded);
  cpu_baseline:  the FP64 CPU oracle timed on one complete restore of the
                 same input on the host's cores.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cg_pass_b_disk6_4096.json")
KERNEL_SOURCES = ["paper_2311_03010_amd/csrc/eecmg_device.h", "paper_2311_03010_amd/csrc/eecmg_sm_box.hip",
                  "paper_2311_03010_amd/csrc/eecmg_internal.h"]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (scaled by the copy-kernel calibration), or
    None when the kernel sources changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def copy_probe():
    """A plain device copy of known size, for calibrating the HBM counters."""
    import torch

    n = 256 << 20  # floats: 1 GiB per buffer
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 5}))


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(p, stats):
    """The FP64 CPU oracle (OpenMP over the pixel loops of its stencils) timed
    on one complete restore of the same input, same parameters."""
    import oracle

    g = p.g_delta.astype(np.float32).astype(np.float64) if p.precision != "f64" else p.g_delta
    t0 = time.perf_counter()
    _, st = oracle.restore(g, p.psf, p.n_levels, delta=p.delta, k=p.k,
                           guard_eps=1e-6 if p.precision != "f64" else 1e-14)
    dt = time.perf_counter() - t0
    return {"value": round(p.shape[0] * p.shape[1] / dt / 1e6, 4), "unit": "Mpixel/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one complete restore of the same {p.shape[0]}x{p.shape[1]} input ({dt:.1f} s); "
                      f"oracle iterations per level {st['iters']} (GPU {stats['iters']})"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", type=int, default=3, choices=[1, 2, 3])
    ap.add_argument("--batch", type=int, default=4, help="images in the batched leg (0 = skip)")
    ap.add_argument("--copy-probe", action="store_true", help="only run the HBM counter calibration copy")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
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

    # finest-level launches only: every tile is at most 64 rows tall, and the
    # next level has a quarter of the pixels
    fine_tiles = ((W + 63) // 64) * ((H + 63) // 64)
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

    # dominant kernel: finest-level CGLS pass B (r -= alpha q, s = H^T r, u += alpha p).
    # Algorithmic HBM bytes per pixel and iteration are 32 (u, r, p, s each
    # read and written once): 12 in pass A (read s, p; write p) and 20 in
    # pass B (read r, u; write r, u, s).  The two passes actually move 16 and
    # 28 (q is stored by A and read by B, p is read again by B).
    kern = {}
    for name, bpp, moved in (("cg_pass_a", 12, 16), ("cg_pass_b", 20, 28)):
        n, ms, px = eecmg.profile_read(name)
        if n:
            avg_ms = ms / n
            px_launch = px / n
            kern[name] = {"launches": n, "avg_us": avg_ms * 1e3, "alg_bytes_per_px": bpp,
                          "gbs": bpp * px_launch / (avg_ms * 1e-3) / 1e9, "moved_bytes_per_px": moved,
                          "moved_gbs": moved * px_launch / (avg_ms * 1e-3) / 1e9}
    for name in ("cg_init_r", "cg_init_s", "transfer_fused"):
        n, ms, px = eecmg.profile_read(name)
        if n:
            kern[name] = {"launches": n, "avg_us": ms / n * 1e3}
    rb = kern.get("cg_pass_b")
    roofline = None
    if rb:
        ach = rb["gbs"]
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                    "kernel": "k_cg_b<float, ConvBox<float, 6>> (finest level, 4096^2)",
                    "avg_launch_us": round(rb["avg_us"], 2), "alg_bytes_per_launch": int(20 * H * W)}
    extra = {"kernels": kern, "iters_per_level": stats["iters"], "stop_reason": stats["reason"]}

    batched = None
    if args.batch > 0:
        # copies of the same input (identical work per image), all images in
        # one batched cascade: every stage is one launch for all of them
        _log(f"bench: batched leg, {args.batch} images")
        gs = [g.clone() for _ in range(args.batch)]
        outs = [torch.empty_like(x) for x in gs]
        bkw = dict(precision=prec, params=[{"delta": p.delta}] * len(gs))
        for _ in range(max(1, args.warmup)):
            eecmg.restore_batch_dev(gs, [p.psf] * len(gs), [p.n_levels] * len(gs), outs=outs, **bkw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            eecmg.restore_batch_dev(gs, [p.psf] * len(gs), [p.n_levels] * len(gs), outs=outs, **bkw)
        torch.cuda.synchronize()
        bdt = time.perf_counter() - t0
        batched = {"images": len(gs), "value": round(len(gs) * H * W * args.steps / bdt / 1e6, 3),
                   "unit": "Mpixel/s", "ms_per_step": round(bdt / args.steps * 1e3, 3),
                   "speedup_vs_plain": round(len(gs) * H * W * args.steps / bdt / 1e6 / value, 3)}

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
            "roofline": roofline, "cpu_baseline": cpu, "batched": batched, "detail": extra}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
