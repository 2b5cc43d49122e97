"""Benchmark: restored Mpixel/s of the EECMG cascade on one MI355X.

Workload (default): one 4096 x 4096 FP32 image (2000 shapes + 200 texture
patches), out-of-focus disk PSF of radius 6, N(0,1) noise, 9 levels
16 -> 4096, the paper's economic iteration counts as caps and the
discrepancy stopping rule (c = 1.1).  A step is one complete restore
(restriction, every level's smoother and transfer) of a device-resident
input into a device-resident output.

Prints one JSON line.  Besides the throughput (`value`, the plain form) it
reports
  batched:       the same image restored as a batch of copies in one
                 batched cascade;
  uneven_set:    256 images with sides log-uniform in [128, 2048] and a mix
                 of Gaussian and disk PSFs, restored one call per image
                 (plain) and as one batched cascade, with the bitwise
                 agreement of the two;
  edge:          the edge-preservation workload (edge-dense 1024^2 scene,
                 Gaussian sigma=3, half bandwidth 11) with EECMG(MR) and
                 EECMG(CG): throughput, PSNR and edge recovery of input and
                 results;
  served:        requests (sides log-uniform in [64, 4096]) through the
                 create/submit/poll loop: closed-loop capacity, then Poisson
                 arrivals at 0.7 of it, with p50/p99 latency from arrival to
                 the poll that returns the result;
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


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Measured HBM bandwidth of a plain device copy (bytes read + written per
    second), the practical ceiling the roofline fraction is also quoted against."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


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


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def edge_leg(torch, eecmg, synth, steps, H=1024, n_levels=7):
    """Edge-preservation workload: edge-dense scene, Gaussian sigma=3 with
    half bandwidth 11, N(0,1) noise, restored with EECMG(MR) (the paper's
    edge experiment) and EECMG(CG); throughput and the quality measures of
    input and results."""
    from paper_2311_03010_amd import metrics

    p = synth.edge_workload(H=H, n_levels=n_levels)
    g = torch.from_numpy(p.g_delta.astype(np.float32)).to("cuda:0")
    out = {"workload": f"{p.name}: edge-dense scene, Gaussian sigma=3 half bandwidth 11, N(0,1) noise, "
                       f"{n_levels} levels, FP32",
           "input": {"psnr": round(metrics.psnr(p.u_true, p.g_delta), 3),
                     "edge_recall": round(metrics.edge_recall(p.u_true, p.g_delta), 4),
                     "edge_error": round(metrics.edge_error(p.u_true, p.g_delta), 4)}}
    for sm in ("mr", "cgls"):
        kw = dict(precision="f32", delta=p.delta, k=p.k, smoother=sm)
        u, st = eecmg.restore_dev(g, p.psf, n_levels, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            eecmg.restore_dev(g, p.psf, n_levels, out=u, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        uh = u.cpu().numpy()
        out["eecmg_" + sm] = {"value": round(H * H / dt / 1e6, 3), "unit": "Mpixel/s", "ms_per_step": round(dt * 1e3, 3),
                              "iters_per_level": st["iters"], "psnr": round(metrics.psnr(p.u_true, uh), 3),
                              "edge_recall": round(metrics.edge_recall(p.u_true, uh), 4),
                              "edge_error": round(metrics.edge_error(p.u_true, uh), 4)}
    return out


def set_leg(torch, eecmg, synth, n_images, steps, form="both"):
    """The uneven batch: n_images images with sides log-uniform in
    [128, 2048] and a mix of Gaussian and disk PSFs, each restored with its
    own level count.  Plain = one restore call per image in turn; batched =
    one batched cascade for the whole set.  Both read device-resident inputs
    and write device-resident outputs; their results must agree bit for bit."""
    probs = synth.batch_problems(n_images)
    gs = [torch.from_numpy(q.g_delta.astype(np.float32)).to("cuda:0") for q in probs]
    px = sum(q.g_delta.size for q in probs)
    po = [torch.empty_like(g) for g in gs]
    bo = [torch.empty_like(g) for g in gs]
    psfs = [q.psf for q in probs]
    Ls = [q.n_levels for q in probs]
    ks = [q.k for q in probs]
    prm = [{"delta": q.delta} for q in probs]

    def plain():
        for q, g, o in zip(probs, gs, po):
            eecmg.restore_dev(g, q.psf, q.n_levels, out=o, precision="f32", delta=q.delta, k=q.k)

    def batched():
        eecmg.restore_batch_dev(gs, psfs, Ls, ks=ks, outs=bo, precision="f32", params=prm)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tp = timed(plain) if form != "batched" else float("nan")
    tb = timed(batched) if form != "plain" else float("nan")
    equal = form == "both" and all(torch.equal(a, b) for a, b in zip(po, bo))
    return {"workload": f"uneven batch of {n_images} images, sides log-uniform in [128, 2048], "
                        "Gaussian sigma U[1,4] / disk r U{2..6} PSFs, FP32",
            "images": n_images, "mpixels": round(px / 1e6, 3), "steps": steps,
            "plain": {"value": round(px / tp / 1e6, 3), "unit": "Mpixel/s", "ms_per_step": round(tp * 1e3, 3)},
            "batched": {"value": round(px / tb / 1e6, 3), "unit": "Mpixel/s", "ms_per_step": round(tb * 1e3, 3)},
            "speedup_vs_plain": round(tp / tb, 3), "bitwise_equal_to_plain": bool(equal)}


def served_leg(torch, eecmg, synth, n_req, pool_n, load=0.7, check_every=8):
    """Served requests through the create/submit/poll loop.  Request images
    come from a pool of pool_n distinct images with sides log-uniform in
    [64, 4096]; each request is host in, host out (the context stages it
    through pinned memory).  First the closed-loop capacity (the whole pool
    submitted at once), then Poisson arrivals at `load` times that capacity;
    latency runs from a request's scheduled arrival to the poll that returns
    its result.  Every check_every-th served result is compared bit for bit
    with a plain device restore of the same image."""
    import threading

    pool = synth.served_pool(pool_n)
    ins = [np.ascontiguousarray(q.g_delta.astype(np.float32)) for q in pool]
    pxs = [q.g_delta.size for q in pool]
    kw = [dict(precision="f32", delta=q.delta, k=q.k) for q in pool]
    # plain: one host-in / host-out restore call per image in turn
    eecmg.restore(ins[0], pool[0].psf, pool[0].n_levels, **kw[0])
    t0 = time.perf_counter()
    refs = [eecmg.restore(x, q.psf, q.n_levels, **k)[0] for q, x, k in zip(pool, ins, kw)]
    dt_plain = time.perf_counter() - t0
    budget = 24 << 30
    with eecmg.Context(hbm_budget_bytes=budget, max_slots=64, max_queue=n_req + pool_n) as ctx:
        outs = [np.empty_like(x) for x in ins]  # reused, as a server reuses its buffers

        def closed():
            t0 = time.perf_counter()
            rs = [ctx.submit(x, q.psf, q.n_levels, **k) for q, x, k in zip(pool, ins, kw)]
            for r, o in zip(rs, outs):
                ctx.wait(r, out=o)
            return time.perf_counter() - t0, outs

        closed()
        # host-bound and noisy: the median of three passes over the pool
        dt_c = float(np.median([closed()[0] for _ in range(3)]))
        closed_ok = all(np.array_equal(a, b) for a, b in zip(outs, refs))
        cap_qps = pool_n / dt_c
        qps = load * cap_qps
        arr = synth.poisson_arrivals(n_req, qps)
        scratch = [np.empty_like(x) for x in ins]
        done_t = np.zeros(n_req)
        # result buffers of the checked requests, touched before the run
        checked = {i: np.zeros_like(ins[i % pool_n]) for i in range(0, n_req, check_every)}
        pending = []
        lock = threading.Lock()
        finished = threading.Event()
        submitted = [0]

        def poller():
            live = []
            n_done = 0
            while n_done < n_req:
                with lock:
                    live.extend(pending)
                    pending.clear()
                hit = False
                still = []
                for i, req, buf in live:
                    if ctx.poll(req, out=buf) is not None:
                        done_t[i] = time.perf_counter()
                        n_done += 1
                        hit = True
                    else:
                        still.append((i, req, buf))
                live = still
                if not hit:
                    time.sleep(0.0001)
            finished.set()

        th = threading.Thread(target=poller, daemon=True)
        th.start()
        start = time.perf_counter()
        for i in range(n_req):
            wait = start + arr[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            j = i % pool_n
            buf = checked.get(i, scratch[j])
            req = ctx.submit(ins[j], pool[j].psf, pool[j].n_levels, **kw[j])
            with lock:
                pending.append((i, req, buf))
            submitted[0] += 1
        finished.wait()
        th.join()
    lat = (done_t - (start + arr)) * 1e3
    span = done_t.max() - start
    px_total = sum(pxs[i % pool_n] for i in range(n_req))
    served_ok = all(np.array_equal(buf, refs[i % pool_n]) for i, buf in checked.items())
    return {"workload": f"{n_req} requests, Poisson arrivals, image sides log-uniform in [64, 4096] "
                        f"(pool of {pool_n} distinct images), Gaussian/disk PSF mix, FP32, host in / host out",
            "requests": n_req, "pool_images": pool_n, "hbm_budget_bytes": budget, "max_slots": 64,
            "closed_loop_capacity": {"value": round(sum(pxs) / dt_c / 1e6, 3), "unit": "Mpixel/s",
                                     "requests_per_s": round(cap_qps, 2)},
            "offered_qps": round(qps, 2), "load_vs_capacity": load,
            "value": round(px_total / span / 1e6, 3), "unit": "Mpixel/s",
            "latency_ms": {"p50": round(_pct(lat, 50), 3), "p99": round(_pct(lat, 99), 3),
                           "mean": round(float(lat.mean()), 3), "max": round(float(lat.max()), 3)},
            "plain": {"value": round(sum(pxs) / dt_plain / 1e6, 3), "unit": "Mpixel/s",
                      "form": "one eecmg_restore call (host in / host out) per pool image in turn"},
            "closed_loop_speedup_vs_plain": round(dt_plain / dt_c, 3),
            "bitwise_equal_to_plain": bool(closed_ok and served_ok), "checked": len(checked) + pool_n}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", type=int, default=3, choices=[1, 2, 3])
    ap.add_argument("--batch", type=int, default=4, help="images in the batched leg (0 = skip)")
    ap.add_argument("--set-images", type=int, default=256,
                    help="images in the uneven plain-vs-batched set (0 = skip)")
    ap.add_argument("--set-steps", type=int, default=2)
    ap.add_argument("--set-form", default="both", choices=["both", "plain", "batched"],
                    help="which forms of the uneven set to run (profiling one form)")
    ap.add_argument("--served-requests", type=int, default=2000, help="served requests (0 = skip)")
    ap.add_argument("--served-pool", type=int, default=64)
    ap.add_argument("--no-edge", action="store_true", help="skip the edge-preservation workload")
    ap.add_argument("--copy-probe", action="store_true", help="only run the HBM counter calibration copy")
    ap.add_argument("--only-set", action="store_true", help="only run the uneven set (for profiling it)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.only_set:
        import torch

        from paper_2311_03010_amd import eecmg, synth

        print(json.dumps(set_leg(torch, eecmg, synth, args.set_images, args.set_steps, args.set_form)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is designed but not implemented", file=sys.stderr)
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

    # finest-level launches only (the job's level holds all H x W pixels)
    eecmg.profile_reset()
    eecmg.profile_enable(True, min_pixels=H * W)
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
    # pass B (read r, u; write r, u, s).  The two passes actually move 16 and,
    # on average, 26 bytes: q is stored by A and read by B; B reads p again;
    # on levels of >= 1024^2 pixels B updates u every second iteration
    # (alternately 20 bytes without u and p, 32 with u and two directions).
    # FP32 levels with a streaming blur kernel run the pass B that recomputes
    # q = H p (pass A then stores no q): pass A moves 12 bytes, pass B 16 and
    # 28 alternately (22 on average: it reads p for q instead of q).
    try:
        dconv = eecmg.profile_read("cg_pass_b_dconv")[0] > 0
    except eecmg.EecmgError:  # a library without that stage
        dconv = False
    kern = {}
    for name, src, bpp, moved in (("cg_pass_a", "cg_pass_a", 12, 12 if dconv else 16),
                                  ("cg_pass_b", "cg_pass_b_dconv" if dconv else "cg_pass_b", 20, 22 if dconv else 26)):
        n, ms, px = eecmg.profile_read(src)
        if n:
            avg_ms = ms / n
            px_launch = px / n
            kern[name] = {"launches": n, "avg_us": avg_ms * 1e3, "alg_bytes_per_px": bpp,
                          "kernel": src, "gbs": bpp * px_launch / (avg_ms * 1e-3) / 1e9, "moved_bytes_per_px": moved,
                          "moved_gbs": moved * px_launch / (avg_ms * 1e-3) / 1e9}
    for name in ("cg_init_r", "cg_init_s", "transfer_fused"):
        n, ms, px = eecmg.profile_read(name)
        if n:
            kern[name] = {"launches": n, "avg_us": ms / n * 1e3}
    rb = kern.get("cg_pass_b")
    roofline = None
    if rb:
        ach = rb["gbs"]
        cbw = copy_bandwidth(torch)
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                    "copy_gbs": round(cbw, 1), "frac_vs_copy": round(ach / cbw, 4),
                    "kernel": ("k_cg_bd<float, ConvBox<float, 6>>" if dconv else "k_cg_b<float, ConvBox<float, 6, true>>")
                    + " (finest level, 4096^2" + ("" if dconv else ", tall strips") + ")",
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

    uneven = None
    if args.set_images > 0:
        _log(f"bench: uneven set, {args.set_images} images, plain vs batched")
        uneven = set_leg(torch, eecmg, synth, args.set_images, args.set_steps, args.set_form)

    edge = None
    if not args.no_edge:
        _log("bench: edge-preservation workload")
        edge = edge_leg(torch, eecmg, synth, args.steps)

    served = None
    if args.served_requests > 0:
        _log(f"bench: served, {args.served_requests} requests")
        served = served_leg(torch, eecmg, synth, args.served_requests, args.served_pool)

    cpu = None
    if not args.no_cpu_baseline:
        _log("bench: cpu baseline (oracle sample)")
        cpu = cpu_baseline(p, stats)

    metric = ("restored Mpixel/s plain vs batched at 4096\u00b2; p50/p99 latency; % HBM roofline"
              if args.workload == 3 else "restored Mpixel/s")
    line = {"metric": metric,
            "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if prec != "f64" else "f64", "data": "synthetic",
            "config": {"workload": p.name, "H": H, "W": W, "psf": "disk r=6" if args.workload == 3 else "gaussian",
                       "n_levels": p.n_levels, "precision": prec, "stop_rule": "discrepancy c=1.1",
                       "caps": "economic m_l rule", "form": "plain"},
            "roofline": roofline, "cpu_baseline": cpu, "batched": batched, "uneven_set": uneven,
            "served": served, "edge": edge, "detail": extra}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
