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
                 the library's launch stream, over a timed region of its own
                 (launches that found their level already stopped are
                 excluded); roofline.cascade: the whole restore's algorithmic
                 bytes / ms_per_step, and per level the algorithmic bytes /
                 the summed kernel time of that level (HIP events around every
                 launch, in one more timed region);
  workloads:     the 64^2 FP64 and 1024^2 FP32 workloads: throughput and the
                 error against the FP64 oracle;
  one_level:     the 1024^2 workload restored by the one-level smoother with
                 the stopping rule (CGLS and MR) next to the cascade: PSNR and
                 time;
  cpu_baseline:  the FP64 CPU oracle timed on one complete restore of the
                 same input on all of the host's cores; cpu_oracle: the oracle
                 on one core and on all cores for the three single-image
                 workloads, with the host's CPU model and core count.
`value` comes from a timed region with kernel timing off; the profiled
regions come after it.
"""
from __future__ import annotations

import argparse
import gc
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


def host_cpu():
    """CPU model and core counts of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable": usable}


def oracle_restore(p, threads=None):
    """One complete FP64 oracle restore of the workload's input (rounded to
    the GPU run's storage precision first), same parameters; (u, stats, s)."""
    import oracle

    if threads is not None:
        oracle.set_num_threads(threads)
    g = p.g_delta.astype(np.float32).astype(np.float64) if p.precision != "f64" else p.g_delta
    t0 = time.perf_counter()
    u, st = oracle.restore(g, p.psf, p.n_levels, delta=p.delta, k=p.k,
                           guard_eps=1e-6 if p.precision != "f64" else 1e-14)
    return u, st, time.perf_counter() - t0


def accuracy(p, u_gpu, u_ref, st_gpu, st_ref):
    import oracle

    u = np.asarray(u_gpu, np.float64)
    return {"rel_l2_vs_oracle": float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)),
            "dpsnr_db": round(abs(oracle.psnr(p.u_true, u) - oracle.psnr(p.u_true, u_ref)), 6),
            "psnr_db": round(oracle.psnr(p.u_true, u), 4), "iters_equal": st_gpu["iters"] == st_ref["iters"]}


def cpu_baseline(p, stats, u_gpu):
    """The FP64 CPU oracle (OpenMP over the pixel loops of its stencils) timed
    on one complete restore of the same input on all host cores."""
    import oracle

    oracle.set_num_threads(host_cpu()["usable"])
    u, st, dt = oracle_restore(p)
    acc = accuracy(p, u_gpu, u, stats, st)
    return {"value": round(p.shape[0] * p.shape[1] / dt / 1e6, 4), "unit": "Mpixel/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one complete restore of the same {p.shape[0]}x{p.shape[1]} input ({dt:.1f} s); "
                      f"oracle iterations per level {st['iters']} (GPU {stats['iters']})"}, acc


def cpu_oracle_table(synth, ids, one_core):
    """The oracle on one core and on all usable cores, per workload (full
    restores; one run each)."""
    import oracle

    cpu = host_cpu()
    out = {"host": cpu, "workloads": {}}
    for wid in ids:
        p = synth.workload(wid)
        row = {}
        for label, th in (("all_cores", cpu["usable"]), ("one_core", 1)):
            if label == "one_core" and not one_core:
                continue
            _, _, dt = oracle_restore(p, threads=th)
            row[label] = {"threads": th, "seconds": round(dt, 3),
                          "mpixel_s": round(p.shape[0] * p.shape[1] / dt / 1e6, 4)}
        out["workloads"][p.name] = row
    oracle.set_num_threads(cpu["usable"])
    return out


# Algorithmic HBM bytes per pixel (FP32; FP64 doubles them): a CGLS iteration
# reads and writes u, r, p, s once (32); its start r = g - H u0, s = H^T r
# reads g, u0, r and writes r, s (20); an MR iteration reads r, q, u and
# writes them (24), its start 12; the transfer into a level reads the two
# coarser solutions and writes the extrapolated one (Pi: 2.25 per fine
# pixel), then reads that and writes the level's start (prolongation, S, D:
# 5); the restriction reads the even rows of the input (2) and writes every
# coarser right-hand side.
def level_bytes(sizes, iters, esz, smoother="cgls", cascade="eecmg"):
    f = esz / 4.0
    it_b, init_b = (32.0, 20.0) if smoother == "cgls" else (24.0, 12.0)
    out = []
    for l, ((h, w), k) in enumerate(zip(sizes, iters)):
        px = h * w
        b = (it_b * k + init_b) * px
        if (cascade == "eecmg" and l >= 2) or (cascade != "eecmg" and l >= 1):
            b += (7.25 if cascade == "eecmg" else 5.0) * px
        out.append(b * f)
    fine = sizes[-1][0] * sizes[-1][1]
    restrict_b = (2.0 * fine + 4.0 * sum(h * w for h, w in sizes[:-1])) * f
    return out, restrict_b


def cascade_roofline(eecmg, restore_once, p, stats, steps, ms_step, copy_gbs):
    """Per-level and whole-restore fractions of the HBM roofline."""
    sizes = [tuple(s) for s in stats["sizes"]]
    esz = 8 if p.precision == "f64" else 4
    lb, rb = level_bytes(sizes, stats["iters"], esz)
    coarse = 0  # the levels the library's one-block cascade solves (EECMG_COARSE_MAX_PIXELS)
    coarse_px = int(os.environ.get("EECMG_COARSE_MAX_PIXELS", 64 * 64))
    while coarse < len(sizes) and sizes[coarse][0] * sizes[coarse][1] <= coarse_px:
        coarse += 1
    eecmg.profile_reset()
    eecmg.profile_enable(True, min_pixels=0)
    for _ in range(steps):
        restore_once()
    eecmg.profile_enable(False)
    rows = []
    kern_ms = 0.0
    other = {}
    for st in ("restrict", "out_copy"):
        n, ms, _ = eecmg.profile_read(st)
        other[st] = (n, ms / steps)
        kern_ms += ms / steps
    for l in range(len(sizes)):
        if 0 < l < coarse:
            continue
        lv = list(range(coarse)) if (l == 0 and coarse > 0) else [l]
        if l == 0 and coarse > 0:
            # the coarse levels are solved inside the restriction launch
            n, ms = other["restrict"]
            b = sum(lb[i] for i in lv) + rb
            name = "restriction + "
        else:
            n, ms = eecmg.profile_read_level(l)
            ms /= steps
            kern_ms += ms
            b = sum(lb[i] for i in lv)
            name = ""
        ws = 6 * sizes[l][0] * sizes[l][1] * esz
        rows.append({"levels": name + f"{sizes[lv[0]][0]}x{sizes[lv[0]][1]}" +
                     (f"..{sizes[lv[-1]][0]}x{sizes[lv[-1]][1]}" if len(lv) > 1 else ""),
                     "iters": [stats["iters"][i] for i in lv], "launches_per_step": round(n / steps, 1),
                     "alg_mb": round(b / 1e6, 3), "us": round(ms * 1e3, 1),
                     "achieved_gbs": round(b / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                     "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else None,
                     "fits_mall": ws <= (256 << 20)})
    other = {k: round(v[1] * 1e3, 1) for k, v in other.items()}
    total_b = sum(lb) + rb
    ach = total_b / (ms_step * 1e-3) / 1e9
    return {"alg_bytes_per_step": int(total_b), "ms_per_step": round(ms_step, 4), "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "frac_vs_copy": round(ach / copy_gbs, 4) if copy_gbs else None,
            "kernel_ms_per_step": round(kern_ms, 4), "gap_ms_per_step": round(ms_step - kern_ms, 4),
            "restrict_us": other["restrict"], "out_copy_us": other["out_copy"], "per_level": rows,
            "restrict_note": "the restriction launch also solves the coarse levels (first per-level row)"
            if coarse > 0 else None,
            "bytes": "CGLS 32 B/px per iteration + 20 at its start; transfer 7.25 per fine px (Pi 2.25, "
                     "prolongation+S+D 5); restriction 2 per fine px + the coarser right-hand sides (FP32)"}


def plain_leg(torch, eecmg, synth, wid, steps, warmup, with_oracle=True):
    """Throughput of one workload restored plain, and its error against the
    oracle (same input rounded to the storage precision)."""
    p = synth.workload(wid)
    prec = p.precision
    g = torch.from_numpy(p.g_delta.astype(np.float64 if prec == "f64" else np.float32)).to("cuda:0")
    out = torch.empty_like(g)
    kw = dict(precision=prec, delta=p.delta, k=p.k)
    for _ in range(warmup):
        eecmg.restore_dev(g, p.psf, p.n_levels, out=out, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = eecmg.restore_dev(g, p.psf, p.n_levels, out=out, **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    res = {"workload": p.name, "H": p.shape[0], "W": p.shape[1], "precision": prec, "n_levels": p.n_levels,
           "value": round(p.shape[0] * p.shape[1] / dt / 1e6, 3), "unit": "Mpixel/s", "ms_per_step": round(dt * 1e3, 4),
           "iters_per_level": st["iters"]}
    if with_oracle:
        u_ref, st_ref, _ = oracle_restore(p)
        res["accuracy"] = accuracy(p, out.cpu().numpy(), u_ref, st, st_ref)
    return res


def one_level_leg(torch, eecmg, synth, steps):
    """The 1024^2 workload (Gaussian sigma=3) restored by the one-level
    smoother with the discrepancy stopping rule (the one-level baseline of the
    paper's Table 1, here with the stopping rule instead of 4 fixed
    iterations) next to the 7-level cascade: PSNR and time, CGLS and MR."""
    import oracle

    p = synth.workload(2)
    g = torch.from_numpy(p.g_delta.astype(np.float32)).to("cuda:0")
    out = torch.empty_like(g)
    res = {"workload": f"{p.name}, FP32, discrepancy stopping rule c=1.1",
           "input_psnr": round(oracle.psnr(p.u_true, p.g_delta), 4)}
    for sm in ("cgls", "mr"):
        for name, L, caps in (("one_level", 1, [1000]), ("cascade", p.n_levels, None)):
            kw = dict(precision="f32", delta=p.delta, k=p.k, smoother=sm)
            eecmg.restore_dev(g, p.psf, L, caps=caps, out=out, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, st = eecmg.restore_dev(g, p.psf, L, caps=caps, out=out, **kw)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res[f"{name}_{sm}"] = {"ms": round(dt * 1e3, 4), "iters_per_level": st["iters"],
                                   "psnr": round(oracle.psnr(p.u_true, out.cpu().numpy().astype(np.float64)), 4)}
    return res


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
        # every step timed on its own, the interpreter's cyclic garbage
        # collector paused meanwhile (a collection over the many image objects
        # takes tens of ms); the median step is reported
        fn()
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        ts = []
        try:
            for _ in range(steps):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
        finally:
            gc.enable()
        return float(np.median(ts)), [round(t * 1e3, 3) for t in ts]

    tp, tps = timed(plain) if form != "batched" else (float("nan"), [])
    tb, tbs = timed(batched) if form != "plain" else (float("nan"), [])
    equal = form == "both" and all(torch.equal(a, b) for a, b in zip(po, bo))
    return {"workload": f"uneven batch of {n_images} images, sides log-uniform in [128, 2048], "
                        "Gaussian sigma U[1,4] / disk r U{2..6} PSFs, FP32",
            "images": n_images, "mpixels": round(px / 1e6, 3), "steps": steps,
            "plain": {"value": round(px / tp / 1e6, 3), "unit": "Mpixel/s", "ms_per_step": round(tp * 1e3, 3),
                      "ms_each": tps},
            "batched": {"value": round(px / tb / 1e6, 3), "unit": "Mpixel/s", "ms_per_step": round(tb * 1e3, 3),
                        "ms_each": tbs},
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
    ap.add_argument("--no-oracle-table", action="store_true",
                    help="skip the one-core / all-core oracle timings of the three workloads")
    ap.add_argument("--workload", type=int, default=3, choices=[1, 2, 3])
    ap.add_argument("--batch", type=int, default=4, help="images in the batched leg (0 = skip)")
    ap.add_argument("--set-images", type=int, default=256,
                    help="images in the uneven plain-vs-batched set (0 = skip)")
    ap.add_argument("--set-steps", type=int, default=5)
    ap.add_argument("--set-form", default="both", choices=["both", "plain", "batched"],
                    help="which forms of the uneven set to run (profiling one form)")
    ap.add_argument("--served-requests", type=int, default=2000, help="served requests (0 = skip)")
    ap.add_argument("--served-pool", type=int, default=64)
    ap.add_argument("--no-edge", action="store_true", help="skip the edge-preservation workload")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads and the one-level leg")
    ap.add_argument("--copy-probe", action="store_true", help="only run the HBM counter calibration copy")
    ap.add_argument("--only-set", action="store_true", help="only run the uneven set (for profiling it)")
    ap.add_argument("--no-profile", action="store_true",
                    help="no profiled regions (for runs under an external profiler)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run with the library's default thresholds (no autotuning)")
    ap.add_argument("--tune-cache", default=None, help="autotune cache file (default: the package's tuning.json)")
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

    tuning = None
    if not args.no_autotune:
        from paper_2311_03010_amd import autotune

        _log("bench: autotune (launch-shape thresholds)")
        tuning = autotune.load_or_tune(torch, eecmg, synth, cache=args.tune_cache or autotune.CACHE, log=_log)

    _log(f"bench: generating workload {args.workload}")
    p = synth.workload(args.workload)
    prec = p.precision
    H, W = p.shape
    g = torch.from_numpy(p.g_delta.astype(np.float64 if prec == "f64" else np.float32)).to("cuda:0")
    out = torch.empty_like(g)
    kw = dict(precision=prec, delta=p.delta, k=p.k)

    def restore_once():
        return eecmg.restore_dev(g, p.psf, p.n_levels, out=out, **kw)

    _log("bench: warmup")
    for _ in range(args.warmup):
        restore_once()
    torch.cuda.synchronize()

    # the throughput: kernel timing off, the interpreter's cyclic garbage
    # collector paused
    _log(f"bench: timing {args.steps} steps")
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(args.steps):
        _, stats = restore_once()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gc.enable()
    ms_step = dt / args.steps * 1e3
    value = H * W * args.steps / dt / 1e6
    u_gpu = out.cpu().numpy()

    roofline = None
    kern = {}
    if not args.no_profile:
        # dominant kernel: finest-level CGLS pass B (r -= alpha q, s = H^T r),
        # timed with HIP events on the library's launch stream around each
        # finest-level launch (the job's level holds all H x W pixels) in a
        # timed region of its own.  Algorithmic HBM bytes per pixel and
        # iteration are 32 (u, r, p, s each read and written once): 12 in
        # pass A (read s, p; write p), 12 in pass B (read r; write r, s) and 8
        # for the solution update (read u, write u), which on levels of >=
        # 1024^2 pixels a flush applies for up to seven iterations at once
        # (reading u and those directions once, writing u).  The passes
        # actually move 16 and 16 bytes: q is stored by A and read by B.
        _log("bench: profiled region (finest level)")
        eecmg.profile_reset()
        eecmg.profile_enable(True, min_pixels=H * W)
        tp0 = time.perf_counter()
        for _ in range(args.steps):
            restore_once()
        torch.cuda.synchronize()
        ms_prof = (time.perf_counter() - tp0) / args.steps * 1e3
        eecmg.profile_enable(False)
        for name, bpp, moved in (("cg_pass_a", 12, 16), ("cg_pass_b", 12, 16)):
            n, ms, px = eecmg.profile_read(name)
            if n:
                avg_ms = ms / n
                px_launch = px / n
                kern[name] = {"launches": n, "avg_us": avg_ms * 1e3, "alg_bytes_per_px": bpp,
                              "gbs": bpp * px_launch / (avg_ms * 1e-3) / 1e9, "moved_bytes_per_px": moved,
                              "moved_gbs": moved * px_launch / (avg_ms * 1e-3) / 1e9}
        for name in ("cg_init_r", "cg_init_s", "transfer_fused", "extrapolate", "flush_u", "cg_fin_a", "cg_fin_b"):
            n, ms, px = eecmg.profile_read(name)
            if n:
                kern[name] = {"launches": n, "avg_us": ms / n * 1e3}
        rb = kern.get("cg_pass_b")
        cbw = copy_bandwidth(torch)
        if rb:
            ach = rb["gbs"]
            roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                        "copy_gbs": round(cbw, 1), "frac_vs_copy": round(ach / cbw, 4),
                        "kernel": "k_cg_b<float, ConvBox<float, 6, true>> (finest level, 4096^2, tall strips)",
                        "avg_launch_us": round(rb["avg_us"], 2), "alg_bytes_per_launch": int(12 * H * W),
                        "ms_per_step_profiled": round(ms_prof, 4)}
        _log("bench: profiled region (every level)")
        casc = cascade_roofline(eecmg, restore_once, p, stats, args.steps, ms_step, cbw)
        if roofline is None:
            roofline = {"bound": "hbm", "achieved": casc["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": casc["frac"], "traffic": None, "kernel": "whole cascade"}
        roofline["cascade"] = casc
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
        same = all(torch.equal(o, out) for o in outs)
        batched = {"images": len(gs), "value": round(len(gs) * H * W * args.steps / bdt / 1e6, 3),
                   "unit": "Mpixel/s", "ms_per_step": round(bdt / args.steps * 1e3, 3),
                   "speedup_vs_plain": round(len(gs) * H * W * args.steps / bdt / 1e6 / value, 3),
                   "bitwise_equal_to_plain": bool(same)}

    uneven = None
    if args.set_images > 0:
        _log(f"bench: uneven set, {args.set_images} images, plain vs batched")
        uneven = set_leg(torch, eecmg, synth, args.set_images, args.set_steps, args.set_form)

    edge = None
    if not args.no_edge:
        _log("bench: edge-preservation workload")
        edge = edge_leg(torch, eecmg, synth, args.steps)

    workloads = None
    one_level = None
    if not args.no_extra:
        _log("bench: the other single-image workloads and the one-level leg")
        workloads = [plain_leg(torch, eecmg, synth, wid, max(args.steps, 20), args.warmup)
                     for wid in (1, 2, 3) if wid != args.workload]
        one_level = one_level_leg(torch, eecmg, synth, args.steps)

    served = None
    if args.served_requests > 0:
        _log(f"bench: served, {args.served_requests} requests")
        served = served_leg(torch, eecmg, synth, args.served_requests, args.served_pool)

    cpu = None
    cpu_table = None
    acc = None
    if not args.no_cpu_baseline:
        _log("bench: cpu baseline (oracle, all cores)")
        cpu, acc = cpu_baseline(p, stats, u_gpu)
        if not args.no_oracle_table:
            _log("bench: oracle on one core and on all cores")
            cpu_table = cpu_oracle_table(synth, (1, 2, 3), one_core=True)

    metric = ("restored Mpixel/s plain vs batched at 4096\u00b2; p50/p99 latency; % HBM roofline"
              if args.workload == 3 else "restored Mpixel/s")
    line = {"metric": metric,
            "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if prec != "f64" else "f64", "data": "synthetic",
            "config": {"workload": p.name, "H": H, "W": W,
                       "psf": {1: "gaussian sigma=2 r=4", 2: "gaussian sigma=3 r=7", 3: "disk r=6"}[args.workload],
                       "n_levels": p.n_levels, "precision": prec, "stop_rule": "discrepancy c=1.1",
                       "caps": "economic m_l rule", "form": "plain"},
            "roofline": roofline, "cpu_baseline": cpu, "accuracy_vs_oracle": acc, "batched": batched,
            "uneven_set": uneven, "served": served, "edge": edge, "workloads": workloads, "one_level": one_level,
            "cpu_oracle": cpu_table, "autotune": tuning, "detail": extra}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
