"""GPU parity against the oracle for the slices of the method that run on the
multi-level engine rather than inside the one-block coarse cascade:
  - Algorithm 1 (IECMG-L with the linear prolongation of eq. 15, IECMG-P with
    the quadratic interpolation of Section 3.2) on cascades whose levels
    exceed 64^2, CGLS and MR;
  - the one-level smoother with the discrepancy stopping rule (the one-level
    baseline of Section 5, Table 1), CGLS and MR, at 1024^2;
  - images of the uneven batch recipe (sides in [128, 2048], Gaussian sigma up
    to 4 with support 2 ceil(3 sigma) + 1, disk radii 2..6) whose finest level
    reaches the streaming separable kernels with radius 9 and 12, plain and in
    one batch;
  - an FP64 cascade with a 1024^2 level.
Bars as for every cascade: FP64 relative L2 <= 1e-12, FP32 <= 1e-4, PSNR
within 0.01 dB, identical per-level iteration counts and stop reasons.
"""
import numpy as np
import pytest

import oracle
from paper_2311_03010_amd import eecmg, synth

pytestmark = pytest.mark.gpu

REL = {"f64": 1e-12, "f32": 1e-4}
GUARD = {"f64": 1e-14, "f32": 1e-6}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _dt(prec):
    return np.float64 if prec == "f64" else np.float32


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _oracle(p, prec, caps=None, stop_rule=True, smoother="cgls", cascade="eecmg"):
    g = p.g_delta.astype(_dt(prec)).astype(np.float64)
    return oracle.restore(g, p.psf, p.n_levels, caps=caps, delta=p.delta, k=p.k, stop_rule=stop_rule,
                          guard_eps=GUARD[prec], smoother=eecmg.SMOOTHERS[smoother],
                          cascade=eecmg.CASCADES[cascade])


def _check(p, prec, u, st, u_ref, st_ref):
    print(f"  {p.name} {p.shape} iters gpu={st['iters']} oracle={st_ref['iters']} reasons={st['reason']}",
          flush=True)
    assert st["iters"] == st_ref["iters"]
    assert st["reason"] == st_ref["reason"]
    rel = _rel(u, u_ref)
    dpsnr = abs(oracle.psnr(p.u_true, np.asarray(u, np.float64)) - oracle.psnr(p.u_true, u_ref))
    print(f"  rel_l2={rel:.3e} dPSNR={dpsnr:.2e}", flush=True)
    assert rel <= REL[prec]
    assert dpsnr <= 0.01


def _gpu(t, p, prec, **kw):
    g = t.from_numpy(p.g_delta.astype(_dt(prec))).to("cuda:0")
    print(f"  gpu restore {p.name} {p.shape} L={p.n_levels} {prec} {kw}", flush=True)
    u, st = eecmg.restore_dev(g, p.psf, p.n_levels, precision=prec, delta=p.delta, k=p.k, **kw)
    t.cuda.synchronize()
    return u.cpu().numpy(), st


# ------------------------------------------------------------- Algorithm 1
@pytest.mark.parametrize("cascade", ["iecmg_l", "iecmg_p"])
@pytest.mark.parametrize("smoother", ["cgls", "mr"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_algorithm1_on_engine_levels(torch_cuda, cascade, smoother, prec):
    # 257 x 190 with 4 levels: 33 x 24, 65 x 48 (coarse cascade), 129 x 95 and
    # 257 x 190 on the engine, ragged on both axes
    p = synth.workload(3, H=257, W=190, n_levels=4, n_shapes=30, n_textures=3, precision=prec)
    u, st = _gpu(torch_cuda, p, prec, smoother=smoother, cascade=cascade)
    _check(p, prec, u, st, *_oracle(p, prec, smoother=smoother, cascade=cascade))


@pytest.mark.parametrize("cascade", ["iecmg_l", "iecmg_p"])
@pytest.mark.parametrize("smoother", ["cgls", "mr"])
def test_algorithm1_full_size_1024(torch_cuda, cascade, smoother):
    p = synth.workload(2)  # 1024^2, Gaussian sigma=3 on 15 x 15, 7 levels
    u, st = _gpu(torch_cuda, p, "f32", smoother=smoother, cascade=cascade)
    _check(p, "f32", u, st, *_oracle(p, "f32", smoother=smoother, cascade=cascade))


# ------------------------------------------------- one level, stopping rule
@pytest.mark.parametrize("smoother", ["cgls", "mr"])
def test_one_level_with_discrepancy_stop_1024(torch_cuda, smoother):
    base = synth.workload(2)
    p = synth.Problem(name="gauss3_1024_one_level", u_true=base.u_true, psf=base.psf, g_delta=base.g_delta,
                      delta=base.delta, n_levels=1, precision="f32")
    caps = [200]
    u, st = _gpu(torch_cuda, p, "f32", caps=caps, smoother=smoother)
    u_ref, st_ref = _oracle(p, "f32", caps=caps, smoother=smoother)
    assert st_ref["reason"] == [1]  # the discrepancy principle ends it, not the cap
    _check(p, "f32", u, st, u_ref, st_ref)


# ------------------------------------------------ uneven batch recipe
def _batch_recipe_images():
    specs = [(1100, 1301, synth.gaussian_psf(4.0, 12), "gauss sigma=4 r=12"),
             (1024, 1536, synth.gaussian_psf(3.0, 9), "gauss sigma=3 r=9"),
             (333, 517, synth.disk_psf(2), "disk r=2"),
             (1500, 700, synth.disk_psf(5), "disk r=5")]
    probs = []
    for i, (H, W, psf, name) in enumerate(specs):
        q = synth.make_problem(f"batch_recipe_{i}", H, W, psf, max(8, int(round(200 * H * W / 1e6))),
                               synth.SEED_BASE + 40 + i, synth.levels_for(H, W), "f32", meta={"psf": name})
        probs.append(q)
    return probs


def test_batch_recipe_images_plain_and_batched_match_oracle(torch_cuda):
    t = torch_cuda
    probs = _batch_recipe_images()
    gs = [t.from_numpy(q.g_delta.astype(np.float32)).to("cuda:0") for q in probs]
    plain = []
    for q, g in zip(probs, gs):
        print(f"  plain {q.name} {q.shape} L={q.n_levels} {q.meta['psf']}", flush=True)
        u, st = eecmg.restore_dev(g, q.psf, q.n_levels, precision="f32", delta=q.delta, k=q.k)
        plain.append((u.cpu().numpy(), st))
    print("  batched", flush=True)
    outs, sts = eecmg.restore_batch_dev(gs, [q.psf for q in probs], [q.n_levels for q in probs],
                                        ks=[q.k for q in probs], precision="f32",
                                        params=[{"delta": q.delta} for q in probs])
    t.cuda.synchronize()
    for q, (u, st), ub, sb in zip(probs, plain, outs, sts):
        np.testing.assert_array_equal(u, ub.cpu().numpy())
        assert st == sb
        _check(q, "f32", u, st, *_oracle(q, "f32"))


# ----------------------------------------------------------- FP64 1024^2
def test_fp64_cascade_with_1024_level(torch_cuda):
    p = synth.workload(2, precision="f64")
    u, st = _gpu(torch_cuda, p, "f64")
    _check(p, "f64", u, st, *_oracle(p, "f64"))


# ------------------------------------------------------------ short strips
@pytest.mark.parametrize("psfname", ["gauss7", "symdisk5", "disk5"])
def test_short_strip_smoother_parity(torch_cuda, monkeypatch, psfname):
    """A 700 x 900 FP32 level gives the streaming kernels too few strips of
    the usual height, so it runs on short strips: CGLS from zero matches the
    oracle with the separable, symmetric-disk and uniform-disk kernels, and the
    usual strips (EECMG_SHORT_MAX_TILES=0) to FP32 rounding (the partial sums
    are grouped by other tiles)."""
    H, W = 700, 900
    rng = np.random.Generator(np.random.PCG64(H + 3 * len(psfname)))
    a = np.arange(-5, 6)
    d2 = a[:, None] ** 2 + a[None, :] ** 2
    symdisk = np.where(d2 <= 25, 1.0 / (1.0 + d2), 0.0)
    psf = {"gauss7": synth.gaussian_psf(2.5, 7), "symdisk5": symdisk / symdisk.sum(), "disk5": synth.disk_psf(5)}[psfname]
    u_true = synth.scene(H, W, 120, rng)
    g = (synth.blur(u_true, psf) + rng.standard_normal((H, W))).astype(np.float32).astype(np.float64)
    cap = 6
    t = torch_cuda
    gd = t.from_numpy(g.astype(np.float32)).to("cuda:0")
    res = {}
    for mode, env in (("short", "2048"), ("usual", "0")):
        monkeypatch.setenv("EECMG_SHORT_MAX_TILES", env)
        print(f"  {psfname} {mode} strips", flush=True)
        ud = t.zeros_like(gd)
        u, st = eecmg.smoother_dev(gd, ud, psf, cap, precision="f32", stop_rule=False)
        t.cuda.synchronize()
        res[mode] = (u.cpu().numpy().astype(np.float64), st)
    u_ref, it, hist, why = oracle.cgls(g, psf, u0=np.zeros_like(g), cap=cap, eps=GUARD["f32"])
    for mode in ("short", "usual"):
        u, st = res[mode]
        print(f"  {mode}: iters gpu={st['iters']} oracle={it} rel={_rel(u, u_ref):.2e}", flush=True)
        assert st["iters"] == it and st["reason"] == why
        assert _rel(u, u_ref) <= 2e-5
    assert _rel(res["short"][0], res["usual"][0]) <= 1e-5


# ------------------------------------------------ strips inside the image
@pytest.mark.parametrize("smoother", ["cgls", "mr"])
@pytest.mark.parametrize("psfname", ["disk3", "symdisk3"])
def test_f64_streaming_smoother_parity_on_a_ragged_level(torch_cuda, smoother, psfname):
    """A 1100 x 1000 FP64 level runs the streaming kernels on usual strips
    (uniform-disk and symmetric-disk policies): most strips lie inside the
    image and walk their middle row groups without per-row tests, the
    strips of the last strip row and column are ragged.  CGLS and MR from a
    smoothed start match the FP64 oracle."""
    H, W = 1100, 1000
    rng = np.random.Generator(np.random.PCG64(H + W + len(psfname) + len(smoother)))
    a = np.arange(-3, 4)
    d2 = a[:, None] ** 2 + a[None, :] ** 2
    symdisk = np.where(d2 <= 9, 1.0 / (1.0 + d2), 0.0)
    psf = {"disk3": synth.disk_psf(3), "symdisk3": symdisk / symdisk.sum()}[psfname]
    u_true = synth.scene(H, W, 60, rng)
    g = synth.blur(u_true, psf) + rng.standard_normal((H, W))
    u0 = synth.blur(g, synth.gaussian_psf(1.0, 2))
    cap = 5
    t = torch_cuda
    print(f"  {smoother} {psfname} {H}x{W} f64", flush=True)
    gd = t.from_numpy(g).to("cuda:0")
    ud = t.from_numpy(u0).to("cuda:0")
    u, st = eecmg.smoother_dev(gd, ud, psf, cap, precision="f64", smoother=smoother, stop_rule=False)
    t.cuda.synchronize()
    fn = oracle.cgls if smoother == "cgls" else oracle.mr
    u_ref, it, hist, why = fn(g, psf, u0=u0, cap=cap, eps=GUARD["f64"])
    print(f"  iters gpu={st['iters']} oracle={it} rel={_rel(u.cpu().numpy(), u_ref):.2e}", flush=True)
    assert st["iters"] == it and st["reason"] == why
    assert _rel(u.cpu().numpy(), u_ref) <= 1e-12


# ------------------------------------------------------------ step pacing
def test_step_pacing_depth_leaves_batched_results_bitwise_unchanged(torch_cuda, monkeypatch):
    """The scheduler's step pacing (how many steps it keeps queued on the
    device before issuing the next) only regroups jobs into launches: a batch
    of uneven-set images gives the same bits and per-level statistics with
    pacing off, at depth 2 and at depth 3, and the same as each image alone."""
    t = torch_cuda
    probs = synth.batch_problems(24)
    gs = [t.from_numpy(q.g_delta.astype(np.float32)).to("cuda:0") for q in probs]
    kw = dict(ks=[q.k for q in probs], precision="f32", params=[{"delta": q.delta} for q in probs])
    res = {}
    for depth in ("0", "2", "3"):
        monkeypatch.setenv("EECMG_PACE_STEPS", depth)
        print(f"  batched, pacing depth {depth}", flush=True)
        outs, sts = eecmg.restore_batch_dev(gs, [q.psf for q in probs], [q.n_levels for q in probs], **kw)
        t.cuda.synchronize()
        res[depth] = ([o.cpu().numpy() for o in outs], sts)
    monkeypatch.setenv("EECMG_PACE_STEPS", "2")
    for i in (0, 7, 23):
        q = probs[i]
        print(f"  alone {q.name} {q.shape}", flush=True)
        u, st = eecmg.restore_dev(gs[i], q.psf, q.n_levels, precision="f32", delta=q.delta, k=q.k)
        t.cuda.synchronize()
        np.testing.assert_array_equal(u.cpu().numpy(), res["2"][0][i])
        assert st == res["2"][1][i]
    for depth in ("0", "3"):
        for a, b in zip(res[depth][0], res["2"][0]):
            np.testing.assert_array_equal(a, b)
        assert res[depth][1] == res["2"][1]


# ------------------------------------------------------------ batch lanes
def test_batch_lanes_leave_results_bitwise_unchanged(torch_cuda, monkeypatch):
    """A batched call split over several lanes (engines with their own
    streams and host threads) gives the same bits and per-level statistics as
    one lane: each image's arithmetic does not depend on what shares its
    launches."""
    t = torch_cuda
    probs = synth.batch_problems(24)
    gs = [t.from_numpy(q.g_delta.astype(np.float32)).to("cuda:0") for q in probs]
    kw = dict(ks=[q.k for q in probs], precision="f32", params=[{"delta": q.delta} for q in probs])
    res = {}
    for lanes in ("1", "2", "3"):
        monkeypatch.setenv("EECMG_BATCH_LANES", lanes)
        print(f"  batched, {lanes} lane(s)", flush=True)
        outs, sts = eecmg.restore_batch_dev(gs, [q.psf for q in probs], [q.n_levels for q in probs], **kw)
        t.cuda.synchronize()
        res[lanes] = ([o.cpu().numpy() for o in outs], sts)
    for lanes in ("2", "3"):
        for a, b in zip(res[lanes][0], res["1"][0]):
            np.testing.assert_array_equal(a, b)
        assert res[lanes][1] == res["1"][1]


# ------------------------------------------------------ restriction launch
def test_served_step_with_both_precisions_and_every_coarse_layout(torch_cuda):
    """Requests admitted in one served step share the restriction launch,
    which also solves each job's coarse levels: it runs once per precision,
    over jobs whose levels are all coarse (no restriction tiles), partly
    coarse (a coarse block and tiles) or not coarse at all (one level: tiles
    only).  Every result equals the request restored alone, bit for bit, and
    FP32 and FP64 requests submitted together both match the oracle."""
    t = torch_cuda
    cases = [(synth.workload(1, H=64, W=64), "f64"),
             (synth.workload(3, H=130, W=200, n_levels=4, n_shapes=20, n_textures=2), "f32"),
             (synth.workload(3, H=130, W=200, n_levels=4, n_shapes=20, n_textures=2), "f64"),
             (synth.workload(1, H=48, W=40, n_levels=3), "f32"),
             (synth.workload(2, H=150, W=120, n_levels=1, n_shapes=20), "f32")]
    alone = [_gpu(t, p, prec) for p, prec in cases]
    with eecmg.Context(hbm_budget_bytes=256 << 20, max_slots=8) as ctx:
        reqs = [ctx.submit(p.g_delta.astype(_dt(prec)), p.psf, p.n_levels, precision=prec, delta=p.delta, k=p.k)
                for p, prec in cases]
        got = [ctx.wait(r) for r in reqs]
    for (p, prec), (ua, sa), (ub, sb) in zip(cases, alone, got):
        print(f"  served {p.name} {p.shape} L={p.n_levels} {prec}", flush=True)
        np.testing.assert_array_equal(ua, ub)
        assert sa == sb
    for i in (1, 2):
        p, prec = cases[i]
        _check(p, prec, got[i][0], got[i][1], *_oracle(p, prec))


# ------------------------------------------------- deferred updates, shared
def test_deferred_updates_in_shared_launches_match_eager_plain(torch_cuda, monkeypatch):
    """Deferred solution updates forced on every level, with iteration counts
    below, at and across the seven-term flush groups, for several jobs that
    share each launch (batched call and served context: launches whose jobs
    flush at different iterations, and no folded finalizes): every result
    equals the eager per-iteration update of the image restored alone, bit
    for bit, with the same statistics."""
    t = torch_cuda
    cases = [(synth.workload(3, H=200, W=160, n_levels=3, n_shapes=20, n_textures=2), [2, 9, 14]),
             (synth.workload(3, H=96, W=130, n_levels=3, n_shapes=10), [7, 3, 17]),
             (synth.workload(2, H=150, W=120, n_levels=3, n_shapes=20), [1, 6, 8]),
             (synth.workload(1, H=100, W=90, n_levels=3, n_shapes=10), [5, 13, 21])]
    gs = [t.from_numpy(p.g_delta.astype(np.float32)).to("cuda:0") for p, _ in cases]
    monkeypatch.setenv("EECMG_LAZY_MIN_PIXELS", str(1 << 40))
    ref = []
    for (p, cl), g in zip(cases, gs):
        u, st = eecmg.restore_dev(g, p.psf, p.n_levels, caps=cl, precision="f32", delta=p.delta, stop_rule=False)
        t.cuda.synchronize()
        ref.append((u.cpu().numpy(), st))
    monkeypatch.setenv("EECMG_LAZY_MIN_PIXELS", "1")
    print("  batched, deferred updates on every level", flush=True)
    outs, sts = eecmg.restore_batch_dev(gs, [p.psf for p, _ in cases], [p.n_levels for p, _ in cases],
                                        caps=[cl for _, cl in cases], precision="f32",
                                        params=[{"delta": p.delta, "stop_rule": False} for p, _ in cases])
    t.cuda.synchronize()
    for (ua, sa), ub, sb in zip(ref, outs, sts):
        np.testing.assert_array_equal(ua, ub.cpu().numpy())
        assert sa == sb
    print("  served, deferred updates on every level", flush=True)
    with eecmg.Context(hbm_budget_bytes=256 << 20, max_slots=8) as ctx:
        reqs = [ctx.submit(p.g_delta.astype(np.float32), p.psf, p.n_levels, caps=cl, precision="f32",
                           delta=p.delta, stop_rule=False) for p, cl in cases]
        got = [ctx.wait(r) for r in reqs]
    for (ua, sa), (ub, sb) in zip(ref, got):
        np.testing.assert_array_equal(ua, ub)
        assert sa == sb
