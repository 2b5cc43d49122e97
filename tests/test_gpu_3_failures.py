"""Failure handling of the host scheduler, forced from the host.

No kernel is made to fail: the conditions are produced by host-side knobs
while every kernel runs and completes normally.
  - stall guard: with a run-ahead of one iteration (EECMG_MAX_AHEAD=1) a
    level with folded finalizes cannot confirm its first iteration (the next
    iteration's pass A would publish it), so the device goes idle with nothing
    left to launch; the guard must report EDEVICE instead of spinning, and
  - an error reported by the HIP runtime (EECMG_TEST_FAIL_STEP: the engine
    records an error at a given step without launching anything).
In both cases the call returns EDEVICE with every admitted job released, and
the next call on the same engine or context succeeds with the same bits as
before.
"""
import numpy as np
import pytest

from paper_2311_03010_amd import eecmg, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _problem():
    # 256^2, 5 levels: 128^2 and 256^2 run on the engine with folded finalizes
    return synth.workload(2, H=256, W=256, n_levels=5, n_shapes=40)


def _reference(t, p):
    g = t.from_numpy(p.g_delta.astype(np.float32)).to("cuda:0")
    u, st = eecmg.restore_dev(g, p.psf, p.n_levels, precision="f32", delta=p.delta)
    t.cuda.synchronize()
    return g, u.cpu().numpy(), st


def test_stall_guard_reports_edevice_and_engine_recovers(torch_cuda, monkeypatch):
    t = torch_cuda
    p = _problem()
    g, u_ref, st_ref = _reference(t, p)
    assert st_ref["iters"][3] >= 1, st_ref  # the first engine level runs an iteration
    monkeypatch.setenv("EECMG_MAX_AHEAD", "1")
    monkeypatch.setenv("EECMG_STALL_STEPS", "16")
    monkeypatch.setenv("EECMG_STALL_MS", "50")
    print("stall guard: restore_dev 256^2 with run-ahead 1", flush=True)
    with pytest.raises(eecmg.EecmgError) as e:
        eecmg.restore_dev(g, p.psf, p.n_levels, precision="f32", delta=p.delta)
    assert e.value.status == eecmg.EDEVICE
    assert "stall" in str(e.value)
    for k in ("EECMG_MAX_AHEAD", "EECMG_STALL_STEPS", "EECMG_STALL_MS"):
        monkeypatch.delenv(k)
    print("stall guard: the next restore", flush=True)
    u, st = eecmg.restore_dev(g, p.psf, p.n_levels, precision="f32", delta=p.delta)
    t.cuda.synchronize()
    np.testing.assert_array_equal(u.cpu().numpy(), u_ref)
    assert st == st_ref


@pytest.mark.parametrize("step", [1, 3, 6])
def test_hip_error_releases_jobs_and_next_call_succeeds(torch_cuda, monkeypatch, step):
    t = torch_cuda
    p = _problem()
    g, u_ref, st_ref = _reference(t, p)
    monkeypatch.setenv("EECMG_TEST_FAIL_STEP", str(step))
    print(f"injected error at step {step}: restore_dev and batch", flush=True)
    with pytest.raises(eecmg.EecmgError) as e:
        eecmg.restore_dev(g, p.psf, p.n_levels, precision="f32", delta=p.delta)
    assert e.value.status == eecmg.EDEVICE
    with pytest.raises(eecmg.EecmgError) as e:
        eecmg.restore_batch_dev([g, g.clone()], [p.psf] * 2, [p.n_levels] * 2, precision="f32",
                                params=[{"delta": p.delta}] * 2)
    assert e.value.status == eecmg.EDEVICE
    with pytest.raises(eecmg.EecmgError) as e:
        eecmg.restore(p.g_delta.astype(np.float32), p.psf, p.n_levels, precision="f32", delta=p.delta)
    assert e.value.status == eecmg.EDEVICE
    monkeypatch.delenv("EECMG_TEST_FAIL_STEP")
    print("injected error: the next calls", flush=True)
    u, st = eecmg.restore_dev(g, p.psf, p.n_levels, precision="f32", delta=p.delta)
    outs, sts = eecmg.restore_batch_dev([g, g.clone()], [p.psf] * 2, [p.n_levels] * 2, precision="f32",
                                        params=[{"delta": p.delta}] * 2)
    t.cuda.synchronize()
    np.testing.assert_array_equal(u.cpu().numpy(), u_ref)
    assert st == st_ref
    for o, s in zip(outs, sts):
        np.testing.assert_array_equal(o.cpu().numpy(), u_ref)
        assert s == st_ref
    uh, sh = eecmg.restore(p.g_delta.astype(np.float32), p.psf, p.n_levels, precision="f32", delta=p.delta)
    np.testing.assert_array_equal(uh, u_ref)


def test_served_requests_fail_with_edevice_and_context_recovers(torch_cuda, monkeypatch):
    t = torch_cuda
    p = _problem()
    _, u_ref, st_ref = _reference(t, p)
    # the context's progress thread reads the knob when it starts
    monkeypatch.setenv("EECMG_TEST_FAIL_STEP", "2")
    print("served: injected error at step 2", flush=True)
    with eecmg.Context(hbm_budget_bytes=512 << 20, max_slots=4) as ctx:
        monkeypatch.delenv("EECMG_TEST_FAIL_STEP")
        reqs = [ctx.submit(p.g_delta.astype(np.float32), p.psf, p.n_levels, precision="f32", delta=p.delta)
                for _ in range(2)]
        codes = []
        for r in reqs:
            try:
                ctx.wait(r)
                codes.append(eecmg.OK)
            except eecmg.EecmgError as e:
                codes.append(e.status)
        assert eecmg.EDEVICE in codes, codes
        assert all(c in (eecmg.OK, eecmg.EDEVICE) for c in codes)
        info = ctx.info()
        assert info["active"] == 0 and info["bytes_in_use"] == 0, info
        print("served: a request after the failure", flush=True)
        r = ctx.submit(p.g_delta.astype(np.float32), p.psf, p.n_levels, precision="f32", delta=p.delta)
        u, st = ctx.wait(r)
    np.testing.assert_array_equal(u, u_ref)
    assert st == st_ref
