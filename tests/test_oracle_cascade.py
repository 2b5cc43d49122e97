"""Pins of the oracle's complete cascades (Algorithm 1 and 2)."""
import numpy as np
import pytest

import oracle
from paper_2311_03010_amd import synth


@pytest.mark.parametrize("cascade", [0, 1, 2])
@pytest.mark.parametrize("smoother", [0, 1])
def test_identity_psf_zero_noise_recovers_g(rng, cascade, smoother):
    # H = I and no noise: every level's smoother returns its right-hand side,
    # so the cascade output is g itself
    g = rng.uniform(0, 255, size=(33, 40))
    u, st = oracle.restore(g, np.ones((1, 1)), 3, caps=[5, 5, 5], stop_rule=False, delta=0.0,
                           smoother=smoother, cascade=cascade, guard_eps=1e-14)
    np.testing.assert_allclose(u, g, rtol=1e-13, atol=1e-11)
    assert st["radius"] == [0, 0, 0]


def test_transpose_equivariance():
    p = synth.workload(1)
    u, st = oracle.restore(p.g_delta, p.psf, 3, delta=p.delta)
    ut, stt = oracle.restore(p.g_delta.T.copy(), p.psf.T.copy(), 3, delta=p.delta)
    np.testing.assert_allclose(ut, u.T, rtol=1e-12, atol=1e-10)
    assert st["iters"] == stt["iters"]


def test_workload1_cascade_improves_psnr_and_respects_caps():
    p = synth.workload(1)
    u, st = oracle.restore(p.g_delta, p.psf, p.n_levels, delta=p.delta)
    assert st["caps"] == [2, 9, 3]
    assert st["radius"] == [1, 2, 4]
    assert all(0 <= it <= cap for it, cap in zip(st["iters"], st["caps"]))
    assert np.isfinite(u).all()
    assert oracle.psnr(p.u_true, u) > oracle.psnr(p.u_true, p.g_delta)


def test_one_level_is_plain_smoother(rng):
    p = synth.workload(1)
    u, st = oracle.restore(p.g_delta, p.psf, 1, caps=[4], stop_rule=False)
    u2, it, _, _ = oracle.cgls(p.g_delta, p.psf, cap=4)
    np.testing.assert_array_equal(u, u2)


def test_two_level_output_is_level2_smoother():
    p = synth.workload(1)
    u, st = oracle.restore(p.g_delta, p.psf, 2, caps=[3, 4], stop_rule=False)
    u2, it, _, _ = oracle.cgls(p.g_delta, p.psf, cap=4)
    np.testing.assert_array_equal(u, u2)


def test_invalid_arguments():
    g = np.zeros((64, 64))
    with pytest.raises(ValueError):
        oracle.restore(g, np.ones((1, 1)), 6)  # coarsest 2x2
    with pytest.raises(ValueError):
        oracle.restore(g, np.ones((1, 1)), 3, tau=0.3)
    with pytest.raises(ValueError):
        oracle.restore(g, np.ones((1, 1)), 3, c=1.0)


def test_cascade_is_well_conditioned_in_rounding(rng):
    # a relative perturbation of 1e-15 in g must not be amplified beyond
    # ~1e-13 (guards the numerical stability of every transfer operator)
    p = synth.workload(1)
    g2 = p.g_delta * (1 + 1e-15 * rng.standard_normal(p.g_delta.shape))
    a, sa = oracle.restore(p.g_delta, p.psf, 3, delta=p.delta, stop_rule=False)
    b, sb = oracle.restore(g2, p.psf, 3, delta=p.delta, stop_rule=False)
    assert np.linalg.norm(b - a) / np.linalg.norm(a) < 1e-13
