"""Pins of the oracle's smoothers (CGLS read as the paper's "CG", and the
minimal-residual iteration read as "MR") against Krylov least squares,
direct solves and monotonicity, all built with dense NumPy linear algebra."""
import numpy as np
import pytest

import oracle
from tests.conftest import dense_conv_matrix


def _problem(rng, H=6, W=5, r=1, symmetric=False):
    psf = rng.uniform(0.0, 1.0, size=(2 * r + 1, 2 * r + 1))
    if symmetric:
        psf = 0.5 * (psf + psf[::-1, ::-1])
    psf /= psf.sum()
    g = rng.uniform(0, 100, size=(H, W))
    u0 = rng.uniform(0, 100, size=(H, W))
    return psf, g, u0


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_cgls_iterate_is_krylov_least_squares_minimiser(rng, k):
    # CGLS after k steps minimises ||g - H u|| over u0 + K_k(H^T H, H^T r0)
    psf, g, u0 = _problem(rng)
    H_, W_ = g.shape
    M = dense_conv_matrix(psf, H_, W_)
    r0 = g.ravel() - M @ u0.ravel()
    A = M.T @ M
    v = M.T @ r0
    basis = []
    for _ in range(k):
        basis.append(v)
        v = A @ v
    Q, _ = np.linalg.qr(np.stack(basis, axis=1))
    c, *_ = np.linalg.lstsq(M @ Q, r0, rcond=None)
    u_ref = u0.ravel() + Q @ c
    u, it, hist, why = oracle.cgls(g, psf, u0=u0, cap=k)
    assert it == k and why == oracle.STOP_CAP
    np.testing.assert_allclose(u.ravel(), u_ref, rtol=1e-8, atol=1e-8 * np.abs(u_ref).max())


def test_cgls_residual_monotone_and_reaches_solution(rng):
    # well-conditioned (diagonally dominant) blur: CGLS reaches the exact solve
    psf = np.array([[0.0, 0.1, 0.0], [0.1, 1.0, 0.1], [0.0, 0.1, 0.0]])
    g = rng.uniform(0, 100, size=(5, 5))
    M = dense_conv_matrix(psf, 5, 5)
    u_ref = np.linalg.solve(M, g.ravel())
    u, it, hist, why = oracle.cgls(g, psf, cap=200, eps=1e-13)
    np.testing.assert_allclose(u.ravel(), u_ref, rtol=1e-10, atol=1e-10)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])


def test_cgls_residual_monotone_on_ill_conditioned_blur(rng):
    from paper_2311_03010_amd import synth
    psf = synth.disk_psf(3)
    g = rng.uniform(0, 255, size=(40, 33))
    u, it, hist, why = oracle.cgls(g, psf, cap=30)
    assert it == 30
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])


def test_cgls_identity_psf_one_step(rng):
    g = rng.uniform(0, 255, size=(8, 7))
    u0 = rng.uniform(0, 255, size=(8, 7))
    u, it, hist, why = oracle.cgls(g, np.ones((1, 1)), u0=u0, cap=50, eps=1e-14)
    assert it == 1 and why == oracle.STOP_GUARD
    np.testing.assert_allclose(u, g, rtol=1e-15, atol=1e-12)


def test_cgls_stopping_rule(rng):
    psf, g, u0 = _problem(rng)
    u, it, hist, why = oracle.cgls(g, psf, u0=u0, cap=10, stop_rule=True, cdelta=1e9)
    assert it == 0 and why == oracle.STOP_DISCREPANCY
    np.testing.assert_array_equal(u, u0)
    u, it, hist, why = oracle.cgls(g, psf, u0=u0, cap=50, stop_rule=True, cdelta=0.5 * 1.0)
    assert why in (oracle.STOP_DISCREPANCY, oracle.STOP_GUARD)
    if why == oracle.STOP_DISCREPANCY:
        assert hist[-1] <= 0.5 and np.all(hist[:-1] > 0.5)
    u, it, hist, why = oracle.cgls(g, psf, u0=u0, cap=0)
    assert it == 0 and why == oracle.STOP_CAP


def test_mr_residual_monotone_and_step_optimal(rng):
    psf, g, u0 = _problem(rng, symmetric=True)
    u, it, hist, why = oracle.mr(g, psf, u0=u0, cap=20)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    # one MR step minimises ||g - H (u0 + t r0)|| over the scalar t
    u1, _, _, _ = oracle.mr(g, psf, u0=u0, cap=1)
    M = dense_conv_matrix(psf, *g.shape)
    r0 = g.ravel() - M @ u0.ravel()
    t = (u1 - u0).ravel() @ r0 / (r0 @ r0)
    np.testing.assert_allclose((u1 - u0).ravel(), t * r0, rtol=1e-10, atol=1e-10)

    def res(tt):
        return np.linalg.norm(g.ravel() - M @ (u0.ravel() + tt * r0))
    assert res(t) <= res(t * (1 + 1e-3)) and res(t) <= res(t * (1 - 1e-3))


def test_mr_converges_on_spd_blur(rng):
    psf = np.array([[0.0, 0.1, 0.0], [0.1, 1.0, 0.1], [0.0, 0.1, 0.0]])  # SPD (diagonally dominant)
    g = rng.uniform(0, 100, size=(6, 6))
    M = dense_conv_matrix(psf, 6, 6)
    u_ref = np.linalg.solve(M, g.ravel())
    u, it, hist, why = oracle.mr(g, psf, cap=500, eps=1e-13)
    np.testing.assert_allclose(u.ravel(), u_ref, rtol=1e-9, atol=1e-9)
