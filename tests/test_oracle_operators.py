"""Pins of the oracle's blur operator, grid hierarchy and iteration-count rule
against statements independent of the oracle's code (CPU only)."""
import numpy as np
import pytest
from scipy.signal import convolve2d, fftconvolve

import oracle
from paper_2311_03010_amd import synth
from tests.conftest import dense_conv_matrix, read_golden


def test_conv_matches_dense_matrix(rng):
    # non-symmetric PSF, non-square image: H and H^T against the dense operator
    for H, W, r in [(7, 9, 2), (5, 4, 1), (6, 6, 3), (3, 11, 0)]:
        psf = rng.standard_normal((2 * r + 1, 2 * r + 1))
        x = rng.standard_normal((H, W))
        M = dense_conv_matrix(psf, H, W)
        np.testing.assert_allclose(oracle.conv(x, psf).ravel(), M @ x.ravel(), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(oracle.conv(x, psf, transpose=True).ravel(), M.T @ x.ravel(), rtol=1e-13,
                                   atol=1e-13)


def test_gaussian_is_kronecker_of_banded_toeplitz():
    # Section 5: H = h (x) h with h the banded Toeplitz Gaussian
    sigma, band, n = 2.0, 4, 10
    psf = synth.gaussian_psf(sigma, band)
    t = np.arange(-band, band + 1)
    h1 = np.exp(-(t * t) / (2 * sigma * sigma))
    h1 /= h1.sum()
    h = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if abs(i - j) <= band:
                h[i, j] = h1[i - j + band]
    K = np.kron(h, h)
    M = np.stack([oracle.conv(e.reshape(n, n), psf).ravel() for e in np.eye(n * n)], axis=1)
    np.testing.assert_allclose(M, K, rtol=0, atol=1e-15)
    # symmetric PSF: H is symmetric (block Toeplitz), eq. 7
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-15)


def test_adjoint_identity(rng):
    psf = rng.standard_normal((7, 7))
    x = rng.standard_normal((23, 17))
    y = rng.standard_normal((23, 17))
    lhs = np.sum(oracle.conv(x, psf) * y)
    rhs = np.sum(x * oracle.conv(y, psf, transpose=True))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_conv_matches_library_convolution_large(rng):
    x = rng.uniform(0, 255, size=(200, 131))
    for psf in (synth.disk_psf(6), synth.gaussian_psf(3.0, 7), rng.standard_normal((5, 5))):
        ref = convolve2d(x, psf, mode="same", boundary="fill")
        np.testing.assert_allclose(oracle.conv(x, psf), ref, rtol=1e-12, atol=1e-9)
        ref_fft = fftconvolve(x, psf, mode="same")
        np.testing.assert_allclose(oracle.conv(x, psf), ref_fft, rtol=1e-9, atol=1e-8)


def test_delta_psf_is_identity(rng):
    x = rng.standard_normal((9, 13))
    np.testing.assert_array_equal(oracle.conv(x, np.ones((1, 1))), x)
    psf = np.zeros((5, 5)); psf[2, 2] = 1.0
    np.testing.assert_array_equal(oracle.conv(x, psf), x)


def test_restrict_is_bitwise_injection(rng):
    g = rng.standard_normal((37, 64))
    sizes = oracle.level_sizes(37, 64, 3)
    (Hc, Wc) = sizes[1]
    np.testing.assert_array_equal(oracle.restrict(g, Hc, Wc), g[::2, ::2])


def test_level_sizes():
    assert oracle.level_sizes(64, 64, 3) == [(16, 16), (32, 32), (64, 64)]
    assert oracle.level_sizes(4096, 4096, 9)[0] == (16, 16)
    # odd case of Section 2: N_{l-1} = (sqrt(N_l) + 1)^2 / 4
    assert oracle.level_sizes(65, 65, 3) == [(17, 17), (33, 33), (65, 65)]
    assert oracle.level_sizes(100, 37, 3) == [(25, 10), (50, 19), (100, 37)]
    with pytest.raises(ValueError):
        oracle.level_sizes(8, 8, 3)


def test_iteration_caps_match_hand_table():
    for row in read_golden("iteration_caps.txt"):
        L = int(row[0])
        assert oracle.iteration_caps(L) == [int(v) for v in row[1:]], L


@pytest.mark.parametrize("Hf,Wf,r", [(12, 10, 2), (11, 9, 3), (8, 13, 4)])
def test_coarse_operator_is_R_H_Rt(rng, Hf, Wf, r):
    # eq. 14: H_l = R H R^* with R the injection of eq. 12; mode 2 is the
    # Euclidean adjoint, mode 1 scales it by 4, mode 0 by sum-preservation
    psf = rng.uniform(0.1, 1.0, size=(2 * r + 1, 2 * r + 1))
    Hc, Wc = (Hf + 1) // 2, (Wf + 1) // 2
    Rm = np.zeros((Hc * Wc, Hf * Wf))
    for a in range(Hc):
        for b in range(Wc):
            Rm[a * Wc + b, (2 * a) * Wf + 2 * b] = 1.0
    M = dense_conv_matrix(psf, Hf, Wf)
    RHR = Rm @ M @ Rm.T
    rc = r // 2
    sub = sum(psf[2 * a + r, 2 * b + r] for a in range(-rc, rc + 1) for b in range(-rc, rc + 1))
    for mode, scale in [(2, 1.0), (1, 4.0), (0, psf.sum() / sub)]:
        pc = oracle.coarse_psf(psf, mode)
        assert pc.shape == (2 * rc + 1, 2 * rc + 1)
        Mc = dense_conv_matrix(pc, Hc, Wc)
        np.testing.assert_allclose(Mc, scale * RHR, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("sigma,r", [(2.0, 4), (3.0, 7), (4.0, 12), (1.0, 3)])
def test_gaussian_self_similarity(sigma, r):
    # decimating a unit-sum Gaussian by 2 and renormalising gives the
    # Gaussian of half the width on half the support (closed form)
    pc = oracle.coarse_psf(synth.gaussian_psf(sigma, r), 0)
    np.testing.assert_allclose(pc, synth.gaussian_psf(sigma / 2, r // 2), rtol=1e-13, atol=1e-16)


def test_coarse_psf_of_unit_sum_keeps_unit_sum():
    pc = oracle.coarse_psf(synth.disk_psf(6), 0)
    assert abs(pc.sum() - 1.0) < 1e-14
    # unit-sum operator maps constants to constants away from the border
    x = np.ones((30, 30))
    y = oracle.conv(x, pc)
    np.testing.assert_allclose(y[5:-5, 5:-5], 1.0, rtol=1e-14)


def test_rms_and_psnr_definitions(rng):
    x = rng.standard_normal(1000)
    assert abs(oracle.rms(x) - np.sqrt(np.mean(x * x))) < 1e-14
    u = rng.uniform(0, 255, 500)
    v = u + 2.0
    assert abs(oracle.psnr(u, v) - 20 * np.log10(255 / 2.0)) < 1e-12
