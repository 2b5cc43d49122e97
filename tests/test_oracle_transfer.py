"""Pins of the oracle's level transfer: new extrapolation Pi, quadratic
interpolation P (against the 1-D coefficients printed in Section 3.2 and
polynomial exactness), linear prolongation L (eq. 15), local smoothing S
(against brute-force weighted least squares) and Perona-Malik denoising D
(conservation, maximum principle, heat-step limit)."""
import numpy as np
import pytest
from scipy.ndimage import laplace

import oracle
from tests.conftest import read_golden


def _grids(HC, WC):
    HB, WB = (HC + 1) // 2, (WC + 1) // 2
    HA, WA = (HB + 1) // 2, (WB + 1) // 2
    return (HA, WA), (HB, WB), (HC, WC)


def _sample(f, H, W, step):
    i = np.arange(H, dtype=np.float64)[:, None] * step
    j = np.arange(W, dtype=np.float64)[None, :] * step
    return f(i, j) + 0 * i * j


def _transfer(uA, uB, HC, WC):
    return oracle.prolong_quad(oracle.extrapolate(uA, uB), HC, WC)


def test_pi_p_matches_paper_1d_coefficients(rng):
    # images constant along i reduce the 2-D operator to the 1-D rule of
    # Section 3.2 along j; compare with the printed raw-value coefficients
    rows = {r[0]: np.array([float(v) for v in r[1:]]) / 16.0 for r in read_golden("pi_p_1d_coefficients.txt")}
    (HA, WA), (HB, WB), (HC, WC) = _grids(17, 33)
    fA = rng.standard_normal(WA)
    fB = rng.standard_normal(WB)
    uA = np.tile(fA, (HA, 1))
    uB = np.tile(fB, (HB, 1))
    out = _transfer(uA, uB, HC, WC)
    for a in range(WA - 1):
        raw = np.array([fB[2 * a], fB[2 * a + 1], fB[2 * a + 2], fA[a], fA[a + 1]])
        q = rows["quarter"] @ raw
        t = rows["three_quarter"] @ raw
        for i in range(HC):
            assert abs(out[i, 4 * a + 1] - q) < 1e-12
            assert abs(out[i, 4 * a + 3] - t) < 1e-12
        # nodes: (5 u2 - u1)/4; half node: u2 + (d_i + d_{i+1})/8
        assert abs(out[3, 4 * a] - (5 * fB[2 * a] - fA[a]) / 4) < 1e-12
        d0, d1 = fB[2 * a] - fA[a], fB[2 * a + 2] - fA[a + 1]
        assert abs(out[3, 4 * a + 2] - (fB[2 * a + 1] + (d0 + d1) / 8)) < 1e-12


def _biquadratic(rng):
    c = rng.standard_normal((3, 3))

    def f(x, y):
        X = [np.ones_like(x), x / 50, (x / 50) ** 2]
        Y = [np.ones_like(y), y / 50, (y / 50) ** 2]
        return sum(c[p, q] * X[p] * Y[q] for p in range(3) for q in range(3))
    return f


@pytest.mark.parametrize("HC,WC", [(33, 33), (32, 32), (34, 30), (31, 29), (20, 45)])
def test_quadratic_exactness(rng, HC, WC):
    # grid A node a sits at fine coordinate 4a, B node p at 2p, C node I at I
    f = _biquadratic(rng)
    (HA, WA), (HB, WB), _ = _grids(HC, WC)
    out = _transfer(_sample(f, HA, WA, 4), _sample(f, HB, WB, 2), HC, WC)
    np.testing.assert_allclose(out, _sample(f, HC, WC, 1), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("HC,WC", [(33, 33), (32, 32), (34, 30), (31, 29)])
def test_richardson_affine_exactness(rng, HC, WC):
    # u_B = q + 4e, u_A = q + 16e with e affine: the extrapolation removes
    # the h^2 term and returns exactly q + e on the next level
    f = _biquadratic(rng)
    al, be, ga = rng.standard_normal(3)

    def e(x, y):
        return al + be * x / 40 + ga * y / 40
    (HA, WA), (HB, WB), _ = _grids(HC, WC)
    uA = _sample(lambda x, y: f(x, y) + 16 * e(x, y), HA, WA, 4)
    uB = _sample(lambda x, y: f(x, y) + 4 * e(x, y), HB, WB, 2)
    out = _transfer(uA, uB, HC, WC)
    np.testing.assert_allclose(out, _sample(lambda x, y: f(x, y) + e(x, y), HC, WC, 1), rtol=1e-11, atol=1e-11)


def test_transfer_linear_and_flip_equivariant(rng):
    (HA, WA), (HB, WB), (HC, WC) = _grids(33, 33)
    X = [rng.standard_normal((HA, WA)), rng.standard_normal((HB, WB))]
    Y = [rng.standard_normal((HA, WA)), rng.standard_normal((HB, WB))]
    a, b = 1.7, -0.3
    lhs = _transfer(a * X[0] + b * Y[0], a * X[1] + b * Y[1], HC, WC)
    rhs = a * _transfer(*X, HC, WC) + b * _transfer(*Y, HC, WC)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    # odd sizes 4m+1: the panel structure is symmetric under reflection
    out = _transfer(*X, HC, WC)
    np.testing.assert_allclose(_transfer(X[0][::-1, ::-1], X[1][::-1, ::-1], HC, WC), out[::-1, ::-1],
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(_transfer(X[0].T, X[1].T, HC, WC), out.T, rtol=1e-12, atol=1e-12)


def test_linear_prolongation_eq15(rng):
    B = rng.standard_normal((5, 6))
    C = oracle.prolong_linear(B, 9, 11)
    np.testing.assert_array_equal(C[::2, ::2], B)
    assert abs(C[0, 1] - 0.5 * (B[0, 0] + B[0, 1])) < 1e-15
    assert abs(C[1, 0] - 0.5 * (B[0, 0] + B[1, 0])) < 1e-15
    # cell centres along the (a,b)-(a+1,b+1) diagonal
    assert abs(C[1, 1] - 0.5 * (B[0, 0] + B[1, 1])) < 1e-15
    assert abs(C[3, 5] - 0.5 * (B[1, 2] + B[2, 3])) < 1e-15
    # affine exactness, including the even-size border
    f = lambda x, y: 3.0 + 0.2 * x - 0.7 * y  # noqa: E731
    for HC, WC in [(9, 11), (10, 12)]:
        HB, WB = (HC + 1) // 2, (WC + 1) // 2
        out = oracle.prolong_linear(_sample(f, HB, WB, 2), HC, WC)
        np.testing.assert_allclose(out, _sample(f, HC, WC, 1), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- S (eq. 18-19)
def _wls_bruteforce(u, i, j, h=1.0):
    H, W = u.shape
    rows, ys, ws = [], [], []
    for s in (-1, 0, 1):
        for t in (-1, 0, 1):
            ii, jj = i + s, j + t
            if 0 <= ii < H and 0 <= jj < W:
                z = ((u[i, j] - u[ii, jj]) / h) ** 2
                w = 0.0 if z > 30 else np.exp(-z)
                rows.append([1.0, s, t]); ys.append(u[ii, jj]); ws.append(w)
    sw = np.sqrt(np.array(ws))
    coef, *_ = np.linalg.lstsq(np.array(rows) * sw[:, None], np.array(ys) * sw, rcond=None)
    return coef[0]


def test_local_smooth_matches_weighted_lstsq(rng):
    u = 100 + 1.5 * rng.standard_normal((12, 10))
    u[3:7, 2:5] += 40  # an edge: weights across it vanish
    u[9, 8] += 3.0
    out = oracle.local_smooth(u)
    for i in range(u.shape[0]):
        for j in range(u.shape[1]):
            assert abs(out[i, j] - _wls_bruteforce(u, i, j)) < 1e-9, (i, j)


def test_local_smooth_reproduces_affine_and_constant(rng):
    for slope in (0.3, 1.0, 8.0):
        ii, jj = np.meshgrid(np.arange(9.0), np.arange(11.0), indexing="ij")
        u = 50 + slope * ii - 0.5 * slope * jj
        np.testing.assert_allclose(oracle.local_smooth(u), u, rtol=1e-12, atol=1e-10)
    c = np.full((6, 7), 42.0)
    np.testing.assert_allclose(oracle.local_smooth(c), c, rtol=1e-15)


def test_local_smooth_scale_parameter(rng):
    u = 100 + 5 * rng.standard_normal((8, 8))
    # with a large h the weights are ~1 everywhere: plain least-squares plane fit
    out = oracle.local_smooth(u, h=1e8)
    ii, jj = 4, 4
    A = np.array([[1.0, s, t] for s in (-1, 0, 1) for t in (-1, 0, 1)])
    y = np.array([u[ii + s, jj + t] for s in (-1, 0, 1) for t in (-1, 0, 1)])
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    assert abs(out[ii, jj] - coef[0]) < 1e-9


# ---------------------------------------------------------------- D (eq. 21-26)
def test_pm_conserves_mass_and_max_principle(rng):
    u = rng.uniform(0, 255, size=(17, 23))
    out = oracle.pm_step(u, k=10.0, tau=0.25)
    assert abs(out.sum() - u.sum()) < 1e-9 * abs(u.sum())
    assert out.min() >= u.min() - 1e-12 and out.max() <= u.max() + 1e-12
    c = np.full((5, 6), 7.0)
    np.testing.assert_array_equal(oracle.pm_step(c), c)


def test_pm_large_k_is_heat_step(rng):
    # k -> infinity: c = 1 and D is the explicit 5-point heat step with
    # zero-flux (replicated) borders
    u = rng.uniform(0, 255, size=(13, 9))
    out = oracle.pm_step(u, k=1e30, tau=0.2)
    np.testing.assert_allclose(out, u + 0.2 * laplace(u, mode="nearest"), rtol=1e-13, atol=1e-11)


def test_pm_ramp_closed_form():
    # u = beta*i: interior |grad u| = beta, border rows beta/2 (replicated
    # central difference); interior fluxes cancel, the top row gains
    # tau*beta*(c + c_b)/2, the bottom row loses the same.
    beta, k, tau, H, W = 3.0, 4.0, 0.2, 8, 5
    u = beta * np.tile(np.arange(H, dtype=np.float64)[:, None], (1, W))
    out = oracle.pm_step(u, k=k, tau=tau)
    c = 1 / (1 + beta ** 2 / k ** 2)
    cb = 1 / (1 + (beta / 2) ** 2 / k ** 2)
    np.testing.assert_allclose(out[2:-2], u[2:-2], rtol=0, atol=1e-12)
    np.testing.assert_allclose(out[0], u[0] + tau * beta * (c + cb) / 2, rtol=1e-14, atol=1e-12)
    np.testing.assert_allclose(out[-1], u[-1] - tau * beta * (c + cb) / 2, rtol=1e-14, atol=1e-12)
