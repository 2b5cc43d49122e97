"""GPU parity of every operator entry point against the oracle, through the
C ABI.  FP64 results must match to ~1e-13 relative, FP32 to ~1e-6 (one FP32
rounding of inputs, taps and outputs); integer/copy work is bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2311_03010_amd import eecmg, synth

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 2e-6}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _dt(prec):
    return np.float64 if prec == "f64" else np.float32


def _dev(torch, a, prec):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=_dt(prec))).to("cuda:0")


def _close(got, ref, prec, what=""):
    got = np.asarray(got, dtype=np.float64)
    scale = max(np.abs(ref).max(), 1e-30)
    err = np.abs(got - ref).max() / scale
    assert err <= TOL[prec], f"{what}: max rel err {err:.3e}"


def _psf(kind, r, rng):
    """PSFs that select each blur-operator kernel family."""
    if kind == "general":  # no symmetry
        return rng.uniform(-0.2, 1.0, size=(2 * r + 1, 2 * r + 1))
    if kind == "separable":  # rank one (Gaussian)
        return synth.gaussian_psf(max(r, 1) / 2.5, r)
    if kind == "disk":  # uniform disk (out-of-focus blur): the uniform-disk kernels
        return synth.disk_psf(r)
    # symmetric in both axes, full square support ("symsq") or disk support
    # with unequal weights ("symdisk")
    q = rng.uniform(0.0, 1.0, size=(r + 1, r + 1))
    full = np.zeros((2 * r + 1, 2 * r + 1))
    for a in range(-r, r + 1):
        for b in range(-r, r + 1):
            if kind == "symsq" or a * a + b * b <= r * r:
                full[a + r, b + r] = q[abs(a), abs(b)]
    return full / full.sum()


CONV_CASES = [("general", 37, 70, 0), ("general", 64, 64, 1), ("general", 97, 130, 3), ("general", 33, 200, 6),
              ("general", 130, 65, 7), ("general", 70, 70, 12), ("general", 5, 3, 2), ("general", 1, 1, 4),
              ("separable", 37, 70, 0), ("separable", 97, 130, 4), ("separable", 130, 200, 7),
              ("separable", 70, 33, 12), ("disk", 65, 129, 1), ("disk", 97, 130, 3), ("disk", 200, 130, 6),
              ("disk", 33, 70, 8), ("disk", 300, 77, 5), ("disk", 2, 70, 2), ("symdisk", 65, 129, 1),
              ("symdisk", 97, 130, 3), ("symdisk", 200, 130, 6), ("symdisk", 33, 70, 8), ("symsq", 97, 130, 2),
              ("symsq", 64, 200, 6), ("symsq", 3, 5, 1)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,H,W,r", CONV_CASES)
@pytest.mark.parametrize("transpose", [False, True])
def test_conv_parity(torch_cuda, prec, kind, H, W, r, transpose):
    rng = np.random.Generator(np.random.PCG64(H * 1000 + W * 10 + r))
    psf = _psf(kind, r, rng)
    x = rng.uniform(0, 255, size=(H, W)).astype(_dt(prec)).astype(np.float64)
    psf_used = psf.astype(_dt(prec)).astype(np.float64)
    y = eecmg.conv_dev(_dev(torch_cuda, x, prec), psf, transpose=transpose, precision=prec)
    ref = oracle.conv(x, psf_used, transpose=transpose)
    # elementwise bound of a recursive/FMA sum of n terms: n u sum |w x|
    unit = 2.0 ** -53 if prec == "f64" else 2.0 ** -24
    n = (2 * r + 1) ** 2
    bound = (n + 2) * unit * oracle.conv(np.abs(x), np.abs(psf_used), transpose=transpose) + 1e-300
    err = np.abs(y.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound), f"conv {kind} {H}x{W} r={r} T={transpose}: worst ratio {np.max(err / bound):.3f}"


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("H,W", [(64, 64), (37, 101), (3, 3), (4096, 4096)])
def test_restrict_bitwise(torch_cuda, prec, H, W):
    rng = np.random.Generator(np.random.PCG64(7))
    g = rng.standard_normal((H, W)).astype(_dt(prec))
    out = eecmg.restrict_dev(_dev(torch_cuda, g, prec), precision=prec).cpu().numpy()
    np.testing.assert_array_equal(out, g[::2, ::2])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("HC,WC", [(33, 33), (32, 32), (34, 30), (129, 70), (1026, 515)])
def test_transfer_operators_parity(torch_cuda, prec, HC, WC):
    rng = np.random.Generator(np.random.PCG64(HC * 7 + WC))
    HB, WB = (HC + 1) // 2, (WC + 1) // 2
    HA, WA = (HB + 1) // 2, (WB + 1) // 2
    uA = rng.uniform(0, 255, size=(HA, WA)).astype(_dt(prec)).astype(np.float64)
    uB = rng.uniform(0, 255, size=(HB, WB)).astype(_dt(prec)).astype(np.float64)
    t = torch_cuda
    ut = eecmg.extrapolate_dev(_dev(t, uA, prec), _dev(t, uB, prec), precision=prec)
    _close(ut.cpu().numpy(), oracle.extrapolate(uA, uB), prec, "extrapolate")
    ut_host = ut.cpu().numpy().astype(np.float64)
    uC = eecmg.prolong_quad_dev(ut, HC, WC, precision=prec)
    _close(uC.cpu().numpy(), oracle.prolong_quad(ut_host, HC, WC), prec, "prolong_quad")
    uL = eecmg.prolong_linear_dev(_dev(t, uB, prec), HC, WC, precision=prec)
    _close(uL.cpu().numpy(), oracle.prolong_linear(uB, HC, WC), prec, "prolong_linear")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("H,W", [(40, 40), (67, 131), (3, 5), (515, 1030)])
def test_smooth_and_denoise_parity(torch_cuda, prec, H, W):
    rng = np.random.Generator(np.random.PCG64(H + 17 * W))
    u = 100 + 2.0 * rng.standard_normal((H, W))
    u[H // 4: H // 2, W // 3: W // 2] += 60.0  # edges: weights cut off
    u = u.astype(_dt(prec)).astype(np.float64)
    t = torch_cuda
    for hs in (1.0, 3.0):
        s = eecmg.local_smooth_dev(_dev(t, u, prec), smooth_h=hs, precision=prec)
        _close(s.cpu().numpy(), oracle.local_smooth(u, hs), prec, f"local_smooth h={hs}")
    for k, tau in ((10.0, 0.2), (2.0, 0.25)):
        d = eecmg.pm_step_dev(_dev(t, u, prec), k=k, tau=tau, precision=prec)
        _close(d.cpu().numpy(), oracle.pm_step(u, k, tau), prec, f"pm_step k={k}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("prolong", ["quad", "linear"])
@pytest.mark.parametrize("HC,WC", [(5, 5), (33, 33), (34, 30), (129, 70), (97, 200), (515, 1030)])
def test_fused_transfer_parity(torch_cuda, prec, prolong, HC, WC):
    """The fused prolongation -> S (-> D) kernel against (a) the separate
    operator kernels run in sequence (bit-identical) and (b) the oracle's
    operators composed with the same rounding to the storage precision
    between stages.  Sizes span several 64 x 32 tiles, ragged edges and the
    smallest grid the quadratic interpolation allows."""
    rng = np.random.Generator(np.random.PCG64(HC * 31 + WC + (prolong == "quad")))
    HB, WB = (HC + 1) // 2, (WC + 1) // 2
    ub = 100 + 3.0 * rng.standard_normal((HB, WB))
    ub[HB // 4: HB // 2, WB // 3: WB // 2] += 50.0  # an edge: S weights cut off, D slows down
    ub = ub.astype(_dt(prec)).astype(np.float64)
    t = torch_cuda
    dt = _dt(prec)
    for hs, steps, k, tau in ((1.0, 1, 10.0, 0.2), (2.5, 0, 10.0, 0.2), (0.7, 1, 3.0, 0.25)):
        got = eecmg.transfer_dev(_dev(t, ub, prec), HC, WC, prolongation=prolong, smooth_h=hs, pm_steps=steps, k=k,
                                 tau=tau, precision=prec).cpu().numpy()
        # (a) separate kernels
        if prolong == "quad":
            x = eecmg.prolong_quad_dev(_dev(t, ub, prec), HC, WC, precision=prec)
        else:
            x = eecmg.prolong_linear_dev(_dev(t, ub, prec), HC, WC, precision=prec)
        x = eecmg.local_smooth_dev(x, smooth_h=hs, precision=prec)
        if steps:
            x = eecmg.pm_step_dev(x, k=k, tau=tau, precision=prec)
        np.testing.assert_array_equal(got, x.cpu().numpy(), err_msg=f"fused != separate (h={hs}, D steps {steps})")
        # (b) oracle, rounded to the storage precision between stages
        y = oracle.prolong_quad(ub, HC, WC) if prolong == "quad" else oracle.prolong_linear(ub, HC, WC)
        y = oracle.local_smooth(y.astype(dt).astype(np.float64), hs)
        if steps:
            y = oracle.pm_step(y.astype(dt).astype(np.float64), k, tau)
        _close(got, y, prec, f"fused transfer h={hs} steps={steps}")


def test_operator_errors(torch_cuda):
    t = torch_cuda
    x = t.zeros((8, 8), dtype=t.float32, device="cuda:0")
    with pytest.raises(eecmg.EecmgError) as e:
        eecmg.conv_dev(x, np.ones((27, 27)))  # radius 13 > 12
    assert e.value.status == eecmg.EINVAL
    with pytest.raises(eecmg.EecmgError):
        eecmg.pm_step_dev(x, k=10.0, tau=0.3)
    with pytest.raises(eecmg.EecmgError):
        eecmg.local_smooth_dev(x, smooth_h=0.0)
    with pytest.raises(eecmg.EecmgError):
        eecmg.transfer_dev(x, 16, 16, pm_steps=2)
    with pytest.raises(eecmg.EecmgError):
        eecmg.transfer_dev(x, 4, 4)  # the quadratic interpolation needs 3 coarse nodes per axis
