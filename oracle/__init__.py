"""EECMG oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.

NumPy/ctypes front end of ``eecmg_oracle.c``: a plain FP64 CPU implementation
of the extrapolation economy cascadic multigrid restoration of Chu, Yan and Li
(arXiv 2311.03010), written from the paper.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import this package; the HIP
library never calls it and shares no code with it.

Parity status per function (pins live in ``tests/test_oracle_*.py``):
  conv / conv_t          pinned (dense matrix, Kronecker form, FFT, adjoint)
  restrict / coarse_psf  pinned (bitwise injection, dense R H R^T, Gaussian
                         self-similarity)
  iteration_caps         pinned (hand-evaluated tables of the m_l rule)
  cgls / mr              pinned (Krylov least-squares minimiser, exact solve,
                         monotone residual, identity PSF)
  extrapolate / prolong  pinned (1-D coefficients printed in Section 3.2,
                         quadratic and Richardson-affine exactness)
  local_smooth           pinned (affine reproduction, brute-force lstsq)
  pm_step                pinned (mass conservation, maximum principle,
                         heat-step limit)
  restore                pinned on its composition (rebuilt from the pinned
                         operators in the order of Algorithms 1 and 2, bit for
                         bit), identity-PSF / zero-noise recovery and
                         symmetry; the paper's PSNR tables use an image that
                         is not available: parity unpinned for those values.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_SRC = os.path.join(_HERE, "eecmg_oracle.c")

STOP_NONE, STOP_DISCREPANCY, STOP_CAP, STOP_GUARD = 0, 1, 2, 3

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over pixel loops)."""
    import subprocess

    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-result",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    i, d, l = ctypes.c_int, ctypes.c_double, ctypes.c_long
    sig = {
        "or_dot": (d, [dp, dp, l]),
        "or_rms": (d, [dp, l]),
        "or_psnr": (d, [dp, dp, l]),
        "or_level_sizes": (i, [i, i, i, ip, ip]),
        "or_iteration_caps": (i, [i, ip]),
        "or_restrict": (None, [dp, i, i, dp, i, i]),
        "or_coarse_psf": (i, [dp, i, i, dp]),
        "or_conv": (None, [dp, i, i, dp, i, i, dp]),
        "or_cgls": (i, [dp, i, i, dp, i, dp, i, i, d, d, ip, dp, ip]),
        "or_mr": (i, [dp, i, i, dp, i, dp, i, i, d, d, ip, dp, ip]),
        "or_extrapolate": (i, [dp, i, i, dp, i, i, dp]),
        "or_prolong_quad": (i, [dp, i, i, dp, i, i]),
        "or_prolong_linear": (i, [dp, i, i, dp, i, i]),
        "or_local_smooth": (None, [dp, i, i, d, dp]),
        "or_pm_step": (None, [dp, i, i, d, d, dp]),
        "or_restore": (i, [dp, i, i, dp, i, i, ip, d, i, d, d, d, i, d, i, d, i, i, dp, ip, dp, ip, ip]),
        "or_num_threads": (i, []),
        "or_set_num_threads": (None, [i]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _psf(psf):
    psf = _f64(psf)
    n = psf.shape[0]
    if psf.ndim != 2 or psf.shape[1] != n or n % 2 != 1:
        raise ValueError("psf must be a square (2r+1)x(2r+1) array")
    return psf, (n - 1) // 2


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the pixel loops (the results do not depend on it)."""
    _load().or_set_num_threads(int(n))


def dot(x, y) -> float:
    x, y = _f64(x).ravel(), _f64(y).ravel()
    return float(_load().or_dot(_dp(x), _dp(y), x.size))


def rms(x) -> float:
    x = _f64(x).ravel()
    return float(_load().or_rms(_dp(x), x.size))


def psnr(u_true, u_hat) -> float:
    a, b = _f64(u_true).ravel(), _f64(u_hat).ravel()
    return float(_load().or_psnr(_dp(a), _dp(b), a.size))


def level_sizes(H: int, W: int, L: int):
    hs = np.zeros(L, np.int32)
    ws = np.zeros(L, np.int32)
    rc = _load().or_level_sizes(H, W, L, _ip(hs), _ip(ws))
    if rc != 0:
        raise ValueError(f"invalid level plan H={H} W={W} L={L}")
    return [(int(h), int(w)) for h, w in zip(hs, ws)]


def iteration_caps(L: int):
    m = np.zeros(L, np.int32)
    if _load().or_iteration_caps(L, _ip(m)) != 0:
        raise ValueError("L must be >= 1")
    return [int(v) for v in m]


def restrict(g_fine, Hc: int, Wc: int):
    g = _f64(g_fine)
    out = np.zeros((Hc, Wc))
    _load().or_restrict(_dp(g), g.shape[0], g.shape[1], _dp(out), Hc, Wc)
    return out


def coarse_psf(psf, mode: int = 0):
    psf, r = _psf(psf)
    rc = r // 2
    out = np.zeros((2 * rc + 1, 2 * rc + 1))
    if _load().or_coarse_psf(_dp(psf), r, mode, _dp(out)) != 0:
        raise ValueError("coarse psf undefined (zero decimated sum or bad mode)")
    return out


def conv(x, psf, transpose: bool = False):
    x = _f64(x)
    psf, r = _psf(psf)
    y = np.zeros_like(x)
    _load().or_conv(_dp(x), x.shape[0], x.shape[1], _dp(psf), r, 1 if transpose else 0, _dp(y))
    return y


def _smoother(name, g, psf, u0, cap, stop_rule, cdelta, eps):
    g = _f64(g)
    psf, r = _psf(psf)
    u = np.array(u0, dtype=np.float64, copy=True) if u0 is not None else np.zeros_like(g)
    hist = np.zeros(cap + 1)
    it = np.zeros(1, np.int32)
    why = np.zeros(1, np.int32)
    fn = getattr(_load(), name)
    rc = fn(_dp(g), g.shape[0], g.shape[1], _dp(psf), r, _dp(u), int(cap), 1 if stop_rule else 0, float(cdelta),
            float(eps), _ip(it), _dp(hist), _ip(why))
    if rc != 0:
        raise RuntimeError(f"{name} failed ({rc})")
    k = int(it[0])
    return u, k, hist[: k + 1].copy(), int(why[0])


def cgls(g, psf, u0=None, cap=10, stop_rule=False, cdelta=0.0, eps=0.0):
    """Returns (u, iterations, rms history, stop reason)."""
    return _smoother("or_cgls", g, psf, u0, cap, stop_rule, cdelta, eps)


def mr(g, psf, u0=None, cap=10, stop_rule=False, cdelta=0.0, eps=0.0):
    return _smoother("or_mr", g, psf, u0, cap, stop_rule, cdelta, eps)


def extrapolate(uA, uB):
    uA, uB = _f64(uA), _f64(uB)
    out = np.zeros_like(uB)
    rc = _load().or_extrapolate(_dp(uA), uA.shape[0], uA.shape[1], _dp(uB), uB.shape[0], uB.shape[1], _dp(out))
    if rc != 0:
        raise ValueError("extrapolate: incompatible sizes")
    return out


def prolong_quad(ut, HC: int, WC: int):
    ut = _f64(ut)
    out = np.zeros((HC, WC))
    if _load().or_prolong_quad(_dp(ut), ut.shape[0], ut.shape[1], _dp(out), HC, WC) != 0:
        raise ValueError("prolong_quad: incompatible sizes")
    return out


def prolong_linear(uB, HC: int, WC: int):
    uB = _f64(uB)
    out = np.zeros((HC, WC))
    if _load().or_prolong_linear(_dp(uB), uB.shape[0], uB.shape[1], _dp(out), HC, WC) != 0:
        raise ValueError("prolong_linear: incompatible sizes")
    return out


def local_smooth(u, h: float = 1.0):
    u = _f64(u)
    out = np.zeros_like(u)
    _load().or_local_smooth(_dp(u), u.shape[0], u.shape[1], float(h), _dp(out))
    return out


def pm_step(u, k: float = 10.0, tau: float = 0.2):
    u = _f64(u)
    out = np.zeros_like(u)
    _load().or_pm_step(_dp(u), u.shape[0], u.shape[1], float(k), float(tau), _dp(out))
    return out


def restore(g_delta, psf, n_levels, caps=None, k=10.0, stop_rule=True, delta=1.0, c=1.1, tau=0.2, pm_steps=1,
            smooth_h=1.0, coarse_psf_mode=0, guard_eps=1e-14, smoother=0, cascade=0):
    """Full cascade.  Returns (u, stats) with per-level iterations, final
    residual RMS, stop reason and PSF radius (coarsest first)."""
    g = _f64(g_delta)
    psf, r = _psf(psf)
    L = int(n_levels)
    H, W = g.shape
    u = np.zeros_like(g)
    it = np.zeros(L, np.int32)
    rm = np.zeros(L)
    why = np.zeros(L, np.int32)
    rad = np.zeros(L, np.int32)
    caps_arr = None
    if caps is not None:
        caps_arr = np.ascontiguousarray(caps, dtype=np.int32)
        if caps_arr.size != L:
            raise ValueError("caps must have n_levels entries")
    rc = _load().or_restore(_dp(g), H, W, _dp(psf), r, L, _ip(caps_arr) if caps_arr is not None else None,
                            float(k), 1 if stop_rule else 0, float(delta), float(c), float(tau), int(pm_steps),
                            float(smooth_h), int(coarse_psf_mode), float(guard_eps), int(smoother), int(cascade),
                            _dp(u), _ip(it), _dp(rm), _ip(why), _ip(rad))
    if rc != 0:
        raise ValueError(f"oracle restore failed ({rc})")
    stats = {"iters": [int(v) for v in it], "final_rms": [float(v) for v in rm],
             "reason": [int(v) for v in why], "radius": [int(v) for v in rad],
             "sizes": level_sizes(H, W, L),
             "caps": [int(v) for v in (caps_arr if caps_arr is not None else iteration_caps(L))]}
    return u, stats
