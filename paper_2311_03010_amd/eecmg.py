"""Python binding of libeecmg.so (the C ABI in include/eecmg.h).

Argument marshalling only: every step of the restoration runs in the HIP
library.  PyTorch is used for device memory and streams.  If the library is
not built, every call raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeecmg.so")
MAX_LEVELS = 16
MAX_SLOTS = 240

OK, PENDING, EINVAL, ENOMEM, EAGAIN, EDEVICE, ENOTFOUND, ENUMERIC, ECANCELED = 0, 1, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "EINVAL", -2: "ENOMEM", -3: "EAGAIN", -4: "EDEVICE", -5: "ENOTFOUND",
                -6: "ENUMERIC", -7: "ECANCELED"}
PRECISIONS = {"f64": 0, "f32": 1, "f32_f16coarse": 2}
CASCADES = {"eecmg": 0, "iecmg_l": 1, "iecmg_p": 2}
SMOOTHERS = {"cgls": 0, "mr": 1}
STOP_NAMES = {0: "none", 1: "discrepancy", 2: "cap", 3: "guard", 4: "nonfinite"}


class EecmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32), ("stop_rule", ctypes.c_int32),
                ("delta", ctypes.c_double), ("c", ctypes.c_double), ("tau", ctypes.c_double),
                ("pm_steps", ctypes.c_int32), ("smooth_h", ctypes.c_double), ("coarse_psf_mode", ctypes.c_int32),
                ("guard_eps", ctypes.c_double), ("smoother", ctypes.c_int32), ("cascade", ctypes.c_int32),
                ("stats", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_levels", ctypes.c_int32),
                ("level_h", ctypes.c_int32 * MAX_LEVELS), ("level_w", ctypes.c_int32 * MAX_LEVELS),
                ("psf_radius", ctypes.c_int32 * MAX_LEVELS), ("caps", ctypes.c_int32 * MAX_LEVELS),
                ("iters", ctypes.c_int32 * MAX_LEVELS), ("stop_reason", ctypes.c_int32 * MAX_LEVELS),
                ("final_rms", ctypes.c_double * MAX_LEVELS)]

    def to_dict(self):
        L = self.n_levels
        # (slicing a ctypes array returns a list)
        return {"sizes": list(zip(self.level_h[:L], self.level_w[:L])),
                "radius": self.psf_radius[:L], "caps": self.caps[:L], "iters": self.iters[:L],
                "reason": self.stop_reason[:L], "final_rms": self.final_rms[:L]}


class CtxConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t),
                ("max_slots", ctypes.c_int32), ("max_queue", ctypes.c_int32)]


_lib = None


def lib():
    """Load libeecmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp, i, d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double
    sig = {
        "eecmg_params_default": [ctypes.POINTER(Params)],
        "eecmg_restore": [vp, i, i, dp, i, i, ip, d, ctypes.POINTER(Params), vp],
        # (the per-call device entry points take every pointer as an address)
        "eecmg_restore_dev": [vp, i, i, vp, i, i, vp, d, vp, vp, vp],
        "eecmg_restore_dev_noalloc": [vp, i, i, vp, i, i, vp, d, vp, vp, vp],
        "eecmg_restore_batch_dev": [i, ctypes.POINTER(vp), ip, ip, ctypes.POINTER(dp), ip, ip, ctypes.POINTER(ip), dp,
                                    ctypes.POINTER(Params), ctypes.POINTER(vp), vp],
        "eecmg_ctx_config_default": [ctypes.POINTER(CtxConfig)],
        "eecmg_create": [ctypes.POINTER(CtxConfig), ctypes.POINTER(vp)],
        "eecmg_submit": [vp, vp, i, i, dp, i, i, ip, d, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_uint64)],
        "eecmg_poll": [vp, ctypes.c_uint64, vp, ctypes.POINTER(Stats)],
        "eecmg_wait": [vp, ctypes.c_uint64, vp, ctypes.POINTER(Stats)],
        "eecmg_cancel": [vp, ctypes.c_uint64],
        "eecmg_ctx_info": [vp, ip, ip, ctypes.POINTER(ctypes.c_size_t)],
        "eecmg_destroy": [vp],
        "eecmg_op_conv_dev": [vp, vp, i, i, dp, i, i, i, vp],
        "eecmg_op_smoother_dev": [vp, vp, i, i, dp, i, i, ctypes.POINTER(Params), ctypes.POINTER(Stats), vp],
        "eecmg_op_restrict_dev": [vp, i, i, vp, i, vp],
        "eecmg_op_coarse_psf": [dp, i, i, dp],
        "eecmg_op_extrapolate_dev": [vp, vp, i, i, vp, i, vp],
        "eecmg_op_prolong_quad_dev": [vp, i, i, vp, i, vp],
        "eecmg_op_prolong_linear_dev": [vp, i, i, vp, i, vp],
        "eecmg_op_local_smooth_dev": [vp, vp, i, i, d, i, vp],
        "eecmg_op_pm_step_dev": [vp, vp, i, i, d, d, i, vp],
        "eecmg_op_transfer_dev": [vp, i, i, vp, i, d, i, d, d, i, vp],
        "eecmg_profile_enable": [i, i],
        "eecmg_profile_min_pixels": [d],
        "eecmg_profile_reset": [],
        "eecmg_profile_read": [i, ip, dp, dp],
        "eecmg_profile_read_level": [i, i, ip, dp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.eecmg_last_error.restype = ctypes.c_char_p
    L.eecmg_last_error.argtypes = []
    L.eecmg_version.restype = ctypes.c_char_p
    L.eecmg_version.argtypes = []
    _lib = L
    return L


def exported_symbols():
    return [n for n in dir(lib()) if n.startswith("eecmg_")]


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        msg = lib().eecmg_last_error().decode(errors="replace")
        raise EecmgError(rc, msg)
    return rc


def _psf_arr(psf):
    psf = np.ascontiguousarray(psf, dtype=np.float64)
    n = psf.shape[0]
    if psf.ndim != 2 or psf.shape[1] != n or n % 2 != 1:
        raise ValueError("psf must be a square (2r+1)x(2r+1) array")
    return psf, (n - 1) // 2


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _caps_arr(caps, L):
    if caps is None:
        return None
    c = np.ascontiguousarray(caps, dtype=np.int32)
    if c.size != L:
        raise ValueError("caps must have n_levels entries")
    return c


def make_params(precision="f32", stop_rule=True, delta=1.0, c=1.1, tau=0.2, pm_steps=1, smooth_h=1.0,
                coarse_psf_mode=0, guard_eps=0.0, smoother="cgls", cascade="eecmg") -> Params:
    p = Params()
    _check(lib().eecmg_params_default(ctypes.byref(p)))
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.stop_rule = 1 if stop_rule else 0
    p.delta = float(delta)
    p.c = float(c)
    p.tau = float(tau)
    p.pm_steps = int(pm_steps)
    p.smooth_h = float(smooth_h)
    p.coarse_psf_mode = int(coarse_psf_mode)
    p.guard_eps = float(guard_eps)
    p.smoother = SMOOTHERS[smoother] if isinstance(smoother, str) else int(smoother)
    p.cascade = CASCADES[cascade] if isinstance(cascade, str) else int(cascade)
    return p


def np_dtype(precision):
    return np.float64 if (precision == "f64" or precision == 0) else np.float32


def restore(g_delta, psf, n_levels, caps=None, k=10.0, **kw):
    """Host-buffer restore.  Returns (u, stats dict)."""
    p = make_params(**kw)
    st = Stats()
    st.struct_size = ctypes.sizeof(Stats)
    p.stats = ctypes.cast(ctypes.pointer(st), ctypes.c_void_p)
    dt = np_dtype(kw.get("precision", "f32"))
    g = np.ascontiguousarray(g_delta, dtype=dt)
    u = np.empty_like(g)
    psf, r = _psf_arr(psf)
    c = _caps_arr(caps, n_levels)
    rc = lib().eecmg_restore(g.ctypes.data, g.shape[0], g.shape[1], _dptr(psf), r, int(n_levels),
                             c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if c is not None else None, float(k),
                             ctypes.byref(p), u.ctypes.data)
    _check(rc)
    return u, st.to_dict()


def _stream_handle(stream):
    """The raw HIP stream of a torch stream, else of the current device's
    current stream (read without building a torch.cuda.Stream object where
    torch offers that)."""
    import torch

    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return ctypes.c_void_p(raw(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _torch_dtype(precision):
    import torch

    return torch.float64 if (precision == "f64" or precision == 0) else torch.float32


def restore_dev(g_delta, psf, n_levels, caps=None, k=10.0, out=None, stream=None, noalloc=False, **kw):
    """Device restore on torch tensors (contiguous H x W on the current GPU).
    Returns (u tensor, stats dict); the result is ready after the stream
    synchronises.  noalloc=True calls eecmg_restore_dev_noalloc (no device
    allocation; images up to the library's fixed scratch region)."""
    import torch

    prec = kw.get("precision", "f32")
    dt = _torch_dtype(prec)
    if g_delta.dtype != dt or not g_delta.is_cuda or not g_delta.is_contiguous():
        raise ValueError(f"g_delta must be a contiguous {dt} CUDA tensor")
    if out is None:
        out = torch.empty_like(g_delta)
    p = _params_for(kw)
    st = Stats()
    st.struct_size = ctypes.sizeof(Stats)
    p.stats = ctypes.addressof(st)
    psf, r = _psf_arr(psf)
    c = _caps_arr(caps, n_levels)
    fn = lib().eecmg_restore_dev_noalloc if noalloc else lib().eecmg_restore_dev
    rc = fn(g_delta.data_ptr(), g_delta.shape[0], g_delta.shape[1], psf.__array_interface__["data"][0], r,
            int(n_levels), c.__array_interface__["data"][0] if c is not None else None, float(k),
            ctypes.addressof(p), out.data_ptr(), _stream_handle(stream))
    _check(rc)
    return out, st.to_dict()


_PARAMS_CACHE = {}


def _params_for(kw):
    """A fresh eecmg_params struct for these keyword arguments (copied from a
    cached one: filling the struct field by field costs more than the copy)."""
    try:
        key = tuple(sorted(kw.items()))
        t = _PARAMS_CACHE.get(key)
    except TypeError:  # an unhashable value: no caching
        return make_params(**kw)
    if t is None:
        t = make_params(**kw)
        if len(_PARAMS_CACHE) < 256:
            _PARAMS_CACHE[key] = t
    return Params.from_buffer_copy(t)


def _override_params(p, kv):
    """Set the given fields of an eecmg_params struct (as make_params does)."""
    for k, v in kv.items():
        conv = _PARAM_CONV.get(k)
        if conv is None:
            raise TypeError(f"unknown parameter {k!r}")
        setattr(p, k, conv(v))


_PARAM_CONV = {
    "precision": lambda v: PRECISIONS[v] if isinstance(v, str) else int(v),
    "stop_rule": lambda v: 1 if v else 0,
    "delta": float, "c": float, "tau": float, "pm_steps": int, "smooth_h": float, "coarse_psf_mode": int,
    "guard_eps": float,
    "smoother": lambda v: SMOOTHERS[v] if isinstance(v, str) else int(v),
    "cascade": lambda v: CASCADES[v] if isinstance(v, str) else int(v),
}


def restore_batch_dev(gs, psfs, n_levels, caps=None, ks=None, outs=None, stream=None, params=None, **kw):
    """Batched device restore of a list of tensors with per-image PSFs and
    level counts.  params: optional list of per-image keyword dicts (override
    kw).  Returns (list of outputs, list of stats dicts)."""
    import torch

    n = len(gs)
    if outs is None:
        outs = [torch.empty_like(g) for g in gs]
    # one default struct with kw applied, copied per image and overridden
    # with that image's params (marshalling stays small next to the cascade)
    base = make_params(**kw)
    P = (Params * n)()
    sts = (Stats * n)()
    stats_size = ctypes.sizeof(Stats)
    psf_arrs, radii = [], []
    for i in range(n):
        P[i] = base
        pi = P[i]
        if params is not None and params[i]:
            _override_params(pi, params[i])
        sts[i].struct_size = stats_size
        pi.stats = ctypes.addressof(sts[i])
        a, r = _psf_arr(psfs[i])
        psf_arrs.append(a)
        radii.append(r)
    vp = ctypes.c_void_p
    g_ptrs = (vp * n)(*[g.data_ptr() for g in gs])
    o_ptrs = (vp * n)(*[o.data_ptr() for o in outs])
    Hs = (ctypes.c_int * n)(*[g.shape[0] for g in gs])
    Ws = (ctypes.c_int * n)(*[g.shape[1] for g in gs])
    psf_ptrs = ctypes.cast((vp * n)(*[a.ctypes.data for a in psf_arrs]),
                           ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))
    rads = (ctypes.c_int * n)(*radii)
    Ls = (ctypes.c_int * n)(*[int(x) for x in n_levels])
    kk = (ctypes.c_double * n)(*[float(x) for x in (ks if ks is not None else [10.0] * n)])
    caps_keep = []
    caps_ptrs = None
    if caps is not None:
        caps_ptrs = (ctypes.POINTER(ctypes.c_int) * n)()
        for i in range(n):
            if caps[i] is not None:
                c = _caps_arr(caps[i], n_levels[i])
                caps_keep.append(c)
                caps_ptrs[i] = c.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    rc = lib().eecmg_restore_batch_dev(n, g_ptrs, Hs, Ws, psf_ptrs, rads, Ls, caps_ptrs, kk, P, o_ptrs,
                                       _stream_handle(stream))
    _check(rc)
    return outs, [s.to_dict() for s in sts]


# ------------------------------------------------------------------ operators
def _prec_code(precision):
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def conv_dev(x, psf, transpose=False, precision="f32", out=None, stream=None):
    import torch

    out = torch.empty_like(x) if out is None else out
    psf, r = _psf_arr(psf)
    _check(lib().eecmg_op_conv_dev(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), x.shape[0],
                                   x.shape[1], _dptr(psf), r, 1 if transpose else 0, _prec_code(precision),
                                   _stream_handle(stream)))
    return out


def smoother_dev(g, u0, psf, cap, stream=None, **kw):
    """One level of the smoother from u0 (updated in place).  Returns (u, stats)."""
    p = make_params(**kw)
    st = Stats()
    st.struct_size = ctypes.sizeof(Stats)
    psf, r = _psf_arr(psf)
    _check(lib().eecmg_op_smoother_dev(ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(u0.data_ptr()), g.shape[0],
                                       g.shape[1], _dptr(psf), r, int(cap), ctypes.byref(p), ctypes.byref(st),
                                       _stream_handle(stream)))
    d = st.to_dict()
    return u0, {"iters": d["iters"][0], "reason": d["reason"][0], "final_rms": d["final_rms"][0]}


def restrict_dev(g, precision="f32", stream=None):
    import torch

    Hc, Wc = (g.shape[0] + 1) // 2, (g.shape[1] + 1) // 2
    out = torch.empty((Hc, Wc), dtype=g.dtype, device=g.device)
    _check(lib().eecmg_op_restrict_dev(ctypes.c_void_p(g.data_ptr()), g.shape[0], g.shape[1],
                                       ctypes.c_void_p(out.data_ptr()), _prec_code(precision), _stream_handle(stream)))
    return out


def coarse_psf(psf, mode=0):
    psf, r = _psf_arr(psf)
    rc = r // 2
    out = np.zeros((2 * rc + 1, 2 * rc + 1))
    _check(lib().eecmg_op_coarse_psf(_dptr(psf), r, int(mode), _dptr(out)))
    return out


def extrapolate_dev(uA, uB, precision="f32", stream=None):
    import torch

    out = torch.empty_like(uB)
    _check(lib().eecmg_op_extrapolate_dev(ctypes.c_void_p(uA.data_ptr()), ctypes.c_void_p(uB.data_ptr()), uB.shape[0],
                                          uB.shape[1], ctypes.c_void_p(out.data_ptr()), _prec_code(precision),
                                          _stream_handle(stream)))
    return out


def prolong_quad_dev(ut, HC, WC, precision="f32", stream=None):
    import torch

    out = torch.empty((HC, WC), dtype=ut.dtype, device=ut.device)
    _check(lib().eecmg_op_prolong_quad_dev(ctypes.c_void_p(ut.data_ptr()), HC, WC, ctypes.c_void_p(out.data_ptr()),
                                           _prec_code(precision), _stream_handle(stream)))
    return out


def prolong_linear_dev(uB, HC, WC, precision="f32", stream=None):
    import torch

    out = torch.empty((HC, WC), dtype=uB.dtype, device=uB.device)
    _check(lib().eecmg_op_prolong_linear_dev(ctypes.c_void_p(uB.data_ptr()), HC, WC, ctypes.c_void_p(out.data_ptr()),
                                             _prec_code(precision), _stream_handle(stream)))
    return out


def local_smooth_dev(u, smooth_h=1.0, precision="f32", stream=None):
    import torch

    out = torch.empty_like(u)
    _check(lib().eecmg_op_local_smooth_dev(ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), u.shape[0],
                                           u.shape[1], float(smooth_h), _prec_code(precision), _stream_handle(stream)))
    return out


def pm_step_dev(u, k=10.0, tau=0.2, precision="f32", stream=None):
    import torch

    out = torch.empty_like(u)
    _check(lib().eecmg_op_pm_step_dev(ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), u.shape[0],
                                      u.shape[1], float(k), float(tau), _prec_code(precision), _stream_handle(stream)))
    return out


def transfer_dev(ub, HC, WC, prolongation="quad", smooth_h=1.0, pm_steps=1, k=10.0, tau=0.2, precision="f32",
                 stream=None):
    """Fused prolongation (quadratic or linear) -> S -> pm_steps (0/1) D steps."""
    import torch

    out = torch.empty((HC, WC), dtype=ub.dtype, device=ub.device)
    _check(lib().eecmg_op_transfer_dev(ctypes.c_void_p(ub.data_ptr()), HC, WC, ctypes.c_void_p(out.data_ptr()),
                                       0 if prolongation == "quad" else 1, float(smooth_h), int(pm_steps), float(k),
                                       float(tau), _prec_code(precision), _stream_handle(stream)))
    return out


# ------------------------------------------------------------ kernel timing
STAGES = {"restrict": 0, "cg_init_r": 1, "cg_init_s": 2, "cg_fin_init": 3, "cg_pass_a": 4, "cg_fin_a": 5,
          "cg_pass_b": 6, "cg_fin_b": 7, "mr_init": 8, "mr_fin_init": 9, "mr_pass": 10, "mr_fin": 11,
          "extrapolate": 12, "prolong_quad": 13, "prolong_linear": 14, "local_smooth": 15, "pm_step": 16,
          "out_copy": 17, "transfer_fused": 18, "transfer_fused_small": 19, "flush_u": 21}


def profile_enable(enable=True, min_blocks=0, min_pixels=0.0):
    """Time launches of at least min_blocks blocks whose levels hold at least
    min_pixels pixels (summed over the jobs of the launch)."""
    _check(lib().eecmg_profile_min_pixels(float(min_pixels)))
    _check(lib().eecmg_profile_enable(1 if enable else 0, int(min_blocks)))


def profile_reset():
    _check(lib().eecmg_profile_reset())


def profile_read(stage):
    """(launches, total_ms, total_pixels) of one stage since the last reset."""
    n, ms, px = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    sid = STAGES[stage] if isinstance(stage, str) else int(stage)
    _check(lib().eecmg_profile_read(sid, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(px)))
    return n.value, ms.value, px.value


def profile_read_level(level, stage=None):
    """(launches, total_ms) of the launches working on level index `level`
    (0 = coarsest) since the last reset: one stage, or all (stage None)."""
    n, ms = ctypes.c_int(), ctypes.c_double()
    sid = -1 if stage is None else (STAGES[stage] if isinstance(stage, str) else int(stage))
    _check(lib().eecmg_profile_read_level(sid, int(level), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ------------------------------------------------------------ request loop
@dataclass
class Request:
    id: int
    shape: tuple
    dtype: type


class Context:
    """Continuous-batching request loop (eecmg_create / submit / poll)."""

    def __init__(self, device=0, hbm_budget_bytes=8 << 30, max_slots=64, max_queue=4096):
        cfg = CtxConfig()
        _check(lib().eecmg_ctx_config_default(ctypes.byref(cfg)))
        cfg.device = device
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.max_slots = max_slots
        cfg.max_queue = max_queue
        h = ctypes.c_void_p()
        _check(lib().eecmg_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def submit(self, g_delta, psf, n_levels, caps=None, k=10.0, **kw) -> Request:
        p = make_params(**kw)
        dt = np_dtype(kw.get("precision", "f32"))
        g = np.ascontiguousarray(g_delta, dtype=dt)
        psf, r = _psf_arr(psf)
        c = _caps_arr(caps, n_levels)
        rid = ctypes.c_uint64()
        _check(lib().eecmg_submit(self._h, g.ctypes.data, g.shape[0], g.shape[1], _dptr(psf), r, int(n_levels),
                                  c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if c is not None else None, float(k),
                                  ctypes.byref(p), ctypes.byref(rid)))
        return Request(rid.value, g.shape, dt)

    def poll(self, req: Request, out=None):
        """None while pending, else (u, stats).  out: optional preallocated
        array of the request's shape and dtype that receives u."""
        u = np.empty(req.shape, dtype=req.dtype) if out is None else out
        if u.shape != tuple(req.shape) or u.dtype != req.dtype or not u.flags.c_contiguous:
            raise ValueError("out must be a contiguous array of the request's shape and dtype")
        st = Stats()
        rc = lib().eecmg_poll(self._h, req.id, u.ctypes.data, ctypes.byref(st))
        if rc == PENDING:
            return None
        _check(rc)
        return u, st.to_dict()

    def wait(self, req: Request, out=None):
        """Block until the request finishes; (u, stats).  out: optional
        preallocated array of the request's shape and dtype."""
        u = np.empty(req.shape, dtype=req.dtype) if out is None else out
        if u.shape != tuple(req.shape) or u.dtype != req.dtype or not u.flags.c_contiguous:
            raise ValueError("out must be a contiguous array of the request's shape and dtype")
        st = Stats()
        _check(lib().eecmg_wait(self._h, req.id, u.ctypes.data, ctypes.byref(st)))
        return u, st.to_dict()

    def cancel(self, req: Request):
        _check(lib().eecmg_cancel(self._h, req.id))

    def info(self):
        q, a, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(lib().eecmg_ctx_info(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(b)))
        return {"queued": q.value, "active": a.value, "bytes_in_use": b.value}

    def close(self):
        if self._h:
            _check(lib().eecmg_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
