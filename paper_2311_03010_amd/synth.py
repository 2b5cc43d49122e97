"""Seeded synthetic workloads shaped like the paper's restoration experiments.

The paper restores one unnamed natural image under Gaussian blur and
Gaussian noise (Section 5); that image is not available, so these inputs
stand in for it.  This module only builds inputs -- scenes, PSFs, blurred
noisy data -- and holds none of the restoration method's arithmetic.  Both
the HIP path's tests/benchmark and the CPU oracle's tests take their inputs
from here.

Scene recipe (piecewise constant, like the paper's test images):
  * a linear ramp background a + b*i/(H-1) + c*j/(W-1), a, b, c ~ U[0, 64];
  * shapes painted in order (later ones overwrite): rectangle or disk with
    probability 1/2 each, centre uniform, size log-uniform in
    [max(2, min(H,W)/64), min(H,W)/6], intensity ~ U[0, 255];
  * optionally sinusoidal texture patches 20 sin(2 pi (fx x + fy y) + phi),
    f ~ U[1/32, 1/4] cycles/pixel, inside random rectangles.
Degradation (eq. 1, 8): g = psf * u (zero boundary, computed with SciPy's FFT
convolution in FP64) plus e ~ N(0, 1); delta = RMS(e) (eq. 10).
Random streams: NumPy PCG64 seeded with 2311030100 + workload id (+1000 i for
the i-th image of a multi-image workload).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2311030100


# --------------------------------------------------------------------------
# PSFs (Section 5 blur; disk PSF for the out-of-focus workload)
# --------------------------------------------------------------------------
def gaussian_psf(sigma: float, r: int) -> np.ndarray:
    """Truncated Gaussian h(t) ~ exp(-t^2 / (2 sigma^2)), |t| <= r, normalised
    to unit sum, and its Kronecker square (the paper's H = h (x) h)."""
    t = np.arange(-r, r + 1, dtype=np.float64)
    h = np.exp(-(t * t) / (2.0 * sigma * sigma))
    h /= h.sum()
    return np.outer(h, h)


def disk_psf(r: int) -> np.ndarray:
    """Uniform out-of-focus disk: 1/n on a^2 + b^2 <= r^2 (n taps)."""
    a = np.arange(-r, r + 1)
    m = (a[:, None] ** 2 + a[None, :] ** 2) <= r * r
    p = m.astype(np.float64)
    return p / p.sum()


def blur(u: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """psf * u with zero boundary conditions ('same' size, FP64)."""
    from scipy.signal import fftconvolve

    return fftconvolve(u, psf, mode="same")


# --------------------------------------------------------------------------
# Scenes
# --------------------------------------------------------------------------
def scene(H: int, W: int, n_shapes: int, rng: np.random.Generator, n_textures: int = 0,
          texture_amp: float = 20.0) -> np.ndarray:
    a, b, c = rng.uniform(0.0, 64.0, size=3)
    ii = np.arange(H, dtype=np.float64)[:, None]
    jj = np.arange(W, dtype=np.float64)[None, :]
    u = a + b * ii / max(H - 1, 1) + c * jj / max(W - 1, 1)
    u = np.ascontiguousarray(np.broadcast_to(u, (H, W)), dtype=np.float64).copy()
    m = min(H, W)
    lo, hi = max(2.0, m / 64.0), max(m / 6.0, 2.5)
    for _ in range(n_shapes):
        is_rect = rng.random() < 0.5
        ci, cj = rng.uniform(0, H), rng.uniform(0, W)
        size = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        val = rng.uniform(0.0, 255.0)
        if is_rect:
            size2 = math.exp(rng.uniform(math.log(lo), math.log(hi)))
            i0, i1 = int(max(0, ci - size / 2)), int(min(H, ci + size / 2 + 1))
            j0, j1 = int(max(0, cj - size2 / 2)), int(min(W, cj + size2 / 2 + 1))
            u[i0:i1, j0:j1] = val
        else:
            rad = size / 2
            i0, i1 = int(max(0, ci - rad)), int(min(H, ci + rad + 1))
            j0, j1 = int(max(0, cj - rad)), int(min(W, cj + rad + 1))
            if i1 <= i0 or j1 <= j0:
                continue
            yi = np.arange(i0, i1)[:, None] - ci
            xj = np.arange(j0, j1)[None, :] - cj
            msk = yi * yi + xj * xj <= rad * rad
            sub = u[i0:i1, j0:j1]
            sub[msk] = val
    for _ in range(n_textures):
        sh = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        sw = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        ci, cj = rng.uniform(0, H), rng.uniform(0, W)
        fx, fy = rng.uniform(1 / 32, 1 / 4, size=2)
        phi = rng.uniform(0, 2 * math.pi)
        i0, i1 = int(max(0, ci - sh / 2)), int(min(H, ci + sh / 2 + 1))
        j0, j1 = int(max(0, cj - sw / 2)), int(min(W, cj + sw / 2 + 1))
        if i1 <= i0 or j1 <= j0:
            continue
        yi = np.arange(i0, i1, dtype=np.float64)[:, None]
        xj = np.arange(j0, j1, dtype=np.float64)[None, :]
        u[i0:i1, j0:j1] += texture_amp * np.sin(2 * math.pi * (fx * xj + fy * yi) + phi)
    return u


# --------------------------------------------------------------------------
# Problems
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """One restoration problem H u = g_delta."""

    name: str
    u_true: np.ndarray
    psf: np.ndarray
    g_delta: np.ndarray
    delta: float
    n_levels: int
    precision: str  # "f64" | "f32" | "f32_f16coarse"
    k: float = 10.0
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.g_delta.shape

    @property
    def radius(self) -> int:
        return (self.psf.shape[0] - 1) // 2


def make_problem(name: str, H: int, W: int, psf: np.ndarray, n_shapes: int, seed: int, n_levels: int,
                 precision: str, n_textures: int = 0, meta: dict | None = None) -> Problem:
    rng = np.random.Generator(np.random.PCG64(seed))
    u = scene(H, W, n_shapes, rng, n_textures=n_textures)
    g = blur(u, psf)
    e = rng.standard_normal((H, W))
    delta = float(np.sqrt(np.mean(e * e)))
    return Problem(name=name, u_true=u, psf=psf, g_delta=g + e, delta=delta, n_levels=n_levels,
                   precision=precision, meta=dict(meta or {}, seed=seed))


def levels_for(H: int, W: int) -> int:
    """Number of levels so that the coarsest grid is about 16 pixels across."""
    return 1 + int(math.floor(math.log2(min(H, W) / 16.0)))


def random_psf(rng: np.random.Generator):
    """Half Gaussian (sigma ~ U[1,4], r = ceil(3 sigma)), half disk (r ~ U{2..6})."""
    if rng.random() < 0.5:
        sigma = float(rng.uniform(1.0, 4.0))
        r = int(math.ceil(3.0 * sigma))
        return gaussian_psf(sigma, r), {"psf": "gaussian", "sigma": sigma, "r": r}
    r = int(rng.integers(2, 7))
    return disk_psf(r), {"psf": "disk", "r": r}


def workload(wid: int, **kw) -> Problem:
    """Single-image workloads.
    1: 64x64 FP64, 16 shapes, Gaussian sigma=2 on 9x9, 3 levels (16-32-64)
    2: 1024x1024 FP32 bulk, 200 shapes, Gaussian sigma=3 on 15x15, 7 levels
    3: 4096x4096 FP32, 2000 shapes + 200 texture patches, disk r=6, 9 levels
    Keyword overrides (H, W, n_levels, precision) give scaled variants of the
    same recipe for parity tests."""
    seed = SEED_BASE + wid
    if wid == 1:
        H = kw.get("H", 64); W = kw.get("W", H)
        return make_problem("gauss2_64", H, W, gaussian_psf(2.0, 4), kw.get("n_shapes", 16), seed,
                            kw.get("n_levels", 3), kw.get("precision", "f64"))
    if wid == 2:
        H = kw.get("H", 1024); W = kw.get("W", H)
        return make_problem("gauss3_1024", H, W, gaussian_psf(3.0, 7), kw.get("n_shapes", 200), seed,
                            kw.get("n_levels", 7), kw.get("precision", "f32"))
    if wid == 3:
        H = kw.get("H", 4096); W = kw.get("W", H)
        return make_problem("disk6_4096", H, W, disk_psf(6), kw.get("n_shapes", 2000), seed,
                            kw.get("n_levels", 9), kw.get("precision", "f32"),
                            n_textures=kw.get("n_textures", 200))
    raise ValueError(f"unknown single-image workload {wid}")


def edge_scene(H: int, W: int, rng: np.random.Generator, density: float = 3000.0) -> np.ndarray:
    """Edge-dense piecewise-constant scene: a flat background, many small
    rectangles and disks (sides 3-48 px, `density` per Mpixel) and thin bars
    one to three pixels wide across the image, every region at its own
    intensity in [0, 255]."""
    u = np.full((H, W), float(rng.uniform(0.0, 255.0)))
    n = max(8, int(round(density * H * W / 1e6)))
    for _ in range(n):
        ci, cj = rng.uniform(0, H), rng.uniform(0, W)
        a = math.exp(rng.uniform(math.log(3.0), math.log(48.0)))
        b = math.exp(rng.uniform(math.log(3.0), math.log(48.0)))
        val = rng.uniform(0.0, 255.0)
        i0, i1 = int(max(0, ci - a / 2)), int(min(H, ci + a / 2 + 1))
        j0, j1 = int(max(0, cj - b / 2)), int(min(W, cj + b / 2 + 1))
        if i1 <= i0 or j1 <= j0:
            continue
        if rng.random() < 0.5:
            u[i0:i1, j0:j1] = val
        else:
            yi = np.arange(i0, i1)[:, None] - ci
            xj = np.arange(j0, j1)[None, :] - cj
            sub = u[i0:i1, j0:j1]
            sub[(yi / (a / 2)) ** 2 + (xj / (b / 2)) ** 2 <= 1.0] = val
    for _ in range(max(2, int(round(40 * math.sqrt(H * W) / 1024)))):
        width = int(rng.integers(1, 4))
        val = rng.uniform(0.0, 255.0)
        if rng.random() < 0.5:
            i = int(rng.integers(0, max(1, H - width)))
            u[i:i + width, :] = val
        else:
            j = int(rng.integers(0, max(1, W - width)))
            u[:, j:j + width] = val
    return u


def edge_workload(H: int = 1024, W: int | None = None, n_levels: int = 7, precision: str = "f32") -> Problem:
    """Edge-preservation workload: the edge-dense scene blurred with the
    paper's strongest Gaussian case that its edge experiment uses (sigma = 3,
    half bandwidth 11, normalised to unit sum) plus N(0,1) noise."""
    W = H if W is None else W
    seed = SEED_BASE + 6
    rng = np.random.Generator(np.random.PCG64(seed))
    u = edge_scene(H, W, rng)
    psf = gaussian_psf(3.0, 11)
    g = blur(u, psf)
    e = rng.standard_normal((H, W))
    delta = float(np.sqrt(np.mean(e * e)))
    return Problem(name=f"edges_b3_{H}x{W}", u_true=u, psf=psf, g_delta=g + e, delta=delta, n_levels=n_levels,
                   precision=precision, meta={"seed": seed, "psf": "gaussian sigma=3 r=11"})


def batch_specs(n_images: int = 256, lo: int = 128, hi: int = 2048, wid: int = 4):
    """Sizes and PSFs of the uneven batch: H and W independently log-uniform
    in [lo, hi]; shapes proportional to area (200 per Mpixel, at least 8)."""
    specs = []
    for i in range(n_images):
        rng = np.random.Generator(np.random.PCG64(SEED_BASE + wid + 1000 * i))
        H = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        W = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        psf, pmeta = random_psf(rng)
        specs.append({"H": H, "W": W, "psf": psf, "pmeta": pmeta,
                      "n_shapes": max(8, int(round(200 * H * W / 1e6))),
                      "seed": SEED_BASE + wid + 1000 * i + 7, "n_levels": levels_for(H, W)})
    return specs


def batch_problems(n_images: int = 256, lo: int = 128, hi: int = 2048, wid: int = 4,
                   precision: str = "f32"):
    out = []
    for i, s in enumerate(batch_specs(n_images, lo, hi, wid)):
        out.append(make_problem(f"batch{wid}_{i}", s["H"], s["W"], s["psf"], s["n_shapes"], s["seed"],
                                s["n_levels"], precision, meta=s["pmeta"]))
    return out


def served_pool(n_images: int = 64, lo: int = 64, hi: int = 4096, precision: str = "f32"):
    """Distinct request images of the served workload: sides log-uniform in
    [lo, hi], the PSF mix of the uneven batch.  Requests draw from this pool
    in turn (generating every request's image would dominate the run)."""
    return batch_problems(n_images, lo, hi, wid=5, precision=precision)


def poisson_arrivals(n: int, qps: float, seed: int = SEED_BASE + 5) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process at rate qps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, size=n))
