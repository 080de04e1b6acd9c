"""Seeded synthetic rectified IR stereo pairs.

Recipe (stands in for the paper's rendered IR captures, which are not available):

* Left image: every pixel independently is a projector dot with probability
  ``dot_density`` (intensity uniform on the integers ``dot_lo..dot_hi``) or
  background (uniform on ``bg_lo..bg_hi``).  Dots are single pixels.
* Disparity field, defined on the right-image grid: ``planes`` seed points drawn
  uniformly in the image; each pixel belongs to the Voronoi cell of its nearest
  seed (ties go to the lowest index) and takes that cell's plane
  ``c + gx*(x - sx) + gy*(y - sy)`` with ``c ~ U[dmin, dmax]`` and
  ``gx, gy ~ U[-0.05, 0.05]``, clamped to ``[dmin, dmax]``.
* Right image: ``right(x, y) = left(x + d(x, y), y)`` by linear interpolation,
  rounded half-to-even; where ``x + d > W - 1`` a fresh dot/background value is
  drawn.
* IR noise draws (the random inputs of the multiplicative-speckle plus
  additive-thermal noise model, Sec. VI-C, Eqs. (7)-(8)): per image and pixel a
  gain ``gamma`` and an offset ``n`` as float32.  Modes: ``none`` (gamma = 1,
  n = 0), ``gauss`` (gamma ~ N(1, gain_sd^2), n ~ N(mu, sigma^2)), ``paper``
  (gamma ~ Gamma(k, theta), n ~ N(mu, sigma^2) with the D415 fit of Sec. VII-C:
  mu = -0.231, sigma = 0.83, k = 3.98, theta = 0.254).  A noise scale ``s``
  maps gamma -> 1 + s (gamma - 1) and n -> s n.
* Ground truth: forward splat of the field onto the left grid (largest
  disparity wins); used only for sanity statistics, never for parity.

All randomness comes from numpy's Philox4x32-10 bit generator keyed by
``(seed, stream)`` so every array is reproducible on any host.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

# stream identifiers: one independent Philox stream per purpose
_S_LEFT, _S_PLANES, _S_FILL, _S_NOISE_L, _S_NOISE_R = 1, 2, 3, 4, 5

PAPER_NOISE = dict(mu=-0.231, sigma=0.83, k=3.98, theta=0.254)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed), int(stream)])))


def pair_seed(workload_index: int, pair_index: int) -> int:
    """Seed of pair ``pair_index`` of workload ``workload_index``."""
    return 1_000_000 * int(workload_index) + int(pair_index)


@dataclasses.dataclass(frozen=True)
class PairSpec:
    width: int
    height: int
    planes: int = 6
    dmin: float = 4.0
    dmax: float = 60.0
    dot_density: float = 0.15
    dot_lo: int = 150
    dot_hi: int = 255
    bg_lo: int = 10
    bg_hi: int = 40
    noise: str = "gauss"          # none | gauss | paper
    sigma: float = 3.0            # additive thermal noise SD (DN)
    mu: float = 0.0               # additive thermal noise mean (DN)
    gain_sd: float = 0.0          # SD of the multiplicative gain in gauss mode
    noise_scale: float = 1.0


@dataclasses.dataclass
class StereoPair:
    left: np.ndarray          # uint8 [H, W], clean
    right: np.ndarray         # uint8 [H, W], clean
    gamma_l: np.ndarray       # float32 [H, W]
    n_l: np.ndarray           # float32 [H, W]
    gamma_r: np.ndarray       # float32 [H, W]
    n_r: np.ndarray           # float32 [H, W]
    gt_disp: np.ndarray       # float32 [H, W] on the left grid, 0 = unknown
    field: np.ndarray         # float32 [H, W] disparity field on the right grid


def _speckle(rng: np.random.Generator, shape, spec: PairSpec) -> np.ndarray:
    is_dot = rng.random(shape) < spec.dot_density
    dots = rng.integers(spec.dot_lo, spec.dot_hi + 1, size=shape)
    bg = rng.integers(spec.bg_lo, spec.bg_hi + 1, size=shape)
    return np.where(is_dot, dots, bg).astype(np.uint8)


def _plane_field(rng: np.random.Generator, spec: PairSpec) -> np.ndarray:
    W, H, K = spec.width, spec.height, spec.planes
    sx = rng.random(K) * W
    sy = rng.random(K) * H
    c = spec.dmin + rng.random(K) * (spec.dmax - spec.dmin)
    gx = rng.uniform(-0.05, 0.05, K)
    gy = rng.uniform(-0.05, 0.05, K)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    best = np.full((H, W), np.inf)
    region = np.zeros((H, W), dtype=np.int64)
    for k in range(K):  # strict < keeps the lowest index on ties
        dist = (xs - sx[k]) ** 2 + (ys - sy[k]) ** 2
        take = dist < best
        best = np.where(take, dist, best)
        region = np.where(take, k, region)
    d = c[region] + gx[region] * (xs - sx[region]) + gy[region] * (ys - sy[region])
    return np.clip(d, spec.dmin, spec.dmax).astype(np.float32)


def noise_draws(spec: PairSpec, shape, seed: int, stream: int):
    """Gain and offset draws for one image (float32, shape ``shape``)."""
    rng = _rng(seed, stream)
    if spec.noise == "none":
        gamma = np.ones(shape, np.float64)
        n = np.zeros(shape, np.float64)
    elif spec.noise == "gauss":
        gamma = 1.0 + spec.gain_sd * rng.standard_normal(shape) if spec.gain_sd > 0 else np.ones(shape)
        n = spec.mu + spec.sigma * rng.standard_normal(shape)
    elif spec.noise == "paper":
        gamma = rng.gamma(PAPER_NOISE["k"], PAPER_NOISE["theta"], shape)
        n = PAPER_NOISE["mu"] + PAPER_NOISE["sigma"] * rng.standard_normal(shape)
    else:
        raise ValueError(f"unknown noise mode {spec.noise!r}")
    s = spec.noise_scale
    gamma = 1.0 + s * (gamma - 1.0)
    n = s * n
    return gamma.astype(np.float32), n.astype(np.float32)


def make_pair(spec: PairSpec, seed: int) -> StereoPair:
    W, H = spec.width, spec.height
    left = _speckle(_rng(seed, _S_LEFT), (H, W), spec)
    field = _plane_field(_rng(seed, _S_PLANES), spec)
    fill = _speckle(_rng(seed, _S_FILL), (H, W), spec)

    xs = np.arange(W, dtype=np.float64)[None, :] + field.astype(np.float64)
    x0 = np.floor(xs).astype(np.int64)
    f = xs - x0
    inside = xs <= W - 1
    x0c = np.clip(x0, 0, W - 1)
    x1c = np.clip(x0 + 1, 0, W - 1)
    rows = np.arange(H)[:, None]
    lf = left.astype(np.float64)
    interp = (1.0 - f) * lf[rows, x0c] + f * lf[rows, x1c]
    right = np.where(inside, np.rint(interp), fill).astype(np.uint8)

    # forward splat of the field onto the left grid; the largest disparity wins
    gt = np.zeros((H, W), np.float32)
    xl = np.rint(xs).astype(np.int64)
    ok = inside & (xl >= 0) & (xl <= W - 1)
    yy = np.broadcast_to(rows, (H, W))[ok]
    np.maximum.at(gt, (yy, xl[ok]), field[ok])

    g_l, n_l = noise_draws(spec, (H, W), seed, _S_NOISE_L)
    g_r, n_r = noise_draws(spec, (H, W), seed, _S_NOISE_R)
    return StereoPair(left, right, g_l, n_l, g_r, n_r, gt, field)


def make_shift_pair(width: int, height: int, d0: int, seed: int, spec: Optional[PairSpec] = None):
    """Noise-free pair related by one constant integer shift: right(x) = left(x + d0)."""
    spec = spec or PairSpec(width, height)
    left = _speckle(_rng(seed, _S_LEFT), (height, width), spec)
    fill = _speckle(_rng(seed, _S_FILL), (height, width), spec)
    right = fill.copy()
    if d0 < width:
        right[:, : width - d0] = left[:, d0:]
    return left, right


# Workloads.  ``params`` is the depth-path parameter set of each workload
# (plain numbers; the method's arithmetic lives in the oracle and the kernels).
_BASE = dict(census_w=7, census_h=9, census_mode=0, p1=7, p2=86, uniqueness_pct=10,
             lr_max_diff=1, num_paths=8, median=3, subpixel=1, baseline_m=0.055)

CONFIGS: Dict[str, dict] = {
    "pair_320x240_d64": dict(spec=PairSpec(320, 240, planes=6, dmin=4, dmax=60, noise="gauss", sigma=3.0),
               params=dict(_BASE, width=320, height=240, max_disp=64, focal_px=400.0),
               pairs=1),
    "pair_1280x720_d128": dict(spec=PairSpec(1280, 720, planes=12, dmin=8, dmax=120, noise="gauss", sigma=4.0,
                             gain_sd=0.05),
               params=dict(_BASE, width=1280, height=720, max_disp=128, focal_px=920.0),
               pairs=1),
}


def sensor_like(width: int, height: int, max_disp: int) -> dict:
    """A pair recipe and parameter set generated as for the 1280x720 sensor workload."""
    dmax = min(120.0, max_disp - 8.0)
    return dict(spec=PairSpec(width, height, planes=12, dmin=min(8.0, dmax), dmax=dmax,
                              noise="gauss", sigma=4.0, gain_sd=0.05),
                params=dict(_BASE, width=width, height=height, max_disp=max_disp, focal_px=920.0))
