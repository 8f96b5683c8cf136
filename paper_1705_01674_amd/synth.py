"""Seeded synthetic inputs for SG-WLS filtering.

The paper evaluates on natural photographs, HDR images and depth/colour
datasets that are not available here, so every input is synthetic: piecewise
constant random rectangles (edges for the edge-aware weights to respect), an
optional smooth sinusoidal gradient, and Gaussian noise.  This module holds
none of the filter's arithmetic; it only draws inputs, and both the GPU
library's tests and the CPU oracle's tests consume the same arrays.

Recipe (numpy PCG64 via ``default_rng(seed)``; float32 after generation):

1. background: one constant per channel, U[0, 1];
2. ``n_rect`` rectangles painted in order: height U_int[ceil(M/16), ceil(M/2)],
   width U_int[ceil(N/16), ceil(N/2)], top-left uniform over valid positions,
   one intensity per channel U[0, 1];
3. optionally ``0.1*sin(2*pi*(x/Px + y/Py) + phi)`` with Px ~ U[N/8, N/2],
   Py ~ U[M/8, M/2], phi ~ U[0, 2*pi), shared by all channels;
4. iid N(0, sigma^2) noise, no clipping.

The guidance of an RGB image is its BT.601 luma 0.299 R + 0.587 G + 0.114 B;
a grey image is its own guidance.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def image(M: int, N: int, C: int = 1, n_rect: int = 50, sigma: float = 0.05,
          seed: int = 0, sinus: bool = False) -> np.ndarray:
    """A (C, M, N) float32 image drawn by the recipe above."""
    rng = np.random.default_rng(seed)
    img = np.empty((C, M, N), dtype=np.float64)
    img[:] = rng.uniform(0.0, 1.0, size=C)[:, None, None]
    hmin, hmax = math.ceil(M / 16), math.ceil(M / 2)
    wmin, wmax = math.ceil(N / 16), math.ceil(N / 2)
    for _ in range(n_rect):
        h = int(rng.integers(hmin, hmax + 1))
        w = int(rng.integers(wmin, wmax + 1))
        i0 = int(rng.integers(0, M - h + 1))
        j0 = int(rng.integers(0, N - w + 1))
        img[:, i0:i0 + h, j0:j0 + w] = rng.uniform(0.0, 1.0, size=C)[:, None, None]
    if sinus:
        px = rng.uniform(N / 8, N / 2)
        py = rng.uniform(M / 8, M / 2)
        phi = rng.uniform(0.0, 2 * math.pi)
        y, x = np.mgrid[0:M, 0:N]
        img += 0.1 * np.sin(2 * math.pi * (x / px + y / py) + phi)[None]
    img += rng.normal(0.0, sigma, size=img.shape)
    return img.astype(np.float32)


def luma(img: np.ndarray) -> np.ndarray:
    """BT.601 luma of a (3, M, N) image; a (1, M, N) image is returned as (M, N)."""
    if img.shape[0] == 1:
        return np.ascontiguousarray(img[0])
    if img.shape[0] != 3:
        raise ValueError("luma needs 1 or 3 channels")
    y = 0.299 * img[0].astype(np.float64) + 0.587 * img[1] + 0.114 * img[2]
    return y.astype(np.float32)


@dataclass
class Workload:
    """One synthetic workload: images, guidance and filter parameters."""
    name: str
    f: np.ndarray            # (C, M, N) float32
    g: np.ndarray            # (M, N) float32
    params: dict = field(default_factory=dict)  # lam, r, iters, stride, kind, sigma_s, sigma_r


def _exp_params(lam, r, iters, stride=1):
    return dict(lam=float(lam), r=int(r), iters=int(iters), stride=int(stride), kind="exp",
                sigma_s=float(r), sigma_r=0.1, alpha_s=1.2, alpha_r=1.2, eps=1e-4)


def single(name: str, M: int, N: int, C: int, n_rect: int, sigma: float, seed: int,
           lam: float, r: int, iters: int, stride: int = 1, sinus: bool = False) -> Workload:
    f = image(M, N, C, n_rect, sigma, seed, sinus)
    return Workload(name, f, luma(f), _exp_params(lam, r, iters, stride))


def grey256(seed: int = 1000) -> Workload:
    """256x256 grey, 50 rectangles, noise 0.05, guidance = input; r=1, T=1, lambda=1."""
    return single("grey256_r1_T1", 256, 256, 1, 50, 0.05, seed, 1.0, 1, 1)


def rgb768x1024(seed: int = 1001) -> Workload:
    """768x1024 RGB, 200 rectangles, noise 0.03, luma guidance; r=1, T=3, lambda=4."""
    return single("rgb768x1024_r1_T3", 768, 1024, 3, 200, 0.03, seed, 4.0, 1, 3)


def rgb1080p(r: int = 1, lam: float = 4.0, iters: int = 3, stride: int = 1,
             seed: int = 1000) -> Workload:
    """1080x1920 RGB, 200 rectangles, noise 0.03, sinusoidal gradient, luma guidance."""
    return single(f"rgb1080p_r{r}_T{iters}_s{stride}_lam{lam:g}", 1080, 1920, 3, 200, 0.03,
                  seed, lam, r, iters, stride, sinus=True)


def rgb1024_ctx(seed: int = 1000) -> Workload:
    """1024x1024 RGB (the size of the paper's timing image), r = 1, T = 4, lambda = 4,
    same generator as rgb1080p."""
    return single("rgb1024_r1_T4_s1_lam4", 1024, 1024, 3, 200, 0.03, seed, 4.0, 1, 4, 1,
                  sinus=True)


@dataclass
class SparseWorkload:
    """Inputs of guided sparse interpolation (Eq. 21)."""
    name: str
    f: np.ndarray            # (C, M, N) float32, 0 where unknown
    h: np.ndarray            # (M, N) float32 index map
    g: np.ndarray            # (M, N) float32 guidance
    params: dict = field(default_factory=dict)


def depth_upsample(M: int = 1080, N: int = 1920, factor: int = 8, seed: int = 1000,
                   iters: int = 3) -> SparseWorkload:
    """Guided depth upsampling stand-in: the depth is channel 0 of the
    noise-free image with the same rectangles as the colour guidance; it is
    known on the regular grid of every factor-th pixel (offset factor/2) with
    N(0, 0.01^2) noise.  Guidance = 255 x luma of the noisy colour image, so
    that sigma_r = 3 is on the scale the paper's setting assumes.  r = 4,
    stride 4, sigma_s = 4, sigma_r = 3, lambda = 100 / 200 / 400 for factors
    2 / 4 / 8 (the paper's depth-upsampling settings)."""
    color = image(M, N, 3, 200, 0.03, seed, sinus=True)
    depth = image(M, N, 3, 200, 0.0, seed)[0].astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    h = np.zeros((M, N), dtype=np.float32)
    h[factor // 2::factor, factor // 2::factor] = 1.0
    f = (h * (depth + rng.normal(0.0, 0.01, size=(M, N)))).astype(np.float32)[None]
    g = (255.0 * luma(color).astype(np.float64)).astype(np.float32)
    lam = {2: 100.0, 4: 200.0, 8: 400.0}.get(factor, 400.0)
    params = dict(lam=lam, r=4, iters=int(iters), stride=4, kind="exp", sigma_s=4.0, sigma_r=3.0,
                  alpha_s=1.2, alpha_r=1.2, eps=1e-4)
    return SparseWorkload(f"depth{M}x{N}_up{factor}", np.ascontiguousarray(f), h, g, params)


def colorize_scribbles(M: int = 512, N: int = 512, n_strokes: int = 60, seed: int = 1000,
                       iters: int = 3) -> SparseWorkload:
    """Scribble colourisation stand-in: the two chrominance planes (BT.601
    U, V) of a synthetic colour image are known on n_strokes random
    horizontal or vertical strokes (length U_int[N/16, N/4], 3 pixels wide);
    guidance = 255 x luma.  r = 4, stride 2, sigma_s = 4, sigma_r = 2,
    lambda = 900 (the paper's colourisation settings)."""
    color = image(M, N, 3, 200, 0.01, seed).astype(np.float64)
    y = 0.299 * color[0] + 0.587 * color[1] + 0.114 * color[2]
    uv = np.stack([0.492 * (color[2] - y), 0.877 * (color[0] - y)])
    rng = np.random.default_rng(seed + 2)
    h = np.zeros((M, N), dtype=np.float32)
    for _ in range(n_strokes):
        length = int(rng.integers(max(1, N // 16), max(2, N // 4) + 1))
        i0, j0 = int(rng.integers(0, M)), int(rng.integers(0, N))
        if rng.uniform() < 0.5:
            h[max(0, i0 - 1):i0 + 2, j0:j0 + length] = 1.0
        else:
            h[i0:i0 + length, max(0, j0 - 1):j0 + 2] = 1.0
    f = (h[None] * uv).astype(np.float32)
    g = (255.0 * y).astype(np.float32)
    params = dict(lam=900.0, r=4, iters=int(iters), stride=2, kind="exp", sigma_s=4.0,
                  sigma_r=2.0, alpha_s=1.2, alpha_r=1.2, eps=1e-4)
    return SparseWorkload(f"colorize{M}x{N}", np.ascontiguousarray(f), h, g, params)


def batch_uneven(B: int = 64, seed_base: int = 4000, min_side: int = 256,
                 max_side: int = 2048, iters: int = 3):
    """B grey images with independent sides U_int[min_side, max_side], 200 rectangles,
    noise 0.03, guidance = input; per image r in {1, 2} and lambda = 2^U[-1, 5]."""
    rng = np.random.default_rng(seed_base)
    out = []
    for b in range(B):
        M = int(rng.integers(min_side, max_side + 1))
        N = int(rng.integers(min_side, max_side + 1))
        r = int(rng.integers(1, 3))
        lam = float(2.0 ** rng.uniform(-1.0, 5.0))
        f = image(M, N, 1, 200, 0.03, seed_base + 1 + b)
        out.append(Workload(f"batch{b}", f, luma(f), _exp_params(lam, r, iters)))
    return out


def rgb_batch_with_target(B: int = 16, M: int = 512, N: int = 512, seed_base: int = 5000):
    """B RGB images with luma guidance and a target drawn from the same seed with the
    noise switched off (a clean version of each input)."""
    fs, gs, ts = [], [], []
    for b in range(B):
        f = image(M, N, 3, 200, 0.03, seed_base + b)
        t = image(M, N, 3, 200, 0.0, seed_base + b)
        fs.append(f)
        gs.append(luma(f))
        ts.append(t)
    return np.stack(fs), np.stack(gs), np.stack(ts)
