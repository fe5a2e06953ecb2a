"""Seeded synthetic hyperspectral cubes.

This module only draws input data. It holds none of the segmentation
arithmetic, so both the GPU path and the CPU oracle read the same cubes from
here without sharing any of the method's code.

The paper measures on AVIRIS Indian Pines (220 bands) and ROSIS Pavia scenes
(102/103 bands), cropped to 64^2 .. 512^2 pixels (Section 5.1.1). Those
datasets are not available, so these generators stand in for them with the
same band counts and image sizes and with region structure of the same kind:
spatially coherent classes with smooth spectra and additive noise.

Every cube is laid out band-interleaved-by-pixel: an H x W x B C-contiguous
array (bands contiguous per pixel), which is the row-major region-by-band
layout the paper's kernel indexes (Section 4.2, Figure 4.8).

Values are quantised so that every FP64 band sum over any set of pixels is
exact:
  * float32 cubes lie on a 2^-6 grid with |x| < 2^11 (17 significant bits);
  * float16 cubes lie on the 2^-4 grid clamped to [0, 2047] and are then
    rounded to the nearest float16 (spacing 2^-4 .. 1); the result is still a
    multiple of 2^-4 below 2^11.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

F32_GRID = 2.0 ** -6
F16_GRID = 2.0 ** -4
F32_CLAMP = 2048.0 - F32_GRID  # keep |x| < 2^11 on the 2^-6 grid
F16_MAX = 2047.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def voronoi_labels(rng: np.random.Generator, H: int, W: int, K: int) -> np.ndarray:
    """Assign every pixel centre to its nearest of K uniform seeds.

    Ties go to the lower seed index. Returns an int32 H x W class map.
    """
    from scipy.spatial import cKDTree

    seeds = np.stack([rng.uniform(0.0, W, size=K), rng.uniform(0.0, H, size=K)], axis=1)
    yy, xx = np.mgrid[0:H, 0:W]
    pts = np.stack([xx.ravel() + 0.5, yy.ravel() + 0.5], axis=1)
    k = min(2, K)
    dist, idx = cKDTree(seeds).query(pts, k=k)
    if k == 1:
        return idx.reshape(H, W).astype(np.int32)
    # exact squared distances for the two nearest, to apply the tie rule
    d0 = ((pts - seeds[idx[:, 0]]) ** 2).sum(1)
    d1 = ((pts - seeds[idx[:, 1]]) ** 2).sum(1)
    first = np.where((d1 < d0) | ((d1 == d0) & (idx[:, 1] < idx[:, 0])), idx[:, 1], idx[:, 0])
    return first.reshape(H, W).astype(np.int32)


def smooth_spectra(rng: np.random.Generator, K: int, B: int) -> np.ndarray:
    """K class spectra: a level in [0,1000] plus three low cosine harmonics."""
    level = rng.uniform(0.0, 1000.0, size=K)
    u = rng.uniform(-1.0, 1.0, size=(K, 3))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(K, 3))
    t = np.arange(B, dtype=np.float64) / max(B - 1, 1)
    m = np.repeat(level[:, None], B, axis=1)
    for k in range(1, 4):
        m += 100.0 * (u[:, k - 1, None] / k) * np.cos(np.pi * k * t[None, :] + phi[:, k - 1, None])
    return m


def endmember_spectra(rng: np.random.Generator, K: int, B: int, n_end: int = 8) -> np.ndarray:
    """K class spectra mixed from n_end Gaussian-bump endmembers.

    Endmember k is a sum of 2..4 bumps with height in [100,1000], centre in
    [0,1] and width in [0.03,0.2] on the normalised band axis. Class weights
    are Dirichlet(0.5).
    """
    t = np.arange(B, dtype=np.float64) / max(B - 1, 1)
    ends = np.zeros((n_end, B))
    for k in range(n_end):
        J = int(rng.integers(2, 5))
        h = rng.uniform(100.0, 1000.0, size=J)
        c = rng.uniform(0.0, 1.0, size=J)
        s = rng.uniform(0.03, 0.2, size=J)
        ends[k] = (h[:, None] * np.exp(-((t[None, :] - c[:, None]) ** 2) / (2.0 * s[:, None] ** 2))).sum(0)
    a = rng.dirichlet(0.5 * np.ones(n_end), size=K)
    return a @ ends


def quantise_f32(x: np.ndarray) -> np.ndarray:
    q = np.round(x / F32_GRID) * F32_GRID
    return np.clip(q, -F32_CLAMP, F32_CLAMP).astype(np.float32)


def quantise_f16(x: np.ndarray) -> np.ndarray:
    q = np.round(x / F16_GRID) * F16_GRID
    return np.clip(q, 0.0, F16_MAX).astype(np.float16)


def _noisy_cube(rng: np.random.Generator, spec: np.ndarray, cls: np.ndarray, sigma: float, dtype: str,
                rows: int = 32) -> np.ndarray:
    """quantise(spec[cls] + N(0, sigma^2)), drawn and quantised a band of
    `rows` image rows at a time. The normal draws come from one stream in
    pixel-major order, so the values are those of a single draw over the
    whole H x W x B array (the chunking only bounds the temporaries)."""
    H, W = cls.shape
    B = spec.shape[1]
    out = np.empty((H, W, B), dtype=np.float32 if dtype == "f32" else np.float16)
    for r0 in range(0, H, rows):
        r1 = min(H, r0 + rows)
        x = spec[cls[r0:r1]] + rng.normal(0.0, sigma, size=(r1 - r0, W, B))
        out[r0:r1] = quantise_f32(x) if dtype == "f32" else quantise_f16(x)
    return out


@dataclasses.dataclass
class Scene:
    cube: np.ndarray          # H x W x B, float32 or float16
    classes: np.ndarray       # H x W int32 ground-truth class map
    seed: int
    recipe: str


def voronoi_scene(H: int, W: int, B: int, K: int, sigma: float, seed: int,
                  dtype: str = "f32") -> Scene:
    """Voronoi cells, one class each, smooth spectra, Gaussian noise."""
    rng = _rng(seed)
    cls = voronoi_labels(rng, H, W, K)
    spec = smooth_spectra(rng, K, B)
    cube = _noisy_cube(rng, spec, cls, sigma, dtype)
    return Scene(cube, cls, seed,
                 f"voronoi H={H} W={W} B={B} K={K} sigma={sigma} seed={seed} {dtype}")


def mixer_scene(H: int, W: int, B: int, K: int, sigma: float, seed: int,
                salt: float = 0.0, dtype: str = "f32") -> Scene:
    """Voronoi cells whose spectra are Dirichlet mixtures of 8 endmembers.

    With salt > 0, a Bernoulli(salt) subset of pixels is set to 2000.0 in
    every band: identical spectra, hence exact zero-dissimilarity ties.
    """
    rng = _rng(seed)
    cls = voronoi_labels(rng, H, W, K)
    spec = endmember_spectra(rng, K, B)
    cube = _noisy_cube(rng, spec, cls, sigma, dtype)
    if salt > 0.0:
        # 2000.0 lies on both quantisation grids, so setting it after quantising is the same
        m = rng.random(size=(H, W)) < salt
        cube[m] = 2000.0
    return Scene(cube, cls, seed,
                 f"mixer H={H} W={W} B={B} K={K} sigma={sigma} salt={salt} seed={seed} {dtype}")


def random_cube(H: int, W: int, B: int, seed: int, kind: str = "continuous") -> np.ndarray:
    """Small test cubes.

    continuous : uniform on the 2^-6 grid in [-1000, 1000) (practically tie-free)
    integer    : small integers 0..3 (tie-heavy; exercises the tie-break)
    """
    rng = _rng(seed)
    if kind == "continuous":
        return quantise_f32(rng.uniform(-1000.0, 1000.0, size=(H, W, B)))
    if kind == "integer":
        return rng.integers(0, 4, size=(H, W, B)).astype(np.float32)
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# The benchmark workloads. Each returns (cube, run parameters as a dict).
# ---------------------------------------------------------------------------

def ladder(start: int, stop: int) -> List[int]:
    """Powers-of-two ladder start, start/2, ..., stop (inclusive)."""
    out = []
    c = start
    while c >= stop:
        out.append(c)
        c //= 2
    if out[-1] != stop:
        out.append(stop)
    return out


def workload(name: str):
    """Synthetic stand-ins for the five benchmark configurations."""
    if name == "hswo64":
        sc = voronoi_scene(64, 64, 32, 40, 20.0, 101)
        params = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=256,
                      target_regions=2, section_regions=0, rnb_levels=1,
                      level_counts=ladder(2048, 2))
        return sc, params
    if name == "rhseg512":
        sc = voronoi_scene(512, 512, 128, 200, 30.0, 202)
        params = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=1024,
                      target_regions=8, section_regions=256, rnb_levels=4,
                      level_counts=ladder(1024, 8))
        return sc, params
    if name == "rhseg1024_salt":
        sc = mixer_scene(1024, 1024, 220, 300, 25.0, 303, salt=0.05)
        params = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=1024,
                      target_regions=8, section_regions=256, rnb_levels=5,
                      level_counts=ladder(1024, 8))
        return sc, params
    if name == "rhseg2048_f16":
        sc = mixer_scene(2048, 2048, 224, 500, 25.0, 505, dtype="f16")
        params = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=2048,
                      target_regions=16, section_regions=512, rnb_levels=5,
                      level_counts=ladder(2048, 16))
        return sc, params
    raise KeyError(name)


def batch_sections(n: int = 256, base_seed: int = 404000) -> List[Tuple[np.ndarray, int]]:
    """Uneven independent sections: side U{32..128}, bands U{64,96,...,224},
    10..120 Voronoi classes, sigma 30; section s uses seed base_seed + s."""
    out = []
    for s in range(n):
        rng = _rng(base_seed + s)
        side = int(rng.integers(32, 129))
        B = int(rng.choice(np.arange(64, 225, 32)))
        K = int(rng.integers(10, 121))
        sc = voronoi_scene(side, side, B, K, 30.0, base_seed + s)
        out.append((sc.cube, base_seed + s))
    return out


BATCH_PARAMS = dict(connectivity=4, seam_connectivity=8, spclust_wght=0.5, spclust_max=1024,
                    target_regions=256, section_regions=0, rnb_levels=1, level_counts=[256])
