"""Seeded synthetic test images (no filter arithmetic lives here).

The paper measures on the 256x256 *Peppers* photograph, which is not
available; these piecewise-constant images with noise stand in for it: flat
regions separated by sharp edges, which is what an edge-preserving filter is
exercised by.

Recipe (all draws from ``numpy.random.default_rng(seed)``, in this order):
  1. ``K`` seed points uniform in ``[0, H) x [0, W)`` (an array of shape (K, 2),
     rows then columns);
  2. ``K`` cell intensities uniform in ``[0, 255]``;
  3. every pixel centre ``(y + 0.5, x + 0.5)`` takes the intensity of its
     nearest seed (Euclidean distance, k-d tree);
  4. optionally a linear ramp: ``0.5 * voronoi + 0.5 * 255 * (x/(W-1) + y/(H-1)) / 2``;
  5. i.i.d. Gaussian noise of standard deviation ``noise`` (one draw per pixel,
     row-major), then clipping to ``[0, 255]`` and conversion to float32.

Also here: the parameter draws of the batched workload and the named
workloads used by the tests and the benchmark.
"""
import math

import numpy as np
from scipy.spatial import cKDTree


def voronoi_image(H, W, cells, seed, noise=10.0, ramp=False):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(cells, 2)) * np.array([H, W], dtype=np.float64)
    vals = rng.uniform(0.0, 255.0, size=cells)
    tree = cKDTree(pts)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64) + 0.5, np.arange(W, dtype=np.float64) + 0.5, indexing="ij")
    q = np.stack([yy.ravel(), xx.ravel()], axis=1)
    _, idx = tree.query(q, k=1, workers=-1)
    img = vals[idx].reshape(H, W)
    if ramp:
        ry = yy - 0.5
        rx = xx - 0.5
        ramp_v = 255.0 * (rx / max(W - 1, 1) + ry / max(H - 1, 1)) / 2.0
        img = 0.5 * img + 0.5 * ramp_v
    if noise > 0:
        img = img + rng.normal(0.0, noise, size=(H, W))
    return np.clip(img, 0.0, 255.0).astype(np.float32)


def cells_for(H, W, density_cells=40, density_px=65536):
    """Cell count that keeps the density of 40 cells per 256x256 image."""
    return max(1, int(math.ceil(density_cells * H * W / density_px)))


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def small_256():
    """256x256, 40 cells, noise 10: the small forward case (sigma_s 3, sigma_r 30)."""
    return voronoi_image(256, 256, 40, seed=1)


def mid_1024():
    """1024x1024, 200 cells: the sigma_s sweep {2, 5, 10, 20} at sigma_r 30."""
    return voronoi_image(1024, 1024, 200, seed=2)


def large_4096():
    """4096x4096 (16 MP), 2000 cells + ramp + noise: sigma_s 10, sigma_r 20."""
    return voronoi_image(4096, 4096, 2000, seed=3, ramp=True)


def batched_64(count=64, seed=4, lo=128, hi=2048):
    """Uneven batch: side lengths uniform in [lo, hi] (H and W drawn
    separately), sigma_s uniform in [1, 16], sigma_r uniform in [10, 50].
    Returns a list of (image, sigma_s, sigma_r)."""
    rng = np.random.default_rng(seed)
    Hs = rng.integers(lo, hi + 1, size=count)
    Ws = rng.integers(lo, hi + 1, size=count)
    ss = rng.uniform(1.0, 16.0, size=count)
    sr = rng.uniform(10.0, 50.0, size=count)
    out = []
    for i in range(count):
        H, W = int(Hs[i]), int(Ws[i])
        img = voronoi_image(H, W, cells_for(H, W), seed=10_000 + 100 * seed + i)
        out.append((img, float(ss[i]), float(sr[i])))
    return out


def grad_batch(count=16, H=512, W=512):
    """Sixteen 512x512 images (200 cells) and a target image of the same size."""
    imgs = np.stack([voronoi_image(H, W, 200, seed=500 + i) for i in range(count)])
    target = voronoi_image(H, W, 200, seed=1005)
    return imgs, target
