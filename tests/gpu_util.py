"""Helpers shared by the GPU parity tests (no filter arithmetic here)."""
import sys

import numpy as np
import torch

import oracle


def note(msg):
    """Names the case about to run on the GPU (flushed, so a crash keeps it)."""
    sys.stderr.write(f"[gpu case] {msg}\n")
    sys.stderr.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_gp(img, sigma_s, sigma_r, N, mode, center=oracle.CENTER_MEAN):
    f = np.asarray(img, np.float64)
    k, _ = oracle.spatial_table(mode, sigma_s, *f.shape)
    return oracle.gp_alg1(f, sigma_r, N, k, center)


def oracle_gp_at(img, y, x, sigma_s, sigma_r, N, mode, reach=None):
    """Oracle output at one pixel of a large image: the FP64 mean of the whole
    image is the centre; only the pixel's neighbourhood (the FIR or box window,
    or 25 sigma_s of the recursive kernel, beyond which its weights are below
    1e-18) is filtered, with the centred crop and no further centring."""
    f = np.asarray(img, np.float64)
    H, W = f.shape
    tc = float(f.mean())
    if reach is None:
        reach = oracle.fir_radius(sigma_s) if mode in ("fir", "box") else int(np.ceil(25 * sigma_s))
    y0, y1 = max(0, y - reach), min(H, y + reach + 1)
    x0, x1 = max(0, x - reach), min(W, x + reach + 1)
    crop = f[y0:y1, x0:x1] - tc
    if mode == "fir":
        k = oracle.gauss_table(sigma_s, oracle.fir_radius(sigma_s))
    elif mode == "box":
        k = oracle.box_table(oracle.fir_radius(sigma_s))
    else:
        k = oracle.deriche_table(sigma_s, max(crop.shape) - 1)
    out = oracle.gp_alg1(crop, sigma_r, N, k, oracle.CENTER_NONE)
    return out[y - y0, x - x0] + tc
