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


def oracle_lines(img, sigma_s, sigma_r, N, mode, rows=(), cols=(), reach=None):
    """Oracle outputs along whole rows and whole columns of a large image:
    the FP64 mean of the whole image is the centre, and each row (column) is
    taken from the oracle run on the band of rows (columns) within `reach` of
    it, centred, with no further centring.  The band spans the image in the
    other direction, so only the filter's reach across the band is cut.  For
    the recursive kernel the default reach is 15 sigma_s, where the kernel
    and its tail mass have fallen below 1e-9 of their peak (the cut changes
    an output on 0..255 data by well under 1e-6); for the FIR window it is the
    window radius (exact).  Returns ({row: values}, {col: values})."""
    f = np.asarray(img, np.float64)
    H, W = f.shape
    tc = float(f.mean())
    if reach is None:
        reach = oracle.fir_radius(sigma_s) if mode in ("fir", "box") else int(np.ceil(15 * sigma_s))

    def table(extent):
        if mode == "fir":
            return oracle.gauss_table(sigma_s, oracle.fir_radius(sigma_s))
        if mode == "box":
            return oracle.box_table(oracle.fir_radius(sigma_s))
        return oracle.deriche_table(sigma_s, max(1, min(extent - 1, oracle.iir_radius(sigma_s, H, W))))

    out_r, out_c = {}, {}
    for y in rows:
        y0, y1 = max(0, y - reach), min(H, y + reach + 1)
        crop = f[y0:y1] - tc
        out_r[y] = oracle.gp_alg1(crop, sigma_r, N, table(max(crop.shape)), oracle.CENTER_NONE)[y - y0] + tc
    for x in cols:
        x0, x1 = max(0, x - reach), min(W, x + reach + 1)
        crop = f[:, x0:x1] - tc
        out_c[x] = oracle.gp_alg1(crop, sigma_r, N, table(max(crop.shape)), oracle.CENTER_NONE)[:, x - x0] + tc
    return out_r, out_c
