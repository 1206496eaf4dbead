"""FP64 CPU oracle for the Gauss-polynomial bilateral filter (arXiv 1505.00077).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark use this package; the product library never imports it.
It shares no code with the GPU path.

Thin ctypes wrappers around ``oracle.c`` (plain C, double precision, OpenMP),
plus NumPy brute-force routines for tiny images that are written directly from
the paper's equations and are used to pin the C routines.

Conventions (also stated in the C source):
  * images are 2-D float64 arrays, row-major;
  * spatial kernels are symmetric tables ``k[0..R]``; the 2-D weight is
    ``k[|dy|] * k[|dx|]``;
  * neighbours outside the image are skipped (zero extension).
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")

CENTER_MEAN, CENTER_MIDRANGE, CENTER_NONE = 0, 1, 2

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i, d = ctypes.c_int, ctypes.c_double
    lib.or_gauss_table.argtypes = [d, i, dp]
    lib.or_gauss_dtable.argtypes = [d, i, dp]
    lib.or_deriche_table.argtypes = [d, i, dp]
    lib.or_deriche_dtable.argtypes = [d, i, dp]
    lib.or_deriche_h.argtypes = [d]
    lib.or_deriche_h.restype = d
    lib.or_spatial.argtypes = [dp, dp, i, i, dp, i]
    lib.or_direct.argtypes = [dp, dp, i, i, dp, i, d]
    lib.or_center.argtypes = [dp, i, i, i]
    lib.or_center.restype = d
    lib.or_gp_alg1.argtypes = [dp, dp, i, i, d, i, dp, i, i]
    lib.or_gp_rescaled.argtypes = [dp, dp, dp, dp, i, i, d, i, dp, i, i]
    lib.or_gp_grad.argtypes = [dp, dp, i, i, d, i, dp, dp, i, i, dp, dp, dp]
    lib.or_spatial3.argtypes = [dp, dp, i, i, i, dp, i, dp, i]
    lib.or_volume_direct.argtypes = [dp, dp, i, i, i, dp, i, dp, i, d]
    lib.or_volume_gp.argtypes = [dp, dp, i, i, i, d, i, dp, i, dp, i, i]
    lib.or_joint_direct.argtypes = [dp, dp, dp, i, i, dp, i, d]
    lib.or_joint_gp.argtypes = [dp, dp, dp, i, i, d, i, dp, i, i]
    lib.or_gauss_poly.argtypes = [d, d, d, i]
    lib.or_gauss_poly.restype = d
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _img(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim != 2:
        raise ValueError("expected a 2-D image")
    return f


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with status {rc}")


# --------------------------------------------------------------------------
# spatial kernels
# --------------------------------------------------------------------------

def fir_radius(sigma_s):
    """Window half-width of eq. (1), W = 3 sigma_s, rounded up (at least 1).
    A relative excess below 1e-6 (float32 rounding of sigma_s) does not round
    up: W = ceil(3 sigma_s (1 - 1e-6))."""
    return max(1, int(math.ceil(3.0 * sigma_s * (1.0 - 1e-6))))


def gauss_table(sigma_s, R):
    """Sampled spatial Gaussian of eq. (2) on offsets 0..R."""
    k = np.empty(R + 1)
    _load().or_gauss_table(float(sigma_s), int(R), _p(k))
    return k


def gauss_dtable(sigma_s, R):
    """d gauss_table / d log(sigma_s) at fixed R."""
    k = np.empty(R + 1)
    _load().or_gauss_dtable(float(sigma_s), int(R), _p(k))
    return k


def deriche_table(sigma_s, R):
    """Closed-form impulse response of Deriche's recursive Gaussian, 0..R."""
    k = np.empty(R + 1)
    _load().or_deriche_table(float(sigma_s), int(R), _p(k))
    return k


def deriche_dtable(sigma_s, R):
    k = np.empty(R + 1)
    _load().or_deriche_dtable(float(sigma_s), int(R), _p(k))
    return k


def deriche_h(t):
    return _load().or_deriche_h(float(t))


def iir_radius(sigma_s, H, W):
    """Support used for the Deriche kernel: the whole image, capped where the
    response has decayed below 1e-29 of its peak (40 sigma_s)."""
    return int(min(max(H, W) - 1, math.ceil(40.0 * sigma_s)))


def box_table(R):
    """Box spatial kernel on offsets 0..R: weight 1 everywhere in the window
    (Section 3 notes, after eq. (11), that any spatial filter with a
    constant-time implementation, a box for instance, can replace the
    Gaussian of eq. (8))."""
    return np.ones(int(R) + 1)


def spatial_table(mode, sigma_s, H, W):
    """(table, R) for spatial mode 'fir' (eq. (8) over W = ceil(3 sigma_s)),
    'iir' (Deriche's recursive Gaussian, untruncated) or 'box' (uniform
    weights over the same window as 'fir')."""
    if mode == "fir":
        R = fir_radius(sigma_s)
        return gauss_table(sigma_s, R), R
    if mode == "iir":
        R = max(1, iir_radius(sigma_s, H, W))
        return deriche_table(sigma_s, R), R
    if mode == "box":
        R = fir_radius(sigma_s)
        return box_table(R), R
    raise ValueError(mode)


def spatial_dtable(mode, sigma_s, H, W):
    if mode == "fir":
        R = fir_radius(sigma_s)
        return gauss_dtable(sigma_s, R), R
    if mode == "iir":
        R = max(1, iir_radius(sigma_s, H, W))
        return deriche_dtable(sigma_s, R), R
    raise ValueError(mode)


def spatial(img, k):
    """Eq. (8): separable zero-extended filtering of img with table k."""
    f = _img(img)
    out = np.empty_like(f)
    _check(_load().or_spatial(_p(f), _p(out), f.shape[0], f.shape[1], _p(np.ascontiguousarray(k, np.float64)), len(k) - 1), "spatial")
    return out


# --------------------------------------------------------------------------
# filters
# --------------------------------------------------------------------------

def direct(img, sigma_r, k):
    """Eq. (1) with spatial table k (window R = len(k) - 1)."""
    f = _img(img)
    out = np.empty_like(f)
    k = np.ascontiguousarray(k, np.float64)
    _check(_load().or_direct(_p(f), _p(out), f.shape[0], f.shape[1], _p(k), len(k) - 1, float(sigma_r)), "direct")
    return out


def direct_gauss(img, sigma_s, sigma_r, window=None):
    """Eq. (1) with the Gaussian of eq. (2) over W = ceil(3 sigma_s)."""
    R = fir_radius(sigma_s) if window is None or window < 0 else int(window)
    return direct(img, sigma_r, gauss_table(sigma_s, R))


def center(img, mode=CENTER_MEAN):
    f = _img(img)
    return _load().or_center(_p(f), f.shape[0], f.shape[1], int(mode))


def gp_alg1(img, sigma_r, N, k, center_mode=CENTER_MEAN):
    """The Gauss-polynomial filter of Section 3 (eqs. (7)-(11) on the
    centred image, eq. (6); Algorithm 1 summarises it) with spatial table k."""
    f = _img(img)
    out = np.empty_like(f)
    k = np.ascontiguousarray(k, np.float64)
    _check(_load().or_gp_alg1(_p(f), _p(out), f.shape[0], f.shape[1], float(sigma_r), int(N), _p(k), len(k) - 1, int(center_mode)), "gp_alg1")
    return out


def gp_rescaled(img, sigma_r, N, k, center_mode=CENTER_MEAN, return_dm=False):
    """The same approximation in bounded channels u_n (see oracle.c)."""
    f = _img(img)
    out = np.empty_like(f)
    D = np.empty_like(f)
    M = np.empty_like(f)
    k = np.ascontiguousarray(k, np.float64)
    _check(_load().or_gp_rescaled(_p(f), _p(out), _p(D), _p(M), f.shape[0], f.shape[1], float(sigma_r), int(N), _p(k), len(k) - 1, int(center_mode)), "gp_rescaled")
    return (out, D, M) if return_dm else out


def gp(img, sigma_s, sigma_r, N, mode="fir", center_mode=CENTER_MEAN):
    """Algorithm 1 with the spatial filter of the given mode ('fir'/'iir'/'box')."""
    f = _img(img)
    k, _ = spatial_table(mode, sigma_s, *f.shape)
    return gp_alg1(f, sigma_r, N, k, center_mode)


def gp_grad(img, gout, sigma_r, N, k, kt, center_mode=CENTER_MEAN):
    """Analytic gradient of the rescaled form: (dL/df, dL/dlog s_s, dL/dlog s_r)."""
    f = _img(img)
    g = _img(gout)
    gf = np.empty_like(f)
    lss = ctypes.c_double()
    lsr = ctypes.c_double()
    k = np.ascontiguousarray(k, np.float64)
    kt = np.ascontiguousarray(kt, np.float64)
    assert len(k) == len(kt)
    _check(_load().or_gp_grad(_p(f), _p(g), f.shape[0], f.shape[1], float(sigma_r), int(N), _p(k), _p(kt), len(k) - 1,
                              int(center_mode), _p(gf), ctypes.byref(lss), ctypes.byref(lsr)), "gp_grad")
    return gf, lss.value, lsr.value


def gp_grad_mode(img, gout, sigma_s, sigma_r, N, mode="fir"):
    f = _img(img)
    k, R = spatial_table(mode, sigma_s, *f.shape)
    kt, R2 = spatial_dtable(mode, sigma_s, *f.shape)
    assert R == R2
    return gp_grad(f, gout, sigma_r, N, k, kt)


def _vol(v):
    a = np.ascontiguousarray(v, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("expected a T x H x W volume")
    return a


def spatial3(vol, kt, ks):
    """Separable zero-extended filtering of a volume: kt along axis 0, ks along
    axes 1 and 2."""
    v = _vol(vol)
    out = np.empty_like(v)
    kt = np.ascontiguousarray(kt, np.float64)
    ks = np.ascontiguousarray(ks, np.float64)
    _check(_load().or_spatial3(_p(v), _p(out), *v.shape, _p(kt), len(kt) - 1, _p(ks), len(ks) - 1), "spatial3")
    return out


def volume_direct(vol, sigma_r, kt, ks):
    """Eq. (1) over a volume, computed directly (small volumes)."""
    v = _vol(vol)
    out = np.empty_like(v)
    kt = np.ascontiguousarray(kt, np.float64)
    ks = np.ascontiguousarray(ks, np.float64)
    _check(_load().or_volume_direct(_p(v), _p(out), *v.shape, _p(kt), len(kt) - 1, _p(ks), len(ks) - 1,
                                    float(sigma_r)), "volume_direct")
    return out


def volume_gp(vol, sigma_r, N, kt, ks, center_mode=CENTER_MEAN):
    """Algorithm 1 over a volume (separable filtering over all three axes)."""
    v = _vol(vol)
    out = np.empty_like(v)
    kt = np.ascontiguousarray(kt, np.float64)
    ks = np.ascontiguousarray(ks, np.float64)
    _check(_load().or_volume_gp(_p(v), _p(out), *v.shape, float(sigma_r), int(N), _p(kt), len(kt) - 1, _p(ks),
                                len(ks) - 1, int(center_mode)), "volume_gp")
    return out


def volume_tables(sigma_t, sigma_s, T, H, W):
    """Deriche tables over the whole extent of each axis (the recursive mode)."""
    return (deriche_table(sigma_t, max(1, iir_radius(sigma_t, T, T))),
            deriche_table(sigma_s, max(1, iir_radius(sigma_s, H, W))))


def joint_direct(guide, data, sigma_r, k):
    """Joint (cross) bilateral filter computed directly: eq. (1) with the range
    argument taken from the guide and the average taken of the data."""
    g, f = _img(guide), _img(data)
    if g.shape != f.shape:
        raise ValueError("guide and data shapes differ")
    out = np.empty_like(g)
    k = np.ascontiguousarray(k, np.float64)
    _check(_load().or_joint_direct(_p(g), _p(f), _p(out), g.shape[0], g.shape[1], _p(k), len(k) - 1,
                                   float(sigma_r)), "joint_direct")
    return out


def joint_gp(guide, data, sigma_r, N, k, center_mode=CENTER_MEAN):
    """Gauss-polynomial approximation of the joint filter: Algorithm 1 with
    the guide in every range term (see oracle.c)."""
    g, f = _img(guide), _img(data)
    if g.shape != f.shape:
        raise ValueError("guide and data shapes differ")
    out = np.empty_like(g)
    k = np.ascontiguousarray(k, np.float64)
    _check(_load().or_joint_gp(_p(g), _p(f), _p(out), g.shape[0], g.shape[1], float(sigma_r), int(N), _p(k),
                               len(k) - 1, int(center_mode)), "joint_gp")
    return out


def brute_joint(guide, data, sigma_r, N, k, center_value=None):
    """The joint GP filter as one explicit double sum per pixel (tiny images):
    weights k(j) exp(-(t^2 + tau^2)/2) T_N(t tau) on the guide's centred
    values, T_N the degree-N Taylor polynomial of exp (eq. (5))."""
    g = np.asarray(guide, np.float64)
    f = np.asarray(data, np.float64)
    H, W = g.shape
    tc = g.mean() if center_value is None else center_value
    x = (g - tc) / sigma_r
    R = len(k) - 1
    out = np.empty_like(g)
    fact = np.array([math.factorial(n) for n in range(N + 1)], np.float64)
    for yi in range(H):
        for xi in range(W):
            tau = x[yi, xi]
            num = den = 0.0
            for yj in range(max(0, yi - R), min(H, yi + R + 1)):
                for xj in range(max(0, xi - R), min(W, xi + R + 1)):
                    t = x[yj, xj]
                    w = k[abs(yi - yj)] * k[abs(xi - xj)] * math.exp(-(t * t + tau * tau) / 2) * \
                        float(np.sum((t * tau) ** np.arange(N + 1) / fact))
                    num += w * f[yj, xj]
                    den += w
            out[yi, xi] = num / den
    return out


def gauss_poly(t, tau, sigma_r, N):
    """Eq. (5) at one (t, tau)."""
    return _load().or_gauss_poly(float(t), float(tau), float(sigma_r), int(N))


def mse_db(a, b):
    """The paper's error measure: 10 log10 of the mean squared difference."""
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return 10.0 * math.log10(float(np.mean(d * d)))


# --------------------------------------------------------------------------
# NumPy brute force for tiny images (independent of oracle.c)
# --------------------------------------------------------------------------

def brute_gp(img, sigma_r, N, k, center_value=None):
    """The GP filter as one explicit double sum per pixel: eq. (1) with the
    range kernel replaced by its Gauss-polynomial eq. (5) on centred data
    (the Proposition, eq. (6)).  O(|I| * (2R+1)^2 * N); tiny images only."""
    f = np.asarray(img, np.float64)
    Hh, Ww = f.shape
    R = len(k) - 1
    tc = f.mean() if center_value is None else center_value
    h = f - tc
    r2 = sigma_r * sigma_r
    fact = np.array([math.factorial(m) for m in range(N + 1)], dtype=np.float64)
    out = np.empty_like(f)
    for y in range(Hh):
        for x in range(Ww):
            tau = h[y, x]
            num = den = 0.0
            for dy in range(-R, R + 1):
                yy = y - dy
                if not 0 <= yy < Hh:
                    continue
                for dx in range(-R, R + 1):
                    xx = x - dx
                    if not 0 <= xx < Ww:
                        continue
                    t = h[yy, xx]
                    z = tau * t / r2
                    poly = float(np.sum(z ** np.arange(N + 1) / fact))
                    w = k[abs(dy)] * k[abs(dx)] * math.exp(-tau * tau / (2 * r2)) * math.exp(-t * t / (2 * r2)) * poly
                    num += w * t
                    den += w
            out[y, x] = num / den + tc
    return out


def brute_direct(img, sigma_r, k):
    """Eq. (1) as an explicit double sum (tiny images)."""
    f = np.asarray(img, np.float64)
    Hh, Ww = f.shape
    R = len(k) - 1
    out = np.empty_like(f)
    for y in range(Hh):
        for x in range(Ww):
            num = den = 0.0
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    yy, xx = y - dy, x - dx
                    if 0 <= yy < Hh and 0 <= xx < Ww:
                        w = k[abs(dy)] * k[abs(dx)] * math.exp(-(f[yy, xx] - f[y, x]) ** 2 / (2 * sigma_r ** 2))
                        num += w * f[yy, xx]
                        den += w
            out[y, x] = num / den
    return out


def brute_spatial(img, k):
    """Eq. (8) as a 2-D double sum (tiny images)."""
    f = np.asarray(img, np.float64)
    Hh, Ww = f.shape
    R = len(k) - 1
    out = np.zeros_like(f)
    for y in range(Hh):
        for x in range(Ww):
            s = 0.0
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    yy, xx = y - dy, x - dx
                    if 0 <= yy < Hh and 0 <= xx < Ww:
                        s += k[abs(dy)] * k[abs(dx)] * f[yy, xx]
            out[y, x] = s
    return out
