"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a brute force
written independently in NumPy, a closed form, a library routine (SciPy), an
invariant that the paper states, a printed number of the paper, or finite
differences.  Images are non-square so that a swapped row/column index fails.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage, special

import oracle
from synthimg import voronoi_image

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_img(H, W, seed, lo=0.0, hi=255.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=(H, W))


# ---------------------------------------------------------------------------
# eqs. (3)-(5): the factorisation and the Gauss-polynomial
# ---------------------------------------------------------------------------

def test_fig1_scaling_factor():
    g = json.load(open(os.path.join(GOLDEN, "fig1_decomposition.json")))
    tau, sr = g["tau"], g["sigma_r"]
    # first factor of eq. (3): the scaling between panel (a) and (b)x(c)
    factor = math.exp(-tau * tau / (2 * sr * sr))
    assert abs(factor - g["scaling_factor_about"]) <= g["scaling_factor_rel_tol"] * g["scaling_factor_about"]
    # eq. (3) is exact: with enough Taylor terms, eq. (5) reproduces g_r(t - tau)
    for t in np.linspace(*g["range"], 52):
        ref = math.exp(-(t - tau) ** 2 / (2 * sr * sr))
        assert oracle.gauss_poly(t, tau, sr, 250) == pytest.approx(ref, rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("N", [10, 20])
@pytest.mark.parametrize("tau", [0.0, 10.0, 50.0, 120.0])
def test_gauss_poly_incomplete_gamma(N, tau):
    # Fig. 2/3 settings (sigma_r = 30, degree 10 / 20, tau in {0,10,50,120}).
    # The truncated exponential series is e^x Q(N+1, x) for x >= 0.
    sr = 30.0
    for t in np.linspace(0.0, 255.0, 35):
        x = tau * t / sr ** 2
        TN = math.exp(x) * special.gammaincc(N + 1, x) if x > 0 else 1.0
        ref = math.exp(-tau ** 2 / (2 * sr ** 2)) * math.exp(-t ** 2 / (2 * sr ** 2)) * TN
        assert oracle.gauss_poly(t, tau, sr, N) == pytest.approx(ref, rel=1e-11, abs=1e-300)


def test_gauss_poly_exact_at_tau_zero():
    # "when tau = 0 there is nothing to approximate"
    for t in np.linspace(-200, 200, 41):
        assert oracle.gauss_poly(t, 0.0, 30.0, 0) == pytest.approx(math.exp(-t * t / 1800.0), rel=1e-14)


def test_gauss_poly_error_grows_with_tau():
    # Fig. 3(a): for a fixed degree the error grows with |tau|; centring helps
    sr, N = 30.0, 20
    ts = np.linspace(0, 255, 256)

    def maxerr(tau, shift=0.0):
        return max(abs(oracle.gauss_poly(t - shift, tau - shift, sr, N) - math.exp(-(t - tau) ** 2 / (2 * sr * sr))) for t in ts)

    errs = [maxerr(tau) for tau in (0.0, 10.0, 50.0, 120.0)]
    assert errs[0] < 1e-15 or errs[0] <= errs[1]
    assert errs[1] < errs[2] < errs[3]
    # centring the range at 127.5 reduces the worst error for tau = 120
    assert maxerr(120.0, shift=127.5) < 1e-3 * errs[3]


def test_even_degree_positive_odd_not():
    # T_N(x) > 0 for all real x when N is even; odd N goes negative
    xs = np.linspace(-25, 25, 2001)
    for N in (2, 10, 20, 40):
        vals = [oracle.gauss_poly(x, 1.0, 1.0, N) for x in xs]
        assert min(vals) > 0
    assert min(oracle.gauss_poly(x, 1.0, 1.0, 21) for x in xs) < 0


# ---------------------------------------------------------------------------
# spatial filter, eq. (8), and the kernel tables
# ---------------------------------------------------------------------------

def test_spatial_matches_2d_double_sum():
    f = rand_img(7, 11, 1)
    for k in (oracle.gauss_table(1.3, 4), oracle.deriche_table(1.7, 6)):
        assert np.allclose(oracle.spatial(f, k), oracle.brute_spatial(f, k), rtol=1e-13, atol=1e-10)


def test_spatial_matches_scipy():
    f = rand_img(23, 17, 2)
    k = oracle.gauss_table(2.0, 6)
    w = np.concatenate([k[:0:-1], k])
    ref = ndimage.correlate1d(ndimage.correlate1d(f, w, axis=0, mode="constant"), w, axis=1, mode="constant")
    assert np.allclose(oracle.spatial(f, k), ref, rtol=1e-13, atol=1e-10)


def test_gauss_table_closed_form():
    k = oracle.gauss_table(2.5, 8)
    assert np.allclose(k, np.exp(-np.arange(9) ** 2 / 12.5), rtol=1e-15)


def test_deriche_fit_to_gaussian():
    # the published constants approximate exp(-t^2/2) with a small error
    ts = np.linspace(0, 8, 801)
    h = np.array([oracle.deriche_h(t) for t in ts])
    assert np.max(np.abs(h - np.exp(-ts ** 2 / 2))) < 6e-4
    assert h[0] == pytest.approx(1.680 - 0.6803, rel=1e-15)
    tt = np.linspace(0, 40, 400001)
    hh = np.array([oracle.deriche_h(t) for t in tt[::100]])
    integ = 2 * np.trapezoid(np.array([oracle.deriche_h(t) for t in tt]), tt)
    assert integ == pytest.approx(math.sqrt(2 * math.pi), rel=3e-4)
    assert hh[-1] < 1e-28
    # sampled tables agree with the sampled Gaussian at every scale
    for s in (1.0, 3.0, 10.0, 20.0):
        R = int(6 * s)
        assert np.max(np.abs(oracle.deriche_table(s, R) - oracle.gauss_table(s, R))) < 6e-4


@pytest.mark.parametrize("kind", ["gauss", "deriche"])
def test_dtables_are_log_sigma_derivatives(kind):
    tab = oracle.gauss_table if kind == "gauss" else oracle.deriche_table
    dtab = oracle.gauss_dtable if kind == "gauss" else oracle.deriche_dtable
    s, R, h = 2.3, 14, 1e-5
    fd = (tab(s * math.exp(h), R) - tab(s * math.exp(-h), R)) / (2 * h)
    assert np.allclose(dtab(s, R), fd, rtol=1e-7, atol=1e-10)


# ---------------------------------------------------------------------------
# eq. (1), the direct filter
# ---------------------------------------------------------------------------

def test_direct_matches_double_sum():
    f = rand_img(6, 9, 3)
    for s, r in ((1.0, 30.0), (1.5, 10.0)):
        k = oracle.gauss_table(s, oracle.fir_radius(s))
        assert np.allclose(oracle.direct(f, r, k), oracle.brute_direct(f, r, k), rtol=1e-13, atol=1e-10)


def test_direct_wide_range_kernel_is_normalised_blur():
    f = rand_img(21, 30, 4)
    k = oracle.gauss_table(2.0, 6)
    w = np.concatenate([k[:0:-1], k])

    def blur(a):
        return ndimage.correlate1d(ndimage.correlate1d(a, w, axis=0, mode="constant"), w, axis=1, mode="constant")

    ref = blur(f) / blur(np.ones_like(f))
    assert np.allclose(oracle.direct(f, 1e8, k), ref, rtol=1e-9, atol=1e-8)


def test_direct_constant_image():
    f = np.full((9, 13), 77.25)
    assert np.allclose(oracle.direct_gauss(f, 2.0, 30.0), 77.25, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Algorithm 1 against brute force, the rescaled form and the limits
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", range(6))
def test_alg1_matches_explicit_double_sum(case):
    rng = np.random.default_rng(100 + case)
    H, W = int(rng.integers(5, 9)), int(rng.integers(6, 11))
    f = rng.uniform(0, 255, size=(H, W))
    s = float(rng.uniform(0.6, 1.8))
    r = float(rng.uniform(25, 70))
    N = [0, 2, 5, 8, 12, 20][case]
    for kind in ("gauss", "deriche"):
        R = oracle.fir_radius(s) if kind == "gauss" else 2 * oracle.fir_radius(s)
        k = oracle.gauss_table(s, R) if kind == "gauss" else oracle.deriche_table(s, R)
        ref = oracle.brute_gp(f, r, N, k)
        got = oracle.gp_alg1(f, r, N, k)
        assert np.allclose(got, ref, rtol=0, atol=1e-9), (kind, np.max(np.abs(got - ref)))


def test_alg1_odd_degree_matches_double_sum():
    f = rand_img(6, 7, 9, 80, 180)
    k = oracle.gauss_table(1.2, 4)
    for N in (1, 3, 7):
        assert np.allclose(oracle.gp_alg1(f, 60.0, N, k), oracle.brute_gp(f, 60.0, N, k), rtol=0, atol=1e-9)


def test_alg1_equals_rescaled_form():
    f = voronoi_image(64, 48, 12, seed=7).astype(np.float64)
    for mode, s in (("fir", 3.0), ("iir", 2.5)):
        k, _ = oracle.spatial_table(mode, s, *f.shape)
        a = oracle.gp_alg1(f, 30.0, 20, k)
        b = oracle.gp_rescaled(f, 30.0, 20, k)
        assert np.max(np.abs(a - b)) < 1e-9


def test_alg1_converges_to_direct_as_degree_grows():
    f = voronoi_image(40, 56, 10, seed=8).astype(np.float64)
    s, r = 2.0, 30.0
    k = oracle.gauss_table(s, oracle.fir_radius(s))
    ref = oracle.direct(f, r, k)
    errs = [np.max(np.abs(oracle.gp_alg1(f, r, N, k) - ref)) for N in (10, 20, 40, 60)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-6
    # the same holds with the recursive-Gaussian kernel and its own direct filter
    kd, _ = oracle.spatial_table("iir", s, *f.shape)
    assert np.max(np.abs(oracle.gp_alg1(f, r, 60, kd) - oracle.direct(f, r, kd))) < 1e-6


def test_alg1_wide_range_kernel_is_normalised_blur():
    f = rand_img(19, 26, 10)
    k = oracle.gauss_table(1.5, 5)
    w = np.concatenate([k[:0:-1], k])

    def blur(a):
        return ndimage.correlate1d(ndimage.correlate1d(a, w, axis=0, mode="constant"), w, axis=1, mode="constant")

    ref = blur(f) / blur(np.ones_like(f))
    assert np.allclose(oracle.gp_alg1(f, 1e7, 2, k), ref, rtol=0, atol=1e-7)


def test_alg1_constant_image_unchanged():
    f = np.full((11, 8), 201.5)
    for N in (0, 1, 20):
        out = oracle.gp(f, 2.0, 30.0, N)
        assert np.max(np.abs(out - 201.5)) < 1e-12


def test_alg1_translation_equivariance():
    # the Proposition, eq. (6): shifting the intensities shifts the output
    f = voronoi_image(30, 41, 8, seed=11).astype(np.float64)
    a = oracle.gp(f, 2.0, 30.0, 20)
    b = oracle.gp(f + 37.5, 2.0, 30.0, 20)
    assert np.max(np.abs(b - (a + 37.5))) < 1e-9


def test_alg1_negation_and_scale():
    f = voronoi_image(33, 27, 8, seed=12).astype(np.float64)
    a = oracle.gp(f, 2.0, 30.0, 20)
    assert np.max(np.abs(oracle.gp(-f, 2.0, 30.0, 20) + a)) < 1e-9
    assert np.max(np.abs(oracle.gp(2.5 * f, 2.0, 75.0, 20) - 2.5 * a)) < 1e-8


def test_alg1_transpose_and_flips():
    f = voronoi_image(29, 37, 9, seed=13).astype(np.float64)
    for mode in ("fir", "iir"):
        a = oracle.gp(f, 2.0, 30.0, 20, mode)
        assert np.max(np.abs(oracle.gp(f.T.copy(), 2.0, 30.0, 20, mode) - a.T)) < 1e-9
        assert np.max(np.abs(oracle.gp(f[::-1].copy(), 2.0, 30.0, 20, mode) - a[::-1])) < 1e-9
        assert np.max(np.abs(oracle.gp(f[:, ::-1].copy(), 2.0, 30.0, 20, mode) - a[:, ::-1])) < 1e-9


def test_alg1_even_degree_stays_in_range():
    f = voronoi_image(48, 40, 15, seed=14).astype(np.float64)
    for N in (2, 8, 20):
        out = oracle.gp(f, 2.0, 25.0, N)
        assert out.min() >= f.min() - 1e-9 and out.max() <= f.max() + 1e-9


def test_alg1_kernel_gain_invariance():
    f = rand_img(17, 22, 15)
    k = oracle.gauss_table(1.5, 5)
    assert np.max(np.abs(oracle.gp_alg1(f, 30.0, 20, k) - oracle.gp_alg1(f, 30.0, 20, 3.7 * k))) < 1e-9


def test_centres_agree_in_the_limit_and_differ_at_low_degree():
    f = voronoi_image(24, 31, 7, seed=16).astype(np.float64)
    k = oracle.gauss_table(1.5, 5)
    outs = [oracle.gp_alg1(f, 30.0, 60, k, c) for c in (oracle.CENTER_MEAN, oracle.CENTER_MIDRANGE)]
    assert np.max(np.abs(outs[0] - outs[1])) < 1e-6
    # without centring |tau t| / sigma_r^2 reaches (255/30)^2 = 72, so the
    # series needs a far higher degree before it reaches the same limit
    uncentred = oracle.gp_alg1(f, 30.0, 150, k, oracle.CENTER_NONE)
    assert np.max(np.abs(outs[0] - uncentred)) < 1e-6
    low = [oracle.gp_alg1(f, 30.0, 8, k, c) for c in (oracle.CENTER_MEAN, oracle.CENTER_NONE)]
    ref = oracle.direct(f, 30.0, k)
    # centring reduces the error of a low-degree approximation
    assert np.max(np.abs(low[0] - ref)) < np.max(np.abs(low[1] - ref))


@pytest.mark.parametrize("N", [2, 6, 12])
def test_midrange_centre_matches_double_sum_about_the_midrange(N):
    # Proposition eq. (6) with t_c the midpoint of the intensity range: the
    # filter equals the explicit double sum with the Gauss-polynomial weights
    # taken about (min + max) / 2.  The image is skewed (most pixels dark), so
    # the mean and the midrange differ by far more than the tolerance and a
    # midrange that silently fell back to the mean would fail.
    rng = np.random.default_rng(140 + N)
    f = rng.uniform(0, 80, size=(7, 9))
    f[0, 0], f[6, 8] = 5.0, 250.0
    k = oracle.gauss_table(1.3, 4)
    mid = 0.5 * (f.min() + f.max())
    assert abs(mid - f.mean()) > 50.0
    assert oracle.center(f, oracle.CENTER_MIDRANGE) == mid
    got = oracle.gp_alg1(f, 40.0, N, k, oracle.CENTER_MIDRANGE)
    ref = oracle.brute_gp(f, 40.0, N, k, center_value=mid)
    assert np.allclose(got, ref, rtol=0, atol=1e-9), np.max(np.abs(got - ref))
    # at these low degrees the centre changes the result
    other = oracle.brute_gp(f, 40.0, N, k, center_value=f.mean())
    assert np.max(np.abs(ref - other)) > 1e-3


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------

def _loss(f, target, s, r, N, mode, R):
    k = oracle.gauss_table(s, R) if mode == "fir" else oracle.deriche_table(s, R)
    out = oracle.gp_alg1(f, r, N, k)
    return 0.5 * float(np.sum((out - target) ** 2)), out


@pytest.mark.parametrize("mode", ["fir", "iir"])
def test_gradients_match_finite_differences(mode):
    f = voronoi_image(9, 11, 4, seed=17).astype(np.float64)
    target = voronoi_image(9, 11, 4, seed=18).astype(np.float64)
    s, r, N = 1.3, 25.0, 8
    R = oracle.fir_radius(s) if mode == "fir" else 10
    _, out = _loss(f, target, s, r, N, mode, R)
    k = oracle.gauss_table(s, R) if mode == "fir" else oracle.deriche_table(s, R)
    kt = oracle.gauss_dtable(s, R) if mode == "fir" else oracle.deriche_dtable(s, R)
    gf, gls, glr = oracle.gp_grad(f, out - target, r, N, k, kt)
    h = 1e-4
    fd_f = np.empty_like(f)
    for idx in np.ndindex(f.shape):
        fp = f.copy(); fp[idx] += h
        fm = f.copy(); fm[idx] -= h
        fd_f[idx] = (_loss(fp, target, s, r, N, mode, R)[0] - _loss(fm, target, s, r, N, mode, R)[0]) / (2 * h)
    scale = np.max(np.abs(fd_f))
    assert np.max(np.abs(gf - fd_f)) < 1e-6 * scale
    fd_s = (_loss(f, target, s * math.exp(h), r, N, mode, R)[0] - _loss(f, target, s * math.exp(-h), r, N, mode, R)[0]) / (2 * h)
    fd_r = (_loss(f, target, s, r * math.exp(h), N, mode, R)[0] - _loss(f, target, s, r * math.exp(-h), N, mode, R)[0]) / (2 * h)
    assert gls == pytest.approx(fd_s, rel=1e-6, abs=1e-8 * scale)
    assert glr == pytest.approx(fd_r, rel=1e-6, abs=1e-8 * scale)


def test_sigma_s_gradient_ignores_kernel_gain():
    f = rand_img(10, 8, 19)
    g = rand_img(10, 8, 20, -1, 1)
    k = oracle.gauss_table(1.4, 5)
    kt = oracle.gauss_dtable(1.4, 5)
    _, a, _ = oracle.gp_grad(f, g, 30.0, 10, k, kt)
    _, b, _ = oracle.gp_grad(f, g, 30.0, 10, k, kt + 0.37 * k)
    assert b == pytest.approx(a, rel=1e-9, abs=1e-9)


# ---------------------------------------------------------------------------
# error measure and the Table 1 trend
# ---------------------------------------------------------------------------

def test_mse_db_definition():
    a = np.zeros((4, 4))
    assert oracle.mse_db(a, a + 1.0) == pytest.approx(0.0)
    assert oracle.mse_db(a, a + 10.0) == pytest.approx(20.0)


def test_table1_trend_error_grows_with_sigma_s():
    # Table 1: at sigma_r = 30 and N = 20 the GP error to eq. (1) rises with
    # sigma_s (the Peppers values themselves are not reproducible here)
    g = json.load(open(os.path.join(GOLDEN, "table1_setting.json")))
    f = voronoi_image(64, 64, 10, seed=21).astype(np.float64)
    db = []
    for s in g["sigma_s"][:4]:
        db.append(oracle.mse_db(oracle.gp(f, s, g["sigma_r"], g["N"]), oracle.direct_gauss(f, s, g["sigma_r"])))
    assert all(b > a for a, b in zip(db, db[1:])), db


# ---------------------------------------------------------------------------
# joint (cross) bilateral filter: range kernel on a guide, average of data
# ---------------------------------------------------------------------------

def test_joint_direct_reduces_to_eq1_when_guide_is_data():
    f = rand_img(9, 14, 21)
    k = oracle.gauss_table(1.5, oracle.fir_radius(1.5))
    assert np.allclose(oracle.joint_direct(f, f, 25.0, k), oracle.direct(f, 25.0, k), rtol=0, atol=1e-11)


def test_joint_direct_matches_double_sum():
    g, f = rand_img(6, 8, 22), rand_img(6, 8, 23)
    k = oracle.gauss_table(1.2, 4)
    ref = np.empty_like(g)
    for yi in range(6):
        for xi in range(8):
            num = den = 0.0
            for yj in range(6):
                for xj in range(8):
                    if abs(yi - yj) > 4 or abs(xi - xj) > 4:
                        continue
                    w = k[abs(yi - yj)] * k[abs(xi - xj)] * math.exp(-(g[yj, xj] - g[yi, xi]) ** 2 / (2 * 30.0 ** 2))
                    num += w * f[yj, xj]
                    den += w
            ref[yi, xi] = num / den
    assert np.allclose(oracle.joint_direct(g, f, 30.0, k), ref, rtol=0, atol=1e-10)


@pytest.mark.parametrize("N", [0, 3, 8, 20])
def test_joint_gp_reduces_to_alg1_when_guide_is_data(N):
    # with g = f, F f = t_c F + sigma_r F H, so the joint numerator is
    # t_c Q + sigma_r P of Algorithm 1 and the outputs agree exactly
    f = voronoi_image(30, 44, 9, seed=24).astype(np.float64)
    for mode, s in (("fir", 2.0), ("iir", 3.0)):
        k, _ = oracle.spatial_table(mode, s, *f.shape)
        assert np.max(np.abs(oracle.joint_gp(f, f, 30.0, N, k) - oracle.gp_alg1(f, 30.0, N, k))) < 1e-9


@pytest.mark.parametrize("case", range(4))
def test_joint_gp_matches_explicit_double_sum(case):
    rng = np.random.default_rng(300 + case)
    H, W = int(rng.integers(5, 8)), int(rng.integers(6, 10))
    g = rng.uniform(0, 255, size=(H, W))
    f = rng.uniform(0, 255, size=(H, W))
    s = float(rng.uniform(0.6, 1.6))
    r = float(rng.uniform(30, 70))
    N = [0, 4, 10, 20][case]
    for kind in ("gauss", "deriche"):
        R = oracle.fir_radius(s) if kind == "gauss" else 2 * oracle.fir_radius(s)
        k = oracle.gauss_table(s, R) if kind == "gauss" else oracle.deriche_table(s, R)
        ref = oracle.brute_joint(g, f, r, N, k)
        assert np.allclose(oracle.joint_gp(g, f, r, N, k), ref, rtol=0, atol=1e-9), kind


def test_joint_gp_linear_in_data_and_constant_data():
    g = voronoi_image(20, 33, 7, seed=25).astype(np.float64)
    f1, f2 = rand_img(20, 33, 26), rand_img(20, 33, 27)
    k = oracle.gauss_table(2.0, 6)
    a = oracle.joint_gp(g, 2.0 * f1 - 3.0 * f2, 25.0, 12, k)
    b = 2.0 * oracle.joint_gp(g, f1, 25.0, 12, k) - 3.0 * oracle.joint_gp(g, f2, 25.0, 12, k)
    assert np.max(np.abs(a - b)) < 1e-9
    # constant data come back unchanged, whatever the guide (even degree)
    assert np.max(np.abs(oracle.joint_gp(g, np.full_like(g, 42.5), 25.0, 12, k) - 42.5)) < 1e-11


def test_joint_gp_wide_range_kernel_is_normalised_blur_of_data():
    g, f = rand_img(17, 23, 28), rand_img(17, 23, 29)
    k = oracle.gauss_table(1.5, 5)
    w = np.concatenate([k[:0:-1], k])

    def blur(a):
        return ndimage.correlate1d(ndimage.correlate1d(a, w, axis=0, mode="constant"), w, axis=1, mode="constant")

    assert np.allclose(oracle.joint_gp(g, f, 1e7, 2, k), blur(f) / blur(np.ones_like(f)), rtol=0, atol=1e-7)


def test_joint_gp_converges_to_joint_direct_and_ignores_guide_offset():
    g = voronoi_image(36, 50, 10, seed=30).astype(np.float64)
    f = voronoi_image(36, 50, 10, seed=31).astype(np.float64)
    k = oracle.gauss_table(2.0, oracle.fir_radius(2.0))
    ref = oracle.joint_direct(g, f, 30.0, k)
    errs = [np.max(np.abs(oracle.joint_gp(g, f, 30.0, N, k) - ref)) for N in (10, 20, 40, 60)]
    assert errs[0] > errs[1] > errs[2] > errs[3] and errs[3] < 1e-6
    # the range kernel sees guide differences only: with mean centring, a
    # constant added to the guide changes nothing
    assert np.max(np.abs(oracle.joint_gp(g + 37.0, f, 30.0, 20, k) - oracle.joint_gp(g, f, 30.0, 20, k))) < 1e-9


# ---------------------------------------------------------------------------
# volumes: separable filtering over three axes
# ---------------------------------------------------------------------------

def test_spatial3_matches_scipy_and_triple_sum():
    v = np.random.default_rng(50).uniform(0, 1, size=(5, 7, 9))
    kt, ks = oracle.gauss_table(0.9, 2), oracle.gauss_table(1.2, 3)
    wt, ws = np.concatenate([kt[:0:-1], kt]), np.concatenate([ks[:0:-1], ks])
    ref = ndimage.correlate1d(v, wt, axis=0, mode="constant")
    ref = ndimage.correlate1d(ref, ws, axis=1, mode="constant")
    ref = ndimage.correlate1d(ref, ws, axis=2, mode="constant")
    got = oracle.spatial3(v, kt, ks)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)
    # one output by the explicit triple sum
    t0, y0, x0 = 2, 3, 4
    acc = 0.0
    for t in range(5):
        for y in range(7):
            for x in range(9):
                if abs(t - t0) <= 2 and abs(y - y0) <= 3 and abs(x - x0) <= 3:
                    acc += kt[abs(t - t0)] * ks[abs(y - y0)] * ks[abs(x - x0)] * v[t, y, x]
    assert got[t0, y0, x0] == pytest.approx(acc, rel=1e-13)


def test_volume_direct_matches_quadruple_sum():
    v = np.random.default_rng(51).uniform(0, 255, size=(3, 5, 6))
    kt, ks = oracle.gauss_table(0.8, 1), oracle.gauss_table(1.0, 2)
    got = oracle.volume_direct(v, 30.0, kt, ks)
    t0, y0, x0 = 1, 2, 3
    num = den = 0.0
    for t in range(3):
        for y in range(5):
            for x in range(6):
                if abs(t - t0) <= 1 and abs(y - y0) <= 2 and abs(x - x0) <= 2:
                    w = kt[abs(t - t0)] * ks[abs(y - y0)] * ks[abs(x - x0)] * \
                        math.exp(-(v[t, y, x] - v[t0, y0, x0]) ** 2 / 1800.0)
                    num += w * v[t, y, x]
                    den += w
    assert got[t0, y0, x0] == pytest.approx(num / den, rel=1e-13)


def test_volume_gp_single_frame_is_alg1():
    # one frame: the time filter multiplies every channel by kt[0], which the
    # ratio cancels
    f = voronoi_image(30, 41, 8, seed=52).astype(np.float64)
    kt, ks = oracle.deriche_table(2.0, 10), oracle.deriche_table(3.0, 40)
    got = oracle.volume_gp(f[None], 30.0, 20, kt, ks)[0]
    assert np.max(np.abs(got - oracle.gp_alg1(f, 30.0, 20, ks))) < 1e-9


def test_volume_gp_against_direct_limits_and_invariants():
    rng = np.random.default_rng(53)
    vol = np.stack([voronoi_image(18, 24, 6, seed=60 + t) for t in range(6)]).astype(np.float64)
    kt, ks = oracle.gauss_table(1.0, 3), oracle.gauss_table(1.5, 5)
    ref = oracle.volume_direct(vol, 30.0, kt, ks)
    errs = [np.max(np.abs(oracle.volume_gp(vol, 30.0, N, kt, ks) - ref)) for N in (10, 20, 40, 60)]
    assert errs[0] > errs[1] > errs[2] > errs[3] and errs[3] < 1e-6
    # constant volume, translation, sigma_r -> inf blur
    c = np.full((4, 9, 11), 99.5)
    assert np.max(np.abs(oracle.volume_gp(c, 30.0, 20, kt, ks) - 99.5)) < 1e-11
    a = oracle.volume_gp(vol + 21.0, 30.0, 20, kt, ks)
    assert np.max(np.abs(a - (oracle.volume_gp(vol, 30.0, 20, kt, ks) + 21.0))) < 1e-9
    u = rng.uniform(0, 255, size=(4, 9, 11))
    blur = oracle.spatial3(u, kt, ks) / oracle.spatial3(np.ones_like(u), kt, ks)
    assert np.allclose(oracle.volume_gp(u, 1e7, 2, kt, ks), blur, rtol=0, atol=1e-7)


# ---------------------------------------------------------------------------
# the degree rule: the Gauss-polynomial weight error and the Poisson tail
# ---------------------------------------------------------------------------

def test_weight_error_is_the_poisson_tail_at_equal_intensities():
    # eq. (5) at t = tau: 1 - w~ = 1 - e^{-lam} T_N(lam) = P(Poisson(lam) > N)
    from scipy import stats
    for tau, N in ((1.0, 4), (2.5, 10), (4.0, 20), (3.0, 6), (0.3, 0)):
        lam = tau * tau
        assert 1.0 - oracle.gauss_poly(30.0 * tau, 30.0 * tau, 30.0, N) == pytest.approx(
            stats.poisson.sf(N, lam), rel=1e-10, abs=1e-15)


def test_poisson_tail_bounds_every_weight_error():
    # for |t|, |tau| <= xmax and N >= xmax^2 - 1, |w - w~| <= P(Poisson(xmax^2) > N)
    from scipy import stats
    rng = np.random.default_rng(70)
    for xmax in (1.0, 2.0, 3.0, 4.0):
        lam = xmax * xmax
        for N in range(int(math.ceil(lam - 1)), int(lam) + 8):
            bound = stats.poisson.sf(N, lam)
            ts = np.concatenate([rng.uniform(-xmax, xmax, 600), [xmax, -xmax]])
            taus = np.concatenate([rng.uniform(-xmax, xmax, 600), [xmax, xmax]])
            for t, tau in zip(ts, taus):
                err = abs(math.exp(-(t - tau) ** 2 / 2) - oracle.gauss_poly(30.0 * t, 30.0 * tau, 30.0, N))
                assert err <= bound * (1 + 1e-9) + 1e-15



# ---------------------------------------------------------------------------
# the box spatial kernel (Section 3, after eq. (11): any constant-time spatial
# filter can stand in for the Gaussian of eq. (8))
# ---------------------------------------------------------------------------

def _box_blur(a, R):
    # SciPy's uniform filter is the window mean with zeros outside the image
    return ndimage.uniform_filter(a, size=2 * R + 1, mode="constant", cval=0.0) * (2 * R + 1) ** 2


def test_box_window_is_the_fir_window():
    for s in (0.3, 1.0, 2.0, 3.4, 10.0, 40.0):
        k, R = oracle.spatial_table("box", s, 64, 64)
        assert R == oracle.fir_radius(s) and np.array_equal(k, np.ones(R + 1))


@pytest.mark.parametrize("R", [1, 3, 7, 30])
def test_box_spatial_matches_scipy_uniform_filter(R):
    # R = 30 is wider than the image: every window clips at the borders
    f = rand_img(23, 17, 200 + R)
    got = oracle.spatial(f, oracle.box_table(R))
    assert np.allclose(got, _box_blur(f, R), rtol=1e-12, atol=1e-9)
    if R <= 3:
        assert np.allclose(got, oracle.brute_spatial(f, oracle.box_table(R)), rtol=1e-13, atol=1e-10)


def test_box_direct_matches_double_sum_and_wide_range_is_box_mean():
    f = rand_img(7, 9, 210)
    k = oracle.box_table(2)
    assert np.allclose(oracle.direct(f, 25.0, k), oracle.brute_direct(f, 25.0, k), rtol=1e-13, atol=1e-10)
    g = rand_img(21, 30, 211)
    ref = _box_blur(g, 4) / _box_blur(np.ones_like(g), 4)
    assert np.allclose(oracle.direct(g, 1e8, oracle.box_table(4)), ref, rtol=1e-9, atol=1e-8)


@pytest.mark.parametrize("N", [0, 4, 10, 20])
def test_box_alg1_matches_explicit_double_sum(N):
    rng = np.random.default_rng(220 + N)
    f = rng.uniform(0, 255, size=(6, 8))
    k = oracle.box_table(2)
    ref = oracle.brute_gp(f, 45.0, N, k)
    assert np.allclose(oracle.gp_alg1(f, 45.0, N, k), ref, rtol=0, atol=1e-9)
    assert np.allclose(oracle.gp_rescaled(f, 45.0, N, k), ref, rtol=0, atol=1e-9)


def test_box_alg1_converges_to_box_direct_and_wide_range_is_box_mean():
    f = voronoi_image(40, 56, 10, seed=230).astype(np.float64)
    k, R = oracle.spatial_table("box", 2.0, *f.shape)
    ref = oracle.direct(f, 30.0, k)
    errs = [np.max(np.abs(oracle.gp_alg1(f, 30.0, N, k) - ref)) for N in (10, 20, 40, 60)]
    assert errs[0] > errs[1] > errs[2] > errs[3] and errs[3] < 1e-6
    blur = _box_blur(f, R) / _box_blur(np.ones_like(f), R)
    assert np.allclose(oracle.gp_alg1(f, 1e7, 2, k), blur, rtol=0, atol=1e-7)


def test_box_covering_the_image_is_a_tone_map():
    # a window wider than the image holds every pixel: the result at i depends
    # on f(i) only, through the Gauss-polynomial weights of eq. (5) over the
    # whole image (with t_c the mean)
    rng = np.random.default_rng(240)
    f = rng.choice(np.array([12.0, 80.0, 81.5, 140.0, 230.0]), size=(9, 12))
    sr, N = 40.0, 12
    out = oracle.gp_alg1(f, sr, N, oracle.box_table(12))
    tc = f.mean()
    h = (f - tc).ravel()
    for v in np.unique(f):
        w = np.array([oracle.gauss_poly(t, v - tc, sr, N) for t in h])
        expect = tc + np.sum(w * h) / np.sum(w)
        assert np.allclose(out[f == v], expect, rtol=0, atol=1e-9)
