"""GP forward on the GPU against the FP64 oracle (element by element).

Tolerance: 1e-3 absolute on 0..255 data, the target the FP32 channels with an
FP64 recombination are held to.  Every case names itself before it runs."""
import numpy as np
import pytest
import torch

import oracle
import synthimg
from gpu_util import note, oracle_gp, oracle_gp_at, oracle_lines, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00077_amd as m
    return m


def run(bf, img, ss, sr, N, spatial, center="mean", check=True):
    note(f"gp_forward {img.shape} ss={ss} sr={sr} N={N} {spatial} {center}")
    out = bf.gp_forward(to_dev(img), ss, sr, N, spatial=spatial, center=center, check=check)
    return to_np(out)


@pytest.mark.parametrize("spatial", ["fir", "iir"])
def test_small_config_matches_oracle(bf, spatial):
    img = synthimg.small_256()
    got = run(bf, img, 3.0, 30.0, 20, spatial)
    ref = oracle_gp(img, 3.0, 30.0, 20, spatial)
    err = np.max(np.abs(got - ref))
    direct = oracle.direct_gauss(img.astype(np.float64), 3.0, 30.0)
    print(f"{spatial}: max|gpu-oracle| {err:.2e}; vs direct: max {np.max(np.abs(got - direct)):.3f}, "
          f"{oracle.mse_db(got, direct):.2f} dB")
    assert err <= TOL


@pytest.mark.parametrize("shape", [(1, 1), (1, 50), (50, 1), (37, 70), (64, 64), (130, 97), (33, 257), (100, 129)])
@pytest.mark.parametrize("spatial", ["fir", "iir"])
def test_ragged_shapes(bf, shape, spatial):
    H, W = shape
    img = synthimg.voronoi_image(H, W, max(1, H * W // 400), seed=H * 1000 + W)
    for ss in (1.0, 2.5):
        got = run(bf, img, ss, 30.0, 20, spatial)
        ref = oracle_gp(img, ss, 30.0, 20, spatial)
        assert np.max(np.abs(got - ref)) <= TOL, (ss, np.max(np.abs(got - ref)))


@pytest.mark.parametrize("ss", [0.4, 4.0, 6.5, 8.0])
def test_fir_radius_range(bf, ss):
    img = synthimg.voronoi_image(90, 150, 30, seed=77)
    got = run(bf, img, ss, 25.0, 20, "fir")
    assert np.max(np.abs(got - oracle_gp(img, ss, 25.0, 20, "fir"))) <= TOL


@pytest.mark.parametrize("ss", [4.3, 4.5, 5.0, 5.33, 5.34])
def test_fir_radii_13_to_17(bf, ss):
    # radii 13..16 run the register-column tile (the widest of them, 15 and
    # 16, are what the tuned crossover sends sigma_s 5 to at 1 MP); radius 17
    # is the first of the region tile, with its 32-row tiles.  Two ragged
    # shapes: several tiles in each direction with a partial last tile.
    R = bf.fir_radius(ss)
    assert R == {4.3: 13, 4.5: 14, 5.0: 15, 5.33: 16, 5.34: 17}[ss]
    for shape, seed in (((90, 150), 77), ((257, 301), 78)):
        img = synthimg.voronoi_image(*shape, 40, seed=seed)
        got = run(bf, img, ss, 25.0, 20, "fir")
        err = np.max(np.abs(got - oracle_gp(img, ss, 25.0, 20, "fir")))
        print(f"R {R} {shape}: {err:.2e}")
        assert err <= TOL


@pytest.mark.parametrize("ss", [0.8, 5.0, 12.0, 20.0])
def test_iir_scales(bf, ss):
    img = synthimg.voronoi_image(150, 140, 30, seed=78)
    got = run(bf, img, ss, 25.0, 20, "iir")
    assert np.max(np.abs(got - oracle_gp(img, ss, 25.0, 20, "iir"))) <= TOL


@pytest.mark.parametrize("shape", [(300, 700), (70, 1500)])
def test_iir_launch_shapes(bf, shape):
    # every split of the IIR passes (band height, channel groups of the column
    # and row passes) computes the same filter: each matches the oracle, and
    # they agree with one another to rounding
    H, W = shape
    img = synthimg.voronoi_image(H, W, 60, seed=H + W)
    ref = oracle_gp(img, 6.0, 25.0, 20, "iir")
    outs = {}
    try:
        for tune in [(0, 0, 0), (32, 1, 1), (64, 0, 0), (64, 1, 1), (64, 3, 2), (64, 8, 4), (32, 2, 8), (32, 4, 3)]:
            bf.set_iir_tuning(*tune)
            note(f"iir tuning {tune} shape {bf.iir_shape(H, W, 20)}")
            outs[tune] = run(bf, img, 6.0, 25.0, 20, "iir")
            assert np.max(np.abs(outs[tune] - ref)) <= TOL, (tune, np.max(np.abs(outs[tune] - ref)))
    finally:
        bf.set_iir_tuning(0, 0, 0)
    base = outs[(0, 0, 0)]
    for tune, o in outs.items():
        assert np.max(np.abs(o - base)) <= 1e-4, tune


@pytest.mark.parametrize("N", [0, 2, 8, 40, 64])
@pytest.mark.parametrize("spatial", ["fir", "iir"])
def test_degrees(bf, N, spatial):
    img = synthimg.voronoi_image(96, 80, 20, seed=79)
    got = run(bf, img, 2.0, 30.0, N, spatial)
    ref = oracle_gp(img, 2.0, 30.0, N, spatial)
    if spatial == "iir" and N == 0:
        # Deriche's kernel dips below zero (about -1.4e-4 of its peak near 5.4
        # sigma_s).  At degree 0 the weights exp(-(t^2 + tau^2)/2) of dark or
        # bright pixels are tiny, so a ring of opposite-intensity pixels seen
        # through these negative lobes nearly cancels the denominator (the
        # FP64 oracle's own D is negative at some pixels).  The FP32 result
        # then legitimately differs from FP64 by the condition number of that
        # sum, cond = (sum |h| w) / |sum h w|.  Compare where cond <= 2 (over
        # 99% of the pixels) and show the rest is genuinely ill-conditioned.
        k, _ = oracle.spatial_table("iir", 2.0, *img.shape)
        f = img.astype(np.float64)
        _, D, _ = oracle.gp_rescaled(f, 30.0, 0, k, return_dm=True)
        _, Da, _ = oracle.gp_rescaled(f, 30.0, 0, np.abs(k), return_dm=True)
        cond = Da / np.abs(D)
        well = cond <= 2.0
        err = np.abs(got - ref)
        worst = np.unravel_index(np.argmax(err), err.shape)
        print(f"N=0 iir: well-conditioned {well.mean():.4f}, max err there {err[well].max():.2e}, "
              f"worst pixel {worst} err {err[worst]:.3e} cond {cond[worst]:.1f}")
        assert well.mean() > 0.99
        assert err[well].max() <= TOL
        return
    assert np.max(np.abs(got - ref)) <= TOL


@pytest.mark.parametrize("N", [1, 3])
def test_odd_degree(bf, N):
    # a wide range kernel keeps every approximate weight positive
    img = synthimg.voronoi_image(64, 72, 12, seed=80)
    for spatial in ("fir", "iir"):
        got = run(bf, img, 2.0, 120.0, N, spatial)
        assert np.max(np.abs(got - oracle_gp(img, 2.0, 120.0, N, spatial))) <= TOL


@pytest.mark.parametrize("center,code", [("midrange", oracle.CENTER_MIDRANGE), ("none", oracle.CENTER_NONE)])
def test_center_modes(bf, center, code):
    img = synthimg.voronoi_image(70, 90, 20, seed=81)
    for spatial in ("fir", "iir"):
        got = run(bf, img, 2.0, 40.0, 20, spatial, center)
        assert np.max(np.abs(got - oracle_gp(img, 2.0, 40.0, 20, spatial, code))) <= TOL


def test_pitched_input_and_output(bf):
    img = synthimg.voronoi_image(80, 100, 20, seed=82)
    big = torch.zeros(80, 128, device="cuda")
    big[:, :100] = to_dev(img)
    view = big[:, :100]
    outbig = torch.full((80, 128), -7.0, device="cuda")
    for spatial in ("fir", "iir"):
        note(f"pitched {spatial}")
        bf.gp_forward(view, 2.0, 30.0, 20, spatial=spatial, out=outbig[:, :100], check=True)
        o = to_np(outbig)
        assert np.max(np.abs(o[:, :100] - oracle_gp(img, 2.0, 30.0, 20, spatial))) <= TOL
        assert np.all(o[:, 100:] == -7.0)


def test_constant_image_unchanged(bf):
    img = np.full((45, 77), 131.5, np.float32)
    for spatial in ("fir", "iir"):
        got = run(bf, img, 3.0, 30.0, 20, spatial)
        assert np.max(np.abs(got - 131.5)) <= 1e-4


@pytest.mark.parametrize("spatial", ["fir", "iir"])
@pytest.mark.parametrize("ss", [1.5, 4.0])
def test_large_x_range(bf, spatial, ss):
    # every |x| in (13.3, 13.8): exp(-x^2/2) is below the FP32 normal range,
    # the channels are carried with a per-sample power-of-two shift (IIR) or
    # formed in double (FIR); no centring keeps the case well conditioned
    v = synthimg.voronoi_image(96, 128, 20, seed=77, noise=0)
    img = (226.0 + 8.0 * (v.astype(np.float64) / 255.0)).astype(np.float32)
    got = run(bf, img, ss, 17.0, 20, spatial, center="none")
    ref = oracle_gp(img, ss, 17.0, 20, spatial, center=oracle.CENTER_NONE)
    assert np.isfinite(got).all()
    assert np.max(np.abs(got - ref)) <= TOL, np.max(np.abs(got - ref))


@pytest.mark.parametrize("N", [46, 47])
def test_fir_degree_variant_boundary(bf, N):
    # the register-column FIR carries unnormalised channels up to degree 46;
    # above it the region variant (double channels) takes over
    img = synthimg.voronoi_image(40, 150, 12, seed=91)
    got = run(bf, img, 2.0, 40.0, N, "fir")
    ref = oracle_gp(img, 2.0, 40.0, N, "fir")
    assert np.max(np.abs(got - ref)) <= TOL


@pytest.mark.parametrize("top", [11.9, 12.1])
def test_fir_range_variant_boundary(bf, top):
    # max |x| just below 12 (register-column variant) and just above it
    # (region variant), no centring: |x| spans [top - 0.6, top]
    v = synthimg.voronoi_image(48, 200, 16, seed=92, noise=0)
    img = ((top - 0.6 + 0.6 * (v.astype(np.float64) / 255.0)) * 20.0).astype(np.float32)
    got = run(bf, img, 3.0, 20.0, 20, "fir", center="none")
    ref = oracle_gp(img, 3.0, 20.0, 20, "fir", center=oracle.CENTER_NONE)
    assert np.isfinite(got).all()
    assert np.max(np.abs(got - ref)) <= TOL, np.max(np.abs(got - ref))


def test_out_of_range_reports_erange(bf):
    img = synthimg.voronoi_image(40, 40, 8, seed=83)
    img[0, 0], img[1, 1] = 0.0, 255.0
    for spatial in ("fir", "iir"):
        note(f"erange {spatial}")
        ws = bf.workspace(40, 40, 20, 2.0, spatial)
        out = bf.gp_forward(to_dev(img), 2.0, 5.0, 20, spatial=spatial, ws=ws)
        assert bf.status(ws) == bf.BF_ERANGE
        assert torch.isnan(out).all()
        bf.gp_forward(to_dev(img), 2.0, 30.0, 20, spatial=spatial, ws=ws)
        assert bf.status(ws) == bf.BF_OK


def test_deterministic(bf):
    img = to_dev(synthimg.voronoi_image(300, 260, 50, seed=84))
    for spatial in ("fir", "iir"):
        note(f"determinism {spatial}")
        a = bf.gp_forward(img, 3.0, 30.0, 20, spatial=spatial).clone()
        b = bf.gp_forward(img, 3.0, 30.0, 20, spatial=spatial)
        assert torch.equal(a, b)


def test_transpose_and_flip(bf):
    img = synthimg.voronoi_image(75, 110, 20, seed=85)
    for spatial in ("fir", "iir"):
        a = run(bf, img, 2.5, 30.0, 20, spatial)
        assert np.max(np.abs(run(bf, img.T.copy(), 2.5, 30.0, 20, spatial) - a.T)) <= TOL
        assert np.max(np.abs(run(bf, img[::-1].copy(), 2.5, 30.0, 20, spatial) - a[::-1])) <= TOL


@pytest.mark.parametrize("ss", [1.0, 2.0, 5.0])
def test_direct_matches_oracle(bf, ss):
    img = synthimg.voronoi_image(70, 101, 20, seed=86)
    note(f"direct ss={ss}")
    got = to_np(bf.direct_forward(to_dev(img), ss, 30.0))
    ref = oracle.direct_gauss(img.astype(np.float64), ss, 30.0)
    assert np.max(np.abs(got - ref)) <= TOL


def test_direct_wide_window_sampled(bf):
    img = synthimg.mid_1024()[:300, :333].copy()
    note("direct ss=20 window 60")
    got = to_np(bf.direct_forward(to_dev(img), 20.0, 30.0))
    f = img.astype(np.float64)
    k = oracle.gauss_table(20.0, 60)
    for (y, x) in [(0, 0), (150, 170), (299, 332), (10, 300)]:
        y0, y1, x0, x1 = max(0, y - 60), min(300, y + 61), max(0, x - 60), min(333, x + 61)
        ref = oracle.direct(f[y0:y1, x0:x1], 30.0, k)[y - y0, x - x0]
        assert abs(got[y, x] - ref) <= TOL


@pytest.fixture
def tuned_table(bf):
    # the crossover table the benchmark installs (measured on this device,
    # cached), restored to the previous state afterwards
    from paper_1505_00077_amd import autotune
    before = bf.get_fir_crossover_table()
    note("tuning the FIR/IIR crossover")
    table = autotune.ensure(20)
    yield table
    bf.set_fir_crossover_table(before)


@pytest.mark.parametrize("ss", [2.0, 5.0, 10.0, 20.0])
def test_mid_config_full_image(bf, tuned_table, ss):
    # the whole 1024^2 sweep image against the oracle, in the mode AUTO takes
    # under the tuned crossover table (what the benchmark times) and in every
    # other mode the radius allows (the FIR tile up to radius 24, IIR always)
    img = synthimg.mid_1024()
    auto = bf.resolve_spatial(ss, shape=img.shape)
    modes = {auto, "iir"} | ({"fir"} if bf.fir_radius(ss) <= bf.FIR_MAX_RADIUS else set())
    outs = {}
    for mode in sorted(modes):
        got = run(bf, img, ss, 30.0, 20, mode)
        outs[mode] = got
        ref = oracle_gp(img, ss, 30.0, 20, mode)
        err = np.max(np.abs(got - ref))
        print(f"sigma_s {ss} {mode}{' (auto)' if mode == auto else ''}: max |gpu - oracle| {err:.2e}")
        assert err <= TOL, (mode, err)
    # AUTO returns the output of the mode it resolves to, bit for bit
    a = run(bf, img, ss, 30.0, 20, "auto")
    assert np.array_equal(a, outs[auto])


def test_mid_config_sweep_sampled(bf):
    img = synthimg.mid_1024()
    rng = np.random.default_rng(5)
    pts = [(0, 0), (1023, 1023), (0, 1023), (512, 3)] + [tuple(rng.integers(0, 1024, 2)) for _ in range(4)]
    for ss in (2.0, 5.0, 10.0, 20.0):
        # the mode AUTO takes for this image size (a size-dependent crossover
        # table, when installed, takes precedence over the process-wide radius)
        mode = bf.resolve_spatial(ss, shape=img.shape)
        got = run(bf, img, ss, 30.0, 20, "auto")
        for (y, x) in pts:
            ref = oracle_gp_at(img, int(y), int(x), ss, 30.0, 20, mode)
            assert abs(got[y, x] - ref) <= TOL, (ss, y, x, got[y, x], ref)


def test_large_config_sampled(bf):
    img = synthimg.large_4096()
    got = run(bf, img, 10.0, 20.0, 20, "auto")
    mode = bf.resolve_spatial(10.0, shape=img.shape)
    for (y, x) in [(0, 0), (4095, 4095), (2047, 3000), (100, 4000)]:
        ref = oracle_gp_at(img, y, x, 10.0, 20.0, 20, mode)
        assert abs(got[y, x] - ref) <= TOL, (y, x, got[y, x], ref)
    assert np.all(np.isfinite(got))


def test_large_config_full_rows_and_columns(bf):
    # the 16-MP image in the recursive mode (AUTO's choice at sigma_s 10 with
    # any crossover table): whole rows at the image edges, at a 32-row band
    # boundary (31 | 32) and in the middle, and the first and last columns
    img = synthimg.large_4096()
    assert bf.resolve_spatial(10.0, shape=img.shape) == "iir"
    got = run(bf, img, 10.0, 20.0, 20, "iir")
    rows, cols = (0, 31, 32, 2047, 4095), (0, 4095)
    note("oracle on the row and column bands")
    ref_r, ref_c = oracle_lines(img, 10.0, 20.0, 20, "iir", rows=rows, cols=cols)
    for y in rows:
        err = np.max(np.abs(got[y] - ref_r[y]))
        print(f"row {y}: {err:.2e}")
        assert err <= TOL, (y, err)
    for x in cols:
        err = np.max(np.abs(got[:, x] - ref_c[x]))
        print(f"column {x}: {err:.2e}")
        assert err <= TOL, (x, err)


@pytest.mark.parametrize("W", [4097, 6000, 8192, 8193, 12000, 16384])
def test_iir_wide_rows(bf, W):
    # rows past 4096 samples run the row pass with 512 threads (8 waves), so
    # the carries cross eight waves of the workgroup; past 8192 the row is cut
    # into segments of 8192 whose end states cross between workgroups (8193:
    # a one-sample last segment)
    img = synthimg.voronoi_image(3, W, 60, seed=W)
    got = run(bf, img, 7.0, 30.0, 20, "iir")
    err = np.max(np.abs(got - oracle_gp(img, 7.0, 30.0, 20, "iir")))
    print(f"W {W}: {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("N", [0, 8, 64])
def test_iir_row_segments_degrees_and_pitch(bf, N):
    # two channels (N 0), a small degree and the largest degree across row
    # segments, with a row pitch larger than the width
    H, W = 3, 9001
    img = synthimg.voronoi_image(H, W, 50, seed=N + 11)
    base = torch.zeros(H, W + 37, device="cuda")
    x = base[:, :W]
    x.copy_(to_dev(img))
    note(f"gp_forward pitched {H}x{W} N={N} iir")
    out = torch.full((H, W + 37), -1.0, device="cuda")[:, :W]
    bf.gp_forward(x, 6.0, 40.0, N, spatial="iir", out=out, check=True)
    got = to_np(out)
    err = np.max(np.abs(got - oracle_gp(img, 6.0, 40.0, N, "iir")))
    print(f"N {N}: {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("shape,ss", [((5, 12000), 25.0), ((37, 12000), 3.0), ((2, 16384), 40.0)])
def test_iir_row_segments(bf, shape, ss):
    # wide support (sigma_s 25 and 40: the response reaches over a whole
    # segment), and bands of rows with segments (37 rows: two bands, a ragged
    # one); an edge step placed on the segment boundary
    H, W = shape
    img = synthimg.voronoi_image(H, W, 80, seed=H * W)
    img[:, 8190:8195] = 255.0 - img[:, 8190:8195]
    got = run(bf, img, ss, 30.0, 20, "iir")
    err = np.max(np.abs(got - oracle_gp(img, ss, 30.0, 20, "iir")))
    print(f"{shape} sigma_s {ss}: {err:.2e}")
    assert err <= TOL
