"""Box spatial mode on the GPU against the FP64 oracle (element by element).

The oracle runs Algorithm 1 with the box table (weight 1 over |d| <=
ceil(3 sigma_s)); the GPU runs the running-sum column pass and the prefix-sum
row pass.  Tolerance: 1e-3 absolute on 0..255 data, as for the other modes.
Every case names itself before it runs."""
import numpy as np
import pytest
import torch

import oracle
import synthimg
from gpu_util import note, oracle_gp, oracle_gp_at, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00077_amd as m
    return m


def run(bf, img, ss, sr, N, center="mean"):
    note(f"box gp_forward {img.shape} ss={ss} sr={sr} N={N} {center}")
    return to_np(bf.gp_forward(to_dev(img), ss, sr, N, spatial="box", center=center, check=True))


def test_small_config_matches_oracle(bf):
    img = synthimg.small_256()
    got = run(bf, img, 3.0, 30.0, 20)
    ref = oracle_gp(img, 3.0, 30.0, 20, "box")
    k = oracle.box_table(oracle.fir_radius(3.0))
    direct = oracle.direct(img.astype(np.float64), 30.0, k)
    print(f"box: max|gpu-oracle| {np.max(np.abs(got - ref)):.2e}; vs the direct box filter: "
          f"max {np.max(np.abs(got - direct)):.3f}, {oracle.mse_db(got, direct):.2f} dB")
    assert np.max(np.abs(got - ref)) <= TOL


@pytest.mark.parametrize("shape", [(1, 1), (1, 50), (50, 1), (37, 70), (130, 97), (33, 257), (100, 129), (300, 41)])
def test_ragged_shapes(bf, shape):
    H, W = shape
    img = synthimg.voronoi_image(H, W, max(1, H * W // 400), seed=H * 1000 + W + 5)
    for ss in (1.0, 2.5):
        got = run(bf, img, ss, 30.0, 20)
        ref = oracle_gp(img, ss, 30.0, 20, "box")
        assert np.max(np.abs(got - ref)) <= TOL, (ss, np.max(np.abs(got - ref)))


@pytest.mark.parametrize("ss", [0.3, 4.0, 10.0, 17.0, 40.0, 400.0])
def test_radii(bf, ss):
    # radius 1 up to windows wider than the image (capped at max(H, W)); the
    # column pass's bands grow with the radius
    img = synthimg.voronoi_image(90, 150, 30, seed=95)
    got = run(bf, img, ss, 25.0, 20)
    assert np.max(np.abs(got - oracle_gp(img, ss, 25.0, 20, "box"))) <= TOL


def test_window_covering_the_image_is_a_tone_map(bf):
    # every window holds the whole image: equal intensities give equal outputs
    rng = np.random.default_rng(96)
    img = rng.choice(np.array([10.0, 60.0, 61.0, 140.0, 250.0], np.float32), size=(70, 90))
    got = run(bf, img, 40.0, 40.0, 20)
    ref = oracle_gp(img, 40.0, 40.0, 20, "box")
    assert np.max(np.abs(got - ref)) <= TOL
    for v in np.unique(img):
        vals = got[img == v]
        assert np.max(vals) - np.min(vals) <= 1e-4


@pytest.mark.parametrize("H", [31, 32, 33, 64, 65, 257])
def test_band_boundaries(bf, H):
    # bands of 32 rows at radius 6 (2 R <= 32), 64 at radius 30
    img = synthimg.voronoi_image(H, 70, 12, seed=H + 97)
    for ss in (2.0, 10.0):
        got = run(bf, img, ss, 30.0, 20)
        assert np.max(np.abs(got - oracle_gp(img, ss, 30.0, 20, "box"))) <= TOL, ss


@pytest.mark.parametrize("N", [0, 2, 8, 22, 23, 40, 64])
def test_degrees(bf, N):
    # N + 2 > 24 channels split over at least two column-pass groups
    img = synthimg.voronoi_image(96, 80, 20, seed=98)
    got = run(bf, img, 2.0, 30.0, N)
    assert np.max(np.abs(got - oracle_gp(img, 2.0, 30.0, N, "box"))) <= TOL


@pytest.mark.parametrize("N", [1, 3])
def test_odd_degree(bf, N):
    img = synthimg.voronoi_image(64, 72, 12, seed=99)
    got = run(bf, img, 2.0, 120.0, N)
    assert np.max(np.abs(got - oracle_gp(img, 2.0, 120.0, N, "box"))) <= TOL


@pytest.mark.parametrize("center,code", [("midrange", oracle.CENTER_MIDRANGE), ("none", oracle.CENTER_NONE)])
def test_center_modes(bf, center, code):
    img = synthimg.voronoi_image(70, 90, 20, seed=100)
    got = run(bf, img, 2.0, 40.0, 20, center)
    assert np.max(np.abs(got - oracle_gp(img, 2.0, 40.0, 20, "box", code))) <= TOL


def test_pitched_input_and_output(bf):
    img = synthimg.voronoi_image(80, 100, 20, seed=101)
    big = torch.zeros(80, 128, device="cuda")
    big[:, :100] = to_dev(img)
    outbig = torch.full((80, 128), -7.0, device="cuda")
    note("box pitched")
    bf.gp_forward(big[:, :100], 2.0, 30.0, 20, spatial="box", out=outbig[:, :100], check=True)
    o = to_np(outbig)
    assert np.max(np.abs(o[:, :100] - oracle_gp(img, 2.0, 30.0, 20, "box"))) <= TOL
    assert np.all(o[:, 100:] == -7.0)


def test_constant_image_unchanged(bf):
    img = np.full((45, 77), 131.5, np.float32)
    assert np.max(np.abs(run(bf, img, 3.0, 30.0, 20) - 131.5)) <= 1e-4


@pytest.mark.parametrize("ss", [1.5, 4.0])
def test_large_x_range(bf, ss):
    # every |x| in (13.3, 13.8): exp(-x^2/2) is formed at a power-of-two shift
    # and taken to double exactly
    v = synthimg.voronoi_image(96, 128, 20, seed=77, noise=0)
    img = (226.0 + 8.0 * (v.astype(np.float64) / 255.0)).astype(np.float32)
    got = run(bf, img, ss, 17.0, 20, center="none")
    ref = oracle_gp(img, ss, 17.0, 20, "box", center=oracle.CENTER_NONE)
    assert np.isfinite(got).all()
    assert np.max(np.abs(got - ref)) <= TOL, np.max(np.abs(got - ref))


def test_out_of_range_reports_erange(bf):
    img = synthimg.voronoi_image(40, 40, 8, seed=102)
    img[0, 0], img[1, 1] = 0.0, 255.0
    note("box erange")
    ws = bf.workspace(40, 40, 20, 2.0, "box")
    out = bf.gp_forward(to_dev(img), 2.0, 5.0, 20, spatial="box", ws=ws)
    assert bf.status(ws) == bf.BF_ERANGE
    assert torch.isnan(out).all()
    bf.gp_forward(to_dev(img), 2.0, 30.0, 20, spatial="box", ws=ws)
    assert bf.status(ws) == bf.BF_OK


def test_deterministic_and_symmetric(bf):
    img = synthimg.voronoi_image(300, 260, 50, seed=103)
    d = to_dev(img)
    note("box determinism")
    a = bf.gp_forward(d, 3.0, 30.0, 20, spatial="box").clone()
    assert torch.equal(a, bf.gp_forward(d, 3.0, 30.0, 20, spatial="box"))
    a = to_np(a)
    assert np.max(np.abs(run(bf, img.T.copy(), 3.0, 30.0, 20) - a.T)) <= TOL
    assert np.max(np.abs(run(bf, img[:, ::-1].copy(), 3.0, 30.0, 20) - a[:, ::-1])) <= TOL


@pytest.mark.parametrize("W", [1024, 1025, 4096, 4097, 6000, 8192, 8193, 12000, 16384])
def test_wide_rows(bf, W):
    # 4 samples per row-pass thread up to 4096 columns (1024 threads), 16
    # up to 8192, 32 beyond (two workgroups per row share the outputs); from
    # about 3000 columns the row's prefix sums need more than 64 KiB of LDS
    img = synthimg.voronoi_image(3, W, 40, seed=W)
    for ss in (2.0, 30.0):
        got = run(bf, img, ss, 30.0, 20)
        assert np.max(np.abs(got - oracle_gp(img, ss, 30.0, 20, "box"))) <= TOL, ss


def test_mid_config_sweep_sampled(bf):
    img = synthimg.mid_1024()
    rng = np.random.default_rng(6)
    pts = [(0, 0), (1023, 1023), (0, 1023), (512, 3)] + [tuple(rng.integers(0, 1024, 2)) for _ in range(4)]
    for ss in (2.0, 5.0, 10.0, 20.0):
        got = run(bf, img, ss, 30.0, 20)
        for (y, x) in pts:
            ref = oracle_gp_at(img, int(y), int(x), ss, 30.0, 20, "box")
            assert abs(got[y, x] - ref) <= TOL, (ss, y, x, got[y, x], ref)


def test_large_config_sampled(bf):
    img = synthimg.large_4096()
    got = run(bf, img, 10.0, 20.0, 20)
    for (y, x) in [(0, 0), (4095, 4095), (2047, 3000), (100, 4000)]:
        ref = oracle_gp_at(img, y, x, 10.0, 20.0, 20, "box")
        assert abs(got[y, x] - ref) <= TOL, (y, x, got[y, x], ref)
    assert np.all(np.isfinite(got))


def test_no_backward_in_box_mode(bf):
    # the box mode is forward only: the autograd path and the backward entry
    # point refuse it with BF_EUNSUPPORTED before any launch
    img = to_dev(synthimg.voronoi_image(32, 40, 6, seed=104))
    ls = torch.tensor(0.5, device="cuda", requires_grad=True)
    lr = torch.tensor(3.0, device="cuda", requires_grad=True)
    note("box autograd refused")
    with pytest.raises(bf.BfError) as e:
        bf.gp_filter(img, ls, lr, 20, spatial="box")
    assert e.value.code == bf.BF_EUNSUPPORTED
