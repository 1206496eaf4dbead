"""Joint (cross) GP filter on the GPU against the FP64 oracle.

The range kernel is evaluated on a guide and the average taken of separate
data (the extension the paper's Conclusion names), in the recursive spatial
mode.  Tolerance: 1e-3 absolute on 0..255 data, as for the filter."""
import numpy as np
import pytest
import torch

import oracle
import synthimg
from gpu_util import note, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00077_amd as m
    return m


def run(bf, guide, data, ss, sr, N, center="mean", check=True):
    note(f"gp_joint_forward {guide.shape} ss={ss} sr={sr} N={N} {center}")
    out = bf.gp_joint_forward(to_dev(guide), to_dev(data), ss, sr, N, center=center, check=check)
    return to_np(out)


def ref(guide, data, ss, sr, N, center=oracle.CENTER_MEAN):
    g = np.asarray(guide, np.float64)
    k, _ = oracle.spatial_table("iir", ss, *g.shape)
    return oracle.joint_gp(g, np.asarray(data, np.float64), sr, N, k, center)


def pair(H, W, seed):
    guide = synthimg.voronoi_image(H, W, max(8, H * W // 400), seed=seed)
    data = synthimg.voronoi_image(H, W, max(8, H * W // 300), seed=seed + 1000)
    return guide, data


@pytest.mark.parametrize("shape,ss,N", [((37, 45), 2.0, 8), ((64, 97), 6.0, 20), ((129, 70), 15.0, 20),
                                         ((1, 60), 3.0, 10), ((60, 1), 3.0, 10), ((33, 257), 4.0, 20)])
def test_joint_matches_oracle(bf, shape, ss, N):
    guide, data = pair(*shape, seed=shape[0] * 7 + shape[1])
    got = run(bf, guide, data, ss, 30.0, N)
    assert np.max(np.abs(got - ref(guide, data, ss, 30.0, N))) <= TOL


def test_joint_with_guide_equal_to_data_is_the_filter(bf):
    img = synthimg.voronoi_image(80, 120, 20, seed=41)
    joint = run(bf, img, img, 8.0, 30.0, 20)
    note("gp_forward iir, same image")
    plain = to_np(bf.gp_forward(to_dev(img), 8.0, 30.0, 20, spatial="iir", check=True))
    assert np.max(np.abs(joint - plain)) <= TOL
    k, _ = oracle.spatial_table("iir", 8.0, *img.shape)
    assert np.max(np.abs(joint - oracle.gp_alg1(img.astype(np.float64), 30.0, 20, k))) <= TOL


def test_joint_constant_data(bf):
    guide = synthimg.voronoi_image(70, 90, 15, seed=42)
    got = run(bf, guide, np.full(guide.shape, 173.25, np.float32), 5.0, 25.0, 20)
    assert np.max(np.abs(got - 173.25)) <= TOL


@pytest.mark.parametrize("tune", [(32, 1, 0), (32, 3, 0), (32, 5, 0), (64, 2, 0), (32, 8, 0)])
def test_joint_channel_groups_and_bands(bf, tune):
    # the column passes split the 2 (N + 1) stack channels into groups that may
    # start on a guide or a data channel; every split gives the same filter
    guide, data = pair(96, 150, seed=43)
    try:
        bf.set_iir_tuning(*tune)
        got = run(bf, guide, data, 7.0, 30.0, 20)
    finally:
        bf.set_iir_tuning(0, 0, 0)
    assert np.max(np.abs(got - ref(guide, data, 7.0, 30.0, 20))) <= TOL


def test_joint_large_x_range(bf):
    # every guide |x| in (13.3, 13.8) (no centring): the channels are carried
    # with a per-sample power-of-two shift
    v = synthimg.voronoi_image(64, 96, 14, seed=44, noise=0)
    guide = (226.0 + 8.0 * (v.astype(np.float64) / 255.0)).astype(np.float32)
    data = synthimg.voronoi_image(64, 96, 14, seed=45)
    got = run(bf, guide, data, 4.0, 17.0, 20, center="none")
    assert np.isfinite(got).all()
    assert np.max(np.abs(got - ref(guide, data, 4.0, 17.0, 20, oracle.CENTER_NONE))) <= TOL


def test_joint_out_of_range_reports_erange(bf):
    guide = synthimg.voronoi_image(40, 40, 8, seed=46)
    guide[0, 0], guide[1, 1] = 0.0, 255.0
    data = synthimg.voronoi_image(40, 40, 8, seed=47)
    ws = bf.joint_workspace(40, 40, 20, 4.0)
    note("joint erange")
    out = bf.gp_joint_forward(to_dev(guide), to_dev(data), 4.0, 5.0, 20, ws=ws)
    assert bf.status(ws) == bf.BF_ERANGE
    assert torch.isnan(out).all()
    bf.gp_joint_forward(to_dev(guide), to_dev(data), 4.0, 30.0, 20, ws=ws)
    assert bf.status(ws) == bf.BF_OK
