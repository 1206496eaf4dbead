"""GP filter of volumes and video on the GPU against the FP64 oracle.

Algorithm 1 with the separable filter over all three axes (the extension to
higher-dimensional signals the paper names), recursive spatial mode, sigma_t
along the first axis.  Tolerance: 1e-3 absolute on 0..255 data."""
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


def video(T, H, W, seed, cells=10):
    """Frames of slowly moving Voronoi cells: each frame's seed points drift."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0, 1, size=(cells, 2)) * np.array([H, W])
    vel = rng.normal(0, 0.7, size=(cells, 2))
    vals = rng.uniform(0, 255, size=cells)
    yy, xx = np.mgrid[0:H, 0:W] + 0.5
    frames = []
    for t in range(T):
        p = pts + t * vel
        d = (yy[..., None] - p[:, 0]) ** 2 + (xx[..., None] - p[:, 1]) ** 2
        f = vals[np.argmin(d, axis=-1)] + rng.normal(0, 10.0, size=(H, W))
        frames.append(np.clip(f, 0, 255))
    return np.stack(frames).astype(np.float32)


def run(bf, vol, ss, st, sr, N, center="mean"):
    note(f"gp_volume_forward {vol.shape} ss={ss} st={st} sr={sr} N={N} {center}")
    out = bf.gp_volume_forward(to_dev(vol), ss, st, sr, N, center=center, check=True)
    return to_np(out)


def ref(vol, ss, st, sr, N, center=oracle.CENTER_MEAN):
    T, H, W = vol.shape
    kt, ks = oracle.volume_tables(st, ss, T, H, W)
    return oracle.volume_gp(vol.astype(np.float64), sr, N, kt, ks, center)


@pytest.mark.parametrize("shape,ss,st,N", [((5, 37, 45), 3.0, 2.0, 20), ((40, 24, 30), 2.0, 4.0, 20),
                                            ((3, 1, 80), 2.5, 1.5, 10), ((70, 3, 5), 1.5, 10.0, 20),
                                            ((9, 65, 33), 6.0, 3.0, 8), ((2, 33, 130), 12.0, 1.0, 20)])
def test_volume_matches_oracle(bf, shape, ss, st, N):
    vol = video(*shape, seed=sum(shape))
    got = run(bf, vol, ss, st, 30.0, N)
    assert np.max(np.abs(got - ref(vol, ss, st, 30.0, N))) <= TOL


@pytest.mark.parametrize("W", [5000, 8192])
def test_volume_wide_frames(bf, W):
    # frame rows past about 4000 samples need more than 64 KiB of LDS in the
    # row pass (one row of 512 threads x 16 samples at 8192)
    vol = video(3, 2, W, seed=W)
    got = run(bf, vol, 3.0, 2.0, 30.0, 20)
    assert np.max(np.abs(got - ref(vol, 3.0, 2.0, 30.0, 20))) <= TOL


def test_single_frame_is_the_image_filter(bf):
    img = synthimg.voronoi_image(70, 90, 15, seed=51)
    got = run(bf, img[None], 5.0, 3.0, 30.0, 20)[0]
    note("gp_forward iir on the same frame")
    plain = to_np(bf.gp_forward(to_dev(img), 5.0, 30.0, 20, spatial="iir", check=True))
    assert np.max(np.abs(got - plain)) <= TOL


def test_constant_volume_and_centre_modes(bf):
    c = np.full((6, 20, 30), 123.5, np.float32)
    assert np.max(np.abs(run(bf, c, 3.0, 2.0, 30.0, 20) - 123.5)) <= TOL
    vol = video(7, 30, 41, seed=52)
    for center, code in (("none", oracle.CENTER_NONE), ("midrange", oracle.CENTER_MIDRANGE)):
        got = run(bf, vol * 0.5 + 40.0, 2.0, 2.0, 40.0, 20, center=center)
        assert np.max(np.abs(got - ref(vol * 0.5 + 40.0, 2.0, 2.0, 40.0, 20, code))) <= TOL


@pytest.mark.parametrize("groups", [(1, 1), (3, 2), (8, 4)])
def test_volume_channel_groups(bf, groups):
    vol = video(12, 40, 70, seed=53)
    try:
        bf.set_iir_tuning(0, groups[0], groups[1])
        got = run(bf, vol, 4.0, 3.0, 30.0, 20)
    finally:
        bf.set_iir_tuning(0, 0, 0)
    assert np.max(np.abs(got - ref(vol, 4.0, 3.0, 30.0, 20))) <= TOL


def test_volume_out_of_range(bf):
    vol = video(4, 20, 20, seed=54)
    vol[0, 0, 0], vol[1, 1, 1] = 0.0, 255.0
    ws = bf.volume_workspace(4, 20, 20, 20, 2.0, 2.0)
    note("volume erange")
    out = bf.gp_volume_forward(to_dev(vol), 2.0, 2.0, 5.0, 20, ws=ws)
    assert bf.status(ws) == bf.BF_ERANGE
    assert torch.isnan(out).all()
