"""Batched path (a graph of grouped per-stage launches over many images)
against single-image calls and the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synthimg
from gpu_util import note, oracle_gp, oracle_gp_at, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00077_amd as m
    return m


def singles(bf, imgs, ss, sr, N=20, spatial="auto"):
    # the batch descriptor holds the sigmas as float32: use the same values;
    # the batch runs its IIR images in 32-row bands without channel groups,
    # which single calls get under the tuning override (32, 1, 1)
    f32 = lambda v: float(np.float32(v))
    try:
        bf.set_iir_tuning(32, 1, 1)
        return [to_np(bf.gp_forward(x, f32(s), f32(r), N, spatial=spatial, check=True))
                for x, s, r in zip(imgs, ss, sr)]
    finally:
        bf.set_iir_tuning(0, 0, 0)


def test_forced_fir_wide_radii(bf):
    # FIR at every radius class the batched plan launches separately
    shapes = [(70, 90), (200, 333), (128, 64)]
    ss = [1.0, 4.5, 8.0]  # radii 3, 14, 24
    sr = [30.0, 25.0, 40.0]
    host = [synthimg.voronoi_image(H, W, 30, seed=700 + i) for i, (H, W) in enumerate(shapes)]
    imgs = [to_dev(h) for h in host]
    note("batched forced FIR, radii 3/14/24")
    plan = bf.BatchPlan(imgs, ss, sr, 20, spatial="fir")
    outs = [to_np(o) for o in plan.run()]
    ref = singles(bf, imgs, ss, sr, spatial="fir")
    for i in range(len(imgs)):
        assert np.array_equal(outs[i], ref[i]), i
        assert np.max(np.abs(outs[i] - oracle_gp(host[i], ss[i], sr[i], 20, "fir"))) <= 1e-3


def test_wide_rows_batch(bf):
    # rows of 5000 and 8192 samples: the row pass of such images needs more
    # than 64 KiB of LDS per workgroup
    shapes = [(3, 5000), (2, 8192), (40, 300)]
    ss, sr = [6.0, 9.0, 7.0], [30.0, 25.0, 35.0]
    host = [synthimg.voronoi_image(H, W, 40, seed=1200 + i) for i, (H, W) in enumerate(shapes)]
    imgs = [to_dev(h) for h in host]
    note("batched wide rows 5000 / 8192")
    plan = bf.BatchPlan(imgs, ss, sr, 20, spatial="iir")
    outs = [to_np(o) for o in plan.run()]
    ref = singles(bf, imgs, ss, sr, spatial="iir")
    f32 = lambda v: float(np.float32(v))
    for i in range(len(imgs)):
        assert np.array_equal(outs[i], ref[i]), i
        err = np.max(np.abs(outs[i] - oracle_gp(host[i], f32(ss[i]), f32(sr[i]), 20, "iir")))
        assert err <= 1e-3, (i, err)


def test_batch_band_rows_64(bf):
    # a plan made under the 64-row band override (end states by weighted sums
    # in four channel groups, the two-wave column pass): equal to single calls
    # under the same override, and to the oracle
    shapes = [(200, 150), (97, 300), (64, 64)]
    ss, sr = [7.0, 10.0, 6.0], [30.0, 25.0, 35.0]
    host = [synthimg.voronoi_image(H, W, 40, seed=1400 + i) for i, (H, W) in enumerate(shapes)]
    imgs = [to_dev(h) for h in host]
    note("batched plan with 64-row bands")
    f32 = lambda v: float(np.float32(v))
    try:
        bf.set_iir_tuning(64, 1, 1)
        plan = bf.BatchPlan(imgs, ss, sr, 20, spatial="iir")
        outs = [to_np(o) for o in plan.run()]
        ref = [to_np(bf.gp_forward(x, f32(s), f32(r), 20, spatial="iir", check=True))
               for x, s, r in zip(imgs, ss, sr)]
    finally:
        bf.set_iir_tuning(0, 0, 0)
    for i in range(len(imgs)):
        assert np.array_equal(outs[i], ref[i]), (i, np.max(np.abs(outs[i] - ref[i])))
        err = np.max(np.abs(outs[i] - oracle_gp(host[i], f32(ss[i]), f32(sr[i]), 20, "iir")))
        assert err <= 1e-3, (i, err)


def test_small_uneven_batch(bf):
    shapes = [(37, 70), (128, 200), (300, 129), (1, 64), (64, 1), (513, 777), (90, 2048), (40, 3000), (20, 300)]
    ss = [1.0, 2.5, 6.0, 3.0, 1.5, 11.0, 4.5, 7.0, 5.0]
    sr = [30.0, 20.0, 45.0, 25.0, 30.0, 15.0, 35.0, 30.0, 30.0]
    host = [synthimg.voronoi_image(H, W, max(1, H * W // 400), seed=300 + i) for i, (H, W) in enumerate(shapes)]
    imgs = [to_dev(h) for h in host]
    note(f"batched plan {len(imgs)} images, modes {[bf.resolve_spatial(s) for s in ss]}")
    plan = bf.BatchPlan(imgs, ss, sr, 20)
    outs = [to_np(o) for o in plan.run()]
    ref = singles(bf, imgs, ss, sr)
    for i in range(len(imgs)):
        assert np.array_equal(outs[i], ref[i]), (i, np.max(np.abs(outs[i] - ref[i])))
    # every image over its whole extent against the oracle, in the mode the
    # plan resolved for it (FIR and recursive images alike; the descriptor's
    # float32 sigmas)
    for i in range(len(imgs)):
        mode = bf.resolve_spatial(ss[i], shape=host[i].shape)
        s32, r32 = float(np.float32(ss[i])), float(np.float32(sr[i]))
        note(f"oracle image {i} {host[i].shape} {mode}")
        err = np.max(np.abs(outs[i] - oracle_gp(host[i], s32, r32, 20, mode)))
        print(f"image {i} {host[i].shape} {mode}: {err:.2e}")
        assert err <= 1e-3, (i, mode, err)


def test_uneven_batch_64(bf):
    batch = synthimg.batched_64()
    host = [b[0] for b in batch]
    ss = [b[1] for b in batch]
    sr = [b[2] for b in batch]
    imgs = [to_dev(h) for h in host]
    note("batched 64 images")
    plan = bf.BatchPlan(imgs, ss, sr, 20)
    outs = [to_np(o) for o in plan.run()]
    ref = singles(bf, imgs, ss, sr)
    # the grouped launches run the single-image arithmetic lane for lane, with
    # the same reduction order for the centre: the outputs are bit-identical
    # (also where a recursive-kernel image with a small sigma_r is
    # ill-conditioned, as image 53 of this batch is)
    diffs = [float(np.max(np.abs(o - r))) for o, r in zip(outs, ref)]
    print(f"batched vs single max abs {max(diffs):.2e}")
    for i, (o, r) in enumerate(zip(outs, ref)):
        assert np.array_equal(o, r), (i, diffs[i])
    # sampled oracle check on three images
    for i in (0, 17, 40):
        H, W = host[i].shape
        mode = bf.resolve_spatial(ss[i], shape=host[i].shape)
        for (y, x) in [(0, 0), (H // 2, W // 3)]:
            ref1 = oracle_gp_at(host[i], y, x, ss[i], sr[i], 20, mode)
            assert abs(outs[i][y, x] - ref1) <= 1e-3, (i, y, x)
    # four recursive-mode images over their whole extent (sigma_s 7.2 to 15,
    # sigma_r 25 to 46, tall, wide and near-square)
    for i in (58, 34, 15, 47):
        mode = bf.resolve_spatial(ss[i], shape=host[i].shape)
        assert mode == "iir"
        s32, r32 = float(np.float32(ss[i])), float(np.float32(sr[i]))
        note(f"oracle image {i} {host[i].shape}")
        err = np.max(np.abs(outs[i] - oracle_gp(host[i], s32, r32, 20, mode)))
        print(f"image {i} {host[i].shape}: {err:.2e}")
        assert err <= 1e-3, (i, err)


def test_graph_replays_match_eager(bf):
    shapes = [(200, 300), (150, 90), (400, 256)]
    ss, sr = [1.5, 5.0, 9.0], [30.0, 25.0, 40.0]
    imgs = [to_dev(synthimg.voronoi_image(H, W, 40, seed=400 + i)) for i, (H, W) in enumerate(shapes)]
    plan = bf.BatchPlan(imgs, ss, sr, 20)
    eager = [o.clone() for o in plan.run()]
    torch.cuda.synchronize()
    note("batched graph capture")
    g = plan.graph()
    for rep in range(3):
        for o in plan.outs:
            o.fill_(-1.0)
        # unrelated eager work between replays
        _ = bf.gp_forward(imgs[0], 2.0, 30.0, 20)
        torch.cuda.synchronize()
        note(f"graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(plan.outs, eager):
            assert torch.equal(o, e)


def test_batched_deterministic(bf):
    imgs = [to_dev(synthimg.voronoi_image(H, W, 30, seed=H)) for H, W in [(100, 300), (257, 129)]]
    plan = bf.BatchPlan(imgs, [2.0, 7.0], [30.0, 20.0], 20)
    a = [o.clone() for o in plan.run()]
    b = plan.run()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
