"""Stacked batch (B images of one size, one launch per stage) against single
calls, bit for bit, and the autograd Function built on it."""
import numpy as np
import pytest
import torch

import synthimg
from gpu_util import note, oracle_gp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00077_amd as m
    return m


def _batch(B, H, W, seed0, K=60):
    return torch.stack([torch.from_numpy(synthimg.voronoi_image(H, W, K, seed=seed0 + i)) for i in range(B)]).cuda()


@pytest.mark.parametrize("spatial,ss,shape,B", [("fir", 2.0, (96, 130), 3), ("fir", 4.0, (200, 77), 5),
                                                 ("iir", 10.0, (96, 130), 3), ("iir", 3.0, (300, 257), 4),
                                                 ("iir", 6.0, (1, 64), 2), ("fir", 1.0, (64, 1), 2)])
def test_stacked_forward_backward_equal_single_calls(bf, spatial, ss, shape, B):
    H, W = shape
    note(f"stacked {spatial} B={B} {shape} sigma_s {ss}")
    x = _batch(B, H, W, 900)
    g = _batch(B, H, W, 950) - 128.0
    sr, N = 30.0, 20
    saved = torch.empty(B, 16 * H * W, dtype=torch.uint8, device="cuda")
    out = bf.gp_forward_stacked(x, ss, sr, N, spatial=spatial, saved=saved)
    gi, gs, gr = bf.gp_backward_stacked(x, g, saved, ss, sr, N, spatial)
    torch.cuda.synchronize()
    for b in range(B):
        sv = bf.saved_buffer(H, W)
        o1 = bf.gp_forward(x[b], ss, sr, N, spatial=spatial, saved=sv)
        gi1, gs1, gr1 = bf.gp_backward(x[b], g[b], sv, ss, sr, N, spatial)
        torch.cuda.synchronize()
        assert torch.equal(out[b], o1), b
        assert torch.equal(saved[b], sv), b
        assert torch.equal(gi[b], gi1), b
        assert float(gs[b]) == float(gs1[0]) and float(gr[b]) == float(gr1[0]), b


@pytest.mark.parametrize("tune", [(64, 0, 0), (64, 2, 1)])
def test_stacked_band_rows_64(bf, tune):
    # 64-row bands (the default of large images) in the stacked launches:
    # still equal to single calls under the same shape, and to the oracle
    B, H, W = 2, 150, 200
    x = _batch(B, H, W, 1100)
    g = _batch(B, H, W, 1150) - 128.0
    try:
        bf.set_iir_tuning(*tune)
        note(f"stacked iir tuning {tune} shape {bf.iir_shape(H, W, 20)}")
        saved = torch.empty(B, 16 * H * W, dtype=torch.uint8, device="cuda")
        out = bf.gp_forward_stacked(x, 7.0, 30.0, 20, spatial="iir", saved=saved)
        gi, gs, gr = bf.gp_backward_stacked(x, g, saved, 7.0, 30.0, 20, "iir")
        torch.cuda.synchronize()
        for b in range(B):
            sv = bf.saved_buffer(H, W)
            o1 = bf.gp_forward(x[b], 7.0, 30.0, 20, spatial="iir", saved=sv)
            gi1, gs1, gr1 = bf.gp_backward(x[b], g[b], sv, 7.0, 30.0, 20, "iir")
            torch.cuda.synchronize()
            assert torch.equal(out[b], o1), b
            assert torch.equal(saved[b], sv), b
            assert torch.equal(gi[b], gi1), b
            assert float(gs[b]) == float(gs1[0]) and float(gr[b]) == float(gr1[0]), b
    finally:
        bf.set_iir_tuning(0, 0, 0)
    ref = oracle_gp(x[1].cpu().numpy(), 7.0, 30.0, 20, "iir")
    assert np.max(np.abs(out[1].cpu().numpy().astype(np.float64) - ref)) <= 1e-3


def test_stacked_pitched_batch_and_forward_without_saved(bf):
    # a batch with padded rows and a gap between images; the plain forward
    # (no saved terms) takes the fused row pass in the recursive mode
    B, H, W = 3, 70, 90
    base = torch.zeros(B, H + 3, 128, device="cuda")
    x = base[:, :H, :W]
    x.copy_(_batch(B, H, W, 700))
    for spatial, ss in (("iir", 8.0), ("fir", 2.0)):
        note(f"stacked pitched {spatial}")
        out = torch.full_like(base, -1.0)[:, :H, :W]
        bf.gp_forward_stacked(x, ss, 25.0, 20, spatial=spatial, out=out)
        torch.cuda.synchronize()
        for b in range(B):
            assert torch.equal(out[b], bf.gp_forward(x[b], ss, 25.0, 20, spatial=spatial)), b


def test_stacked_wide_rows(bf):
    # rows of 6000 samples: the fused row pass then needs more than 64 KiB of
    # LDS per workgroup
    B, H, W = 2, 3, 6000
    x = _batch(B, H, W, 1300)
    note("stacked iir wide rows 6000")
    out = bf.gp_forward_stacked(x, 8.0, 25.0, 20, spatial="iir")
    torch.cuda.synchronize()
    for b in range(B):
        o1 = bf.gp_forward(x[b], 8.0, 25.0, 20, spatial="iir")
        assert torch.equal(out[b], o1), b
        ref = oracle_gp(x[b].cpu().numpy(), 8.0, 25.0, 20, "iir")
        assert np.max(np.abs(out[b].cpu().numpy().astype(np.float64) - ref)) <= 1e-3


def test_gp_filter_batch_uses_stacked_path(bf):
    B, H, W = 4, 64, 80
    x = _batch(B, H, W, 600).requires_grad_(True)
    tgt = _batch(B, H, W, 650)
    for spatial, ss in (("fir", 2.5), ("iir", 9.0)):
        lss = torch.tensor(float(np.log(ss)), dtype=torch.float64, requires_grad=True)
        lsr = torch.tensor(float(np.log(25.0)), dtype=torch.float64, requires_grad=True)
        out = bf.gp_filter(x, lss, lsr, 20, spatial)
        loss = ((out - tgt) ** 2).sum()
        loss.backward()
        # per-image reference: single calls and their gradients
        gsum, rsum = 0.0, 0.0
        for b in range(B):
            sv = bf.saved_buffer(H, W)
            o1 = bf.gp_forward(x.detach()[b], ss, 25.0, 20, spatial=spatial, saved=sv)
            assert torch.equal(out.detach()[b], o1)
            gi1, gs1, gr1 = bf.gp_backward(x.detach()[b], 2 * (o1 - tgt[b]), sv, ss, 25.0, 20, spatial)
            assert torch.equal(x.grad[b], gi1), b
            gsum += float(gs1[0])
            rsum += float(gr1[0])
        assert abs(float(lss.grad) - gsum) <= 1e-12 * max(1.0, abs(gsum))
        assert abs(float(lsr.grad) - rsum) <= 1e-12 * max(1.0, abs(rsum))
        x.grad = None
