"""bf_gp_forward_noalloc against bf_gp_forward through the C ABI (GPU).

The allocation-free entry point runs the same kernels on the library's static
device array, so its output must equal bf_gp_forward's bit for bit.  Two calls
in a row, the second on a smaller image, check that nothing left in the array
by the first call leaks into the second."""
import numpy as np
import pytest
import torch

import paper_1505_00077_amd as bf
from synthimg import voronoi_image

pytestmark = pytest.mark.gpu


def _pair(img, sigma_s, sigma_r, N, spatial, center="mean", save=False):
    H, W = img.shape
    ref = bf.gp_forward(img, sigma_s, sigma_r, N, spatial=spatial, center=center)
    got = bf.gp_forward_noalloc(img, sigma_s, sigma_r, N, spatial=spatial, center=center)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("spatial", ["fir", "iir", "box"])
def test_noalloc_equals_forward_two_calls(spatial):
    dev = torch.device("cuda:0")
    big = torch.from_numpy(voronoi_image(777, 1013, 120, seed=11)).to(dev)
    small = torch.from_numpy(voronoi_image(131, 259, 20, seed=12)).to(dev)
    for img, ss in ((big, 3.0), (small, 7.0)):
        print(f"noalloc {spatial} {tuple(img.shape)} sigma_s {ss}", flush=True)
        ref, got = _pair(img, ss, 30.0, 20, spatial)
        assert torch.equal(ref, got), float((ref - got).abs().max())
        assert torch.isfinite(got).all()


def test_noalloc_saved_terms_and_headline_image():
    dev = torch.device("cuda:0")
    img = torch.from_numpy(voronoi_image(1024, 1024, 200, seed=2)).to(dev)
    for ss in (2.0, 10.0):
        print(f"noalloc auto 1024x1024 sigma_s {ss}", flush=True)
        ref, got = _pair(img, ss, 30.0, 20, "auto")
        assert torch.equal(ref, got)
    # saved terms for the backward, IIR, then a smaller FIR call
    for shape, ss, spatial in (((300, 411), 6.0, "iir"), ((97, 65), 1.5, "fir")):
        im = torch.from_numpy(voronoi_image(*shape, 15, seed=13)).to(dev)
        H, W = shape
        s_ref = bf.saved_buffer(H, W, dev)
        s_got = bf.saved_buffer(H, W, dev)
        ref = bf.gp_forward(im, ss, 25.0, 20, spatial=spatial, saved=s_ref)
        got = bf.gp_forward_noalloc(im, ss, 25.0, 20, spatial=spatial, saved=s_got)
        torch.cuda.synchronize()
        assert torch.equal(ref, got)
        assert torch.equal(s_ref, s_got)


def test_noalloc_wide_rows():
    # rows past 8192 samples: the row segments' states live in the array too;
    # a wide call, then a narrower one
    dev = torch.device("cuda:0")
    for (H, W), ss, spatial in (((3, 12000), 9.0, "iir"), ((5, 9000), 4.0, "box"), ((4, 3000), 9.0, "iir")):
        img = torch.from_numpy(voronoi_image(H, W, 40, seed=W)).to(dev)
        print(f"noalloc {spatial} {H}x{W} sigma_s {ss}", flush=True)
        ref, got = _pair(img, ss, 30.0, 20, spatial)
        assert torch.equal(ref, got), float((ref - got).abs().max())


def test_noalloc_rejects_oversize_without_running():
    dev = torch.device("cuda:0")
    img = torch.zeros(2048, 2048, device=dev)
    out = torch.full_like(img, 7.0)
    with pytest.raises(bf.BfError) as e:
        bf.gp_forward_noalloc(img, 10.0, 30.0, 20, spatial="iir", out=out)
    assert e.value.code == bf.BF_ENOMEM
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
