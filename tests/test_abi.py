"""Host-side contract of libbfgp.so: exports, argument checks, workspace sizes.

Every call here is rejected (or is a pure host query) before any HIP call, so
these tests run without a GPU."""
import ctypes
import os
import re

import pytest

import paper_1505_00077_amd as bf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfgp.h")
FAKE = 0x10000  # never dereferenced: every call below fails validation first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bf_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(bf.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_error_text():
    assert bf.bf_version() >= 10000
    assert isinstance(bf.bf_last_error(), bytes)


def fwd(img=FAKE, out=FAKE + 4096, H=8, W=8, pitch=8, ss=2.0, sr=30.0, N=20, flags=0, saved=None, ws=FAKE + 8192,
        ws_bytes=1 << 30):
    return bf.bf_gp_forward(img, out, H, W, pitch, ss, sr, N, flags, saved, ws, ws_bytes, None)


@pytest.mark.parametrize("kw", [
    dict(img=None), dict(out=None), dict(ws=None), dict(H=0), dict(W=0), dict(H=-3), dict(pitch=7),
    dict(ss=0.0), dict(ss=-1.0), dict(ss=float("nan")), dict(ss=float("inf")), dict(sr=0.0), dict(sr=float("nan")),
    dict(N=-1), dict(N=65), dict(flags=12), dict(flags=16), dict(out=FAKE),
])
def test_forward_rejects_invalid_arguments(kw):
    assert fwd(**kw) == bf.BF_EINVAL
    assert len(bf.bf_last_error()) > 0


def test_forward_rejects_small_workspace():
    need = bf.workspace_bytes(64, 64, 20, 2.0, "iir")
    assert fwd(H=64, W=64, pitch=64, flags=bf.SPATIAL["iir"], ws_bytes=need - 1) == bf.BF_ENOMEM


def test_forward_rejects_unsupported_modes():
    # FIR radius ceil(3 * 9) = 27 > 24
    assert fwd(ss=9.0, flags=bf.SPATIAL["fir"]) == bf.BF_EUNSUPPORTED
    # IIR width limits: rows up to 16384 in the plain forward (row segments
    # of 8192), 8192 where the saved terms are stored
    iir = bf.SPATIAL["iir"]
    assert fwd(H=4, W=16385, pitch=16385, flags=iir) == bf.BF_EUNSUPPORTED
    assert fwd(H=4, W=9000, pitch=9000, flags=iir, saved=FAKE + (1 << 20)) == bf.BF_EUNSUPPORTED
    need = bf.workspace_bytes(4, 12000, 20, 5.0, "iir")
    assert fwd(H=4, W=12000, pitch=12000, flags=iir, ws_bytes=need - 1) == bf.BF_ENOMEM


def test_box_mode_contract():
    box = bf.SPATIAL["box"]
    assert box == 3 and bf.resolve_spatial(2.0, "box") == "box" and bf.resolve_spatial(50.0, "box") == "box"
    # width limit, no saved terms (no backward), small workspace
    assert fwd(H=4, W=16385, pitch=16385, flags=box) == bf.BF_EUNSUPPORTED
    assert fwd(flags=box, saved=FAKE + 65536) == bf.BF_EUNSUPPORTED
    # the column-filtered stack: N + 2 channels of H rows of pitch P (W rounded
    # up to a multiple of 256 up to 4096 columns, of 1024 up to 8192, of 2048
    # beyond), whatever the radius
    for H, W, P in ((64, 64, 256), (100, 1000, 1024), (9, 1025, 1280), (5, 4096, 4096), (7, 4097, 5120),
                    (3, 8192, 8192), (3, 8193, 10240), (2, 12000, 12288), (2, 16384, 16384)):
        need = bf.workspace_bytes(H, W, 20, 2.0, "box")
        assert 22 * H * P * 4 <= need < 22 * H * P * 4 + 8192
        assert bf.workspace_bytes(H, W, 20, 400.0, "box") == need
        assert fwd(H=H, W=W, pitch=W, flags=box, ws_bytes=need - 1) == bf.BF_ENOMEM
    # the other entry points do not run the box mode
    assert bwd(flags=box) == bf.BF_EUNSUPPORTED
    assert bf.bf_gp_backward_workspace_bytes(64, 64, 20, 2.0, box) == 0
    assert jfwd(flags=box) == bf.BF_EUNSUPPORTED
    assert bf.bf_gp_joint_workspace_bytes(64, 64, 20, 2.0, box) == 0
    assert vfwd(flags=box) == bf.BF_EUNSUPPORTED
    assert bf.bf_gp_volume_workspace_bytes(4, 64, 64, 20, 2.0, 2.0, box) == 0
    item = bf.BfGpItem(FAKE, FAKE + 4096, 8, 8, 8, 2.0, 30.0, 20)
    plan = ctypes.c_void_p()
    assert bf.bf_gp_plan_batched(ctypes.byref(item), 1, box, ctypes.byref(plan)) == bf.BF_EUNSUPPORTED
    assert not plan.value


def bwd(img=FAKE, g=FAKE + 4096, saved=FAKE + 8192, H=8, W=8, pitch=8, ss=2.0, sr=30.0, N=20, flags=0,
        gi=FAKE + 65536, ws=FAKE + 131072, ws_bytes=1 << 30):
    return bf.bf_gp_backward(img, g, saved, H, W, pitch, ss, sr, N, flags, gi, None, None, ws, ws_bytes, None)


@pytest.mark.parametrize("kw", [
    dict(img=None), dict(g=None), dict(saved=None), dict(ws=None), dict(H=0), dict(pitch=7), dict(ss=0.0),
    dict(sr=float("inf")), dict(N=65), dict(flags=12), dict(flags=16), dict(gi=FAKE), dict(gi=FAKE + 4096),
    dict(flags=2, gi=FAKE), dict(flags=2, N=-1),
])
def test_backward_rejects_invalid_arguments(kw):
    assert bwd(**kw) == bf.BF_EINVAL


def test_backward_modes_and_workspace():
    fir, iir = bf.SPATIAL["fir"], bf.SPATIAL["iir"]
    # FIR radius limit and the unsupported midrange centre, in both modes
    assert bwd(ss=9.0, flags=fir) == bf.BF_EUNSUPPORTED
    assert bwd(flags=fir | bf.CENTER["midrange"]) == bf.BF_EUNSUPPORTED
    assert bwd(flags=iir | bf.CENTER["midrange"]) == bf.BF_EUNSUPPORTED
    # the recursive backward holds two transposed channel stacks and carries
    need_iir = bf.bf_gp_backward_workspace_bytes(512, 512, 20, 12.0, iir)
    need_fir = bf.bf_gp_backward_workspace_bytes(512, 512, 20, 2.0, fir)
    assert need_iir >= 2 * 22 * 512 * 512 * 4 > need_fir > 0
    assert bwd(H=512, W=512, pitch=512, ss=12.0, flags=iir, ws_bytes=need_iir - 1) == bf.BF_ENOMEM
    # AUTO resolves as the forward does (radius 36 is past any crossover)
    assert bf.bf_gp_backward_workspace_bytes(512, 512, 20, 12.0, 0) == need_iir
    assert bf.bf_gp_backward_workspace_bytes(0, 512, 20, 12.0, iir) == 0


def jfwd(g=FAKE, d=FAKE + 4096, out=FAKE + 8192, H=8, W=8, pitch=8, ss=4.0, sr=30.0, N=20, flags=0,
         ws=FAKE + 65536, ws_bytes=1 << 30):
    return bf.bf_gp_joint_forward(g, d, out, H, W, pitch, ss, sr, N, flags, ws, ws_bytes, None)


@pytest.mark.parametrize("kw", [
    dict(g=None), dict(d=None), dict(out=None), dict(ws=None), dict(H=0), dict(pitch=7), dict(ss=0.0),
    dict(sr=float("nan")), dict(N=65), dict(flags=12), dict(flags=16), dict(out=FAKE), dict(out=FAKE + 4096),
])
def test_joint_rejects_invalid_arguments(kw):
    assert jfwd(**kw) == bf.BF_EINVAL


def test_joint_modes_and_workspace():
    fir, iir = bf.SPATIAL["fir"], bf.SPATIAL["iir"]
    assert jfwd(flags=fir) == bf.BF_EUNSUPPORTED
    assert jfwd(H=4, W=9000, pitch=9000) == bf.BF_EUNSUPPORTED
    # 2 (N + 1) channels: twice the stack of the filter at the same degree
    j = bf.bf_gp_joint_workspace_bytes(256, 300, 20, 4.0, iir)
    assert j >= 42 * 256 * 300 * 4 and j > bf.workspace_bytes(256, 300, 20, 4.0, "iir")
    assert bf.bf_gp_joint_workspace_bytes(256, 300, 20, 4.0, 0) == j
    assert bf.bf_gp_joint_workspace_bytes(256, 300, 20, 4.0, fir) == 0
    assert jfwd(H=256, W=300, pitch=300, ws_bytes=j - 1) == bf.BF_ENOMEM


def vfwd(v=FAKE, out=FAKE + 4096, T=4, H=8, W=8, ss=3.0, st=2.0, sr=30.0, N=20, flags=0, ws=FAKE + 65536,
         ws_bytes=1 << 30):
    return bf.bf_gp_volume_forward(v, out, T, H, W, ss, st, sr, N, flags, ws, ws_bytes, None)


@pytest.mark.parametrize("kw", [
    dict(v=None), dict(out=None), dict(ws=None), dict(T=0), dict(H=0), dict(W=-1), dict(ss=0.0),
    dict(st=0.0), dict(st=float("inf")), dict(sr=-1.0), dict(N=65), dict(flags=12), dict(flags=16), dict(out=FAKE),
])
def test_volume_rejects_invalid_arguments(kw):
    assert vfwd(**kw) == bf.BF_EINVAL


def test_volume_modes_and_workspace():
    fir = bf.SPATIAL["fir"]
    assert vfwd(flags=fir) == bf.BF_EUNSUPPORTED
    assert vfwd(W=9000) == bf.BF_EUNSUPPORTED
    need = bf.bf_gp_volume_workspace_bytes(10, 64, 96, 20, 3.0, 2.0, 0)
    # two channel stacks of the volume
    assert need >= 2 * 22 * 10 * 64 * 96 * 4
    assert bf.bf_gp_volume_workspace_bytes(10, 64, 96, 20, 3.0, 2.0, fir) == 0
    assert bf.bf_gp_volume_workspace_bytes(10, 64, 96, 20, 3.0, 0.0, 0) == 0
    assert vfwd(T=10, H=64, W=96, ws_bytes=need - 1) == bf.BF_ENOMEM


def test_workspace_sizes():
    fir = bf.workspace_bytes(1024, 1024, 20, 2.0, "fir")
    iir = bf.workspace_bytes(1024, 1024, 20, 2.0, "iir")
    assert 0 < fir < 1 << 20
    # the IIR stack holds N + 2 = 22 channels of the image
    assert iir >= 22 * 1024 * 1024 * 4
    assert bf.workspace_bytes(0, 10, 20, 2.0) == 0
    assert bf.workspace_bytes(10, 10, 99, 2.0) == 0


def test_spatial_resolution_and_crossover():
    old = bf.get_fir_crossover()
    try:
        bf.set_fir_crossover(6)
        assert bf.resolve_spatial(2.0) == "fir"      # radius 6
        assert bf.resolve_spatial(2.1) == "iir"      # radius 7
        assert bf.resolve_spatial(10.0, "fir") == "fir"
        assert bf.resolve_spatial(0.5, "iir") == "iir"
        bf.set_fir_crossover(0)
        assert bf.resolve_spatial(0.1) == "iir"
        with pytest.raises(bf.BfError):
            bf.set_fir_crossover(25)
    finally:
        bf.set_fir_crossover(old)


def test_direct_rejects_invalid_arguments():
    f = bf.bf_direct_forward
    assert f(None, FAKE, 8, 8, 8, 2.0, 30.0, -1, None) == bf.BF_EINVAL
    assert f(FAKE, FAKE + 4096, 8, 8, 7, 2.0, 30.0, -1, None) == bf.BF_EINVAL
    assert f(FAKE, FAKE + 4096, 8, 8, 8, 0.0, 30.0, -1, None) == bf.BF_EINVAL
    assert f(FAKE, FAKE + 4096, 8, 8, 8, 2.0, 30.0, 65, None) == bf.BF_EUNSUPPORTED
    assert f(FAKE, FAKE, 8, 8, 8, 2.0, 30.0, -1, None) == bf.BF_EINVAL


def test_status_rejects_null():
    v = ctypes.c_int()
    assert bf.bf_gp_status(None, None, ctypes.byref(v)) == bf.BF_EINVAL


def test_fir_radius_rule():
    # eq. (1): W = 3 sigma_s, rounded up
    assert bf.fir_radius(3.0) == 9
    assert bf.fir_radius(2.0) == 6
    assert bf.fir_radius(0.1) == 1
    assert bf.fir_radius(3.01) == 10
    # float32 rounding of sigma_s does not move the window
    import math
    import numpy as np
    assert bf.fir_radius(math.exp(float(np.float32(math.log(2.0))))) == 6
    assert bf.fir_radius(2.0 * (1 + 1e-5)) == 7


def test_iir_shape_rule_and_overrides():
    # automatic shapes: small images split the channels over more waves
    assert bf.iir_shape(1024, 1024, 20) == dict(band_rows=32, col_groups=4, row_chunk=16, row_threads=64,
                                                row_groups=3)
    # row groups fill three waves per SIMD once (1024 SIMDs): no more
    assert bf.iir_shape(900, 1000, 20)["row_groups"] == 3
    assert bf.iir_shape(1500, 900, 20)["row_groups"] == 2
    assert bf.iir_shape(4096, 4096, 20) == dict(band_rows=64, col_groups=1, row_chunk=16, row_threads=256,
                                                row_groups=1)
    assert bf.iir_shape(512, 512, 20)["col_groups"] == 8
    assert bf.iir_shape(512, 512, 20)["row_groups"] == 4
    assert bf.iir_shape(2048, 2048, 20)["row_groups"] == 1
    assert bf.iir_shape(100, 200, 20)["row_chunk"] == 4
    assert bf.iir_shape(100, 500, 20)["row_chunk"] == 8
    assert bf.iir_shape(100, 640, 20)["row_chunk"] == 12
    assert bf.iir_shape(100, 1500, 20)["row_threads"] == 128
    assert bf.iir_shape(100, 1500, 20)["row_chunk"] == 12
    # every width is covered, with fewer than one chunk of idle samples per wave
    for W in (1, 63, 64, 65, 255, 256, 257, 700, 1023, 1025, 2047, 3000, 4097, 8192):
        s = bf.iir_shape(8, W, 20)
        assert s["row_threads"] % 64 == 0 and s["row_threads"] * s["row_chunk"] >= W
        assert s["row_chunk"] == 4 or s["row_threads"] * (s["row_chunk"] - 4) < W
    # wider rows: segments of 512 threads x 16 samples, one channel group
    for W in (8193, 12000, 16384):
        s = bf.iir_shape(8, W, 20)
        assert (s["row_threads"], s["row_chunk"], s["row_groups"]) == (512, 16, 1)
    with pytest.raises(bf.BfError):
        bf.iir_shape(8, 16385, 20)
    # 64-row bands where the image still gives 1024 column waves at that height
    assert bf.iir_shape(1024, 1024, 20)["band_rows"] == 32
    assert bf.iir_shape(2048, 2048, 20)["band_rows"] == 64
    assert bf.iir_shape(4096, 4096, 20)["band_rows"] == 64
    assert bf.iir_shape(64, 16384, 20)["band_rows"] == 32
    # the joint filter keeps 32-row bands: its workspace at 4096^2 holds the
    # carries of 128 bands
    C = 2 * (20 + 1)
    assert bf.bf_gp_joint_workspace_bytes(4096, 4096, 20, 10.0, bf._flags("iir")) >= 4 * 128 * C * 8 * 4096
    # never more channel groups than channels (N = 0: two channels)
    s = bf.iir_shape(64, 64, 0)
    assert s["col_groups"] <= 2 and s["row_groups"] <= 2
    ws_auto = bf.workspace_bytes(1024, 1024, 20, 8.0, "iir")
    try:
        bf.set_iir_tuning(64, 2, 1)
        s = bf.iir_shape(1024, 1024, 20)
        assert (s["band_rows"], s["col_groups"], s["row_groups"]) == (64, 2, 1)
        # half as many bands: half the carry space
        assert bf.workspace_bytes(1024, 1024, 20, 8.0, "iir") < ws_auto
        bf.set_iir_tuning(0, 2, 0)
        assert bf.iir_shape(512, 512, 20)["col_groups"] == 2
        # row groups are capped by the threads a workgroup can hold and its LDS
        bf.set_iir_tuning(0, 0, 8)
        s = bf.iir_shape(1024, 4096, 20)
        assert s["row_threads"] * s["row_groups"] <= 512
        for bad in ((16, 0, 0), (0, 9, 0), (0, 0, -1)):
            with pytest.raises(bf.BfError):
                bf.set_iir_tuning(*bad)
    finally:
        bf.set_iir_tuning(0, 0, 0)
    assert bf.workspace_bytes(1024, 1024, 20, 8.0, "iir") == ws_auto
    with pytest.raises(bf.BfError):
        bf.iir_shape(10, 16385, 20)


def test_crossover_table():
    old = bf.get_fir_crossover()
    try:
        bf.set_fir_crossover(9)
        bf.set_fir_crossover_table([(300 * 300, 20), (1100 * 1100, 12), (2100 * 2100, 4)])
        assert bf.get_fir_crossover_table() == [(90000, 20), (1210000, 12), (4410000, 4)]
        # sigma_s = 5 -> radius 15
        assert bf.resolve_spatial(5.0, shape=(256, 256)) == "fir"
        assert bf.resolve_spatial(5.0, shape=(1024, 1024)) == "iir"
        assert bf.resolve_spatial(4.0, shape=(1024, 1024)) == "fir"      # radius 12
        assert bf.resolve_spatial(2.0, shape=(2048, 2048)) == "iir"      # radius 6 > 4
        assert bf.resolve_spatial(2.0, shape=(4096, 4096)) == "fir"      # past the table: radius 9
        assert bf.resolve_spatial(5.0) == "iir"                          # no shape: process-wide radius
        # the workspace follows the size-dependent choice
        assert bf.workspace_bytes(256, 256, 20, 5.0) < bf.workspace_bytes(256, 256, 20, 5.0, "iir")
        for bad in ([(100, 3), (100, 4)], [(0, 3)], [(100, 25)], [(100, 1)] * 9):
            with pytest.raises(bf.BfError):
                bf.set_fir_crossover_table(bad)
        assert len(bf.get_fir_crossover_table()) == 3  # unchanged by the rejected calls
    finally:
        bf.set_fir_crossover_table([])
        bf.set_fir_crossover(old)
    assert bf.get_fir_crossover_table() == []


def test_workspace_follows_tuning_overrides():
    # a batch plan and a workspace sized under one set of overrides: the
    # forward refuses a workspace sized for fewer bands
    try:
        bf.set_iir_tuning(64, 0, 0)
        small = bf.workspace_bytes(1000, 700, 20, 8.0, "iir")
        bf.set_iir_tuning(32, 0, 0)
        assert bf.workspace_bytes(1000, 700, 20, 8.0, "iir") > small
    finally:
        bf.set_iir_tuning(0, 0, 0)


def test_degree_rule_against_the_poisson_tail():
    # the rule is host-only: the smallest even N >= xmax^2 - 1 whose Poisson
    # tail P(Poisson(xmax^2) > N) is at most eps (SciPy's survival function)
    from scipy import stats
    for xmax in (0.0, 0.5, 1.0, 2.0, 3.3, 4.0, 5.5):
        for eps in (1e-2, 1e-3, 1e-6, 1e-12):
            lam = xmax * xmax
            try:
                n = bf.degree_for(xmax, eps)
            except bf.BfError as e:
                assert e.code == bf.BF_ERANGE
                assert all(stats.poisson.sf(m, lam) > eps for m in range(0, 65, 2))
                continue
            assert n % 2 == 0 and n >= lam - 1 and n <= 64
            assert stats.poisson.sf(n, lam) <= eps * (1 + 1e-9)
            if n >= 2 and n - 2 >= lam - 1:
                assert stats.poisson.sf(n - 2, lam) > eps
    assert bf.bf_gp_degree_for(-1.0, 1e-3) == bf.BF_EINVAL
    assert bf.bf_gp_degree_for(2.0, 0.0) == bf.BF_EINVAL
    assert bf.bf_gp_degree_for(2.0, 1.0) == bf.BF_EINVAL
    assert bf.bf_gp_degree_for(float("nan"), 1e-3) == bf.BF_EINVAL
    assert bf.bf_gp_degree_for(9.0, 1e-6) == bf.BF_ERANGE



def test_source_fingerprint_ignores_comments_and_layout():
    # the recorded HBM counters stay valid across comment edits, not code edits
    from paper_1505_00077_amd import profiling
    a = 'int f(int x) { // one\n  return x + 1; /* two */ }\nconst char *s = "a // b /* c */";'
    b = 'int f(int x) {\n\n    return x + 1;\n}\n// three\nconst char *s = "a // b /* c */";'
    assert profiling._code_only(a) == profiling._code_only(b)
    assert profiling._code_only(a) != profiling._code_only(a.replace("x + 1", "x + 2"))
    assert "// b /* c */" in profiling._code_only(a)
    assert len(profiling.source_fingerprint()) == 16


def test_noalloc_forward_checks_on_the_host():
    """bf_gp_forward_noalloc runs bf_gp_forward's argument checks, then refuses
    a workspace larger than its static scratch, both before any HIP call."""
    def na(img=FAKE, out=FAKE + 4096, H=8, W=8, pitch=8, ss=2.0, sr=30.0, N=20, flags=0, saved=None):
        return bf.bf_gp_forward_noalloc(img, out, H, W, pitch, ss, sr, N, flags, saved, None)
    assert na(img=None) == bf.BF_EINVAL
    assert na(out=FAKE) == bf.BF_EINVAL  # aliasing
    assert na(pitch=4) == bf.BF_EINVAL
    assert na(N=65) == bf.BF_EINVAL
    assert na(ss=0.0) == bf.BF_EINVAL
    assert na(flags=1 << 5) == bf.BF_EINVAL
    assert na(flags=bf.SPATIAL["box"], saved=FAKE + 12288) == bf.BF_EUNSUPPORTED
    # the IIR mode on an image whose workspace exceeds the static array
    H = W = 2048
    need = bf.workspace_bytes(H, W, 20, 10.0, "iir")
    assert need > bf.NOALLOC_SCRATCH_BYTES
    assert na(H=H, W=W, pitch=W, ss=10.0, flags=bf.SPATIAL["iir"]) == bf.BF_ENOMEM
    assert b"static scratch" in bf.bf_last_error()
    # the headline image fits (IIR at N 20), as does any FIR image
    assert bf.workspace_bytes(1024, 1024, 20, 10.0, "iir") <= bf.NOALLOC_SCRATCH_BYTES
    assert bf.workspace_bytes(8192, 8192, 20, 2.0, "fir") <= bf.NOALLOC_SCRATCH_BYTES


def test_noalloc_scratch_size_matches_the_header():
    text = open(HEADER).read()
    m = re.search(r"#define BF_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == bf.NOALLOC_SCRATCH_BYTES


def test_stacked_entry_points_check_on_the_host():
    """The stacked forward and backward run the single-image checks on image 0,
    then the batch's own: at least one image, a stride covering an image, no
    overlap between the image, output and gradient batches, enough workspace."""
    B, H, W = 4, 8, 8
    stride = H * W
    span = 4 * stride * B
    img, out = FAKE, FAKE + span
    ws = FAKE + 8 * span

    def fwd(img=img, out=out, B=B, pitch=W, stride=stride, flags=0, saved=None, ws=ws, ws_bytes=1 << 30):
        return bf.bf_gp_forward_stacked(img, out, B, H, W, pitch, stride, 2.0, 30.0, 20, flags, saved, ws, ws_bytes,
                                        None)

    assert fwd(B=0) == bf.BF_EINVAL
    assert fwd(stride=H * W - 1) == bf.BF_EINVAL
    assert fwd(out=img + 4 * stride) == bf.BF_EINVAL  # overlaps image 1
    assert fwd(img=None) == bf.BF_EINVAL
    assert fwd(ws=None) == bf.BF_EINVAL
    assert fwd(flags=bf.SPATIAL["box"]) == bf.BF_EUNSUPPORTED
    need = bf.bf_gp_forward_stacked_workspace_bytes(B, H, W, 20, 2.0, 0)
    assert need >= B * bf.workspace_bytes(H, W, 20, 2.0)
    assert fwd(ws_bytes=need - 1) == bf.BF_ENOMEM
    assert bf.bf_gp_forward_stacked_workspace_bytes(0, H, W, 20, 2.0, 0) == 0

    def bwd(img=img, gout=out, saved=FAKE + 4 * span, gimg=FAKE + 2 * span, B=B, stride=stride, flags=0, ws=ws,
            ws_bytes=1 << 30):
        return bf.bf_gp_backward_stacked(img, gout, saved, B, H, W, W, stride, 2.0, 30.0, 20, flags, gimg, None,
                                         None, ws, ws_bytes, None)

    assert bwd(B=0) == bf.BF_EINVAL
    assert bwd(gimg=img + 4) == bf.BF_EINVAL
    assert bwd(gimg=out + 4 * stride) == bf.BF_EINVAL
    assert bwd(saved=None) == bf.BF_EINVAL
    assert bwd(flags=bf.CENTER["midrange"]) == bf.BF_EUNSUPPORTED
    bneed = bf.bf_gp_backward_stacked_workspace_bytes(B, H, W, 20, 2.0, 0)
    assert bneed >= B * bf.bf_gp_backward_workspace_bytes(H, W, 20, 2.0, 0)
    assert bwd(ws_bytes=bneed - 1) == bf.BF_ENOMEM
