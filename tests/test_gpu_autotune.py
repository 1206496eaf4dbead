"""Crossover tuner on the GPU: it times both spatial modes and installs a
table that the AUTO mode then follows (single-image and batched)."""
import numpy as np
import pytest
import torch

import synthimg
from gpu_util import note, oracle_gp, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00077_amd as m
    return m


def test_tune_installs_a_table(bf, tmp_path, monkeypatch):
    from paper_1505_00077_amd import autotune
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "crossover.json"))
    note("autotune 256^2 and 1024^2")
    try:
        res = autotune.tune(N=20, sizes=((256, 256), (1024, 1024)), reps=3)
        table = bf.get_fir_crossover_table()
        assert table == [tuple(t) for t in res["table"]]
        assert [px for px, _ in table] == [256 * 256, 1024 * 1024]
        for (H, W), (_, r) in zip(((256, 256), (1024, 1024)), table):
            d = res["detail"][f"{H}x{W}"]
            assert d["iir_ms"] > 0 and all(v > 0 for v in d["fir_ms"].values())
            # the AUTO mode now follows the measured radius at this size
            if r >= 1:
                assert bf.resolve_spatial(r / 3.0, shape=(H, W)) == "fir"
            if r < bf.FIR_MAX_RADIUS:
                assert bf.resolve_spatial((r + 1) / 3.0, shape=(H, W)) == "iir"
        # the cache round-trips
        bf.set_fir_crossover_table([])
        assert autotune.load(N=20) == table
        assert bf.get_fir_crossover_table() == table
        # AUTO results stay within the parity bound whichever mode was chosen
        img = synthimg.voronoi_image(256, 256, 40, seed=9)
        ss = max(1, table[0][1]) / 3.0
        mode = bf.resolve_spatial(ss, shape=img.shape)
        got = to_np(bf.gp_forward(to_dev(img), ss, 30.0, 20, check=True))
        assert np.max(np.abs(got - oracle_gp(img, ss, 30.0, 20, mode))) <= 1e-3
    finally:
        bf.set_fir_crossover_table([])
