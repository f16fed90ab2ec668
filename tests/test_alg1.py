"""The library's Alg. 1 packer (hmsv_alg1_pack) against the oracle's
(oracle/alg1.py): the same column for every sequence, the same heights,
padding and PRR."""
import numpy as np
import pytest

import synth
from oracle import alg1

hm = pytest.importorskip("paper_1707_09683_amd")


@pytest.mark.parametrize("n,nblocks,width,kind", [
    (8, 1, 2, "hand"), (3000, 8, 16, "uniform"), (5000, 30, 32, "lognormal"),
    (20000, 15, 128, "lognormal"), (100, 4, 64, "uniform"), (0, 3, 4, "uniform")])
def test_packer_matches_oracle(n, nblocks, width, kind):
    rng = np.random.default_rng(n + width)
    if kind == "hand":
        L = np.array([10, 9, 8, 3, 3, 2, 2, 1], np.int64)
    elif kind == "uniform":
        L = rng.integers(0, 600, size=n).astype(np.int64)
    else:
        L = synth.sample_lengths_lognormal(rng, n).astype(np.int64)
    cont, heights, st = hm.alg1_pack(L, nblocks, width)
    exp = alg1.pack(L, nblocks, width)
    assert np.array_equal(cont.astype(np.int64), exp["container"])
    assert np.array_equal(heights, exp["heights"])
    assert st["padding"] == exp["padding"] and st["real"] == exp["real"]
    assert st["ending"] == n
    assert st["prr"] == pytest.approx(exp["prr"], rel=1e-12)
    if n:
        per_block = np.bincount(exp["container"] // width, minlength=nblocks)
        assert st["mean_ending"] == pytest.approx(per_block.mean())
        assert st["sd_ending"] == pytest.approx(per_block.std(), abs=1e-9)
        assert st["max_height"] == exp["heights"].max()
        assert st["efficiency"] == pytest.approx(exp["heights"].mean() / exp["heights"].max())


def test_packer_rejects_bad_arguments():
    with pytest.raises(hm.HmsvError):
        hm.alg1_pack(np.array([3, -1]), 1, 2)
    with pytest.raises(hm.HmsvError):
        hm.alg1_pack(np.array([3, 1]), 0, 2)
