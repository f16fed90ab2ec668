"""Pins of the Alg. 1 packing oracle (oracle/alg1.py): a hand-worked
example, conservation, the first containers' seeds, and the forced
placement onto the last container."""
import numpy as np

from oracle import alg1


def test_hand_worked_example():
    """Lengths 10 9 8 3 3 2 2 1, one block of two columns (footprints L+1):
    C0 = [10], C1 = [9], maxLen 11.  8 (9): fits neither (20, 19 > 11):
    forced onto C1 = 19, maxLen 19.  3 (4): pointer at C1 (23 > 19), then
    C0 (15): C0.  3 (4): pointer below C0: forced onto C1 = 23, maxLen 23.
    2 (3): C1 26 > 23, C0 18: C0.  2 (3): forced, C1 = 26.  1 (2): C1 28,
    C0 20: C0.  Heights: one block of 26; padding 2 x 26 - (20 + 26) = 6;
    real 38; PRR 6/38."""
    out = alg1.pack([10, 9, 8, 3, 3, 2, 2, 1], 1, 2)
    assert list(out["container"]) == [0, 1, 1, 0, 1, 0, 1, 0]
    assert list(out["heights"]) == [26]
    assert out["padding"] == 6 and out["real"] == 38 and out["ending"] == 8
    assert abs(out["prr"] - 6 / 38) < 1e-15


def test_conservation_and_seeds():
    rng = np.random.default_rng(1)
    L = rng.integers(0, 500, size=3000)
    out = alg1.pack(L, 8, 16)
    c = out["container"]
    assert ((c >= 0) & (c < 128)).all()
    tot = np.bincount(c, weights=L + 1, minlength=128)
    assert tot.sum() == L.sum() + len(L)
    # the 128 longest sequences seed the containers in order
    order = np.argsort(-L, kind="stable")
    assert list(c[order[:128]]) == list(range(128))
    # heights are the blocks' tallest containers; padding fills the rest
    h = out["heights"]
    assert (h == tot.reshape(8, 16).max(1)).all()
    assert out["padding"] == int((16 * h - tot.reshape(8, 16).sum(1)).sum())


def test_fewer_sequences_than_containers():
    out = alg1.pack([5, 7], 2, 2)
    assert list(out["container"]) == [1, 0]
    assert list(out["heights"]) == [8, 0]
    assert out["padding"] == 8 - 6
