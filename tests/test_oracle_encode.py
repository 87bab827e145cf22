"""Pins of the BLCO encoder oracle.

* Figure 6 (a: ALTO index l, b: block b and re-encoded key, row order) for the
  Figure 4a tensor with a 32-long encoding line and at most 6 non-zeros per
  block (tests/golden/fig6_blco.txt, with the v = 8.0 row read from its
  Figure 4a coordinates).
* Equal mode widths give Morton (Z-order) interleaving: bit j of mode n at
  position j*N + n.
* The index is a bijection; for power-of-two lengths it is onto [0, prod I).
* Decoding (shift, mask, block top bits) returns the input coordinates for
  any key width and block cap; keys fit K bits; (block, l) is sorted.
* The bit splits worked out by hand for 2^24 x 2^22 x 2^20 x 2^10 (76 bits)
  and 2^20 x 2^18 x 2^16 x 2^12 (66 bits).
The ALTO order of irregular shapes beyond bijectivity is a reading of the
paper (round robin from the least significant bit), not pinned by it.
"""
import itertools

import numpy as np
import pytest

from conftest import read_golden
from oracle import encode as E


def test_figure6_golden(fig4a):
    coords, vals, dims = fig4a
    t = E.encode(coords, vals, dims, key_bits=5, max_block_nnz=6)
    g = read_golden("fig6_blco.txt")
    want_v = [float(r[0]) for r in g]
    want_l = [int(r[1]) for r in g]
    want_b = [int(r[2]) for r in g]
    want_k = [int(r[3]) for r in g]
    assert t["values"].tolist() == want_v
    assert t["keys"].tolist() == want_k
    lo, hi = E.linearize([c[t["order"]] for c in coords], t["layout"]["pos"])
    assert lo.tolist() == want_l and not hi.any()
    per_nnz_block = np.repeat(t["block_ids"], np.diff(t["block_starts"]))
    assert per_nnz_block.tolist() == want_b
    assert t["block_ids"].tolist() == [0, 1]
    assert t["block_starts"].tolist() == [0, 6, 12]
    lay = t["layout"]
    assert lay["T"] == 6 and lay["K"] == 5 and lay["h"] == [0, 0, 1] and lay["w"] == [2, 2, 1]
    back = E.decode(t["keys"], t["block_ids"], t["block_starts"], lay)
    for n in range(3):
        assert back[n].tolist() == coords[n][t["order"]].tolist()


def test_figure6_split_cap():
    # the same tensor with a 3-non-zero cap splits each 6-block into two
    rows = read_golden("fig4a_coo.txt")
    c = [np.array([int(r[m]) - 1 for r in rows], dtype=np.uint32) for m in range(3)]
    v = np.array([float(r[3]) for r in rows], dtype=np.float32)
    t = E.encode(c, v, (4, 4, 4), key_bits=5, max_block_nnz=3)
    assert t["block_ids"].tolist() == [0, 0, 1, 1]
    assert t["block_starts"].tolist() == [0, 3, 6, 9, 12]


@pytest.mark.parametrize("b", [(3, 3, 3), (2, 2, 2, 2), (5, 5)])
def test_equal_widths_are_morton(b):
    pos = E.alto_positions(list(b))
    N = len(b)
    for n in range(N):
        assert pos[n] == [j * N + n for j in range(b[n])]


def test_irregular_positions_round_robin():
    # widths (3, 1, 2): level 0 -> modes 1,2,3; level 1 -> modes 1,3; level 2 -> mode 1
    assert E.alto_positions([3, 1, 2]) == [[0, 3, 5], [1], [2, 4]]


@pytest.mark.parametrize("dims", [(5, 3, 6), (4, 2, 8), (1, 7, 3), (2, 2, 2, 3)])
def test_bijective_and_compact(dims):
    allc = np.array(list(itertools.product(*[range(d) for d in dims])), dtype=np.uint32)
    coords = [np.ascontiguousarray(allc[:, m]) for m in range(len(dims))]
    lay = E.layout(dims)
    lo, hi = E.linearize(coords, lay["pos"])
    assert not hi.any()
    assert len(np.unique(lo)) == len(lo)
    assert int(lo.max()) < (1 << lay["T"])
    if all(d & (d - 1) == 0 for d in dims):
        assert sorted(lo.tolist()) == list(range(int(np.prod(dims))))


@pytest.mark.parametrize("key_bits,cap", [(64, 1 << 27), (12, 64), (8, 6), (5, 1)])
def test_round_trip_and_order(key_bits, cap):
    rng = np.random.default_rng(key_bits)
    dims = (300, 7, 1, 129, 40)
    nnz = 3000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.random(nnz).astype(np.float32)
    t = E.encode(coords, vals, dims, key_bits=key_bits, max_block_nnz=cap)
    lay = t["layout"]
    assert lay["K"] == min(lay["T"], key_bits)
    assert int(t["keys"].max()) < (1 << lay["K"])
    back = E.decode(t["keys"], t["block_ids"], t["block_starts"], lay)
    for n in range(len(dims)):
        np.testing.assert_array_equal(back[n], coords[n][t["order"]])
    np.testing.assert_array_equal(t["values"], vals[t["order"]])
    # sorted by (block, l): recompute l from the decoded coordinates
    lo, hi = E.linearize(back, lay["pos"])
    Lint = [(int(h) << 64) | int(l) for l, h in zip(lo, hi)]
    assert all(a <= b for a, b in zip(Lint, Lint[1:]))
    # blocks: runs of equal block key (brute force) split into caps
    blk = [x >> lay["K"] for x in Lint]
    starts = t["block_starts"].tolist()
    assert starts[0] == 0 and starts[-1] == nnz
    for bi in range(len(starts) - 1):
        a, e = starts[bi], starts[bi + 1]
        assert 0 < e - a <= cap
        assert all(blk[k] == int(t["block_ids"][bi]) for k in range(a, e))
    runs = 0
    for k in range(nnz):
        if k == 0 or blk[k] != blk[k - 1]:
            runs += 1
    assert len(set(blk)) == runs
    assert len(starts) - 1 >= runs


def test_hand_worked_bit_splits():
    lay = E.layout((1 << 24, 1 << 22, 1 << 20, 1 << 10))
    assert (lay["T"], lay["S"], lay["h"], lay["w"]) == (76, 12, [6, 4, 2, 0], [18, 18, 18, 10])
    assert lay["s"] == [0, 18, 36, 54]
    lay = E.layout((1 << 20, 1 << 18, 1 << 16, 1 << 12))
    assert (lay["T"], lay["S"], lay["h"], lay["w"]) == (66, 2, [2, 0, 0, 0], [18, 18, 16, 12])
    lay = E.layout((1 << 22, 1 << 21, 1 << 20))
    assert (lay["T"], lay["S"]) == (63, 0)
    lay = E.layout((1000, 800, 600))
    assert lay["b"] == [10, 10, 10]


def test_wide_tensor_round_trip():
    # 76-bit index: blocks on the top 12 bits
    rng = np.random.default_rng(7)
    dims = (1 << 24, 1 << 22, 1 << 20, 1 << 10)
    nnz = 5000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][:2500] = rng.integers(0, 4, size=2500)  # a dense corner
    vals = rng.random(nnz).astype(np.float32)
    t = E.encode(coords, vals, dims)
    assert len(t["block_ids"]) > 1
    back = E.decode(t["keys"], t["block_ids"], t["block_starts"], t["layout"])
    for n in range(4):
        np.testing.assert_array_equal(back[n], coords[n][t["order"]])
