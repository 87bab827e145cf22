"""BLCO construction on the GPU (blco_build_device) against the oracle encoder
(oracle.encode, numpy) on the same inputs, bit for bit: keys, values in BLCO
order, block keys, block starts and the bit map.  It is also compared with the
host builder (the frequent-row counts, which the oracle does not define, and
MTTKRP results).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from oracle import encode as E  # noqa: E402
import paper_2201_12523_amd as blco  # noqa: E402
import synth  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def same(coords, vals, dims, **kw):
    tg = blco.build_device(coords, vals, dims, **kw)
    b = tg.export()
    ref = E.encode(coords, vals, dims, key_bits=kw.get("key_bits", 64),
                   max_block_nnz=kw.get("max_block_nnz", 1 << 27))
    for x, name in zip(b, ("keys", "values", "block_ids", "block_starts")):
        np.testing.assert_array_equal(x, ref[name], err_msg=f"GPU builder vs oracle: {name}")
    lay, ig = ref["layout"], tg.info()
    assert (ig["total_bits"], ig["key_bits"], ig["block_bits"]) == (lay["T"], lay["K"], lay["S"])
    assert ig["bits"] == lay["b"] and ig["kept"] == lay["w"]
    assert ig["shift"] == lay["s"] and ig["high"] == lay["h"]
    assert ig["nblocks"] == len(ref["block_ids"])
    th = blco.build(coords, vals, dims, placement="host", **kw)
    ih = th.info()
    for k in ("total_bits", "key_bits", "block_bits", "bits", "kept", "shift", "high", "nblocks",
              "nruns", "hot_rows"):
        assert ih[k] == ig[k], k
    return tg


def rand_coords(rng, dims, nnz):
    return [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]


@pytest.mark.parametrize("key_bits,cap", [(64, 1 << 27), (9, 100), (14, 1)])
def test_matches_oracle_encoder(key_bits, cap):
    rng = np.random.default_rng(key_bits)
    dims = (1000, 300, 77, 6)
    coords = rand_coords(rng, dims, 20_000)
    coords[0][:500] = 3                      # duplicates: stable order decides
    coords[1][:500] = 4
    coords[2][:500] = 5
    coords[3][:500] = 1
    vals = rng.standard_normal(20_000).astype(np.float32)
    same(coords, vals, dims, key_bits=key_bits, max_block_nnz=cap)


@pytest.mark.parametrize("key_bits,cap", [(64, 1 << 27), (40, 1 << 27), (64, 1000)])
def test_index_over_64_bits(key_bits, cap):
    # 2^24 x 2^22 x 2^20 x 2^10: 76 bits, blocks on the top 12 (36 at 40 key bits)
    w = synth.WORKLOADS["zipf4"]
    coords, vals = synth.workload_tensor(w, nnz=2_000_000)
    t = same(coords, vals, w.dims, key_bits=key_bits, max_block_nnz=cap)
    assert t.info()["total_bits"] == 76 and t.info()["nruns"] > 1


@pytest.mark.parametrize("dims", [(1 << 24,) * 4, (1 << 24, 1 << 24, 1 << 24, 1 << 25),
                                  (1 << 25,) * 4])
def test_index_of_96_bits_and_over(dims):
    # 96 bits: the two-part sort moves the values and the high 32 bits along; 97 and
    # 100 bits: the (index, number) sort and the gathers
    rng = np.random.default_rng(len(dims) + int(np.log2(dims[-1])))
    nnz = 200_000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.random(nnz).astype(np.float32)
    t = same(coords, vals, dims, key_bits=64, max_block_nnz=5000)
    assert t.info()["total_bits"] == sum(int(np.log2(d)) for d in dims)


def test_zipf_recipe_frequent_rows_and_mttkrp():
    w = synth.WORKLOADS["zipf3"]
    coords, vals = synth.workload_tensor(w, nnz=3_000_000)
    t = same(coords, vals, w.dims)
    assert t.info()["hot_rows"][0] > 0
    A = synth.workload_factors(w, 32)
    F = [torch.from_numpy(a).to(DEV) for a in A]
    th = blco.build(coords, vals, w.dims)
    for n in range(3):
        rows = np.unique(np.concatenate([np.arange(20), [w.dims[n] - 1]])).astype(np.int64)
        assert rows.max() < w.dims[n]
        a = blco.mttkrp(t, n, F)
        b = blco.mttkrp(th, n, F)
        torch.cuda.synchronize()
        M, S = oracle.mttkrp_rows_f32(coords, vals, A, n, rows.astype(np.uint32), w.dims)
        for out in (a, b):
            got = out[torch.from_numpy(rows).to(DEV)].cpu().numpy().astype(np.float64)
            nz = S > 0
            assert np.all(got[~nz] == 0)
            assert float((np.abs(got - M)[nz] / S[nz]).max()) <= 1e-5


def test_edge_cases():
    rng = np.random.default_rng(5)
    same([np.zeros(0, np.uint32)] * 3, np.zeros(0, np.float32), (5, 6, 7))     # empty
    same([np.zeros(10, np.uint32)] * 2, np.ones(10, np.float32), (1, 1))      # no index bits
    same([rng.integers(0, 50, 1).astype(np.uint32)], np.ones(1, np.float32), (50,))
    same(rand_coords(rng, (7, 9, 11, 13, 3, 5, 2, 4), 3000),
         rng.random(3000).astype(np.float32), (7, 9, 11, 13, 3, 5, 2, 4))    # eight modes
    same(rand_coords(rng, (100, 200), 5000), rng.random(5000).astype(np.float32), (100, 200),
         hot_min_count=1)


@pytest.mark.parametrize("nnz", [4095, 4096, 4097, 8192, 3 * 4096 + 1])
def test_sort_tile_boundaries(nnz):
    # the radix sort works on tiles of 4096 keys: full, partial and single-key last tiles
    rng = np.random.default_rng(nnz)
    dims = (300, 200, 100)
    coords = rand_coords(rng, dims, nnz)
    coords[0][: nnz // 5] = 7                  # duplicates: stable order decides
    coords[1][: nnz // 5] = 9
    same(coords, rng.standard_normal(nnz).astype(np.float32), dims)


@pytest.mark.parametrize("span", [1, 8, 256, 1 << 20])
def test_sort_skips_constant_digits(span):
    # only mode 1 varies (its bits sit at index positions 0, 3, 6, 7, 8, ...): 0, 1, 2 or 3
    # of the index's 8-bit digits change between keys, so the sort runs that many passes
    # (none: a copy) and skips the others
    rng = np.random.default_rng(span)
    dims = (1 << 20, 4, 4)
    nnz = 20_000
    coords = [rng.integers(0, span, size=nnz).astype(np.uint32),
              np.zeros(nnz, np.uint32), np.zeros(nnz, np.uint32)]
    same(coords, rng.standard_normal(nnz).astype(np.float32), dims)


def test_errors_and_pinned_placement():
    rng = np.random.default_rng(6)
    dims = (20, 30, 40)
    coords = rand_coords(rng, dims, 1000)
    vals = rng.random(1000).astype(np.float32)
    bad = [c.copy() for c in coords]
    bad[2][777] = 40
    with pytest.raises(blco.BLCOError) as e:
        blco.build_device(bad, vals, dims)
    assert e.value.status == "ERANGE" and "777" in str(e.value)
    with pytest.raises(blco.BLCOError):
        blco.build_device(coords, vals, dims, placement="host")
    tp = blco.build_device(coords, vals, dims, placement="pinned")
    th = blco.build(coords, vals, dims, placement="host")
    ref = E.encode(coords, vals, dims)
    for x, name in zip(tp.export(), ("keys", "values", "block_ids", "block_starts")):
        np.testing.assert_array_equal(x, ref[name], err_msg=name)
    A = [rng.standard_normal((d, 8)).astype(np.float32) for d in dims]
    F = [torch.from_numpy(a).to(DEV) for a in A]
    out = blco.mttkrp_stream(tp, 1, F, device_budget=1 << 30)
    M, S = oracle.mttkrp(coords, vals, A, 1)
    got = out.cpu().numpy().astype(np.float64)
    nz = S > 0
    assert float((np.abs(got - M)[nz] / S[nz]).max()) <= 1e-5
