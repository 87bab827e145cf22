"""The library's host-side BLCO construction against the oracle encoder, bit for bit.

Tensors are built with host placement, which makes no GPU call, and exported;
keys, permuted values, block keys and block starts must equal the oracle's,
and the reported bit map must equal the oracle layout.
"""
import ctypes
import re
import subprocess

import numpy as np
import pytest

import synth
from conftest import ROOT
from oracle import encode as E

blco = pytest.importorskip("paper_2201_12523_amd")


def _lib_or_skip():
    try:
        return blco.lib()
    except RuntimeError as e:  # not built
        pytest.skip(str(e))


def _same(coords, vals, dims, key_bits=64, cap=1 << 27):
    _lib_or_skip()
    t = blco.build(coords, vals, dims, key_bits=key_bits, max_block_nnz=cap, placement="host")
    keys, v, bids, bst = t.export()
    ref = E.encode(coords, vals, dims, key_bits=key_bits, max_block_nnz=cap)
    np.testing.assert_array_equal(keys, ref["keys"])
    np.testing.assert_array_equal(v, ref["values"])
    np.testing.assert_array_equal(bids, ref["block_ids"])
    np.testing.assert_array_equal(bst, ref["block_starts"])
    inf = t.info()
    lay = ref["layout"]
    assert inf["total_bits"] == lay["T"] and inf["key_bits"] == lay["K"]
    assert inf["block_bits"] == lay["S"]
    assert inf["bits"] == lay["b"] and inf["kept"] == lay["w"]
    assert inf["shift"] == lay["s"] and inf["high"] == lay["h"]
    assert inf["nblocks"] == len(ref["block_ids"])
    t.free()
    return ref


def test_figure6(fig4a):
    coords, vals, dims = fig4a
    ref = _same(coords, vals, dims, key_bits=5, cap=6)
    assert ref["keys"].tolist() == [0, 16, 17, 7, 18, 23, 1, 8, 11, 27, 30, 31]


@pytest.mark.parametrize("dims", [(1000, 800, 600), (5, 1, 7), (2 ** 22, 2 ** 21, 2 ** 20),
                                  (1 << 24, 1 << 22, 1 << 20, 1 << 10),
                                  (1 << 20, 1 << 18, 1 << 16, 1 << 12), (3,), (9, 2),
                                  (17, 3, 5, 2, 9, 4, 3, 6)])
def test_random_tensors(dims):
    rng = np.random.default_rng(len(dims) * 100 + dims[0] % 97)
    nnz = 20000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][: nnz // 3] = rng.integers(0, max(1, min(dims[0], 5)), size=nnz // 3)
    vals = rng.random(nnz).astype(np.float32)
    _same(coords, vals, dims)


@pytest.mark.parametrize("key_bits,cap", [(12, 64), (8, 6), (5, 1), (33, 1000), (64, 7)])
def test_forced_blocking(key_bits, cap):
    rng = np.random.default_rng(key_bits + cap)
    dims = (300, 7, 1, 129, 40)
    nnz = 5000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.standard_normal(nnz).astype(np.float32)
    _same(coords, vals, dims, key_bits=key_bits, cap=cap)


def test_duplicates_keep_input_order():
    dims = (8, 8, 8)
    coords = [np.array([1, 1, 1, 0, 1], dtype=np.uint32) for _ in range(3)]
    vals = np.array([1, 2, 3, 4, 5], dtype=np.float32)
    ref = _same(coords, vals, dims)
    assert ref["values"].tolist() == [4, 1, 2, 3, 5]


def test_synthetic_zipf_medium():
    w = synth.WORKLOADS["zipf3"]
    coords, vals = synth.workload_tensor(w, nnz=400_000)
    _same(coords, vals, w.dims)


def test_empty_tensor():
    _lib_or_skip()
    t = blco.build([np.zeros(0, np.uint32)] * 3, np.zeros(0, np.float32), (4, 5, 6),
                   placement="host")
    keys, v, bids, bst = t.export()
    assert len(keys) == 0 and len(bids) == 0 and bst.tolist() == [0]


def test_errors():
    _lib_or_skip()
    c = [np.array([0, 3], dtype=np.uint32), np.array([0, 1], dtype=np.uint32)]
    v = np.ones(2, np.float32)
    with pytest.raises(blco.BLCOError) as e:
        blco.build(c, v, (3, 2), placement="host")
    assert e.value.status == "ERANGE"
    with pytest.raises(blco.BLCOError) as e:
        blco.build([np.zeros(1, np.uint32)] * 9, np.ones(1, np.float32), (2,) * 9, placement="host")
    assert e.value.status == "EUNSUPPORTED"
    with pytest.raises(blco.BLCOError) as e:
        # 8 modes x 32 bits = 256 bits: the block key would exceed 64 bits
        blco.build([np.zeros(1, np.uint32)] * 8, np.ones(1, np.float32), (2 ** 32,) * 8,
                   placement="host")
    assert e.value.status == "EUNSUPPORTED"
    with pytest.raises(blco.BLCOError) as e:
        blco.build(c, v, (4, 2), key_bits=0, placement="host")
    assert e.value.status == "EINVAL"
    with pytest.raises(blco.BLCOError) as e:
        blco.build(c, v, (4, 2), max_block_nnz=0, placement="host")
    assert e.value.status == "EINVAL"
    with pytest.raises(blco.BLCOError) as e:
        blco.build(c, v, (4, 0), placement="host")
    assert e.value.status == "EINVAL"


def test_exports_every_declared_symbol():
    _lib_or_skip()
    header = open(f"{ROOT}/include/blco.h").read()
    declared = sorted(set(re.findall(r"\b(blco_[a-z0-9_]+)\s*\(", header)))
    assert "blco_build" in declared and "blco_mttkrp_stream" in declared
    out = subprocess.check_output(["nm", "-D", "--defined-only", blco.library_path()], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [d for d in declared if d not in exported]
    assert not missing, missing
    L = ctypes.CDLL(blco.library_path())
    for d in declared:
        assert getattr(L, d) is not None


def test_resolution_setting_and_heuristic():
    """Section 5.3: the hierarchical mechanism for a target mode shorter than the
    compute-unit count (at least 100 on any device this runs on), the register-based
    one otherwise; a forced choice sticks, and a mode too long for the LDS stash
    rejects the hierarchical one."""
    _lib_or_skip()
    rng = np.random.default_rng(2)
    dims = (100, 5000, 7)
    coords = [rng.integers(0, d, size=500).astype(np.uint32) for d in dims]
    t = blco.build(coords, rng.random(500).astype(np.float32), dims, placement="host")
    assert [t.resolution(n, 32) for n in range(3)] == ["hierarchical", "register", "hierarchical"]
    t.set_resolution("register")
    assert [t.resolution(n, 32) for n in range(3)] == ["register"] * 3
    t.set_resolution("hierarchical")
    assert t.resolution(0, 1000) == "hierarchical"   # split into rank slices
    with pytest.raises(blco.BLCOError) as e:
        t.resolution(1, 16)
    assert e.value.status == "EUNSUPPORTED"
    L = blco.lib()
    assert L.blco_set_resolution(t.handle, 3) == -1
    assert L.blco_set_resolution(None, 0) == -1
    c = ctypes.c_int(-1)
    assert L.blco_resolution(t.handle, 3, 32, ctypes.byref(c)) == -1
    assert L.blco_resolution(t.handle, 0, 0, ctypes.byref(c)) == -1
    t.set_resolution("auto")
    assert L.blco_resolution(t.handle, 2, 8, ctypes.byref(c)) == 0 and c.value == 2


def test_frequent_rows_recorded_at_build():
    """Rows with at least hot_min_count non-zeros (at most 256 per mode, most
    frequent first); none when disabled or for modes longer than 2^26."""
    _lib_or_skip()
    rng = np.random.default_rng(3)
    nnz = 20_000
    c0 = rng.integers(0, 1000, size=nnz).astype(np.uint32)
    c0[:3000] = 7            # row 7: 3000+ non-zeros
    c0[3000:5500] = 11       # row 11: 2500+
    c1 = rng.integers(0, (1 << 27) + 5, size=nnz).astype(np.uint32)
    c1[:4000] = 0
    dims = (1000, (1 << 27) + 5)
    vals = np.ones(nnz, np.float32)
    t = blco.build([c0, c1], vals, dims, placement="host")
    assert t.info()["hot_rows"] == [2, 0]           # default threshold 2048; mode 1 too long
    t = blco.build([c0, c1], vals, dims, placement="host", hot_min_count=1)
    assert t.info()["hot_rows"] == [256, 0]
    t = blco.build([c0, c1], vals, dims, placement="host", hot_min_count=-1)
    assert t.info()["hot_rows"] == [0, 0]
