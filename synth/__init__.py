"""Seeded synthetic sparse tensors and dense factors.

The workloads stand in for the real-world tensors the paper measures (Table 2):
N-mode coordinates with per-mode power-law (Zipf) or uniform index
distributions, deduplicated so every coordinate is distinct, with U(0,1) or
lognormal values, and N(0,1) factor matrices.  Nothing here computes any part of
the tensor method; the generator library (``synth.c``) only draws numbers.

Streams: config ``k`` uses base key ``12523 * 100 + k``; each quantity (the
coordinates of mode m, the values, the factor of mode m, ...) has its own
stream id, so the pieces are independent and each can be regenerated alone.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None

BASE_SEED = 12523


def build_lib(force: bool = True) -> str:
    """Compile ``synth.c`` into ``libsynth.so`` next to it."""
    if force or not os.path.exists(_SO):
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-pthread", os.path.join(_HERE, "synth.c"),
             "-o", _SO, "-lm"])
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_lib(force=False)
        L = ctypes.CDLL(_SO)
        u64, i64, p = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        L.synth_stream_key.restype = u64
        L.synth_stream_key.argtypes = [u64, u64]
        L.synth_uniform_u32.argtypes = [u64, u64, i64, u64, p]
        L.synth_zipf_cdf.argtypes = [u64, ctypes.c_double, p]
        L.synth_zipf_u32.argtypes = [u64, u64, i64, p, u64, p]
        L.synth_u01_f32.argtypes = [u64, u64, i64, p]
        L.synth_u01_f64.argtypes = [u64, u64, i64, p]
        L.synth_normal_f64.argtypes = [u64, u64, i64, ctypes.c_double, ctypes.c_double, p]
        L.synth_normal_f32.argtypes = [u64, u64, i64, ctypes.c_double, ctypes.c_double, p]
        L.synth_lognormal_f32.argtypes = [u64, u64, i64, ctypes.c_double, ctypes.c_double, p]
        L.synth_dedupe.restype = i64
        L.synth_dedupe.argtypes = [ctypes.c_int, p, i64, p, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def stream_key(seed: int, stream: int) -> int:
    return int(lib().synth_stream_key(seed, stream))


# stream ids
S_COORD = 100   # + mode
S_VALUE = 200
S_FACTOR = 300  # + mode (+ 1000 * variant)
S_TRUTH = 400   # + mode
S_NOISE = 500


@dataclass
class Workload:
    """One synthetic workload: tensor recipe plus factor rank(s)."""
    name: str
    dims: tuple
    nnz: int
    index_dist: tuple          # per mode: ("zipf", alpha) or ("uniform",)
    value_dist: str            # "u01" | "lognormal" | "cp8"
    ranks: tuple
    modes: tuple               # 0-based modes exercised
    seed: int
    notes: str = ""
    budget_bytes: int = 0      # device budget (out-of-memory workload only)
    extra: dict = field(default_factory=dict)


def _z(a):
    return ("zipf", a)


U = ("uniform",)

WORKLOADS = {
    # 3-mode, 1000x800x600, 100k uniform distinct coordinates, R=16, mode 1
    "small": Workload("small", (1000, 800, 600), 100_000, ("linear_uniform",) * 3, "u01", (16,),
                      (0,), BASE_SEED * 100 + 0),
    # 3-mode, 2^22 x 2^21 x 2^20 (63 bits: one block), 50M Zipf(1.1), R=32, all modes
    "zipf3": Workload("zipf3", (1 << 22, 1 << 21, 1 << 20), 50_000_000, (_z(1.1),) * 3, "u01",
                      (32,), (0, 1, 2), BASE_SEED * 100 + 1),
    # same shape with uniform indices: no hot rows (a contention-free reference point)
    "uniform3": Workload("uniform3", (1 << 22, 1 << 21, 1 << 20), 50_000_000, (U,) * 3, "u01",
                         (32,), (0, 1, 2), BASE_SEED * 100 + 5),
    # 4-mode, 2^24 x 2^22 x 2^20 x 2^10 (76 bits: blocked on the top 12), 200M, R=32/64
    "zipf4": Workload("zipf4", (1 << 24, 1 << 22, 1 << 20, 1 << 10), 200_000_000,
                      (_z(1.2), _z(1.2), U, U), "lognormal", (32, 64), (0, 1, 2, 3),
                      BASE_SEED * 100 + 2),
    # out-of-memory: 2^23 x 2^23 x 2^17, 1.5B Zipf(1.05), 8 GB device budget, R=32
    "oom3": Workload("oom3", (1 << 23, 1 << 23, 1 << 17), 1_500_000_000, (_z(1.05),) * 3, "u01",
                     (32,), (0, 1, 2), BASE_SEED * 100 + 3, budget_bytes=8_000_000_000),
    # CP-gradient: 2^20 x 2^18 x 2^16 x 2^12, 80M Zipf(1.1), rank-8 model + noise, R=32
    "cpgrad4": Workload("cpgrad4", (1 << 20, 1 << 18, 1 << 16, 1 << 12), 80_000_000,
                        (_z(1.1),) * 4, "cp8", (32,), (0, 1, 2, 3), BASE_SEED * 100 + 4),
    # short modes: 2^21 x 2^17 x 24 x 168, 50M, Zipf(1.1) on the long modes and uniform on
    # the two modes shorter than the compute-unit count (hierarchical resolution), R=32
    "short4": Workload("short4", (1 << 21, 1 << 17, 24, 168), 50_000_000,
                       (_z(1.1), _z(1.1), U, U), "u01", (32,), (0, 1, 2, 3), BASE_SEED * 100 + 6),
}


_cdf_cache: dict = {}


def zipf_cdf(I: int, alpha: float) -> np.ndarray:
    key = (I, alpha)
    if key not in _cdf_cache:
        cdf = np.empty(I, dtype=np.float64)
        lib().synth_zipf_cdf(I, alpha, _ptr(cdf))
        _cdf_cache.clear()
        _cdf_cache[key] = cdf
    return _cdf_cache[key]


def _draw_mode(seed: int, mode: int, dist: tuple, I: int, start: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    key = stream_key(seed, S_COORD + mode)
    if dist[0] == "zipf":
        cdf = zipf_cdf(I, dist[1])
        lib().synth_zipf_u32(key, start, n, _ptr(cdf), I, _ptr(out))
    else:
        lib().synth_uniform_u32(key, start, n, I, _ptr(out))
    return out


def draw_coords(dims, nnz: int, index_dist, seed: int, log=None):
    """Exactly ``nnz`` distinct coordinates (0-based u32 arrays, one per mode).

    Draws rounds of coordinates per mode (counter-based, so a longer draw
    extends a shorter one), keeps the first occurrence of every coordinate in
    draw order, and tops up with 1.35x the deficit until ``nnz`` are distinct;
    the result is the first ``nnz`` distinct draws, in draw order.
    """
    N = len(dims)
    dims_a = np.asarray(dims, dtype=np.uint64)
    if index_dist[0] == "linear_uniform":
        # uniform over the whole index space: draw a linear index, split it mixed-radix
        total = int(np.prod([int(d) for d in dims]))
        assert total < (1 << 63)
        m = int(nnz * 1.05) + 64
        while True:
            lin = np.empty(m, dtype=np.uint32) if total <= (1 << 32) else None
            key = stream_key(seed, S_COORD)
            if lin is not None:
                lib().synth_uniform_u32(key, 0, m, total, _ptr(lin))
                lin = lin.astype(np.uint64)
            else:
                raise ValueError("linear_uniform needs a product of dims <= 2^32")
            coords = []
            rest = lin.copy()
            for d in dims:
                coords.append((rest % np.uint64(d)).astype(np.uint32))
                rest //= np.uint64(d)
            keep = np.empty(m, dtype=np.uint32)
            arr = (ctypes.c_void_p * N)(*[_ptr(c) for c in coords])
            cnt = lib().synth_dedupe(N, _ptr(dims_a), m, arr, _ptr(keep))
            if cnt >= nnz:
                keep = keep[:nnz]
                return [np.ascontiguousarray(c[keep]) for c in coords]
            m += int((nnz - cnt) * 1.35) + 64
    m = int(nnz * 1.1) + 64
    coords = [np.empty(0, dtype=np.uint32) for _ in range(N)]
    while True:
        if m >= (1 << 32):
            raise ValueError("too many draws")
        have = len(coords[0])
        coords = [np.concatenate([coords[d], _draw_mode(seed, d, index_dist[d], int(dims[d]), have,
                                                         m - have)]) for d in range(N)]
        keep = np.empty(m, dtype=np.uint32)
        arr = (ctypes.c_void_p * N)(*[_ptr(c) for c in coords])
        cnt = lib().synth_dedupe(N, _ptr(dims_a), m, arr, _ptr(keep))
        if log:
            log(f"draws={m} distinct={cnt}")
        if cnt >= nnz:
            keep = keep[:nnz]
            return [np.ascontiguousarray(c[keep]) for c in coords]
        # the marginal duplicate rate exceeds the average one: extrapolate with margin
        m += int((nnz - cnt) * (m / max(cnt, 1)) * 1.25) + 64


def draw_values(nnz: int, dist: str, seed: int) -> np.ndarray:
    out = np.empty(nnz, dtype=np.float32)
    key = stream_key(seed, S_VALUE)
    if dist == "u01":
        lib().synth_u01_f32(key, 0, nnz, _ptr(out))
    elif dist == "lognormal":
        lib().synth_lognormal_f32(key, 0, nnz, 0.0, 1.0, _ptr(out))
    else:
        raise ValueError(dist)
    return out


def draw_factor(I: int, R: int, seed: int, mode: int, variant: int = 0, scale: float = 1.0):
    """I x R row-major fp32 matrix with N(0, scale^2) entries."""
    out = np.empty((I, R), dtype=np.float32)
    key = stream_key(seed, S_FACTOR + mode + 1000 * variant)
    lib().synth_normal_f32(key, 0, I * R, 0.0, float(scale), _ptr(out))
    return out


def draw_u01_matrix(I: int, R: int, seed: int, stream: int) -> np.ndarray:
    """I x R fp64 matrix with U(0,1) entries."""
    out = np.empty((I, R), dtype=np.float64)
    lib().synth_u01_f64(stream_key(seed, stream), 0, I * R, _ptr(out))
    return out


def draw_normal_f64(n: int, sigma: float, seed: int, stream: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().synth_normal_f64(stream_key(seed, stream), 0, n, 0.0, float(sigma), _ptr(out))
    return out


def random_tensor(dims, nnz, seed, index_dist=None, value_dist="u01"):
    """A small or medium tensor for tests: (coords list, values)."""
    if index_dist is None:
        index_dist = (U,) * len(dims)
    coords = draw_coords(dims, nnz, index_dist, seed)
    vals = draw_values(nnz, value_dist, seed)
    return coords, vals


def workload_tensor(w: Workload, nnz: int | None = None, log=None):
    """Coordinates and values of a workload; ``nnz`` may shrink it (same recipe)."""
    n = w.nnz if nnz is None else nnz
    coords = draw_coords(w.dims, n, w.index_dist, w.seed, log=log)
    if w.value_dist == "cp8":
        vals = None  # built from a planted CP model by the caller
    else:
        vals = draw_values(n, w.value_dist, w.seed)
    return coords, vals


def workload_factors(w: Workload, R: int, variant: int = 0, scale: float = 1.0):
    return [draw_factor(int(I), R, w.seed, m, variant, scale) for m, I in enumerate(w.dims)]

