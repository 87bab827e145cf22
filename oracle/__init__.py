"""ORACLE — test infrastructure only.

A plain, slow, obviously correct CPU reference for what the library computes:

* :mod:`oracle.encode` — the BLCO encoding (Section 4) in numpy;
* this module — fp64 sparse MTTKRP (Eq. (1), Figure 3) and the sparse CP fit
  loss and its gradient, through the C file ``mttkrp_oracle.c``.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the library under ``paper_2201_12523_amd``
and the library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import encode  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_lib(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp",
                               os.path.join(_HERE, "mttkrp_oracle.c"), "-o", _SO, "-lm"])
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_lib(force=False)
        L = ctypes.CDLL(_SO)
        p, i64 = ctypes.c_void_p, ctypes.c_int64
        L.oracle_mttkrp.argtypes = [ctypes.c_int, p, i64, p, p, p, ctypes.c_int, ctypes.c_int, p, p]
        L.oracle_mttkrp_rows.argtypes = [ctypes.c_int, p, i64, p, p, p, ctypes.c_int, ctypes.c_int,
                                         i64, p, p, p]
        L.oracle_mttkrp_rows_f32.argtypes = [ctypes.c_int, p, i64, p, p, p, ctypes.c_int,
                                             ctypes.c_int, i64, p, p, p]
        L.oracle_mttkrp_omp.argtypes = [ctypes.c_int, p, i64, p, p, p, ctypes.c_int,
                                        ctypes.c_int, p, p, ctypes.c_int, ctypes.c_int]
        L.oracle_mttkrp_omp.restype = ctypes.c_int
        L.oracle_mttkrp_rows_omp.argtypes = [ctypes.c_int, p, i64, p, p, p, ctypes.c_int,
                                             ctypes.c_int, i64, p, p, p, ctypes.c_int]
        L.oracle_mttkrp_rows_omp.restype = ctypes.c_int
        L.oracle_cp_model_omp.argtypes = [ctypes.c_int, i64, p, p, ctypes.c_int, p, ctypes.c_int]
        L.oracle_cp_model.argtypes = [ctypes.c_int, i64, p, p, ctypes.c_int, p]
        L.oracle_cp_loss.argtypes = [ctypes.c_int, i64, p, p, p, ctypes.c_int, p]
        L.oracle_cp_loss.restype = ctypes.c_double
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptrs(arrs):
    return (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])


def bf16_round(a):
    """fp32 values rounded to bfloat16 (8 significand bits), round to nearest even, as fp32.

    The rounding of factor storage to bf16 is not fixed by the paper (which
    uses fp64); round-to-nearest-even is the reading taken.  NaN is not expected.
    """
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(np.shape(a))


def mttkrp(coords, vals, factors, mode, dims=None, with_scale=True):
    """Mode-``mode`` MTTKRP in fp64: returns (M, S) with S = sum of |terms|.

    coords: list of N integer arrays (0-based); vals: nnz values; factors: list
    of N arrays I_m x R (factors[mode] is not read, only its shape if dims is None).
    All inputs are converted exactly to fp64 / uint32.
    """
    N = len(coords)
    if dims is None:
        dims = [f.shape[0] for f in factors]
    R = int(factors[0].shape[1]) if factors[0] is not None else int(
        [f for f in factors if f is not None][0].shape[1])
    cs = [_c(c, np.uint32) for c in coords]
    fs = [_c(f, np.float64) if f is not None else np.zeros((1, R)) for f in factors]
    v = _c(vals, np.float64)
    d = _c(dims, np.uint64)
    I = int(dims[mode])
    M = np.empty((I, R), dtype=np.float64)
    S = np.empty((I, R), dtype=np.float64) if with_scale else None
    lib().oracle_mttkrp(N, d.ctypes.data, len(v), _ptrs(cs), v.ctypes.data, _ptrs(fs), R, mode,
                        M.ctypes.data, S.ctypes.data if S is not None else None)
    return M, S


def mttkrp_omp(coords, vals, factors, mode, dims=None, with_scale=True, threads=0,
               force_atomic=False):
    """:func:`mttkrp` on several host threads: returns (M, S, threads used, atomic form taken).

    Only the order of the additions differs from :func:`mttkrp` (contiguous
    non-zero chunks per thread; private outputs added in thread order, or
    atomic updates when the private copies would not fit in a quarter of RAM).
    It exists to time the oracle on all host cores.
    """
    N = len(coords)
    if dims is None:
        dims = [f.shape[0] for f in factors]
    R = int([f for f in factors if f is not None][0].shape[1])
    cs = [_c(c, np.uint32) for c in coords]
    fs = [_c(f, np.float64) if f is not None else np.zeros((1, R)) for f in factors]
    v = _c(vals, np.float64)
    d = _c(dims, np.uint64)
    I = int(dims[mode])
    M = np.empty((I, R), dtype=np.float64)
    S = np.empty((I, R), dtype=np.float64) if with_scale else None
    t = lib().oracle_mttkrp_omp(N, d.ctypes.data, len(v), _ptrs(cs), v.ctypes.data, _ptrs(fs), R,
                                mode, M.ctypes.data, S.ctypes.data if S is not None else None,
                                int(threads), int(bool(force_atomic)))
    return M, S, abs(t), t < 0


def mttkrp_rows(coords, vals, factors, mode, rows, dims):
    """Rows ``rows`` (distinct) of the mode-``mode`` MTTKRP: (M_rows, S_rows)."""
    N = len(coords)
    R = int([f for f in factors if f is not None][0].shape[1])
    cs = [_c(c, np.uint32) for c in coords]
    fs = [_c(f, np.float64) if f is not None else np.zeros((1, R)) for f in factors]
    v = _c(vals, np.float64)
    d = _c(dims, np.uint64)
    rw = _c(rows, np.uint32)
    M = np.empty((len(rw), R), dtype=np.float64)
    S = np.empty((len(rw), R), dtype=np.float64)
    lib().oracle_mttkrp_rows(N, d.ctypes.data, len(v), _ptrs(cs), v.ctypes.data, _ptrs(fs), R,
                             mode, len(rw), rw.ctypes.data, M.ctypes.data, S.ctypes.data)
    return M, S


def mttkrp_rows_f32(coords, vals, factors, mode, rows, dims):
    """mttkrp_rows for fp32 values and factors (read and widened exactly, element by element)."""
    N = len(coords)
    R = int([f for f in factors if f is not None][0].shape[1])
    cs = [_c(c, np.uint32) for c in coords]
    fs = [_c(f, np.float32) if f is not None else np.zeros((1, R), np.float32) for f in factors]
    v = _c(vals, np.float32)
    d = _c(dims, np.uint64)
    rw = _c(rows, np.uint32)
    M = np.empty((len(rw), R), dtype=np.float64)
    S = np.empty((len(rw), R), dtype=np.float64)
    lib().oracle_mttkrp_rows_f32(N, d.ctypes.data, len(v), _ptrs(cs), v.ctypes.data, _ptrs(fs), R,
                                 mode, len(rw), rw.ctypes.data, M.ctypes.data, S.ctypes.data)
    return M, S


def mttkrp_rows_omp(coords, vals, factors, mode, rows, dims, threads=0):
    """:func:`mttkrp_rows` on several host threads, with fp64 values and fp32 factors
    (widened exactly as read).  Only the order of the additions differs."""
    N = len(coords)
    R = int([f for f in factors if f is not None][0].shape[1])
    cs = [_c(c, np.uint32) for c in coords]
    fs = [_c(f, np.float32) if f is not None else np.zeros((1, R), np.float32) for f in factors]
    v = _c(vals, np.float64)
    d = _c(dims, np.uint64)
    rw = _c(rows, np.uint32)
    M = np.empty((len(rw), R), dtype=np.float64)
    S = np.empty((len(rw), R), dtype=np.float64)
    lib().oracle_mttkrp_rows_omp(N, d.ctypes.data, len(v), _ptrs(cs), v.ctypes.data, _ptrs(fs), R,
                                 mode, len(rw), rw.ctypes.data, M.ctypes.data, S.ctypes.data,
                                 int(threads))
    return M, S


def cp_model_omp(coords, factors, threads=0):
    """:func:`cp_model` with the non-zeros shared among host threads (bit-identical)."""
    N = len(coords)
    R = int(factors[0].shape[1])
    cs = [_c(c, np.uint32) for c in coords]
    fs = [_c(f, np.float64) for f in factors]
    out = np.empty(len(cs[0]), dtype=np.float64)
    lib().oracle_cp_model_omp(N, len(out), _ptrs(cs), _ptrs(fs), R, out.ctypes.data, int(threads))
    return out


def cp_model(coords, factors):
    """xhat_k = sum_r prod_m A^(m)[i_m^k, r] at every non-zero (fp64)."""
    N = len(coords)
    R = int(factors[0].shape[1])
    cs = [_c(c, np.uint32) for c in coords]
    fs = [_c(f, np.float64) for f in factors]
    out = np.empty(len(cs[0]), dtype=np.float64)
    lib().oracle_cp_model(N, len(out), _ptrs(cs), _ptrs(fs), R, out.ctypes.data)
    return out


def cp_loss(coords, vals, factors):
    """(f, e): f = 1/2 sum_k e_k^2 with e_k = x_k - xhat_k (fp64)."""
    N = len(coords)
    R = int(factors[0].shape[1])
    cs = [_c(c, np.uint32) for c in coords]
    fs = [_c(f, np.float64) for f in factors]
    v = _c(vals, np.float64)
    e = np.empty(len(v), dtype=np.float64)
    f = lib().oracle_cp_loss(N, len(v), _ptrs(cs), v.ctypes.data, _ptrs(fs), R, e.ctypes.data)
    return float(f), e


def cp_grad(coords, vals, factors, dims=None):
    """Gradient of the sparse CP fit loss: G^(n) = -MTTKRP_n(E), E the residual tensor.

    The loss is 1/2 sum_k e_k^2 with e_k = x_k - xhat_k; d xhat_k / d A^(n)[i,r]
    is prod_{m != n} A^(m)[i_m^k, r] when i_n^k = i, so the gradient is the
    mode-n MTTKRP of the tensor holding -e_k at the non-zeros.  Returns
    (f, e, [G^(n)], [S^(n)]) with S^(n) the sum of |terms| of each entry.
    """
    f, e = cp_loss(coords, vals, factors)
    G, S = [], []
    for n in range(len(coords)):
        g, s = mttkrp(coords, -e, factors, n, dims=dims)
        G.append(g)
        S.append(s)
    return f, e, G, S
