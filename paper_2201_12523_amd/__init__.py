"""Python binding of the BLCO sparse MTTKRP library (``libblco.so``, C ABI in include/blco.h).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels.  PyTorch provides device memory and streams.  ``torch`` is
imported before the library is loaded so that the library binds to the HIP
runtime torch already uses (one runtime per process).

Method: Nguyen et al., "Efficient, Out-of-Memory Sparse MTTKRP on Massively
Parallel Architectures", ICS '22 — the BLCO format (Section 4) and its MTTKRP
(Section 5).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (must precede loading libblco.so)

__all__ = ["BLCOTensor", "build", "mttkrp", "mttkrp_acc", "mttkrp_v", "mttkrp_stream",
           "mttkrp_stream_all", "sampled_loss", "cp_grad",
           "cast_bf16", "atomic_probe", "gather_probe", "CPLoss", "BLCOError", "lib", "library_path"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libblco.so")
_lib = None

MAX_MODES = 8
F32, BF16 = 0, 1
PLACEMENTS = {"device": 0, "pinned": 1, "host": 2}
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ERANGE", -5: "EUNSUPPORTED"}

EXPORTED = ["blco_build", "blco_mttkrp", "blco_mttkrp_acc", "blco_mttkrp_v", "blco_mttkrp_stream",
            "blco_mttkrp_stream_all",
            "blco_sampled_loss", "blco_cp_grad", "blco_cp_grad_noalloc", "blco_scale", "blco_cast_bf16", "blco_set_resolution", "blco_resolution",
            "blco_gram", "blco_cp_als", "blco_build_device",
            "blco_atomic_probe", "blco_gather_probe", "blco_frequent_rows", "blco_info", "blco_export", "blco_free",
            "blco_last_error"]


class BLCOError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class _Opts(ctypes.Structure):
    _fields_ = [("key_bits", ctypes.c_int), ("max_block_nnz", ctypes.c_int64),
                ("placement", ctypes.c_int), ("hot_min_count", ctypes.c_int64)]


class _CPALSOpts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int), ("tol", ctypes.c_double), ("factor_dtype", ctypes.c_int)]


class _CPALSReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("pinv_fallbacks", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("nmodes", ctypes.c_int), ("nnz", ctypes.c_int64), ("total_bits", ctypes.c_int),
                ("key_bits", ctypes.c_int), ("block_bits", ctypes.c_int),
                ("bits", ctypes.c_int * MAX_MODES), ("kept", ctypes.c_int * MAX_MODES),
                ("shift", ctypes.c_int * MAX_MODES), ("high", ctypes.c_int * MAX_MODES),
                ("dims", ctypes.c_uint64 * MAX_MODES), ("nblocks", ctypes.c_int64),
                ("nruns", ctypes.c_int64), ("placement", ctypes.c_int),
                ("device_bytes", ctypes.c_size_t), ("host_bytes", ctypes.c_size_t),
                ("stream_peak_bytes", ctypes.c_size_t), ("stream_chunks", ctypes.c_int64),
                ("stream_chunk_nnz", ctypes.c_int64), ("stream_copy_ms", ctypes.c_double),
                ("stream_kernel_ms", ctypes.c_double), ("stream_total_ms", ctypes.c_double),
                ("hot_rows", ctypes.c_int * MAX_MODES),
                ("build_stage_ms", ctypes.c_double * 5)]


def library_path() -> str:
    return _SO


def lib():
    """The loaded ``libblco.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is missing: build it with `python -m paper_2201_12523_amd.buildlib`")
        L = ctypes.CDLL(_SO)
        p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.blco_build.argtypes = [i32, p, i64, p, p, p, ctypes.POINTER(p)]
        L.blco_mttkrp.argtypes = [p, i32, p, i32, i32, p, p]
        L.blco_mttkrp_acc.argtypes = [p, i32, p, i32, i32, p, p]
        L.blco_mttkrp_v.argtypes = [p, i32, p, p, i32, i32, p, ctypes.c_double, p, p]
        L.blco_mttkrp_stream.argtypes = [p, i32, p, i32, i32, p, ctypes.c_size_t, p]
        L.blco_mttkrp_stream_all.argtypes = [p, p, i32, i32, p, ctypes.c_size_t, p]
        L.blco_sampled_loss.argtypes = [p, p, i32, i32, p, p, p]
        L.blco_cast_bf16.argtypes = [p, p, i64, p]
        L.blco_cp_grad.argtypes = [p, p, i32, i32, p, ctypes.c_double, p, p, p, ctypes.c_size_t,
                                   p]
        L.blco_cp_grad_noalloc.argtypes = [p, p, i32, i32, p, ctypes.c_double, p, p, p, p]
        L.blco_scale.argtypes = [p, i64, p, ctypes.c_double, p]
        L.blco_info.argtypes = [p, ctypes.POINTER(_Info)]
        L.blco_export.argtypes = [p, p, p, p, p]
        L.blco_set_resolution.argtypes = [p, i32]
        L.blco_build_device.argtypes = [i32, p, i64, p, p, ctypes.POINTER(_Opts), p,
                                        ctypes.POINTER(p)]
        L.blco_gram.argtypes = [p, i32, i64, i32, p, p]
        L.blco_cp_als.argtypes = [p, p, i32, ctypes.POINTER(_CPALSOpts), p,
                                  ctypes.POINTER(_CPALSReport), p]
        L.blco_resolution.argtypes = [p, i32, i32, ctypes.POINTER(ctypes.c_int)]
        L.blco_frequent_rows.argtypes = [p, i32, i32, ctypes.POINTER(ctypes.c_int)]
        L.blco_atomic_probe.argtypes = [p, i64, i32, p, i64, p]
        L.blco_gather_probe.argtypes = [p, i64, i32, p, i64, p, p]
        L.blco_free.argtypes = [p]
        L.blco_free.restype = None
        L.blco_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("blco_free", "blco_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise BLCOError(rc, lib().blco_last_error().decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


RESOLUTIONS = {"auto": 0, "register": 1, "hierarchical": 2}


class BLCOTensor:
    """A BLCO tensor owned by the library (freed with the object)."""

    def __init__(self, handle, dims):
        self._h = ctypes.c_void_p(handle)
        self.dims = tuple(int(d) for d in dims)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _Info()
        _check(lib().blco_info(self._h, ctypes.byref(inf)))
        N = inf.nmodes
        return dict(nmodes=N, nnz=inf.nnz, total_bits=inf.total_bits, key_bits=inf.key_bits,
                    block_bits=inf.block_bits, bits=list(inf.bits[:N]), kept=list(inf.kept[:N]),
                    shift=list(inf.shift[:N]), high=list(inf.high[:N]), dims=list(inf.dims[:N]),
                    nblocks=inf.nblocks, nruns=inf.nruns, placement=inf.placement,
                    device_bytes=inf.device_bytes, host_bytes=inf.host_bytes,
                    stream_peak_bytes=inf.stream_peak_bytes, stream_chunks=inf.stream_chunks,
                    stream_chunk_nnz=inf.stream_chunk_nnz, stream_copy_ms=inf.stream_copy_ms,
                    stream_kernel_ms=inf.stream_kernel_ms, stream_total_ms=inf.stream_total_ms,
                    hot_rows=list(inf.hot_rows[:N]),
                    build_stage_ms=dict(zip(("linearize", "sort", "encode", "runs",
                                             "frequent_rows"), list(inf.build_stage_ms))))

    @property
    def nnz(self) -> int:
        return self.info()["nnz"]

    @property
    def nmodes(self) -> int:
        return len(self.dims)

    def set_resolution(self, resolution: str):
        """Conflict resolution of later MTTKRP calls: "auto" (Section 5.3 heuristic),
        "register" (Section 5.2) or "hierarchical" (Section 5.1)."""
        if resolution not in RESOLUTIONS:
            raise ValueError(f"resolution {resolution!r}: one of {sorted(RESOLUTIONS)}")
        _check(lib().blco_set_resolution(self._h, RESOLUTIONS[resolution]))

    def resolution(self, mode: int, rank: int) -> str:
        """The mechanism a mode-`mode` MTTKRP at rank `rank` uses on the current device."""
        c = ctypes.c_int(-1)
        _check(lib().blco_resolution(self._h, int(mode), int(rank), ctypes.byref(c)))
        return {v: k for k, v in RESOLUTIONS.items()}[c.value]

    def stash_rows(self, mode: int, rank: int) -> int:
        """Frequent rows of `mode` a register-based MTTKRP at `rank` sums in its LDS stash."""
        c = ctypes.c_int(-1)
        _check(lib().blco_frequent_rows(self._h, int(mode), int(rank), ctypes.byref(c)))
        return c.value

    def export(self):
        """(keys uint64, values float32, block_ids uint64, block_starts int64) on the host."""
        inf = self.info()
        n, nb = inf["nnz"], inf["nblocks"]
        keys = np.empty(n, dtype=np.uint64)
        vals = np.empty(n, dtype=np.float32)
        bids = np.empty(nb, dtype=np.uint64)
        bst = np.empty(nb + 1, dtype=np.int64)
        _check(lib().blco_export(self._h, keys.ctypes.data, vals.ctypes.data, bids.ctypes.data,
                                 bst.ctypes.data))
        return keys, vals, bids, bst

    def free(self):
        if self._h is not None and self._h.value:
            lib().blco_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build(coords, values, dims, key_bits=64, max_block_nnz=1 << 27, placement="device",
          hot_min_count=0):
    """Build a BLCO tensor from 0-based COO coordinates (list of N integer arrays) and values.

    hot_min_count: non-zeros a row needs to count as frequent (0: the library's
    default; negative: no frequent rows)."""
    N = len(dims)
    cs = [np.ascontiguousarray(c, dtype=np.uint32) for c in coords]
    if len(cs) != N:
        raise ValueError("one coordinate array per mode")
    v = np.ascontiguousarray(values, dtype=np.float32)
    d = np.ascontiguousarray(dims, dtype=np.uint64)
    arr = (ctypes.c_void_p * N)(*[c.ctypes.data for c in cs])
    opts = _Opts(key_bits, max_block_nnz, PLACEMENTS[placement], int(hot_min_count))
    h = ctypes.c_void_p()
    _check(lib().blco_build(N, d.ctypes.data, len(v), arr, v.ctypes.data, ctypes.byref(opts),
                            ctypes.byref(h)))
    return BLCOTensor(h.value, dims)


def build_device(coords, values, dims, key_bits=64, max_block_nnz=1 << 27, placement="device",
                 hot_min_count=0, stream=None):
    """blco_build on the GPU.  coords: N index arrays (numpy, or int32 device tensors holding
    the uint32 bits); values: float32 (numpy or device tensor).  Same result as build()."""
    N = len(dims)
    if len(coords) != N:
        raise ValueError("one coordinate array per mode")
    dev = torch.device("cuda", torch.cuda.current_device())
    keep = []
    for c in coords:
        if isinstance(c, torch.Tensor):
            if not c.is_cuda or c.dtype != torch.int32 or not c.is_contiguous():
                raise ValueError("device coordinates must be contiguous int32 tensors")
            keep.append(c)
        else:
            a = np.ascontiguousarray(c, dtype=np.uint32).view(np.int32)
            keep.append(torch.from_numpy(a).to(dev))
    if isinstance(values, torch.Tensor):
        if not values.is_cuda or values.dtype != torch.float32 or not values.is_contiguous():
            raise ValueError("device values must be a contiguous float32 tensor")
        v = values
    else:
        v = torch.from_numpy(np.ascontiguousarray(values, dtype=np.float32)).to(dev)
    nnz = v.numel()
    for c in keep:
        if c.numel() != nnz:
            raise ValueError("coordinate arrays and values differ in length")
    d = np.ascontiguousarray(dims, dtype=np.uint64)
    arr = (ctypes.c_void_p * N)(*[c.data_ptr() for c in keep])
    opts = _Opts(key_bits, max_block_nnz, PLACEMENTS[placement], int(hot_min_count))
    h = ctypes.c_void_p()
    _check(lib().blco_build_device(N, d.ctypes.data, nnz, arr, v.data_ptr(), ctypes.byref(opts),
                                   _stream(stream), ctypes.byref(h)))
    return BLCOTensor(h.value, dims)


def _factor_args(t, factors, mode_skip):
    dt = None
    R = None
    ptrs = []
    keep = []
    for m, f in enumerate(factors):
        if f is None or (mode_skip is not None and m == mode_skip and f is None):
            ptrs.append(None)
            continue
        if not f.is_cuda or not f.is_contiguous() or f.dim() != 2:
            raise ValueError(f"factor {m} must be a contiguous 2-D device tensor")
        if f.shape[0] != t.dims[m]:
            raise ValueError(f"factor {m} has {f.shape[0]} rows, mode length is {t.dims[m]}")
        fd = {torch.float32: F32, torch.bfloat16: BF16}.get(f.dtype)
        if fd is None:
            raise ValueError("factors must be float32 or bfloat16")
        if dt is None:
            dt, R = fd, int(f.shape[1])
        elif fd != dt or int(f.shape[1]) != R:
            raise ValueError("all factors must share dtype and rank")
        ptrs.append(f.data_ptr())
        keep.append(f)
    if R is None:
        raise ValueError("no factor given")
    return (ctypes.c_void_p * len(factors))(*ptrs), dt, R, keep


def _out(t, mode, R, out, device):
    if out is None:
        out = torch.empty((t.dims[mode], R), dtype=torch.float32, device=device)
    elif (out.dtype != torch.float32 or not out.is_contiguous() or
          tuple(out.shape) != (t.dims[mode], R)):
        raise ValueError("out must be a contiguous float32 tensor of shape (I_mode, R)")
    return out


def _device_of(factors):
    for f in factors:
        if f is not None:
            return f.device
    return torch.device("cuda")


def mttkrp(t, mode, factors, out=None, stream=None):
    """Mode-``mode`` MTTKRP of an in-memory BLCO tensor; returns out (I_mode x R, float32)."""
    arr, dt, R, _keep = _factor_args(t, factors, mode)
    out = _out(t, mode, R, out, _device_of(factors))
    _check(lib().blco_mttkrp(t.handle, mode, arr, dt, R, out.data_ptr(), _stream(stream)))
    return out


def mttkrp_acc(t, mode, factors, out, stream=None):
    """out += mode-``mode`` MTTKRP (out is not cleared first)."""
    arr, dt, R, _keep = _factor_args(t, factors, mode)
    out = _out(t, mode, R, out, _device_of(factors))
    _check(lib().blco_mttkrp_acc(t.handle, mode, arr, dt, R, out.data_ptr(), _stream(stream)))
    return out


def mttkrp_v(t, mode, values, factors, out=None, scale=None, alpha=1.0, stream=None):
    """MTTKRP with the values replaced (device float32, BLCO order), scaled by alpha*scale."""
    arr, dt, R, _keep = _factor_args(t, factors, mode)
    out = _out(t, mode, R, out, _device_of(factors))
    if values.dtype != torch.float32 or not values.is_contiguous():
        raise ValueError("values must be contiguous float32")
    sp = None
    if scale is not None:
        if scale.dtype != torch.float64 or scale.numel() != 1:
            raise ValueError("scale must be a one-element float64 device tensor")
        sp = scale.data_ptr()
    _check(lib().blco_mttkrp_v(t.handle, mode, values.data_ptr(), arr, dt, R, sp, float(alpha),
                               out.data_ptr(), _stream(stream)))
    return out


def mttkrp_stream(t, mode, factors, out=None, device_budget=8_000_000_000, stream=None):
    """MTTKRP of a tensor in pinned host memory, streamed under a device-memory budget."""
    arr, dt, R, _keep = _factor_args(t, factors, mode)
    out = _out(t, mode, R, out, _device_of(factors))
    _check(lib().blco_mttkrp_stream(t.handle, mode, arr, dt, R, out.data_ptr(),
                                    int(device_budget), _stream(stream)))
    return out


def mttkrp_stream_all(t, factors, outs=None, device_budget=8_000_000_000, modes=None,
                      stream=None):
    """MTTKRP of several modes (default: all) in one streamed pass over a pinned tensor."""
    arr, dt, R, _keep = _factor_args(t, factors, None)
    dev = _device_of(factors)
    modes = list(range(len(t.dims))) if modes is None else list(modes)
    if outs is None:
        outs = [None] * len(t.dims)
    outs = list(outs)
    for m in modes:
        outs[m] = _out(t, m, R, outs[m], dev)
    ptrs = (ctypes.c_void_p * len(t.dims))(*[outs[m].data_ptr() if m in modes else None
                                               for m in range(len(t.dims))])
    _check(lib().blco_mttkrp_stream_all(t.handle, arr, dt, R, ptrs, int(device_budget),
                                        _stream(stream)))
    return [outs[m] if m in modes else None for m in range(len(t.dims))]


def sampled_loss(t, factors, residual=None, loss=None, stream=None):
    """(loss, residual): 1/2 sum_k (x_k - xhat_k)^2 as a float64 device scalar, and e (BLCO order)."""
    arr, dt, R, _keep = _factor_args(t, factors, None)
    dev = _device_of(factors)
    n = t.nnz
    if residual is None:
        residual = torch.empty(n, dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=dev)
    _check(lib().blco_sampled_loss(t.handle, arr, dt, R, residual.data_ptr(), loss.data_ptr(),
                                   _stream(stream)))
    return loss, residual


def cp_grad(t, factors, grads=None, residual=None, loss=None, scale=None, alpha=1.0,
            device_budget=8_000_000_000, stream=None):
    """(loss, grads, residual): the sparse CP fit loss 1/2 sum_k e_k^2 (float64 device scalar)
    and alpha * scale * dloss/dA^(m) = -alpha * scale * MTTKRP_m(E) for every mode, in one call.

    A device tensor also returns the residual e (BLCO order); a tensor in pinned host
    memory is streamed under `device_budget` (residual None)."""
    arr, dt, R, _keep = _factor_args(t, factors, None)
    dev = _device_of(factors)
    N = len(t.dims)
    if grads is None:
        grads = [None] * N
    grads = [_out(t, m, R, grads[m], dev) for m in range(N)]
    pinned = t.info()["placement"] == PLACEMENTS["pinned"]
    if not pinned and residual is None:
        residual = torch.empty(max(t.nnz, 1), dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=dev)
    sp = None
    if scale is not None:
        if scale.dtype != torch.float64 or scale.numel() != 1:
            raise ValueError("scale must be a one-element float64 device tensor")
        sp = scale.data_ptr()
    ptrs = (ctypes.c_void_p * N)(*[g.data_ptr() for g in grads])
    _check(lib().blco_cp_grad(t.handle, arr, dt, R, sp, float(alpha),
                              None if pinned else residual.data_ptr(), loss.data_ptr(), ptrs,
                              int(device_budget), _stream(stream)))
    return loss, grads, (None if pinned else residual)


def cp_grad_noalloc(t, factors, grads, residual, loss, scale=None, alpha=1.0, stream=None):
    """cp_grad for a device tensor through the entry point that allocates nothing on the
    device: every output (grads, residual of t.nnz floats, a float64 loss) is the caller's."""
    arr, dt, R, _keep = _factor_args(t, factors, None)
    N = len(t.dims)
    if len(grads) != N:
        raise ValueError(f"{N} gradients expected")
    sp = None
    if scale is not None:
        if scale.dtype != torch.float64 or scale.numel() != 1:
            raise ValueError("scale must be a one-element float64 device tensor")
        sp = scale.data_ptr()
    ptrs = (ctypes.c_void_p * N)(*[g.data_ptr() for g in grads])
    _check(lib().blco_cp_grad_noalloc(t.handle, arr, dt, R, sp, float(alpha), residual.data_ptr(),
                                      loss.data_ptr(), ptrs, _stream(stream)))
    return loss, grads, residual


def scale_(x, scale, alpha=1.0, stream=None):
    """x *= alpha * scale (x float32 device tensor, scale a one-element float64 device tensor)."""
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be contiguous float32")
    if scale.dtype != torch.float64 or scale.numel() != 1:
        raise ValueError("scale must be a one-element float64 device tensor")
    _check(lib().blco_scale(x.data_ptr(), x.numel(), scale.data_ptr(), float(alpha),
                            _stream(stream)))
    return x


def cast_bf16(x, stream=None):
    """Round-to-nearest-even bfloat16 copy of a float32 device tensor (library kernel)."""
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be contiguous float32")
    y = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    _check(lib().blco_cast_bf16(x.data_ptr(), y.data_ptr(), x.numel(), _stream(stream)))
    return y


def atomic_probe(out, rows, stream=None):
    """Calibration kernel: out[rows[k], :] += 1 with one device-scope fp32 atomic per entry
    (16-lane groups, the MTTKRP kernels' flush pattern).  out: float32 (I x R) device
    tensor; rows: int32 device tensor of row ids (uint32 bits)."""
    if out.dtype != torch.float32 or not out.is_contiguous() or out.dim() != 2:
        raise ValueError("out must be a contiguous 2-D float32 tensor")
    if rows.dtype != torch.int32 or not rows.is_contiguous():
        raise ValueError("rows must be a contiguous int32 tensor")
    _check(lib().blco_atomic_probe(out.data_ptr(), out.shape[0], out.shape[1], rows.data_ptr(),
                                   rows.numel(), _stream(stream)))
    return out


def gather_probe(table, rows, sink, stream=None):
    """Calibration kernel: reads table[rows[k], :] by 16-lane groups, six rows per group in
    flight (the MTTKRP kernels' gather pattern), one partial sum per group into sink.
    table: float32 (I x R) device tensor; rows: int32 device tensor of row ids (uint32
    bits); sink: float32 device tensor of at least ceil(len(rows) / 6) entries."""
    if table.dtype != torch.float32 or not table.is_contiguous() or table.dim() != 2:
        raise ValueError("table must be a contiguous 2-D float32 tensor")
    if rows.dtype != torch.int32 or not rows.is_contiguous():
        raise ValueError("rows must be a contiguous int32 tensor")
    if sink.dtype != torch.float32 or sink.numel() < (rows.numel() + 5) // 6:
        raise ValueError("sink must be a float32 tensor of at least ceil(len(rows) / 6) entries")
    _check(lib().blco_gather_probe(table.data_ptr(), table.shape[0], table.shape[1],
                                   rows.data_ptr(), rows.numel(), sink.data_ptr(),
                                   _stream(stream)))
    return sink


def gram(A, stream=None):
    """A^T A as a float64 R x R device tensor (fp32 products, fp64 sums; library kernel)."""
    if A.dim() != 2 or not A.is_contiguous() or A.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("A must be a contiguous 2-D float32 or bfloat16 tensor")
    R = A.shape[1]
    G = torch.empty((R, R), dtype=torch.float64, device=A.device)
    dt = BF16 if A.dtype == torch.bfloat16 else F32
    _check(lib().blco_gram(A.data_ptr(), dt, A.shape[0], R, G.data_ptr(), _stream(stream)))
    return G


def cp_als(t, factors, max_iters=25, tol=1e-5, storage="fp32", stream=None):
    """CP-ALS (Algorithm 1) on the device; `factors` (fp32 I_m x R device tensors) are the
    initial values and are overwritten.  Returns (fits per iteration, report dict)."""
    for f in factors:
        if f.dtype != torch.float32 or not f.is_contiguous() or f.dim() != 2:
            raise ValueError("factors must be contiguous 2-D float32 tensors")
    R = factors[0].shape[1]
    arr = (ctypes.c_void_p * len(factors))(*[f.data_ptr() for f in factors])
    if storage not in ("fp32", "bf16"):
        raise ValueError("storage must be 'fp32' or 'bf16'")
    for m, f in enumerate(factors):
        if f.shape[0] != t.dims[m] or f.shape[1] != R:
            raise ValueError(f"factor {m} must be {t.dims[m]} x {R}")
    opts = _CPALSOpts(int(max_iters), float(tol), BF16 if storage == "bf16" else F32)
    fits = np.zeros(int(max_iters), dtype=np.float64)
    rep = _CPALSReport()
    _check(lib().blco_cp_als(t.handle, arr, R, ctypes.byref(opts), fits.ctypes.data,
                             ctypes.byref(rep), _stream(stream)))
    return fits[:rep.iters].tolist(), {"iters": rep.iters, "pinv_fallbacks": rep.pinv_fallbacks}


class CPLoss(torch.autograd.Function):
    """Sparse CP fit loss 1/2 sum_nnz (x - sum_r prod_m A^(m))^2 with a hand-written backward.

    forward(t, storage, *A): A are fp32 factor masters (I_m x R); storage "fp32"
    or "bf16" (round-to-nearest-even copies used by the kernels).  The loss is a
    float64 device scalar.  When any factor needs a gradient, the forward makes one
    blco_cp_grad call: the loss and dL/dA^(m) = -MTTKRP_m(E) for every mode (E the
    residual tensor), the residual formed inside one mode's MTTKRP walk; the backward
    then only scales them by the incoming gradient g.  Otherwise the forward runs the
    sampled-loss kernel alone.  A tensor in pinned host memory is streamed (budget:
    CPLoss.device_budget bytes).
    """

    device_budget = 8_000_000_000

    @staticmethod
    def forward(ctx, t, storage, *A):
        if storage == "bf16":
            F = [cast_bf16(a.contiguous()) for a in A]
        elif storage == "fp32":
            F = [a.contiguous() for a in A]
        else:
            raise ValueError("storage must be 'fp32' or 'bf16'")
        pinned = t.info()["placement"] == PLACEMENTS["pinned"]
        if any(ctx.needs_input_grad[2:]) or pinned:
            loss, grads, _ = cp_grad(t, F, device_budget=CPLoss.device_budget)
            ctx.grads = grads
        else:
            loss, _ = sampled_loss(t, F)
            ctx.grads = None
        return loss

    @staticmethod
    def backward(ctx, g):
        g = g.detach().reshape(1)
        if g.dtype != torch.float64:
            raise ValueError("loss gradient must be float64")
        g = g.contiguous()
        grads = ctx.grads
        ctx.grads = None
        for x in grads:
            scale_(x, g)
        return (None, None, *grads)
