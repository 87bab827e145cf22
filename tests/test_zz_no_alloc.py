"""blco_cp_grad_noalloc, the allocation-free CP loss and gradient, against blco_cp_grad
(run on an MI355X).

Two calls in a row through the C ABI, the second on a smaller tensor (fewer
non-zeros, fewer modes, lower rank), each checked against blco_cp_grad on the same
tensor and factors, and against the fp64 oracle: the residual and the loss bit for
bit (both entry points run the same kernels, and the fused walk's model sum and the
fixed-order fp64 reduction do not depend on atomic order), the gradients within
twice conftest.grad_allowed of each other and within it of the oracle.  Every output
buffer exists before the first call and is filled with NaN, so the call must
overwrite all of it, and the device's free memory must not shrink across the two
calls (the workspace's one-time address lookup happens before them).
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from conftest import grad_allowed  # noqa: E402
import paper_2201_12523_amd as blco  # noqa: E402

DEV = torch.device("cuda:0")


def make(dims, nnz, R, seed):
    rng = np.random.default_rng(seed)
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    for c, d in zip(coords, dims):   # a few frequent rows, so the stash path runs
        c[: nnz // 4] = rng.integers(0, min(d, 5), size=nnz // 4)
    vals = rng.standard_normal(nnz).astype(np.float32)
    N = len(dims)
    A = [(rng.standard_normal((d, R)) * R ** (-1.0 / (2 * N))).astype(np.float32) for d in dims]
    return coords, vals, A


def noalloc(t, F, grads, resid, loss):
    N = len(F)
    fac = (ctypes.c_void_p * N)(*[f.data_ptr() for f in F])
    outs = (ctypes.c_void_p * N)(*[g.data_ptr() for g in grads])
    return blco.lib().blco_cp_grad_noalloc(t.handle, fac, 0, int(F[0].shape[1]), None,
                                           ctypes.c_double(1.0), resid.data_ptr(),
                                           loss.data_ptr(), outs, blco._stream(None))


def test_noalloc_matches_cp_grad_on_two_calls():
    cases = [((700, 400, 300, 40), 60_000, 32, 1), ((300, 200, 120), 15_000, 16, 2)]
    runs = []
    for dims, nnz, R, seed in cases:
        coords, vals, A = make(dims, nnz, R, seed)
        t = blco.build(coords, vals, dims, hot_min_count=1)
        F = [torch.from_numpy(a).to(DEV) for a in A]
        grads = [torch.full((d, R), float("nan"), device=DEV) for d in dims]
        resid = torch.full((nnz,), float("nan"), device=DEV)
        loss = torch.full((), float("nan"), dtype=torch.float64, device=DEV)
        ref = blco.cp_grad(t, F)   # the allocating entry point, for comparison
        runs.append((dims, coords, vals, A, R, t, F, grads, resid, loss, ref))
    # the workspace's address is looked up on a device's first call: take it outside
    # the measured span, on a small tensor of its own
    c0, v0, A0 = make((30, 20, 10), 500, 4, 9)
    t0 = blco.build(c0, v0, (30, 20, 10))
    F0 = [torch.from_numpy(a).to(DEV) for a in A0]
    g0 = [torch.empty((d, 4), device=DEV) for d in (30, 20, 10)]
    r0 = torch.empty(500, device=DEV)
    l0 = torch.empty((), dtype=torch.float64, device=DEV)
    assert noalloc(t0, F0, g0, r0, l0) == 0, blco.lib().blco_last_error()
    torch.cuda.synchronize()
    # two calls in a row, the second on the smaller tensor; nothing else touches the
    # device between the two readings of its free memory
    free0 = torch.cuda.mem_get_info()[0]
    for *_, t, F, grads, resid, loss, _ref in runs:
        assert noalloc(t, F, grads, resid, loss) == 0, blco.lib().blco_last_error()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0, "device memory was allocated"
    for dims, coords, vals, A, R, t, F, grads, resid, loss, (loss_r, grads_r, resid_r) in runs:
        N = len(dims)
        assert torch.equal(resid, resid_r), "residual differs from blco_cp_grad's"
        assert float(loss) == float(loss_r), (float(loss), float(loss_r))
        f, e, G, S = oracle.cp_grad(coords, vals, [a.astype(np.float64) for a in A], dims=dims)
        assert abs(float(loss) - f) <= 1e-6 * f
        Aabs = [np.abs(a).astype(np.float64) for a in A]
        xabs = oracle.cp_model(coords, Aabs)
        for n in range(N):
            W, _ = oracle.mttkrp(coords, xabs, Aabs, n, dims=dims)
            lim = grad_allowed(S[n], W, N, R)
            got = grads[n].cpu().numpy().astype(np.float64)
            other = grads_r[n].cpu().numpy().astype(np.float64)
            assert np.all(np.isfinite(got)), f"mode {n}: entries left unwritten"
            assert np.all(got[S[n] == 0] == 0.0)
            assert np.all(np.abs(got - G[n]) <= lim), f"mode {n} against the oracle"
            assert np.all(np.abs(got - other) <= 2 * lim), f"mode {n} against blco_cp_grad"
        t.free()
    t0.free()


def test_noalloc_refuses_pinned_tensors():
    coords, vals, A = make((50, 40, 30), 1000, 8, 3)
    t = blco.build(coords, vals, (50, 40, 30), placement="pinned")
    F = [torch.from_numpy(a).to(DEV) for a in A]
    grads = [torch.zeros((d, 8), device=DEV) for d in (50, 40, 30)]
    resid = torch.zeros(1000, device=DEV)
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    assert noalloc(t, F, grads, resid, loss) == -1
    assert b"device" in blco.lib().blco_last_error()
    t.free()
