"""The fused CP gradient (blco_cp_grad) against the fp64 oracle (run on an MI355X).

The loss is 1/2 sum_k e_k^2 with e_k = x_k - xhat_k (Section 2.2 model) and the
gradient with respect to A^(n) is -MTTKRP_n(E): the oracle composes its CP loss and
its MTTKRP (oracle.cp_grad), both pinned on the CPU.  Acceptance: loss within 1e-6
relative; each gradient entry within 1e-5 of the sum of |terms| plus the fp32
residual's rounding through the model's magnitude (conftest.grad_allowed); the residual within
1e-5 of |x_k| + sum_r prod_m |a| (its fp32 rounding).  Cases cover the fused walk
(register-based modes, R <= 64), the fallback through the sampled-loss kernel (every
mode hierarchical, or R > 64), frequent-row stashes, blocked keys, out-of-memory
streaming with many chunks, the chain-rule scale, and the argument errors.
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
TOL = 1e-5


def check(got, M, S, W, N, R, label):
    """Gradient entries within grad_allowed: TOL of the sum of |terms| plus the fp32
    residual's rounding through the model's magnitude W."""
    got = np.asarray(got, dtype=np.float64)
    zero = S == 0
    assert np.all(got[zero] == 0.0), f"{label}: non-zero where no term lands"
    lim = grad_allowed(S, W, N, R, TOL)
    worst = float((np.abs(got - M)[~zero] / lim[~zero]).max()) if (~zero).any() else 0.0
    assert worst <= 1.0, f"{label}: max error / allowed {worst:.3e}"


def make(dims, nnz, seed, hot=False):
    rng = np.random.default_rng(seed)
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    if hot:
        for c, d in zip(coords, dims):
            c[: nnz // 3] = rng.integers(0, min(d, 6), size=nnz // 3)
    vals = rng.standard_normal(nnz).astype(np.float32)
    return coords, vals, rng


def run(coords, vals, dims, R, rng, storage="fp32", placement="device", resolution="auto",
        budget=8_000_000_000, key_bits=64, hot_min_count=0, scale=None, alpha=1.0):
    N = len(dims)
    t = blco.build(coords, vals, dims, placement=placement, key_bits=key_bits,
                   hot_min_count=hot_min_count)
    t.set_resolution(resolution)
    A = [(rng.standard_normal((d, R)) * R ** (-1.0 / (2 * N))).astype(np.float32) for d in dims]
    F32 = [torch.from_numpy(a).to(DEV) for a in A]
    F = F32 if storage == "fp32" else [blco.cast_bf16(f) for f in F32]
    Aref = A if storage == "fp32" else [oracle.bf16_round(a) for a in A]
    sc = None if scale is None else torch.tensor([scale], dtype=torch.float64, device=DEV)
    if callable(budget):
        budget = budget(t)
    loss, grads, resid = blco.cp_grad(t, F, scale=sc, alpha=alpha, device_budget=budget)
    torch.cuda.synchronize()
    f, e, G, S = oracle.cp_grad(coords, vals, [a.astype(np.float64) for a in Aref], dims=dims)
    lab = f"dims={dims} R={R} {storage} {placement} {resolution}"
    assert abs(float(loss) - f) <= 1e-6 * f, (lab, float(loss), f)
    k = alpha * (1.0 if scale is None else scale)
    Aabs = [np.abs(a).astype(np.float64) for a in Aref]
    xabs = oracle.cp_model(coords, Aabs)
    for n in range(N):
        W, _ = oracle.mttkrp(coords, xabs, Aabs, n, dims=dims)
        check(grads[n].cpu().numpy(), k * G[n], abs(k) * S[n], abs(k) * W, N, R,
              f"{lab} grad mode {n}")
    if resid is not None:
        order = oracle.encode.encode(coords, vals, dims, key_bits=key_bits)["order"]
        xabs = oracle.cp_model([c[order] for c in coords],
                               [np.abs(a).astype(np.float64) for a in Aref]) + np.abs(vals[order])
        got = resid.cpu().numpy()[: len(vals)].astype(np.float64)
        assert np.max(np.abs(got - e[order]) / xabs) <= TOL, lab
    return t, loss, grads


@pytest.mark.parametrize("R", [1, 16, 32, 64])
@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_fused_walk(R, storage):
    # mode 0 (300 rows) is register-based under the heuristic: it carries the fused walk;
    # the short modes take the hierarchical kernel with the residual
    dims = (300, 200, 100)
    coords, vals, rng = make(dims, 20_000, 10 + R)
    run(coords, vals, dims, R, rng, storage)


@pytest.mark.parametrize("N", [1, 2, 4, 5])
def test_fused_walk_mode_counts(N):
    dims = (400, 37, 300, 11, 260)[:N]
    coords, vals, rng = make(dims, 6000, 20 + N)
    run(coords, vals, dims, 32, rng, resolution="register")


def test_fallback_every_mode_hierarchical():
    dims = (100, 50, 30, 20)
    coords, vals, rng = make(dims, 8000, 31)
    run(coords, vals, dims, 32, rng)


def test_fallback_rank_over_64():
    dims = (300, 200, 100)
    coords, vals, rng = make(dims, 5000, 32)
    run(coords, vals, dims, 100, rng, resolution="register")


def test_frequent_rows_and_blocks():
    dims = (600, 500, 400)
    coords, vals, rng = make(dims, 30_000, 33, hot=True)
    run(coords, vals, dims, 32, rng, resolution="register", hot_min_count=1)
    run(coords, vals, dims, 32, rng, resolution="register", key_bits=14)


def test_scale_and_alpha():
    dims = (300, 200, 100)
    coords, vals, rng = make(dims, 5000, 34)
    run(coords, vals, dims, 16, rng, scale=0.25, alpha=-3.0)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_streamed_many_chunks(storage):
    dims = (700, 300, 260, 9)
    nnz = 40_000
    coords, vals, rng = make(dims, nnz, 35, hot=True)
    R = 32

    sf = 4 if storage == "fp32" else 2   # bytes per stored factor element

    def budget(t):
        # every factor (sf bytes per element) and fp32 gradient, the tables, and two
        # buffers of ~3000 non-zeros (key, value, residual)
        return sum(d * R * (sf + 4) for d in dims) + t.info()["device_bytes"] + 2 * 3000 * 16

    t, loss, grads = run(coords, vals, dims, R, rng, storage, placement="pinned",
                         budget=budget, hot_min_count=1)
    inf = t.info()
    assert inf["stream_chunks"] >= 10 and inf["stream_peak_bytes"] <= budget(t)


def test_cploss_backward_scales_by_the_incoming_gradient():
    dims = (300, 40, 30)
    coords, vals, rng = make(dims, 4000, 36)
    t = blco.build(coords, vals, dims)
    A = [(rng.standard_normal((d, 8)) * 0.5).astype(np.float32) for d in dims]
    P = [torch.from_numpy(a).to(DEV).requires_grad_(True) for a in A]
    loss = blco.CPLoss.apply(t, "fp32", *P)
    (2.5 * loss).backward()
    f, e, G, S = oracle.cp_grad(coords, vals, [a.astype(np.float64) for a in A])
    Aabs = [np.abs(a).astype(np.float64) for a in A]
    xabs = oracle.cp_model(coords, Aabs)
    for n in range(3):
        W, _ = oracle.mttkrp(coords, xabs, Aabs, n, dims=dims)
        check(P[n].grad.cpu().numpy(), 2.5 * G[n], 2.5 * S[n], 2.5 * W, 3, 8,
              f"2.5 * loss, mode {n}")
    # no gradient wanted: the loss alone
    with torch.no_grad():
        l2 = blco.CPLoss.apply(t, "fp32", *[p.detach() for p in P])
    assert abs(float(l2) - f) <= 1e-6 * f


def test_empty_and_errors():
    t = blco.build([np.zeros(0, np.uint32)] * 3, np.zeros(0, np.float32), (4, 5, 6))
    F = [torch.ones((d, 3), device=DEV) for d in (4, 5, 6)]
    grads = [torch.full((d, 3), 9.0, device=DEV) for d in (4, 5, 6)]
    loss, grads, _ = blco.cp_grad(t, F, grads=grads)
    torch.cuda.synchronize()
    assert float(loss) == 0.0 and all(float(g.abs().sum()) == 0.0 for g in grads)
    rng = np.random.default_rng(1)
    dims = (300, 20, 10)
    coords = [rng.integers(0, d, 500).astype(np.uint32) for d in dims]
    t = blco.build(coords, rng.random(500).astype(np.float32), dims)
    F = [torch.ones((d, 4), device=DEV) for d in dims]
    G = [torch.empty((d, 4), device=DEV) for d in dims]
    L = blco.lib()
    fa = (ctypes.c_void_p * 3)(*[f.data_ptr() for f in F])
    ga = (ctypes.c_void_p * 3)(*[g.data_ptr() for g in G])
    lo = torch.empty((), dtype=torch.float64, device=DEV)
    r = torch.empty(500, device=DEV)
    ok = L.blco_cp_grad(t.handle, fa, 0, 4, None, 1.0, r.data_ptr(), lo.data_ptr(), ga, 0, None)
    assert ok == 0
    assert L.blco_cp_grad(t.handle, fa, 0, 4, None, 1.0, None, lo.data_ptr(), ga, 0, None) == -1
    assert b"residual" in L.blco_last_error()
    ga2 = (ctypes.c_void_p * 3)(G[0].data_ptr(), G[0].data_ptr(), G[2].data_ptr())
    assert L.blco_cp_grad(t.handle, fa, 0, 4, None, 1.0, r.data_ptr(), lo.data_ptr(), ga2, 0,
                          None) == -1
    assert b"overlaps" in L.blco_last_error()
    fa2 = (ctypes.c_void_p * 3)(F[0].data_ptr(), None, F[2].data_ptr())
    assert L.blco_cp_grad(t.handle, fa2, 0, 4, None, 1.0, r.data_ptr(), lo.data_ptr(), ga, 0,
                          None) == -1
    tp = blco.build(coords, rng.random(500).astype(np.float32), dims, placement="pinned")
    assert L.blco_cp_grad(tp.handle, fa, 0, 4, None, 1.0, r.data_ptr(), lo.data_ptr(), ga,
                          1 << 30, None) == -1
    torch.cuda.synchronize()
