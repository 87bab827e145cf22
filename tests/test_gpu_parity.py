"""GPU parity of the HIP path against the fp64 oracle (run on an MI355X).

Acceptance for fp32 factors: every output entry satisfies
|M_gpu - M| <= 1e-5 * S, with S the sum of |terms| of that entry, and
M_gpu == 0 exactly where S == 0 (which also catches a missing zero-fill).
bf16 factors: the same bound against the oracle on the bf16-rounded factors,
and |M_gpu - M_fp32| <= ((N-1) * 2^-8 + 1e-5) * S against the fp32 factors.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2201_12523_amd as blco  # noqa: E402
import synth  # noqa: E402
from conftest import read_golden  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev_factors(factors, dtype=torch.float32):
    out = []
    for f in factors:
        t = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(DEV)
        out.append(blco.cast_bf16(t) if dtype == torch.bfloat16 else t)
    return out


_bf16_round = oracle.bf16_round


def check_entries(got, M, S, tol=TOL, label=""):
    got = np.asarray(got, dtype=np.float64)
    zero = S == 0
    assert np.all(got[zero] == 0.0), f"{label}: non-zero output where no term lands"
    err = np.abs(got - M)[~zero] / S[~zero]
    worst = float(err.max()) if err.size else 0.0
    assert worst <= tol, f"{label}: max normalised error {worst:.3e} > {tol:.1e}"
    return worst


def hierarchical_fits(t, n, R):
    """Whether mode n at rank R can take hierarchical conflict resolution."""
    t.set_resolution("hierarchical")
    try:
        t.resolution(n, R)
        return True
    except blco.BLCOError as e:
        assert e.status == "EUNSUPPORTED"
        return False


def run_case(coords, vals, dims, R, modes=None, key_bits=64, cap=1 << 27, seed=0,
             dtypes=("fp32",), label="", resolutions=("register", "hierarchical", "frequent")):
    """Every mode under each conflict-resolution mechanism (hierarchical only where
    the mode fits its LDS stash; "frequent": register-based with every mode's 256
    most frequent rows summed in the workgroup stash) against the oracle."""
    say(f"case {label} dims={dims} nnz={len(vals)} R={R} key_bits={key_bits} cap={cap}")
    t = blco.build(coords, vals, dims, key_bits=key_bits, max_block_nnz=cap, hot_min_count=-1)
    th = blco.build(coords, vals, dims, key_bits=key_bits, max_block_nnz=cap, hot_min_count=1)
    th.set_resolution("register")
    rng = np.random.default_rng(seed)
    A = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    modes = range(len(dims)) if modes is None else modes
    for dt in dtypes:
        if dt == "fp32":
            F = _dev_factors(A)
            Aref = A
        else:
            F = _dev_factors(A, torch.bfloat16)
            Aref = [_bf16_round(a) for a in A]
        for n in modes:
            M, S = oracle.mttkrp(coords, vals, Aref, n)
            for res in resolutions:
                if res == "hierarchical" and not hierarchical_fits(t, n, R):
                    continue
                if res == "frequent":
                    out = blco.mttkrp(th, n, F)
                else:
                    t.set_resolution(res)
                    assert t.resolution(n, R) == res
                    out = blco.mttkrp(t, n, F)
                torch.cuda.synchronize()
                tag = f"{label} {dt} {res} mode {n}"
                check_entries(out.cpu().numpy(), M, S, label=tag)
                if dt == "bf16":
                    M32, S32 = oracle.mttkrp(coords, vals, A, n)
                    bound = (len(dims) - 1) * 2.0 ** -8 + 1e-5
                    check_entries(out.cpu().numpy(), M32, S32, tol=bound,
                                  label=f"{tag} bf16-vs-fp32")
    t.free()
    th.free()


def test_figure4a_worked_example(fig4a):
    coords, vals, dims = fig4a
    t = blco.build(coords, vals, dims, key_bits=5, max_block_nnz=6)
    for case in ("ones", "ramp"):
        col = np.ones(4, np.float32) if case == "ones" else np.arange(1, 5, dtype=np.float32)
        F = _dev_factors([col[:, None]] * 3)
        want = {int(r[1]) - 1: [float(x) for x in r[2:]] for r in read_golden("fig4a_mttkrp.txt")
                if r[0] == case}
        for n in range(3):
            out = blco.mttkrp(t, n, F)
            assert out[:, 0].cpu().tolist() == want[n], (case, n)


def test_small_workload_all_modes():
    w = synth.WORKLOADS["small"]
    coords, vals = synth.workload_tensor(w)
    A = synth.workload_factors(w, 16)
    t = blco.build(coords, vals, w.dims)
    F = _dev_factors(A)
    for n in range(3):
        out = blco.mttkrp(t, n, F)
        M, S = oracle.mttkrp(coords, vals, A, n)
        check_entries(out.cpu().numpy(), M, S, label=f"small mode {n}")


@pytest.mark.parametrize("R", [1, 3, 16, 18, 32, 33, 34, 62, 64, 100])
def test_ranks(R):
    rng = np.random.default_rng(R)
    dims = (97, 61, 45)
    nnz = 3001
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.random(nnz).astype(np.float32)
    # bf16 too: odd ranks gather packed bf16 runs with 2-byte loads, even ones with 4/8-byte
    # (at R = 34 and 62 the 8-byte runs start 4-byte aligned)
    run_case(coords, vals, dims, R, seed=R, label=f"rank{R}", dtypes=("fp32", "bf16"))


@pytest.mark.parametrize("R", [8, 48])
@pytest.mark.parametrize("N", [1, 2, 4, 5, 6, 7, 8])
def test_mode_counts(N, R):
    # R = 48 at N <= 5: the 4096-non-zero window (the largest LDS use at N = 5)
    rng = np.random.default_rng(N + 50 + R)
    dims = tuple([13, 1, 7, 30, 5, 9, 3, 17][:N])
    nnz = 777 if R == 8 else 5000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.standard_normal(nnz).astype(np.float32)
    run_case(coords, vals, dims, R, seed=N, label=f"N{N}R{R}")


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("nnz,R", [(1023, 32), (1025, 32), (2047, 32), (2048, 32), (2049, 32),
                                   (4095, 32), (6145, 32), (2049, 64), (4095, 64), (4096, 64),
                                   (4097, 64), (8193, 64)])
def test_window_boundaries(nnz, R, N):
    """Non-zero counts around the 1024-, 2048- and 4096-non-zero windows (modes without a
    stash take two non-zeros per thread at R <= 32, four at R = 64): a 7-row mode whose
    segments run across many lane groups, a 5000-row mode with short ones, and the
    stash path beside them."""
    rng = np.random.default_rng(nnz * 10 + N + R)
    dims = (7, 300, 5000, 3)[:N]
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.standard_normal(nnz).astype(np.float32)
    run_case(coords, vals, dims, R, seed=nnz, label=f"win{nnz}R{R}N{N}", dtypes=("fp32", "bf16"),
             resolutions=("register", "frequent"))


@pytest.mark.parametrize("dtype,R,exact", [("fp32", 64, False), ("bf16", 64, False),
                                           ("bf16", 34, False), ("fp32", 64, True)])
def test_register_path_factor_past_4gib(dtype, R, exact):
    """Register-based MTTKRP of the two short modes when the long mode's factor is just
    past 4 GiB, so the kernel gathers through 64-bit addresses instead of 32-bit buffer
    offsets, with and without the frequent-row stash (packed bf16 ranks at R = 34); and
    (exact) a factor of exactly 4 GiB at 64 fp32 ranks, which the kernel still reaches with
    32-bit offsets from the factor's base, its last row included."""
    fsz = 4 if dtype == "fp32" else 2
    rows0 = (1 << 32) // (R * fsz) if exact else max(1 << 24, (1 << 32) // (R * fsz) + 1)
    assert rows0 * R * fsz == 1 << 32 if exact else rows0 * R * fsz > 0xFFFFFFFF
    rng = np.random.default_rng(R + fsz)
    dims = (rows0, 100, 60)
    nnz = 300_000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][:1000] = rows0 - 1
    vals = rng.random(nnz).astype(np.float32)
    g = torch.Generator(device=DEV)
    g.manual_seed(R)
    F0 = torch.randn((rows0, R), device=DEV, generator=g)
    if dtype == "bf16":
        F0 = blco.cast_bf16(F0)
    torch.cuda.empty_cache()
    A1 = rng.standard_normal((dims[1], R)).astype(np.float32)
    A2 = rng.standard_normal((dims[2], R)).astype(np.float32)
    F = [F0] + _dev_factors([A1, A2], torch.bfloat16 if dtype == "bf16" else torch.float32)
    used, inv = np.unique(coords[0], return_inverse=True)
    A0 = F0[torch.from_numpy(used.astype(np.int64)).to(DEV)].float().cpu().numpy()
    Aref = [A0] + ([A1, A2] if dtype == "fp32" else [_bf16_round(A1), _bf16_round(A2)])
    small = [inv.astype(np.uint32), coords[1], coords[2]]
    for hot in (0, -1):   # 0: default frequent rows (stash); -1: none
        t = blco.build(coords, vals, dims, hot_min_count=hot)
        t.set_resolution("register")
        for n in (1, 2):
            out = blco.mttkrp(t, n, F)
            M, S = oracle.mttkrp(small, vals, Aref, n)
            say(f"{dtype} R={R} rows0={rows0} hot={hot} mode {n}: stash rows {t.stash_rows(n, R)}")
            check_entries(out.cpu().numpy(), M, S, label=f"{dtype} R={R} hot={hot} mode {n}")
            del out
        t.free()
    del F0, F
    torch.cuda.empty_cache()


@pytest.mark.parametrize("pattern", ["one_row", "distinct", "lane_mod_3", "tail_65", "tail_1"])
def test_conflict_patterns(pattern):
    rng = np.random.default_rng(7)
    dims = (4096, 64, 64)
    nnz = {"tail_65": 65, "tail_1": 1}.get(pattern, 4096 + 37)
    c1 = rng.integers(0, 64, size=nnz).astype(np.uint32)
    c2 = rng.integers(0, 64, size=nnz).astype(np.uint32)
    if pattern == "one_row":
        c0 = np.full(nnz, 17, np.uint32)
    elif pattern == "distinct":
        c0 = rng.permutation(4096)[: min(nnz, 4096)].astype(np.uint32)
        c0 = np.concatenate([c0, np.arange(nnz - len(c0), dtype=np.uint32)])
    elif pattern == "lane_mod_3":
        c0 = (np.arange(nnz) % 3).astype(np.uint32)
    else:
        c0 = rng.integers(0, 4096, size=nnz).astype(np.uint32)
    vals = rng.standard_normal(nnz).astype(np.float32)
    run_case([c0, c1, c2], vals, dims, 32, seed=3, label=pattern)


@pytest.mark.parametrize("key_bits,cap", [(12, 64), (9, 5), (20, 100000), (14, 1)])
def test_blocks_inside_a_wave(key_bits, cap):
    rng = np.random.default_rng(key_bits)
    dims = (1000, 300, 77, 6)
    nnz = 5000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][:2000] = rng.integers(0, 3, size=2000)
    vals = rng.random(nnz).astype(np.float32)
    run_case(coords, vals, dims, 16, key_bits=key_bits, cap=cap, seed=key_bits,
             label=f"blocks{key_bits}/{cap}")


def test_wide_target_index():
    # a mode longer than 2^26 - 1 takes the 64-bit sort path
    rng = np.random.default_rng(11)
    dims = ((1 << 26) + 3, 5, 4)
    nnz = 4000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][:1000] = (1 << 26) + 2
    coords[0][1000:1500] = 0
    vals = rng.random(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims)
    A = [rng.standard_normal((d, 2)).astype(np.float32) if d < 100 else None for d in dims]
    F = [None] + _dev_factors(A[1:])
    out = blco.mttkrp(t, 0, F)
    rows = np.unique(coords[0])
    Afull = [np.zeros((1, 2), np.float32), A[1], A[2]]
    M, S = oracle.mttkrp_rows(coords, vals, Afull, 0, rows, dims)
    got = out[torch.from_numpy(rows.astype(np.int64)).to(DEV)].cpu().numpy()
    check_entries(got, M, S, label="wide")
    assert float(out.abs().sum()) == pytest.approx(float(np.abs(got).sum()), rel=1e-6)


def test_bf16_factors():
    w = synth.WORKLOADS["small"]
    coords, vals = synth.workload_tensor(w)
    run_case(coords, vals, w.dims, 32, seed=5, dtypes=("bf16",), label="bf16")


@pytest.mark.parametrize("res", ["register", "hierarchical"])
def test_mttkrp_v_scaled(res):
    rng = np.random.default_rng(21)
    dims = (50, 40, 30)
    nnz = 2000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.random(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims)
    t.set_resolution(res)
    _, v_blco, _, _ = t.export()
    A = [rng.standard_normal((d, 16)).astype(np.float32) for d in dims]
    F = _dev_factors(A)
    newv = rng.standard_normal(nnz).astype(np.float32)
    # the override is given in BLCO order; the oracle gets it in COO order
    ref_t = oracle.encode.encode(coords, vals, dims)
    v_dev = torch.from_numpy(newv).to(DEV)
    coo_v = np.empty(nnz, np.float32)
    coo_v[ref_t["order"]] = newv
    scale = torch.tensor([0.75], dtype=torch.float64, device=DEV)
    out = blco.mttkrp_v(t, 1, v_dev, F, scale=scale, alpha=-2.0)
    M, S = oracle.mttkrp(coords, coo_v, A, 1)
    check_entries(out.cpu().numpy(), -1.5 * M, 1.5 * S, label="mttkrp_v")


@pytest.mark.parametrize("dtype,R", [("fp32", 32), ("bf16", 32), ("bf16", 33), ("bf16", 64)])
def test_sampled_loss_and_residual(dtype, R):
    rng = np.random.default_rng(31)
    dims = (60, 50, 40, 7)
    nnz = 5000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.standard_normal(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims)
    A = [(rng.standard_normal((d, R)) * 0.6).astype(np.float32) for d in dims]
    F = _dev_factors(A, torch.bfloat16 if dtype == "bf16" else torch.float32)
    if dtype == "bf16":
        A = [_bf16_round(a) for a in A]   # the oracle on the factors the kernel reads
    loss, resid = blco.sampled_loss(t, F)
    f, e = oracle.cp_loss(coords, vals, A)
    assert abs(float(loss) - f) <= 1e-6 * f
    order = oracle.encode.encode(coords, vals, dims)["order"]
    e_blco = e[order]
    xhat_abs = np.abs(np.prod([A[m][coords[m][order]].astype(np.float64) for m in range(4)],
                              axis=0)).sum(axis=1) + np.abs(vals[order])
    assert np.max(np.abs(resid.cpu().numpy() - e_blco) / xhat_abs) <= 1e-5
    # deterministic: the same call gives the same bits
    loss2, resid2 = blco.sampled_loss(t, F)
    assert float(loss2) == float(loss)
    assert torch.equal(resid, resid2)


@pytest.mark.parametrize("res", ["register", "hierarchical"])
@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_cp_gradient(storage, res):
    rng = np.random.default_rng(41)
    dims = (40, 30, 20, 10)
    nnz = 3000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.standard_normal(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims)
    t.set_resolution(res)
    A = [(rng.standard_normal((d, 32)) * 0.6).astype(np.float32) for d in dims]
    P = [torch.from_numpy(a).to(DEV).requires_grad_(True) for a in A]
    loss = blco.CPLoss.apply(t, storage, *P)
    loss.backward()
    Aref = A if storage == "fp32" else [_bf16_round(a) for a in A]
    f, e, G, S = oracle.cp_grad(coords, vals, Aref)
    assert abs(float(loss) - f) <= 1e-6 * f
    for n in range(4):
        check_entries(P[n].grad.cpu().numpy(), G[n], S[n], label=f"grad {storage} mode {n}")


def test_cp_gradient_finite_differences():
    """Central differences of the GPU loss (quadratic in each entry, so exact up to rounding)."""
    rng = np.random.default_rng(51)
    dims = (6, 5, 4)
    nnz = 60
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.standard_normal(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims)
    A = [(rng.standard_normal((d, 3))).astype(np.float32) for d in dims]
    P = [torch.from_numpy(a).to(DEV).requires_grad_(True) for a in A]
    loss = blco.CPLoss.apply(t, "fp32", *P)
    loss.backward()
    h = 0.0625  # a power of two: a +- h is exact in fp32 for these magnitudes
    for n in range(3):
        for i in range(dims[n]):
            for r in range(3):
                Q = [p.detach().clone() for p in P]
                Q[n][i, r] += h
                fp = float(blco.CPLoss.apply(t, "fp32", *Q))
                Q[n][i, r] -= 2 * h
                fm = float(blco.CPLoss.apply(t, "fp32", *Q))
                fd = (fp - fm) / (2 * h)
                g = float(P[n].grad[i, r])
                assert abs(fd - g) <= 2e-4 * max(1.0, float(loss)), (n, i, r, fd, g)


def test_cast_bf16_matches_torch():
    x = torch.randn(100_003, device=DEV) * 3
    x[:6] = torch.tensor([0.0, -0.0, float("inf"), float("-inf"), 1e-40, -3.4e38], device=DEV)
    y = blco.cast_bf16(x)
    assert torch.equal(y.view(torch.int16), x.to(torch.bfloat16).view(torch.int16))
    # ties round to even: 1 + 2^-8 sits halfway between two bf16 values
    z = torch.tensor([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8], device=DEV)
    assert blco.cast_bf16(z).float().cpu().tolist() == [1.0, 1.0 + 2 ** -6]


@pytest.mark.parametrize("res", ["register", "hierarchical"])
@pytest.mark.parametrize("budget_nnz", [64, 1000, 5000])
@pytest.mark.parametrize("R", [16, 64])
def test_stream_matches_in_memory(budget_nnz, res, R):
    rng = np.random.default_rng(budget_nnz + R)
    dims = (300, 200, 100)
    nnz = 20_000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.random(nnz).astype(np.float32)
    A = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    F = _dev_factors(A)
    tp = blco.build(coords, vals, dims, placement="pinned")
    tp.set_resolution(res)
    for n in range(3):
        fixed = dims[n] * R * 4 + sum(dims[m] * R * 4 for m in range(3) if m != n)
        fixed += tp.info()["device_bytes"]
        budget = fixed + 2 * budget_nnz * 12
        out = blco.mttkrp_stream(tp, n, F, device_budget=budget)
        torch.cuda.synchronize()
        inf = tp.info()
        assert inf["stream_peak_bytes"] <= budget
        assert inf["stream_chunks"] == -(-nnz // inf["stream_chunk_nnz"])
        M, S = oracle.mttkrp(coords, vals, A, n)
        check_entries(out.cpu().numpy(), M, S, label=f"stream mode {n}")
    with pytest.raises(blco.BLCOError) as e:
        blco.mttkrp_stream(tp, 0, F, device_budget=1000)
    assert e.value.status == "ENOMEM"


def test_calibration_probes():
    """The two measurement kernels the benchmark times: the atomic probe adds 1 to every
    entry of each listed row (ids past the table skipped), the gather probe leaves in each
    group's sink entry lane 0's sum over its six rows (ranks 0 and 16 at R = 32)."""
    R, I = 32, 1000
    rng = np.random.default_rng(5)
    ids = rng.integers(0, I + 50, size=4001).astype(np.int64)   # some ids past the table
    out = torch.zeros((I, R), dtype=torch.float32, device=DEV)
    rows = torch.from_numpy(ids.astype(np.int32)).to(DEV)
    blco.atomic_probe(out, rows)
    want = np.zeros((I, R))
    for i in ids[ids < I]:
        want[i] += 1.0
    assert np.array_equal(out.cpu().numpy(), want)
    table = (torch.arange(I, dtype=torch.float32, device=DEV)[:, None] * 100.0 +
             torch.arange(R, dtype=torch.float32, device=DEV)[None, :])
    sink = torch.full(((len(ids) + 5) // 6,), -1.0, dtype=torch.float32, device=DEV)
    blco.gather_probe(table, rows, sink)
    tab = table.cpu().numpy().astype(np.float64)
    exp = np.zeros(len(sink))
    for k, i in enumerate(ids):
        if i < I:
            exp[k // 6] += tab[i, 0] + tab[i, 16]
    assert np.allclose(sink.cpu().numpy(), exp, rtol=1e-6)
    with pytest.raises(ValueError):
        blco.gather_probe(table, rows, sink[:10])


def test_argument_errors():
    rng = np.random.default_rng(1)
    dims = (10, 10, 10)
    coords = [rng.integers(0, 10, size=100).astype(np.uint32) for _ in range(3)]
    vals = rng.random(100).astype(np.float32)
    t = blco.build(coords, vals, dims)
    F = _dev_factors([rng.standard_normal((10, 4)).astype(np.float32)] * 3)
    out = torch.empty((10, 4), device=DEV)
    import ctypes
    arr = (ctypes.c_void_p * 3)(*[f.data_ptr() for f in F])
    L = blco.lib()
    assert L.blco_mttkrp(t.handle, 3, arr, 0, 4, out.data_ptr(), None) == -1
    assert L.blco_mttkrp(t.handle, 0, arr, 0, 0, out.data_ptr(), None) == -1
    assert L.blco_mttkrp(t.handle, 0, arr, 7, 4, out.data_ptr(), None) == -1
    assert L.blco_mttkrp(t.handle, 0, arr, 0, 4, None, None) == -1
    assert L.blco_mttkrp(None, 0, arr, 0, 4, out.data_ptr(), None) == -1
    th = blco.build(coords, vals, dims, placement="host")
    assert L.blco_mttkrp(th.handle, 0, arr, 0, 4, out.data_ptr(), None) == -1
    assert b"device" in L.blco_last_error()


def test_empty_tensor_zero_fills():
    t = blco.build([np.zeros(0, np.uint32)] * 3, np.zeros(0, np.float32), (4, 5, 6))
    F = _dev_factors([np.ones((d, 3), np.float32) for d in (4, 5, 6)])
    out = torch.full((5, 3), 7.0, device=DEV)
    blco.mttkrp(t, 1, F, out=out)
    assert float(out.abs().sum()) == 0.0


def test_empty_tensor_loss_is_zero():
    """No non-zeros: loss 0 and no factor row read; NULL factors are still rejected."""
    t = blco.build([np.zeros(0, np.uint32)] * 3, np.zeros(0, np.float32), (4, 5, 6))
    F = _dev_factors([np.ones((d, 3), np.float32) for d in (4, 5, 6)])
    loss = torch.full((), 7.0, dtype=torch.float64, device=DEV)
    blco.sampled_loss(t, F, residual=torch.empty(1, device=DEV), loss=loss)
    torch.cuda.synchronize()
    assert float(loss) == 0.0
    import ctypes
    arr = (ctypes.c_void_p * 3)(F[0].data_ptr(), None, F[2].data_ptr())
    L = blco.lib()
    assert L.blco_sampled_loss(t.handle, arr, 0, 3, None, loss.data_ptr(), None) == -1
    assert b"factors[1]" in L.blco_last_error()


@pytest.mark.skipif(os.environ.get("BLCO_SKIP_FULL") == "1", reason="full-size case disabled")
def test_zipf3_full_size_sampled_rows():
    """The 2^22 x 2^21 x 2^20, 50M-non-zero Zipf(1.1) workload at full size, R = 32,
    all modes, fp32 and bf16: hot and random rows against the oracle row by row, plus
    the cross-mode invariant sum(M^(n) * A^(n)) that holds at any size."""
    w = synth.WORKLOADS["zipf3"]
    say("generating 50M-non-zero workload")
    coords, vals = synth.workload_tensor(w)
    say("building")
    t = blco.build(coords, vals, w.dims)
    A = synth.workload_factors(w, 32)
    rng = np.random.default_rng(99)
    for dt in ("fp32", "bf16"):
        F = _dev_factors(A, torch.float32 if dt == "fp32" else torch.bfloat16)
        Aref = A if dt == "fp32" else [_bf16_round(a) for a in A]
        inner, inner_abs = [], []
        for n in range(3):
            out = blco.mttkrp(t, n, F)
            torch.cuda.synchronize()
            rows = np.unique(np.concatenate([np.arange(8), rng.integers(0, w.dims[n], 56),
                                             [w.dims[n] - 1]]).astype(np.uint32))
            M, S = oracle.mttkrp_rows(coords, vals, Aref, n, rows, w.dims)
            got = out[torch.from_numpy(rows.astype(np.int64)).to(DEV)].cpu().numpy()
            worst = check_entries(got, M, S, label=f"zipf3 {dt} mode {n}")
            say(f"zipf3 {dt} mode {n}: max err {worst:.2e}")
            Fd = F[n].float() if dt == "bf16" else F[n]
            inner.append(float((out.double() * Fd.double()).sum()))
            inner_abs.append(float((out.double().abs() * Fd.double().abs()).sum()))
        assert max(inner) - min(inner) <= 1e-5 * max(inner_abs), (inner, inner_abs)


@pytest.mark.parametrize("placement", ["pinned", "device"])
def test_stream_all_modes_one_pass(placement):
    rng = np.random.default_rng(77)
    dims = (300, 200, 100, 7)
    nnz = 20_000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.random(nnz).astype(np.float32)
    R = 16
    A = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    F = _dev_factors(A)
    t = blco.build(coords, vals, dims, placement=placement)
    fixed = sum(d * R * 4 * 2 for d in dims) + t.info()["device_bytes"]
    budget = fixed + 2 * 1000 * 12
    outs = blco.mttkrp_stream_all(t, F, device_budget=budget)
    torch.cuda.synchronize()
    inf = t.info()
    if placement == "pinned":
        assert inf["stream_chunks"] == -(-nnz // inf["stream_chunk_nnz"]) and inf["stream_chunks"] > 10
        assert inf["stream_peak_bytes"] <= budget
    for n in range(4):
        M, S = oracle.mttkrp(coords, vals, A, n)
        check_entries(outs[n].cpu().numpy(), M, S, label=f"stream_all {placement} mode {n}")
    # a subset of modes, the others untouched
    keep = torch.full((dims[1], R), 5.0, device=DEV)
    outs2 = blco.mttkrp_stream_all(t, F, outs=[None, keep, None, None], modes=[1, 3],
                                   device_budget=budget)
    M, S = oracle.mttkrp(coords, vals, A, 1)
    check_entries(outs2[1].cpu().numpy(), M, S, label="stream_all subset")
    assert outs2[0] is None and outs2[2] is None


def test_stream_with_frequent_rows():
    # every chunk's workgroups sum the frequent rows in LDS and flush them at their end
    rng = np.random.default_rng(77)
    dims = (300, 200, 100)
    nnz = 30_000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][:9000] = rng.integers(0, 5, size=9000)
    vals = rng.random(nnz).astype(np.float32)
    R = 32
    A = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    F = _dev_factors(A)
    tp = blco.build(coords, vals, dims, placement="pinned", hot_min_count=1)
    tp.set_resolution("register")
    assert tp.info()["hot_rows"] == [256, 200, 100]
    for n in range(3):
        fixed = dims[n] * R * 4 + sum(dims[m] * R * 4 for m in range(3) if m != n)
        fixed += tp.info()["device_bytes"]
        out = blco.mttkrp_stream(tp, n, F, device_budget=fixed + 2 * 4000 * 12)
        torch.cuda.synchronize()
        assert tp.info()["stream_chunks"] >= 7
        M, S = oracle.mttkrp(coords, vals, A, n)
        check_entries(out.cpu().numpy(), M, S, label=f"stream frequent rows mode {n}")
