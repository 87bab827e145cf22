"""Hierarchical conflict resolution (Section 5.1) and its selection heuristic
(Section 5.3) on the GPU, against the fp64 oracle.

Acceptance as in test_gpu_parity: |gpu - oracle| <= 1e-5 * sum|terms| per
entry, exact zeros where no term lands.  Cases: the heuristic's choice at the
compute-unit threshold, rank slices (a stash too small for all ranks at once),
every non-zero on one output row, a factor past 4 GiB (64-bit gathers), and
agreement between the two mechanisms on a Zipf tensor with short modes.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2201_12523_amd as blco  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_entries(got, M, S, tol=TOL, label=""):
    got = np.asarray(got, dtype=np.float64)
    zero = S == 0
    assert np.all(got[zero] == 0.0), f"{label}: non-zero output where no term lands"
    err = np.abs(got - M)[~zero] / S[~zero]
    worst = float(err.max()) if err.size else 0.0
    say(f"{label}: max normalised error {worst:.2e}")
    assert worst <= tol, f"{label}: max normalised error {worst:.3e} > {tol:.1e}"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def test_heuristic_threshold_is_the_cu_count():
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    dims = (cus - 1, cus, 5000, 3)
    rng = np.random.default_rng(1)
    coords = [rng.integers(0, d, size=1000).astype(np.uint32) for d in dims]
    t = blco.build(coords, rng.random(1000).astype(np.float32), dims)
    got = [t.resolution(n, 32) for n in range(4)]
    assert got == ["hierarchical", "register", "register", "hierarchical"], (cus, got)
    t.set_resolution("hierarchical")
    t.resolution(0, 32)
    dims3 = (640, 5, 5)
    t3 = blco.build([np.arange(640, dtype=np.uint32) % d for d in dims3],
                    np.ones(640, np.float32), dims3)
    t3.set_resolution("hierarchical")
    with pytest.raises(blco.BLCOError):
        t3.resolution(0, 16)
    t.set_resolution("register")
    assert [t.resolution(n, 32) for n in range(4)] == ["register"] * 4
    t.set_resolution("hierarchical")
    assert t.resolution(1, 32) == "hierarchical"
    # 4 modes: the stash holds at most 895 - 64 * 5 = 575 rows of 16 ranks
    with pytest.raises(blco.BLCOError) as e:
        t.resolution(2, 32)
    assert e.value.status == "EUNSUPPORTED"
    F = [dev(rng.standard_normal((d, 32))) for d in dims]
    with pytest.raises(blco.BLCOError) as e:
        blco.mttkrp(t, 2, F)
    assert e.value.status == "EUNSUPPORTED"
    with pytest.raises(ValueError):
        t.set_resolution("sometimes")


@pytest.mark.parametrize("R", [16, 48, 64, 100, 129])
def test_rank_slices(R):
    # 639 rows (the 3-mode maximum) x R ranks does not fit one stash: the ranks
    # are split into slices
    rng = np.random.default_rng(R)
    dims = (639, 300, 64)
    nnz = 30_000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][:5000] = rng.integers(0, 4, size=5000)
    vals = rng.standard_normal(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims)
    t.set_resolution("hierarchical")
    A = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    F = [dev(a) for a in A]
    for n in range(3):
        out = blco.mttkrp(t, n, F)
        M, S = oracle.mttkrp(coords, vals, A, n)
        check_entries(out.cpu().numpy(), M, S, label=f"slices R={R} mode {n}")


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_every_nonzero_on_one_row(dtype):
    rng = np.random.default_rng(3)
    dims = (37, 2000, 1500)
    nnz = 400_000
    coords = [np.full(nnz, 11, np.uint32)] + [rng.integers(0, d, size=nnz).astype(np.uint32)
                                              for d in dims[1:]]
    vals = rng.random(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims)
    assert t.resolution(0, 32) == "hierarchical"
    A = [rng.standard_normal((d, 32)).astype(np.float32) for d in dims]
    F = [dev(a) for a in A]
    Aref = A
    if dtype == "bf16":
        F = [blco.cast_bf16(f) for f in F]
        Aref = [oracle.bf16_round(a) for a in A]
    out = blco.mttkrp(t, 0, F)
    M, S = oracle.mttkrp(coords, vals, Aref, 0)
    check_entries(out.cpu().numpy(), M, S, label=f"one row {dtype}")


@pytest.mark.parametrize("dtype,R", [("fp32", 64), ("bf16", 64), ("bf16", 34)])
def test_factor_past_4gib(dtype, R):
    # mode 0's factor is just past 4 GiB (2^24 rows at R = 64 in fp32; more rows in
    # bf16), so the hierarchical kernel gathers it with 64-bit addresses; in bf16 at
    # R = 34 the last lane's packed run ends past the row, and past the factor on its
    # last row, which is referenced
    fsz = 4 if dtype == "fp32" else 2
    rows0 = max(1 << 24, (1 << 32) // (R * fsz) + 1)
    assert rows0 * R * fsz > 0xFFFFFFFF
    rng = np.random.default_rng(9)
    dims = (rows0, 100, 60)
    nnz = 300_000
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][:1000] = rows0 - 1
    vals = rng.random(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims)
    g = torch.Generator(device=DEV)
    g.manual_seed(9)
    F0 = torch.randn((dims[0], R), device=DEV, generator=g)
    A1 = rng.standard_normal((dims[1], R)).astype(np.float32)
    A2 = rng.standard_normal((dims[2], R)).astype(np.float32)
    F = [F0, dev(A1), dev(A2)]
    A12 = [A1, A2]
    if dtype == "bf16":
        F = [blco.cast_bf16(f) for f in F]
        del F0
        F0 = F[0]
        torch.cuda.empty_cache()
        A12 = [oracle.bf16_round(a) for a in A12]
    # the oracle sees only the referenced rows of the big factor
    used, inv = np.unique(coords[0], return_inverse=True)
    A0 = F0[torch.from_numpy(used.astype(np.int64)).to(DEV)].float().cpu().numpy()
    small = [inv.astype(np.uint32), coords[1], coords[2]]
    for n in (1, 2):
        assert t.resolution(n, R) == "hierarchical"
        out = blco.mttkrp(t, n, F)
        M, S = oracle.mttkrp(small, vals, [A0] + A12, n)
        check_entries(out.cpu().numpy(), M, S, label=f"4 GiB factor {dtype} R={R} mode {n}")
    del F0, F
    torch.cuda.empty_cache()


def test_mechanisms_agree_on_zipf_short_modes():
    # two long Zipf modes and two short modes, like the short4 bench recipe
    import synth

    dims = (1 << 16, 1 << 14, 24, 168)
    nnz = 2_000_000
    w = synth.Workload("t", dims, nnz, (("zipf", 1.1), ("zipf", 1.1), ("uniform",), ("uniform",)),
                       "u01", (32,), (0, 1, 2, 3), 77)
    coords, vals = synth.workload_tensor(w)
    t = blco.build(coords, vals, dims)
    A = synth.workload_factors(w, 32)
    F = [dev(a) for a in A]
    for n in (2, 3):
        assert t.resolution(n, 32) == "hierarchical"
        M, S = oracle.mttkrp(coords, vals, A, n)
        outs = {}
        for res in ("hierarchical", "register"):
            t.set_resolution(res)
            outs[res] = blco.mttkrp(t, n, F).cpu().numpy()
            check_entries(outs[res], M, S, label=f"zipf short mode {n} {res}")
        t.set_resolution("auto")
