"""Pins of the fp64 MTTKRP oracle against what the paper and the mathematics fix.

* Dense brute force of Eq. (1): materialise X, unfold it in mode n (mode-n
  fibres as columns, Section 2.3), form the Khatri-Rao product
  A^(N) (.) ... (.) A^(n+1) (.) A^(n-1) (.) ... (.) A^(1) column by column with the
  Kronecker product of Section 2.1, and multiply.  Distinct mode lengths make a
  wrong unfolding order or a transposed operand fail.
* N = 2 reduces to sparse-matrix times dense-matrix (scipy).
* All-ones factors give slice sums (numpy bincount).
* The hand-worked Figure 4a example (tests/golden/fig4a_mttkrp.txt).
* Cross-mode invariant, linearity, order invariance.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from conftest import read_golden


def _rand_sparse(dims, nnz, seed, dup=False):
    rng = np.random.default_rng(seed)
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    if dup and nnz >= 2:
        for c in coords:
            c[-1] = c[0]  # one duplicated coordinate
    vals = rng.standard_normal(nnz)
    return coords, vals


def _dense(coords, vals, dims):
    X = np.zeros(dims)
    np.add.at(X, tuple(c.astype(np.int64) for c in coords), vals)
    return X


def _unfold(X, n):
    # column index sum_{k != n} i_k prod_{m < k, m != n} I_m  (first remaining mode fastest)
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


def _khatri_rao_eq1(factors, n):
    """A^(N) (.) ... (.) A^(n+1) (.) A^(n-1) (.) ... (.) A^(1), column-wise Kronecker."""
    R = factors[0].shape[1]
    others = [factors[m] for m in range(len(factors) - 1, -1, -1) if m != n]
    cols = []
    for r in range(R):
        col = np.ones(1)
        for A in others:
            col = np.kron(col, A[:, r])
        cols.append(col)
    return np.stack(cols, axis=1)


CASES = [
    ((5, 3), 3, 11),
    ((3, 1, 5), 2, 9),
    ((4, 3, 2, 5), 5, 40),
    ((2, 3, 1, 2, 3), 1, 20),
    ((7, 6, 5), 4, 60),
]


@pytest.mark.parametrize("dims,R,nnz", CASES)
@pytest.mark.parametrize("dup", [False, True])
def test_dense_brute_force(dims, R, nnz, dup):
    coords, vals = _rand_sparse(dims, nnz, seed=sum(dims) * 7 + R, dup=dup)
    rng = np.random.default_rng(R + len(dims))
    factors = [rng.standard_normal((d, R)) for d in dims]
    X = _dense(coords, vals, dims)
    for n in range(len(dims)):
        M, S = oracle.mttkrp(coords, vals, factors, n)
        ref = _unfold(X, n) @ _khatri_rao_eq1(factors, n)
        assert M.shape == (dims[n], R)
        scale = np.abs(ref).max() + 1e-300
        assert np.max(np.abs(M - ref)) <= 1e-12 * scale
        assert np.all(S >= np.abs(M) - 1e-12 * scale)


def test_two_modes_is_spmm():
    dims = (37, 23)
    coords, vals = _rand_sparse(dims, 150, seed=3)
    rng = np.random.default_rng(4)
    A = [rng.standard_normal((d, 6)) for d in dims]
    X = sp.coo_matrix((vals, (coords[0].astype(np.int64), coords[1].astype(np.int64))), shape=dims)
    M0, _ = oracle.mttkrp(coords, vals, A, 0)
    M1, _ = oracle.mttkrp(coords, vals, A, 1)
    np.testing.assert_allclose(M0, X @ A[1], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(M1, X.T @ A[0], rtol=1e-12, atol=1e-12)


def test_all_ones_gives_slice_sums():
    dims = (50, 40, 30, 3)
    coords, vals = _rand_sparse(dims, 500, seed=5)
    ones = [np.ones((d, 4)) for d in dims]
    for n in range(4):
        M, _ = oracle.mttkrp(coords, vals, ones, n)
        ref = np.bincount(coords[n], weights=vals, minlength=dims[n])
        for r in range(4):
            np.testing.assert_allclose(M[:, r], ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("case", ["ones", "ramp"])
def test_figure4a_worked_example(fig4a, case):
    coords, vals, dims = fig4a
    col = np.ones(4) if case == "ones" else np.arange(1, 5, dtype=np.float64)
    factors = [col[:, None].copy() for _ in range(3)]
    want = {int(r[1]) - 1: [float(x) for x in r[2:]] for r in read_golden("fig4a_mttkrp.txt")
            if r[0] == case}
    for n in range(3):
        M, _ = oracle.mttkrp(coords, vals, factors, n)
        assert M[:, 0].tolist() == want[n]
    if case == "ramp":
        for n in range(3):
            M, _ = oracle.mttkrp(coords, vals, factors, n)
            assert float(M[:, 0] @ col) == 2314.0


def test_cross_mode_invariant_and_linearity():
    dims = (31, 17, 9, 4)
    coords, vals = _rand_sparse(dims, 300, seed=8)
    rng = np.random.default_rng(9)
    A = [rng.standard_normal((d, 5)) for d in dims]
    rowprod = np.prod([A[m][coords[m].astype(np.int64)] for m in range(4)], axis=0)
    target = float(vals @ rowprod.sum(axis=1))
    for n in range(4):
        M, _ = oracle.mttkrp(coords, vals, A, n)
        assert abs(float(np.sum(M * A[n])) - target) <= 1e-11 * (abs(target) + 1)
    # linear in x and in each other factor; invariant to the order of non-zeros
    M, _ = oracle.mttkrp(coords, vals, A, 1)
    M2, _ = oracle.mttkrp(coords, 2.5 * vals, A, 1)
    np.testing.assert_allclose(M2, 2.5 * M, rtol=1e-13, atol=1e-13)
    B = [a.copy() for a in A]
    B[3] = -3.0 * B[3]
    M3, _ = oracle.mttkrp(coords, vals, B, 1)
    np.testing.assert_allclose(M3, -3.0 * M, rtol=1e-13, atol=1e-13)
    perm = np.random.default_rng(10).permutation(len(vals))
    M4, _ = oracle.mttkrp([c[perm] for c in coords], vals[perm], A, 1)
    np.testing.assert_allclose(M4, M, rtol=1e-12, atol=1e-12)


def test_rows_variant_matches_full():
    dims = (64, 33, 20)
    coords, vals = _rand_sparse(dims, 2000, seed=12)
    rng = np.random.default_rng(13)
    A = [rng.standard_normal((d, 7)) for d in dims]
    X = _dense(coords, vals, dims)
    for n in range(3):
        rows = np.array([0, 5, dims[n] - 1, 17 % dims[n]], dtype=np.uint32)
        rows = np.unique(rows)
        Mr, Sr = oracle.mttkrp_rows(coords, vals, A, n, rows, dims)
        ref = (_unfold(X, n) @ _khatri_rao_eq1(A, n))[rows.astype(np.int64)]
        np.testing.assert_allclose(Mr, ref, rtol=1e-12, atol=1e-12)
        M, S = oracle.mttkrp(coords, vals, A, n)
        np.testing.assert_array_equal(Mr, M[rows.astype(np.int64)])
        np.testing.assert_array_equal(Sr, S[rows.astype(np.int64)])


def test_synthetic_workload_small_against_brute_force_rows():
    """The generated 1000x800x600 workload: sampled rows against a dense per-row sum."""
    w = synth.WORKLOADS["small"]
    coords, vals = synth.workload_tensor(w, nnz=20_000)
    A = synth.workload_factors(w, 16)
    n = 0
    rows = np.array([0, 1, 499, 998, 999], dtype=np.uint32)
    Mr, _ = oracle.mttkrp_rows(coords, vals, A, n, rows, w.dims)
    for j, i in enumerate(rows):
        sel = np.flatnonzero(coords[0] == i)
        ref = np.zeros(16)
        for k in sel:
            ref += float(vals[k]) * A[1][coords[1][k]].astype(np.float64) * \
                A[2][coords[2][k]].astype(np.float64)
        np.testing.assert_allclose(Mr[j], ref, rtol=1e-12, atol=1e-12)


def test_bf16_round_pins():
    # bf16 keeps 8 significand bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1);
    # 1 + 3*2^-8 ties between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6); exact values stay
    x = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -7, -2.5, 0.0, 1 + 2.0 ** -9],
                 dtype=np.float32)
    assert oracle.bf16_round(x).tolist() == [1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -2.5, 0.0, 1.0]
    r = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    y = oracle.bf16_round(r)
    assert np.all(np.abs(y - r) <= np.abs(r) * 2.0 ** -8)
    assert np.all(y.view(np.uint32) & 0xFFFF == 0)


def test_rows_f32_variant_matches_fp64():
    dims = (40, 30, 20, 5)
    coords, vals = _rand_sparse(dims, 3000, seed=77)
    vals32 = vals.astype(np.float32)
    rng = np.random.default_rng(78)
    A32 = [rng.standard_normal((d, 6)).astype(np.float32) for d in dims]
    for n in range(4):
        rows = np.unique(np.array([0, 3, dims[n] - 1], dtype=np.uint32))
        M, S = oracle.mttkrp_rows(coords, vals32.astype(np.float64),
                                  [a.astype(np.float64) for a in A32], n, rows, dims)
        M2, S2 = oracle.mttkrp_rows_f32(coords, vals32, A32, n, rows, dims)
        np.testing.assert_array_equal(M, M2)
        np.testing.assert_array_equal(S, S2)


@pytest.mark.parametrize("threads,force_atomic", [(1, False), (3, False), (8, False), (5, True)])
def test_omp_oracle_matches_serial(threads, force_atomic):
    """The multi-threaded oracle (used to time the oracle on all host cores) changes only
    the order of the additions: equal to the serial oracle within fp64 rounding, and
    pinned independently by the dense brute force of Eq. (1)."""
    dims = (37, 11, 23)
    coords, vals = _rand_sparse(dims, 4000, 31 + threads, dup=True)
    rng = np.random.default_rng(9)
    A = [rng.standard_normal((d, 6)) for d in dims]
    X = _dense(coords, vals, dims)
    for n in range(3):
        M, S = oracle.mttkrp(coords, vals, A, n)
        Mo, So, used, atomic = oracle.mttkrp_omp(coords, vals, A, n, threads=threads,
                                                 force_atomic=force_atomic)
        assert used == threads and atomic == force_atomic
        assert np.all(np.abs(Mo - M) <= 1e-12 * S)
        assert np.allclose(So, S, rtol=1e-12, atol=0)
        brute = _unfold(X, n) @ _khatri_rao_eq1(A, n)
        assert np.allclose(Mo, brute, rtol=1e-10, atol=1e-10)


def test_omp_oracle_fewer_nonzeros_than_threads():
    dims = (4, 5)
    coords, vals = _rand_sparse(dims, 3, 2)
    A = [np.ones((d, 2)) for d in dims]
    M, S = oracle.mttkrp(coords, vals, A, 0)
    Mo, So, used, _ = oracle.mttkrp_omp(coords, vals, A, 0, threads=8)
    assert used == 8
    assert np.array_equal(M, Mo) and np.array_equal(S, So)
    # all-ones factors: slice sums
    assert np.allclose(Mo[:, 0], np.bincount(coords[0], weights=vals, minlength=4))


@pytest.mark.parametrize("threads", [1, 4, 7])
def test_omp_rows_oracle_matches_serial(threads):
    """The threaded row-restricted oracle (fp64 values, fp32 factors widened as read) equals
    the serial row oracles within fp64 rounding; the serial ones are pinned above."""
    dims = (50, 13, 29, 4)
    coords, vals = _rand_sparse(dims, 6000, 71 + threads, dup=True)
    rng = np.random.default_rng(3)
    A = [rng.standard_normal((d, 5)).astype(np.float32) for d in dims]
    for n in range(4):
        rows = np.unique(rng.integers(0, dims[n], 9)).astype(np.uint32)
        M, S = oracle.mttkrp_rows(coords, vals, [a.astype(np.float64) for a in A], n, rows, dims)
        Mo, So = oracle.mttkrp_rows_omp(coords, vals, A, n, rows, dims, threads=threads)
        assert np.all(np.abs(Mo - M) <= 1e-12 * S) and np.allclose(So, S, rtol=1e-12, atol=0)
        Mf, Sf = oracle.mttkrp_rows_f32(coords, vals.astype(np.float32), A, n, rows, dims)
        Mo2, So2 = oracle.mttkrp_rows_omp(coords, vals.astype(np.float32), A, n, rows, dims,
                                          threads=threads)
        assert np.all(np.abs(Mo2 - Mf) <= 1e-12 * Sf)


def test_omp_cp_model_bit_identical():
    dims = (30, 20, 10)
    coords, _ = _rand_sparse(dims, 5000, 5)
    rng = np.random.default_rng(8)
    A = [rng.standard_normal((d, 7)) for d in dims]
    assert np.array_equal(oracle.cp_model(coords, A), oracle.cp_model_omp(coords, A, threads=5))
