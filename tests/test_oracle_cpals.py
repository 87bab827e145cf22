"""Pins of the CP-ALS oracle (Algorithm 1) to facts that do not come from its own code.

* rank-1 closed form: with the other factors exact, one update returns the
  exact factor (V and M reduce to scalars times the true column);
* the update solves the least-squares subproblem: A^(n) V = M (normal
  equations), and no perturbation of A^(n) lowers the dense residual;
* block coordinate descent: the dense residual ||X - Xhat||_F never rises
  across updates;
* the fit identity equals the brute-force dense residual on tiny shapes;
* exact recovery: ALS on an exactly rank-2 dense tensor reaches fit ~ 1;
* a singular V (two equal columns) still gives the minimum-norm solution.
"""
import itertools

import numpy as np
import pytest

from oracle import cpals


def dense_tensor_as_coo(X):
    idx = list(itertools.product(*[range(d) for d in X.shape]))
    coords = [np.array([t[m] for t in idx], np.uint32) for m in range(X.ndim)]
    vals = np.array([X[t] for t in idx], np.float64)
    return coords, vals


def rand_factors(rng, dims, R):
    return [rng.standard_normal((d, R)) for d in dims]


def test_rank1_closed_form():
    rng = np.random.default_rng(1)
    dims = (5, 4, 3)
    a, b, c = (rng.standard_normal((d, 1)) for d in dims)
    X = np.einsum("i,j,k->ijk", a[:, 0], b[:, 0], c[:, 0])
    coords, vals = dense_tensor_as_coo(X)
    start = [rng.standard_normal((5, 1)), b, c]
    A1, M, V = cpals.als_update(coords, vals, start, 0, dims)
    # V = (b.b)(c.c) and M = a (b.b)(c.c), so A1 = a
    assert V.shape == (1, 1)
    assert abs(V[0, 0] - float((b.T @ b)[0, 0]) * float((c.T @ c)[0, 0])) <= 1e-12 * V[0, 0]
    np.testing.assert_allclose(A1, a, rtol=1e-12, atol=1e-12)


def test_update_solves_the_least_squares_subproblem():
    rng = np.random.default_rng(2)
    dims = (4, 3, 5)
    X = rng.standard_normal(dims)
    X[rng.random(dims) < 0.5] = 0.0
    coords, vals = dense_tensor_as_coo(X)
    A = rand_factors(rng, dims, 3)
    for n in range(3):
        An, M, V = cpals.als_update(coords, vals, A, n, dims)
        np.testing.assert_allclose(An @ V, M, rtol=1e-10, atol=1e-10)
        A2 = list(A)
        A2[n] = An
        base = np.linalg.norm(X - cpals.dense_model(dims, A2))
        for _ in range(5):
            A3 = list(A2)
            A3[n] = An + 1e-3 * rng.standard_normal(An.shape)
            assert np.linalg.norm(X - cpals.dense_model(dims, A3)) >= base - 1e-12
        A = A2


def test_residual_never_rises():
    rng = np.random.default_rng(3)
    dims = (4, 4, 3)
    X = rng.random(dims)
    coords, vals = dense_tensor_as_coo(X)
    A = rand_factors(rng, dims, 2)
    prev = np.linalg.norm(X - cpals.dense_model(dims, A))
    for _ in range(4):
        for n in range(3):
            A[n], _, _ = cpals.als_update(coords, vals, A, n, dims)
            cur = np.linalg.norm(X - cpals.dense_model(dims, A))
            assert cur <= prev + 1e-12
            prev = cur


@pytest.mark.parametrize("seed", [4, 5])
def test_fit_identity_matches_dense_residual(seed):
    rng = np.random.default_rng(seed)
    dims = (3, 4, 2, 3)
    X = rng.standard_normal(dims)
    X[rng.random(dims) < 0.6] = 0.0
    coords, vals = dense_tensor_as_coo(X)
    keep = vals != 0
    coords = [c[keep] for c in coords]
    vals = vals[keep]
    A = rand_factors(rng, dims, 2)
    want = 1.0 - np.linalg.norm(X - cpals.dense_model(dims, A)) / np.linalg.norm(X)
    assert abs(cpals.fit(coords, vals, A, dims) - want) <= 1e-12


def test_exact_rank2_recovery():
    rng = np.random.default_rng(6)
    dims = (6, 5, 4)
    G = [rng.random((d, 2)) + 0.1 for d in dims]
    X = cpals.dense_model(dims, G)
    coords, vals = dense_tensor_as_coo(X)
    A, fits = cpals.cp_als(coords, vals, rand_factors(rng, dims, 2), dims, max_iters=300,
                           tol=1e-13)
    assert fits[-1] > 1 - 1e-6
    assert np.linalg.norm(X - cpals.dense_model(dims, A)) <= 1e-5 * np.linalg.norm(X)


def test_singular_v_gives_minimum_norm_solution():
    rng = np.random.default_rng(7)
    dims = (4, 3, 3)
    X = rng.random(dims)
    coords, vals = dense_tensor_as_coo(X)
    A = rand_factors(rng, dims, 2)
    A[1][:, 1] = A[1][:, 0]
    A[2][:, 1] = A[2][:, 0]
    An, M, V = cpals.als_update(coords, vals, A, 0, dims)
    assert np.linalg.matrix_rank(V) == 1
    # the two columns of M are equal, and the minimum-norm answer splits them evenly
    np.testing.assert_allclose(M[:, 0], M[:, 1], rtol=1e-12)
    np.testing.assert_allclose(An[:, 0], An[:, 1], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(An @ V, M, rtol=1e-10, atol=1e-10)


def test_one_mode_update_is_the_data():
    # N = 1: V is the empty Hadamard product (all ones); with R = 1 one update
    # returns the vector of values itself
    x = np.array([3.0, 0.0, -1.5, 2.0])
    coords = [np.array([0, 2, 3], np.uint32)]
    vals = x[[0, 2, 3]]
    A1, M, V = cpals.als_update(coords, vals, [np.ones((4, 1))], 0, (4,))
    np.testing.assert_array_equal(V, [[1.0]])
    np.testing.assert_allclose(A1[:, 0], x, rtol=0, atol=0)
