"""Pins of the CP loss / gradient oracle.

* Central finite differences of f = 1/2 sum_k (x_k - xhat_k)^2 (fp64).
* A tensor generated exactly from the model has zero loss and zero gradient.
* <G^(n), A^(n)> = -sum_k e_k xhat_k for every mode n (the model is
  multilinear, so d/dt f(A^(n) (1+t)) at t = 0 equals that sum).
"""
import numpy as np
import pytest

import oracle


def _problem(dims, nnz, R, seed):
    rng = np.random.default_rng(seed)
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    vals = rng.standard_normal(nnz)
    A = [rng.standard_normal((d, R)) * 0.7 for d in dims]
    return coords, vals, A


@pytest.mark.parametrize("dims,R", [((5, 4, 3), 3), ((4, 3, 5, 2), 2), ((6, 7), 4)])
def test_gradient_matches_central_differences(dims, R):
    coords, vals, A = _problem(dims, 25, R, seed=len(dims) * 10 + R)
    f, e, G, _ = oracle.cp_grad(coords, vals, A)
    for n in range(len(dims)):
        for i in range(dims[n]):
            for r in range(R):
                a = A[n][i, r]
                h = 1e-6 * max(1.0, abs(a))
                Ap = [x.copy() for x in A]
                Am = [x.copy() for x in A]
                Ap[n][i, r] = a + h
                Am[n][i, r] = a - h
                fd = (oracle.cp_loss(coords, vals, Ap)[0] - oracle.cp_loss(coords, vals, Am)[0]) / (2 * h)
                assert abs(fd - G[n][i, r]) <= 1e-6 * max(1.0, abs(fd))


def test_zero_residual():
    dims = (6, 5, 4)
    rng = np.random.default_rng(1)
    A = [rng.standard_normal((d, 3)) for d in dims]
    coords = [rng.integers(0, d, size=40).astype(np.uint32) for d in dims]
    # exact model values, computed independently of the oracle
    x = np.prod([A[m][coords[m].astype(np.int64)] for m in range(3)], axis=0).sum(axis=1)
    f, e, G, _ = oracle.cp_grad(coords, x, A)
    assert f < 1e-25
    for g in G:
        assert np.max(np.abs(g)) < 1e-12


def test_inner_product_invariant():
    dims = (9, 8, 7, 3)
    coords, vals, A = _problem(dims, 60, 4, seed=2)
    f, e, G, _ = oracle.cp_grad(coords, vals, A)
    xhat = oracle.cp_model(coords, A)
    target = -float(e @ xhat)
    for n in range(4):
        assert abs(float(np.sum(G[n] * A[n])) - target) <= 1e-10 * (abs(target) + 1)
    # the loss itself
    assert abs(f - 0.5 * float(np.sum((vals - xhat) ** 2))) <= 1e-12 * (f + 1)
