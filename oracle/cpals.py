"""ORACLE — test infrastructure only.

CP-ALS (Algorithm 1) in plain fp64 numpy on top of the fp64 MTTKRP oracle.
Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import it; it shares no code with the library.

Algorithm 1, per iteration and for n = 1..N in turn:
  V      = Hadamard product of the Gram matrices A^(m)T A^(m), m != n;
  M      = mode-n MTTKRP (Eq. (1)) with the current factors;
  A^(n)  = M V^+   (V^+ the Moore-Penrose pseudo-inverse);
repeated until the fit stops improving or an iteration cap is reached.

The paper does not define the fit or the stopping test; the readings taken are
  fit = 1 - ||X - Xhat||_F / ||X||_F,  Xhat = [[A^(1), ..., A^(N)]],
computed without forming Xhat from
  ||X - Xhat||^2 = ||X||^2 - 2 <X, Xhat> + ||Xhat||^2,
  <X, Xhat>      = sum(M_N * A^(N))            (M_N the last MTTKRP of the sweep),
  ||Xhat||^2     = sum of the entries of the Hadamard product of all N Grams,
and "stops improving" = the fit rose by less than ``tol`` over the previous
iteration.  Algorithm 1 has no column normalisation, so none is applied.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import mttkrp as _mttkrp


def gram(A):
    """A^T A in fp64 (a factor of V in Algorithm 1)."""
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A


def hadamard_of_grams(grams, skip=None):
    """Entry-wise product of the given Gram matrices, leaving out index ``skip``
    (all ones, the identity of the entry-wise product, when nothing is left)."""
    V = np.ones_like(grams[0])
    for m, G in enumerate(grams):
        if m != skip:
            V = V * G
    return V


def als_update(coords, vals, factors, n, dims):
    """One update of Algorithm 1 for mode n: returns (A_new, M, V)."""
    grams = [gram(A) for A in factors]
    V = hadamard_of_grams(grams, skip=n)
    M, _ = _mttkrp(coords, vals, factors, n, dims=dims)
    return M @ np.linalg.pinv(V), M, V


def fit(coords, vals, factors, dims, M_last=None):
    """1 - ||X - Xhat||_F / ||X||_F by the norm identity above (fp64)."""
    N = len(factors)
    x2 = float(np.dot(np.asarray(vals, np.float64), np.asarray(vals, np.float64)))
    if M_last is None:
        M_last, _ = _mttkrp(coords, vals, factors, N - 1, dims=dims)
    inner = float(np.sum(M_last * np.asarray(factors[N - 1], np.float64)))
    model2 = float(np.sum(hadamard_of_grams([gram(A) for A in factors])))
    resid2 = max(x2 - 2.0 * inner + model2, 0.0)
    return 1.0 - np.sqrt(resid2) / np.sqrt(x2)


def cp_als(coords, vals, factors, dims, max_iters, tol=0.0):
    """Algorithm 1 from the given initial factors: returns (factors, fits per iteration)."""
    A = [np.array(f, dtype=np.float64, copy=True) for f in factors]
    N = len(A)
    fits = []
    for _ in range(max_iters):
        M = None
        for n in range(N):
            A[n], M, _ = als_update(coords, vals, A, n, dims)
        fits.append(fit(coords, vals, A, dims, M_last=M))
        if len(fits) > 1 and fits[-1] - fits[-2] < tol:
            break
    return A, fits


def dense_model(dims, factors):
    """Every entry of [[A^(1), ..., A^(N)]] by brute force (tiny shapes only)."""
    out = np.zeros(dims, dtype=np.float64)
    R = factors[0].shape[1]
    for idx in itertools.product(*[range(d) for d in dims]):
        s = 0.0
        for r in range(R):
            p = 1.0
            for m, i in enumerate(idx):
                p *= float(factors[m][i, r])
            s += p
        out[idx] = s
    return out
