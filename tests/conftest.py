import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def fig4a():
    """(coords 0-based list of 3 uint32 arrays, values float32, dims)."""
    import numpy as np
    rows = read_golden("fig4a_coo.txt")
    c = np.array([[int(r[0]) - 1, int(r[1]) - 1, int(r[2]) - 1] for r in rows], dtype=np.uint32)
    v = np.array([float(r[3]) for r in rows], dtype=np.float32)
    return [np.ascontiguousarray(c[:, m]) for m in range(3)], v, (4, 4, 4)


# fp32 residuals in CP-gradient checks.  The library forms e_k = x_k - xhat_k in fp32 with
# xhat_k = sum_r prod_m A^(m)[i_m^k, r]: N - 1 products per rank and a sum of R terms, in
# whatever order its kernel uses, so |fl(xhat_k) - xhat_k| <= gamma_{N+R-1} sum_r prod_m |a|
# (gamma_n = n u / (1 - n u), u = 2^-24, any summation order), and the difference adds
# u |e_k|.  A gradient entry sums e_k prod_{m != n} a, so on top of the relative bound on
# its own summation (TOL times the sum of |terms|) it may move by gamma_{N+R} W, with
# W = MTTKRP_n(sum_r prod_m |a|; |A|): the model's magnitude, not the residual's, which a
# near-cancelling residual in a row of few non-zeros exposes.  residual_gamma(N, R) is that
# gamma, rounded up.
def residual_gamma(N, R):
    n = N + R + 1
    u = 2.0 ** -24
    return n * u / (1 - n * u)


def grad_allowed(S, W, N, R, tol=1e-5):
    """Allowed |gpu - oracle| of CP-gradient entries: tol * S (S the sum of |e-terms|) plus
    the fp32 residual's rounding carried through the MTTKRP (W as above)."""
    return tol * S + residual_gamma(N, R) * W
