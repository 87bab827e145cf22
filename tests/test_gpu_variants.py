"""The alternative register-based MTTKRP kernels, chosen per process with
BLCO_KERNEL (stash: hashed LDS segment stash in persistent workgroups; tile:
64-non-zero tiles sorted per wave, the paper's sub-group tile; naive: one
atomic per non-zero and rank), against the fp64 oracle.  Each variant runs in
a child process of its own (the choice is read once per process).
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, ROOT)
import numpy as np, torch
import oracle, paper_2201_12523_amd as blco
rng = np.random.default_rng(3)
cases = [((900, 700, 500), 30_000, 8, 64), ((300, 250, 80, 7), 20_000, 32, 9),
         ((5000, 64, 64), 8_000, 40, 64)]
worst = 0.0
for dims, nnz, R, kb in cases:
    coords = [rng.integers(0, d, size=nnz).astype(np.uint32) for d in dims]
    coords[0][: nnz // 4] = rng.integers(0, 3, size=nnz // 4)
    vals = rng.standard_normal(nnz).astype(np.float32)
    t = blco.build(coords, vals, dims, key_bits=kb, max_block_nnz=5000)
    t.set_resolution("register")
    A = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    for dt in ("fp32", "bf16"):
        F = [torch.from_numpy(a).cuda() for a in A]
        Aref = A
        if dt == "bf16":
            F = [blco.cast_bf16(f) for f in F]
            Aref = [oracle.bf16_round(a) for a in A]
        for n in range(len(dims)):
            out = blco.mttkrp(t, n, F).cpu().numpy().astype(np.float64)
            M, S = oracle.mttkrp(coords, vals, Aref, n)
            nz = S > 0
            assert np.all(out[~nz] == 0), (dims, n, dt)
            e = float((np.abs(out - M)[nz] / S[nz]).max())
            assert e <= 1e-5, (dims, n, dt, e)
            worst = max(worst, e)
print("variant ok, worst normalised error %.2e" % worst, flush=True)
"""


@pytest.mark.parametrize("variant", ["stash", "tile", "naive"])
def test_variant_matches_oracle(variant):
    env = dict(os.environ)
    env["BLCO_KERNEL"] = variant
    code = "ROOT = %r\n" % ROOT + CHILD
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=240)
    print(r.stdout, r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "variant ok" in r.stdout
