"""GPU: the library driven from C alone (tests/c_abi/solve_demo.c, built by build()).

The program builds the 33^3 cylinder's domain with saamg_domain_from_shape, sets up the
hierarchy, solves with hipMalloc'ed buffers, then refreshes the hierarchy for a longer pipe
and solves again.  Its first solution must match the oracle's solve of the same problem to
1e-8 (the fp64 parity bound).
"""
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import operator, solve

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi", "solve_demo")


def test_c_program_matches_the_oracle(tmp_path):
    if not os.path.exists(EXE):
        raise RuntimeError(f"{EXE} is missing: run __graft_entry__.build() first")
    w = W.c1_cylinder33()
    b = W.rhs(w)
    rhs, out = tmp_path / "b.f64", tmp_path / "x.f64"
    np.ascontiguousarray(b, dtype=np.float64).tofile(rhs)
    print("[case] C demo on the 33^3 cylinder", flush=True)
    p = subprocess.run([EXE, str(rhs), str(out)], capture_output=True, text=True, timeout=120)
    print(p.stdout, p.stderr, flush=True)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok")
    x = np.fromfile(out, dtype=np.float64).reshape(b.shape)
    sys_, H = solve.build(w.shape, w.nx, w.ny, w.nz, w.variant)
    ref = solve.solve(sys_, H, b, tol=1e-12)
    xo = sys_.scatter(operator.unscale(sys_, ref.x)).reshape(b.shape)
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
