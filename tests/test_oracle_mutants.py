"""Mutation test of the oracle's pins: each planted mistake (a dropped term, a
wrong sign or index, a transposed operand, a missing step) is compiled into a
private copy of the oracle, and the pin suite must fail on it.  The planted
mistakes live only in those private builds (CPU only)."""
import os
import subprocess
import sys

import pytest

from oracle import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    1: "Gram drops the last column of every row product",
    2: "Gram leaves the upper triangle unset",
    3: "Householder beta halved",
    4: "eigenvector rotation with a wrong sign",
    5: "eigenvalues sorted ascending (bottom-k sketch)",
    6: "one-sided Jacobi rotation with a wrong sign",
    7: "sketch rows taken one eigenvector too far",
    8: "row basis V not orthogonalised",
    9: "R = V Y_r with Y transposed",
    10: "rank-(r+1) output instead of rank-r truncation",
    11: "sketch product reads S as a transposed (m x k) operand",
    12: "QR keeps |R_jj| but not the reflector's sign",
    13: "format rounding breaks ties away from zero",
    14: "format rounding keeps one significant bit too few",
    15: "e4m3 scale one power of two too large",
    16: "Box-Muller radius sqrt(-ln u) instead of sqrt(-2 ln u)",
    17: "sparse sign sketch never uses its last row",
    18: "two-sided SCW drops Sigma_r from L",
    19: "HOOI never updates S (mode 1 stays at the HOSVD guess)",
    20: "block-scaled e4m3 with blocks of 16 instead of 32 elements",
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, mutant):
    so = oracle.build(force=True, out=str(tmp_path / f"libtsko_m{mutant}.so"), mutant=mutant)
    env = dict(os.environ, TSKO_LIB=so, OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py"),
                        os.path.join(ROOT, "tests", "test_oracle_formats.py"),
                        os.path.join(ROOT, "tests", "test_oracle_random.py"),
                        os.path.join(ROOT, "tests", "test_oracle_twosided.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins missed mutant {mutant}: {MUTANTS[mutant]}\n{r.stdout[-2000:]}"
