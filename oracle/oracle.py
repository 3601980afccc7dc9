"""ctypes binding of the FP64 CPU oracle (``libtsko.so``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use this module to obtain reference results.  The GPU product
path never imports it.  Arrays are numpy; inputs are converted to C-contiguous
float32/float64 as the C routine expects, outputs are float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TSKO_LIB") or os.path.join(HERE, "libtsko.so")
SRC = os.path.join(HERE, "tsko.c")

FLAG_RANKDEF, FLAG_TIE, FLAG_NONFIN = 1, 2, 4


def build(force: bool = True, out: str | None = None, mutant: int = 0) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math).
    ``mutant`` > 0 builds a copy with one planted mistake (mutation test)."""
    out = out or os.path.join(HERE, "libtsko.so")
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               f"-DTSKO_MUTANT={int(mutant)}", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "tsko_gram_f32": [_P, _I, _I, _I, _P],
            "tsko_gram_f64": [_P, _I, _I, _I, _P],
            "tsko_eigh": [_P, _I, _P, _P],
            "tsko_eigh_jacobi": [_P, _I, _P, _P],
            "tsko_svd": [_P, _I, _I, _P, _P, _P],
            "tsko_qr": [_P, _I, _I, _P, _P],
            "tsko_train_f32": [_P, _I, _I, _I, _I, _P, _P, _P],
            "tsko_train_from_gram": [_P, _I, _I, _P, _P],
            "tsko_scw": [_P, _I, _I, _P, _I, _I, ctypes.c_int, _P, _P, _P, _P, _P, _P],
            "tsko_scw_basis": [_P, _I, _I, _P, _I, ctypes.c_int, _P, _P],
            "tsko_random_sketch": [ctypes.c_int, _I, _I, ctypes.c_uint64, _P],
            "tsko_gram2_f32": [_P, _I, _I, _I, _P],
            "tsko_train2_f32": [_P, _I, _I, _I, _I, _I, _I, ctypes.c_double, _P, _P, _P, _P],
            "tsko_scw2": [_P, _I, _I, _P, _I, _P, _I, _I, _P, _P, _P, _P, _P],
            "tsko_apply2_f32": [_P, _I, _I, _I, _P, _I, _P, _I, _I, _P, _P, _P, _P, _P],
            "tsko_apply_f32": [_P, _I, _I, _I, _P, _I, _I, _P, _P, _P, _P, _P],
            "tsko_error_f32": [_P, _I, _I, _I, _P, _P, _I, _P],
            "tsko_opt_f32": [_P, _I, _I, _I, _I, _P, _P],
            "tsko_threads": [],
            "tsko_round_bf16": [_P, _I, _P],
            "tsko_round_e4m3": [_P, _I, ctypes.c_float, _P],
            "tsko_e4m3_scale": [_P, _I, _P],
            "tsko_round_e4m3_mx": [_P, _I, _I, _P, _P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.tsko_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.tsko_splitmix64.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _check(st, name):
    if st < 0:
        raise ValueError(f"{name}: invalid arguments")
    return st


def threads() -> int:
    return lib().tsko_threads()


def gram(A: np.ndarray) -> np.ndarray:
    """Mode-1 Gram sum_d A_d A_d^T of a (count, m, n) stack."""
    A = np.asarray(A)
    if A.ndim == 2:
        A = A[None]
    cnt, m, n = A.shape
    G = np.empty((m, m))
    if A.dtype == np.float32:
        A = _f32(A)
        _check(lib().tsko_gram_f32(_p(A), cnt, m, n, _p(G)), "gram")
    else:
        A = _f64(A)
        _check(lib().tsko_gram_f64(_p(A), cnt, m, n, _p(G)), "gram")
    return G


def eigh(G: np.ndarray, vectors: bool = True, method: str = "qr"):
    """Descending eigenvalues (and eigenvector columns) of a symmetric matrix."""
    G = _f64(G)
    m = G.shape[0]
    w = np.empty(m)
    V = np.empty((m, m)) if vectors else None
    f = lib().tsko_eigh if method == "qr" else lib().tsko_eigh_jacobi
    st = _check(f(_p(G), m, _p(w), _p(V)), "eigh")
    if st:
        raise RuntimeError("oracle eigensolver did not converge")
    return (w, V) if vectors else w


def svd(A: np.ndarray):
    """Thin SVD A = U diag(s) Vt (one-sided Jacobi)."""
    A = _f64(A)
    m, n = A.shape
    p = min(m, n)
    U, s, Vt = np.empty((m, p)), np.empty(p), np.empty((p, n))
    _check(lib().tsko_svd(_p(A), m, n, _p(U), _p(s), _p(Vt)), "svd")
    return U, s, Vt


def qr(A: np.ndarray):
    A = _f64(A)
    m, n = A.shape
    Q, R = np.empty((m, n)), np.empty((n, n))
    _check(lib().tsko_qr(_p(A), m, n, _p(Q), _p(R)), "qr")
    return Q, R


def train(A: np.ndarray, k: int, return_fro2: bool = False):
    """Sketch S (k x m, rows = top-k eigenvectors of the mode-1 Gram) and
    lambda_1..lambda_{k+1}."""
    A = _f32(A)
    cnt, m, n = A.shape
    S = np.empty((k, m))
    lam = np.empty(k + 1)
    fro2 = np.empty(1)
    st = _check(lib().tsko_train_f32(_p(A), cnt, m, n, k, _p(S), _p(lam), _p(fro2)), "train")
    if st:
        raise RuntimeError("oracle eigensolver did not converge")
    return (S, lam, float(fro2[0])) if return_fro2 else (S, lam)


def train_from_gram(G: np.ndarray, k: int):
    G = _f64(G)
    m = G.shape[0]
    S = np.empty((k, m))
    lam = np.empty(k + 1)
    st = _check(lib().tsko_train_from_gram(_p(G), m, k, _p(S), _p(lam)), "train_from_gram")
    if st:
        raise RuntimeError("oracle eigensolver did not converge")
    return S, lam


def scw(A: np.ndarray, S: np.ndarray, r: int, vmode: int = 0, want_ahat: bool = False):
    """Algorithm 1 on one matrix.  Returns dict(L, R, sigma, relerr, flags[, Ahat])."""
    A = _f64(A)
    S = _f64(S)
    m, n = A.shape
    k = S.shape[0]
    L, R, sig = np.empty((m, r)), np.empty((n, r)), np.empty(r)
    Ah = np.empty((m, n)) if want_ahat else None
    e = np.empty(1)
    fl = np.zeros(1, dtype=np.int32)
    _check(lib().tsko_scw(_p(A), m, n, _p(S), k, r, vmode, _p(L), _p(R), _p(sig), _p(Ah),
                          _p(e), _p(fl)), "scw")
    out = dict(L=L, R=R, sigma=sig, relerr=float(e[0]), flags=int(fl[0]))
    if want_ahat:
        out["Ahat"] = Ah
    return out


def scw_basis(A: np.ndarray, S: np.ndarray, vmode: int = 0):
    """Step 1 of Algorithm 1: V (n x k, orthonormal columns) spanning the row
    space of S A, and the flags (RANKDEF) of that step."""
    A = _f64(A)
    S = _f64(S)
    m, n = A.shape
    k = S.shape[0]
    V = np.empty((n, k))
    fl = np.zeros(1, dtype=np.int32)
    _check(lib().tsko_scw_basis(_p(A), m, n, _p(S), k, vmode, _p(V), _p(fl)), "scw_basis")
    return V, int(fl[0])


SKETCH_KINDS = {"gaussian": 0, "sign": 1, "sparse": 2}


def gram2(A: np.ndarray) -> np.ndarray:
    """Mode-2 Gram sum_d A_d^T A_d of a (count, m, n) stack."""
    A = _f32(A)
    if A.ndim == 2:
        A = A[None]
    cnt, m, n = A.shape
    G = np.empty((n, n))
    _check(lib().tsko_gram2_f32(_p(A), cnt, m, n, _p(G)), "gram2")
    return G


def train2(A: np.ndarray, k: int, l: int, max_sweeps: int = 50, tol: float = 1e-10):
    """Tucker2 by HOOI: (S (k x m), W (l x n), core2 history, sweeps)."""
    A = _f32(A)
    cnt, m, n = A.shape
    S, W = np.empty((k, m)), np.empty((l, n))
    core2 = np.zeros(max_sweeps + 1)
    sw = np.zeros(1, dtype=np.int64)
    _check(lib().tsko_train2_f32(_p(A), cnt, m, n, k, l, max_sweeps, tol, _p(S), _p(W), _p(core2), _p(sw)),
           "train2")
    return S, W, core2[:int(sw[0]) + 1], int(sw[0])


def scw2(A: np.ndarray, S: np.ndarray, W: np.ndarray, r: int):
    """Two-sided SCW (Algorithm 4) on one matrix."""
    A = _f64(A)
    S = _f64(S)
    W = _f64(W)
    m, n = A.shape
    k, l = S.shape[0], W.shape[0]
    L, R, sig = np.empty((m, r)), np.empty((n, r)), np.empty(r)
    e = np.empty(1)
    fl = np.zeros(1, dtype=np.int32)
    _check(lib().tsko_scw2(_p(A), m, n, _p(S), k, _p(W), l, r, _p(L), _p(R), _p(sig), _p(e), _p(fl)), "scw2")
    return dict(L=L, R=R, sigma=sig, relerr=float(e[0]), flags=int(fl[0]))


def apply2(A: np.ndarray, S: np.ndarray, W: np.ndarray, r: int, factors: bool = True):
    """Two-sided SCW over a (count, m, n) float32 stack (OpenMP across slices)."""
    A = _f32(A)
    S = _f64(S)
    W = _f64(W)
    cnt, m, n = A.shape
    k, l = S.shape[0], W.shape[0]
    L = np.empty((cnt, m, r)) if factors else None
    R = np.empty((cnt, n, r)) if factors else None
    sig = np.empty((cnt, r)) if factors else None
    e = np.empty(cnt)
    fl = np.zeros(cnt, dtype=np.int32)
    _check(lib().tsko_apply2_f32(_p(A), cnt, m, n, _p(S), k, _p(W), l, r, _p(L), _p(R), _p(sig), _p(e),
                                 _p(fl)), "apply2")
    return dict(L=L, R=R, sigma=sig, relerr=e, flags=fl)


def splitmix64(seed: int, c: int) -> int:
    """The c-th output (from 0) of SplitMix64 seeded with `seed`."""
    return int(lib().tsko_splitmix64(seed, c))


def random_sketch(kind: str, k: int, m: int, seed: int) -> np.ndarray:
    """Data-free k x m sketch of the SCW baseline ("gaussian", "sign" or
    "sparse"), float64."""
    S = np.empty((k, m))
    _check(lib().tsko_random_sketch(SKETCH_KINDS[kind], k, m, seed, _p(S)), "random_sketch")
    return S


def apply(A: np.ndarray, S: np.ndarray, r: int, factors: bool = True):
    """Algorithm 1 over a (count, m, n) float32 stack (OpenMP across slices)."""
    A = _f32(A)
    S = _f64(S)
    cnt, m, n = A.shape
    k = S.shape[0]
    L = np.empty((cnt, m, r)) if factors else None
    R = np.empty((cnt, n, r)) if factors else None
    sig = np.empty((cnt, r)) if factors else None
    e = np.empty(cnt)
    fl = np.zeros(cnt, dtype=np.int32)
    _check(lib().tsko_apply_f32(_p(A), cnt, m, n, _p(S), k, r, _p(L), _p(R), _p(sig),
                                _p(e), _p(fl)), "apply")
    return dict(L=L, R=R, sigma=sig, relerr=e, flags=fl)


def error(A: np.ndarray, L: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Explicit ||A_d - L_d R_d^T||_F / ||A_d||_F per slice."""
    A = _f32(A)
    cnt, m, n = A.shape
    L = _f64(L).reshape(cnt, m, -1)
    R = _f64(R).reshape(cnt, n, -1)
    r = L.shape[2]
    e = np.empty(cnt)
    _check(lib().tsko_error_f32(_p(A), cnt, m, n, _p(L), _p(R), r, _p(e)), "error")
    return e


def opt_tail(A: np.ndarray, r: int):
    """||A_d - [A_d]_r||_F and ||A_d||_F per slice (Jacobi SVD)."""
    A = _f32(A)
    if A.ndim == 2:
        A = A[None]
    cnt, m, n = A.shape
    t, f = np.empty(cnt), np.empty(cnt)
    _check(lib().tsko_opt_f32(_p(A), cnt, m, n, r, _p(t), _p(f)), "opt")
    return t, f


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Values of x rounded to bfloat16 (nearest, ties to even), as float32."""
    x = _f32(x)
    y = np.empty_like(x)
    _check(lib().tsko_round_bf16(_p(x), x.size, _p(y)), "round_bf16")
    return y


def round_e4m3(x: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """Values of x * scale rounded to e4m3 (nearest, ties to even, saturating
    at 448), as float32."""
    x = _f32(x)
    y = np.empty_like(x)
    _check(lib().tsko_round_e4m3(_p(x), x.size, ctypes.c_float(scale), _p(y)), "round_e4m3")
    return y


MX_BLOCK = 32


def round_e4m3_mx(x: np.ndarray):
    """Block-scaled e4m3 of x (..., n): one power-of-two scale per block of
    32 consecutive elements of a row.  Returns (decoded values as float32,
    E8M0 exponent bytes (..., ceil(n / 32)))."""
    x = _f32(x)
    n = x.shape[-1]
    rows = x.size // n if n else 0
    nb = (n + MX_BLOCK - 1) // MX_BLOCK
    y = np.empty_like(x)
    e = np.empty(x.shape[:-1] + (nb,), dtype=np.uint8)
    _check(lib().tsko_round_e4m3_mx(_p(x), rows, n, _p(y), _p(e)), "round_e4m3_mx")
    return y, e


def e4m3_scale(x: np.ndarray) -> float:
    """Power-of-two scale 2^floor(log2(448 / max|x|)) of one matrix."""
    x = _f32(x)
    s = np.empty(1, dtype=np.float32)
    _check(lib().tsko_e4m3_scale(_p(x), x.size, _p(s)), "e4m3_scale")
    return float(s[0])
