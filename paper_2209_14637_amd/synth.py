"""Seeded synthetic data streams (inputs only).

This module produces the matrices that both the GPU path and the FP64 CPU
oracle consume. It holds none of the sketching method's arithmetic: no Gram,
no eigensolver, no SCW. It only draws stream matrices and a few structured
test inputs.

Stream model (stand-in for the paper's HSI / Logo / MRI streams, Section 4,
Table 1, which are not available here):

    A_d = U_d diag(sigma) W_d^T + eta * E_d,      d = 1, 2, ...

* U_0   : orthonormal m x rho basis, QR of a Gaussian matrix.
* U_perp: orthonormal m x rho basis of a Gaussian matrix projected off U_0.
* U_d   = cos(theta_d) U_0 + sin(theta_d) U_perp.  Every principal angle
          between span(U_d) and span(U_0) equals theta_d, and the columns
          stay orthonormal (needs m >= 2 rho).
* W_d   : an independent random orthonormal n x rho basis per slice.
* E_d   : i.i.d. standard normal, or Student-t with 3 degrees of freedom.
* sigma : 1-based law, either sigma_i = 2^-i or sigma_i = i^-p.

Training slices are d = 1..n_train, test slices follow in the same stream
(d = n_train+1 .. n_train+n_test).  Every slice is drawn from its own
``numpy.random.SeedSequence([seed, cfg, stream, purpose, d])`` so any slice can
be regenerated alone (purposes: U0=0, Uperp=1, W=2, E=3).  Values are drawn in
float64 and rounded once to float32; that float32 array is THE input, which
the oracle reads exactly (upcast to float64) and the GPU path reads as stored.
"""
from __future__ import annotations

import contextlib
import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

PURPOSE_U0, PURPOSE_UPERP, PURPOSE_W, PURPOSE_E = 0, 1, 2, 3


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(x) for x in key]))


def _single_thread_blas():
    """Context in which BLAS/OpenMP pools run one thread (no-op when
    threadpoolctl is missing)."""
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(1)
    except Exception:
        return contextlib.nullcontext()


def _orth(x: np.ndarray) -> np.ndarray:
    q, _ = np.linalg.qr(x)
    return q


@dataclasses.dataclass(frozen=True)
class StreamSpec:
    m: int
    n: int
    rho: int
    sigma_law: str = "pow"          # "pow2": 2^-i ; "pow": i^-sigma_exp
    sigma_exp: float = 1.5
    eta: float = 1e-3
    noise: str = "gauss"            # "gauss" or "t3"
    theta_scale: float = 0.0        # theta_d = theta_scale * d
    n_train: int = 0
    n_test: int = 0
    k: int = 0
    r: int = 0
    seed: int = 0
    cfg: int = 0
    stream: int = 0

    @property
    def sigma(self) -> np.ndarray:
        i = np.arange(1, self.rho + 1, dtype=np.float64)
        if self.sigma_law == "pow2":
            return 2.0 ** (-i)
        return i ** (-self.sigma_exp)

    def replace(self, **kw) -> "StreamSpec":
        return dataclasses.replace(self, **kw)


class Stream:
    """Generator for one stream; slices are produced on demand."""

    def __init__(self, spec: StreamSpec):
        if spec.m < 2 * spec.rho:
            raise ValueError("drift construction needs m >= 2*rho")
        if spec.n < spec.rho:
            raise ValueError("need n >= rho")
        self.spec = spec
        s = spec
        self.U0 = _orth(_rng(s.seed, s.cfg, s.stream, PURPOSE_U0, 0).standard_normal((s.m, s.rho)))
        x = _rng(s.seed, s.cfg, s.stream, PURPOSE_UPERP, 0).standard_normal((s.m, s.rho))
        x -= self.U0 @ (self.U0.T @ x)
        x -= self.U0 @ (self.U0.T @ x)
        self.Uperp = _orth(x)

    def theta(self, d: int) -> float:
        return self.spec.theta_scale * d

    def signal(self, d: int) -> np.ndarray:
        """Noise-free part U_d diag(sigma) W_d^T in float64."""
        s = self.spec
        th = self.theta(d)
        ud = np.cos(th) * self.U0 + np.sin(th) * self.Uperp
        w = _orth(_rng(s.seed, s.cfg, s.stream, PURPOSE_W, d).standard_normal((s.n, s.rho)))
        return (ud * s.sigma) @ w.T

    def noise(self, d: int) -> np.ndarray:
        s = self.spec
        g = _rng(s.seed, s.cfg, s.stream, PURPOSE_E, d)
        if s.noise == "t3":
            return g.standard_t(3, size=(s.m, s.n))
        return g.standard_normal((s.m, s.n))

    def slice(self, d: int) -> np.ndarray:
        s = self.spec
        a = self.signal(d)
        if s.eta != 0.0:
            a = a + s.eta * self.noise(d)
        return a.astype(np.float32)

    def slices(self, ds, out: np.ndarray | None = None, threads: int | None = None) -> np.ndarray:
        """Slices ds as a (len(ds), m, n) float32 array, drawn by a pool of
        threads (the draws are per-slice, so the result does not depend on
        the split).  Each worker's BLAS runs single-threaded meanwhile, so
        the pool does not oversubscribe the cores; no process is forked, so
        it is safe after GPU work has started."""
        ds = list(ds)
        s = self.spec
        if out is None:
            out = np.empty((len(ds), s.m, s.n), dtype=np.float32)
        nthr = threads or min(16, len(os.sched_getaffinity(0)))

        def work(i):
            out[i] = self.slice(ds[i])

        if nthr <= 1 or len(ds) <= 1:
            for i in range(len(ds)):
                work(i)
        else:
            with _single_thread_blas(), ThreadPoolExecutor(nthr) as ex:
                list(ex.map(work, range(len(ds))))
        return out

    def train(self, count: int | None = None, **kw) -> np.ndarray:
        c = self.spec.n_train if count is None else count
        return self.slices(range(1, c + 1), **kw)

    def test(self, count: int | None = None, start: int = 0, **kw) -> np.ndarray:
        c = self.spec.n_test if count is None else count
        d0 = self.spec.n_train + 1 + start
        return self.slices(range(d0, d0 + c), **kw)


# ---------------------------------------------------------------------------
# Named workloads.  Shapes, laws, ranks and seeds follow the five benchmark
# configurations of this project; the paper's datasets (Table 1) are replaced
# by these synthetic streams.
# ---------------------------------------------------------------------------

def spec_tiny() -> StreamSpec:
    """64x48, 32 train / 16 test, rank-8 law sigma_i = 2^-i, eta 0.01,
    drift 0.01 rad per slice, k=10, r=5."""
    return StreamSpec(m=64, n=48, rho=8, sigma_law="pow2", eta=0.01,
                      theta_scale=0.01, n_train=32, n_test=16, k=10, r=5,
                      seed=0, cfg=1)


def spec_hsi_fp32() -> StreamSpec:
    """1024x768 (the HSI shape), 400 train / 400 test, rank-40 law
    sigma_i = i^-1.5, eta 1e-3, slow drift, k=20, r=10."""
    return StreamSpec(m=1024, n=768, rho=40, sigma_law="pow", sigma_exp=1.5,
                      eta=1e-3, theta_scale=0.48 / 800, n_train=400, n_test=400,
                      k=20, r=10, seed=0, cfg=2)


def spec_bf16_1920() -> StreamSpec:
    """1920x1080, 1000 train / 1000 test, same law, k=40, r=20."""
    return StreamSpec(m=1920, n=1080, rho=40, sigma_law="pow", sigma_exp=1.5,
                      eta=1e-3, theta_scale=0.48 / 2000, n_train=1000, n_test=1000,
                      k=40, r=20, seed=0, cfg=3)


def spec_fp8_1920() -> StreamSpec:
    """1920x1080, 4000 train / 1000 test, Student-t(3) noise at 1e-2, k=40, r=20."""
    return StreamSpec(m=1920, n=1080, rho=40, sigma_law="pow", sigma_exp=1.5,
                      eta=1e-2, noise="t3", theta_scale=0.48 / 5000, n_train=4000,
                      n_test=1000, k=40, r=20, seed=0, cfg=4)


BATCH_SHAPES = [(256, 192), (512, 384), (768, 512), (1024, 768), (1280, 720),
                (1536, 1024), (1920, 1080), (2048, 1536)]


def spec_batch_stream(s: int, n_train: int = 100, n_test: int = 2000) -> StreamSpec:
    """Stream s of the uneven-shape batch workload; k in {10,20,40}, r = k/2."""
    m, n = BATCH_SHAPES[s]
    k = (10, 20, 40)[s % 3]
    return StreamSpec(m=m, n=n, rho=40, sigma_law="pow", sigma_exp=1.5, eta=1e-3,
                      theta_scale=0.48 / (n_train + n_test), n_train=n_train,
                      n_test=n_test, k=k, r=k // 2, seed=0, cfg=5, stream=s)


def batch_order(count: int = 2000, seed: int = 0) -> np.ndarray:
    """Stream id per test slot of the uneven-shape batch workload."""
    return _rng(seed, 5, 99).integers(0, len(BATCH_SHAPES), size=count)


# ---------------------------------------------------------------------------
# Structured inputs for exact tests.
# ---------------------------------------------------------------------------

def integer_stack(count: int, m: int, n: int, seed: int = 0, lo: int = -3, hi: int = 3) -> np.ndarray:
    """Slices with entries in {lo..hi}: every product and partial sum of a Gram
    is an exact integer far below 2^24, so any FP32/BF16/FP8 arithmetic that
    accumulates in FP32 or wider gives the exact value."""
    return _rng(seed, 77, count, m, n).integers(lo, hi + 1, size=(count, m, n)).astype(np.float32)


def gaussian_stack(count: int, m: int, n: int, seed: int = 0) -> np.ndarray:
    return _rng(seed, 78, count, m, n).standard_normal((count, m, n)).astype(np.float32)


def householder_orthogonal(m: int, seed: int = 0, reflectors: int | None = None) -> np.ndarray:
    """Orthogonal m x m matrix as a product of Householder reflectors
    I - 2 v v^T / (v^T v) with Gaussian v (exactly orthogonal up to rounding)."""
    g = _rng(seed, 79, m)
    q = np.eye(m)
    for _ in range(reflectors or m):
        v = g.standard_normal(m)
        q -= np.outer(q @ v, v) * (2.0 / (v @ v))
    return q


def planted_symmetric(lam: np.ndarray, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """G = Q diag(lam) Q^T with Q a Householder product; returns (G, Q)."""
    lam = np.asarray(lam, dtype=np.float64)
    q = householder_orthogonal(lam.size, seed)
    g = (q * lam) @ q.T
    return 0.5 * (g + g.T), q
