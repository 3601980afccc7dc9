"""Thin ctypes binding of libtsk (include/tsk.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libtsk.so.  torch is used for device memory and the current stream.  There
is no fallback: if the library or a gfx950 GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsk.so")

TSK_OK, TSK_E_ARG, TSK_E_SHAPE, TSK_E_NOMEM, TSK_E_DEVICE, TSK_E_NOCONV = range(6)
TSK_F64, TSK_F32, TSK_BF16, TSK_F8E4M3, TSK_MXE4M3 = range(5)
FLAG_RANKDEF, FLAG_TIE, FLAG_NONFIN = 1, 2, 4
KERNELS = ["gram", "gram_reduce", "eig_iter", "eig_rr", "sketch", "qr", "project", "finish", "error", "stage"]

_STATUS = {0: "TSK_OK", 1: "TSK_E_ARG", 2: "TSK_E_SHAPE", 3: "TSK_E_NOMEM", 4: "TSK_E_DEVICE",
           5: "TSK_E_NOCONV"}

EXPORTS = ["tsk_create", "tsk_destroy", "tsk_set_stream", "tsk_last_error", "tsk_stage", "tsk_stage_mx", "tsk_gram",
           "tsk_eig_topk", "tsk_train", "tsk_random_sketch", "tsk_apply", "tsk_apply_noalloc", "tsk_apply_multi",
           "tsk_apply_multi_plan", "tsk_plan_launch", "tsk_plan_destroy", "tsk_error", "tsk_opt_tail",
           "tsk_set_eig_params", "tsk_set_tuning", "tsk_train2", "tsk_apply2",
           "tsk_timing_enable", "tsk_timing_read"]

_DTYPES = {"f32": TSK_F32, "bf16": TSK_BF16, "e4m3": TSK_F8E4M3, "mxe4m3": TSK_MXE4M3}
SKETCH_KINDS = {"gaussian": 0, "sign": 1, "sparse": 2}


class TskError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Stack(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("scale", ctypes.c_void_p),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("count", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("stride", ctypes.c_int64)]


class Problem(ctypes.Structure):
    _fields_ = [("A", Stack), ("S", ctypes.c_void_p), ("k", ctypes.c_int32), ("r", ctypes.c_int32),
                ("L", ctypes.c_void_p), ("R", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("relerr", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


_lib = None


def load(path: str | None = None):
    """Load libtsk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built: run paper_2209_14637_amd/build.py")
    L = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sp = ctypes.POINTER(Stack)
    sig = {
        "tsk_create": ([ctypes.POINTER(P), ctypes.c_int, P], I32),
        "tsk_destroy": ([P], None),
        "tsk_set_stream": ([P, P], I32),
        "tsk_last_error": ([P], ctypes.c_char_p),
        "tsk_stage": ([P, sp, I32, P, I64, I64, P, P], I32),
        "tsk_stage_mx": ([P, sp, P, I64, I64, P], I32),
        "tsk_gram": ([P, sp, I32, P], I32),
        "tsk_eig_topk": ([P, P, I64, I32, P, P, P], I32),
        "tsk_train": ([P, sp, I32, I32, P, P, P], I32),
        "tsk_random_sketch": ([P, I32, I32, I64, ctypes.c_uint64, P], I32),
        "tsk_apply": ([P, P, I32, sp, I32, I32, P, P, P, P, P], I32),
        "tsk_apply_noalloc": ([P, P, I32, sp, I32, I32, P, P, P, P, P], I32),
        "tsk_apply_multi": ([P, ctypes.POINTER(Problem), I32, I32], I32),
        "tsk_apply_multi_plan": ([P, ctypes.POINTER(Problem), I32, I32, ctypes.POINTER(P)], I32),
        "tsk_plan_launch": ([P, ctypes.POINTER(P), I32], I32),
        "tsk_plan_destroy": ([P], None),
        "tsk_error": ([P, sp, P, P, I32, P], I32),
        "tsk_opt_tail": ([P, sp, I32, P, P], I32),
        "tsk_set_eig_params": ([P, I32, I32, D, I32], I32),
        "tsk_set_tuning": ([P, I64, I64, I32, I32, I32, I32], I32),
        "tsk_train2": ([P, sp, I32, I32, I32, D, P, P, P, P], I32),
        "tsk_apply2": ([P, P, I32, P, I32, sp, I32, I32, P, P, P, P, P], I32),
        "tsk_timing_enable": ([P, I32], I32),
        "tsk_timing_read": ([P, I32, P, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class Staged:
    """A stack in a reduced-precision storage format: `data` holds the raw
    elements (torch.bfloat16 for bf16, torch.uint8 bytes for e4m3 and
    mxe4m3) as (count, m, ld); `scale` is the per-slice e4m3 scale (float32),
    the per-block exponents of mxe4m3 (uint8, (count, m, ceil(n / 32))), or
    None for bf16."""

    def __init__(self, data: torch.Tensor, n: int, dtype: str, scale: torch.Tensor | None = None):
        self.data, self.n, self.dtype, self.scale = data, n, dtype, scale

    @property
    def shape(self):
        return (self.data.shape[0], self.data.shape[1], self.n)


def _stack(A) -> Stack:
    if isinstance(A, Staged):
        t = A.data
        if not t.is_cuda or t.dim() != 3 or t.stride(2) != 1:
            raise ValueError("staged data must be a (count, m, ld) CUDA tensor")
        cnt, m, _ = t.shape
        return Stack(t.data_ptr(), _DTYPES[A.dtype], _ptr(A.scale), m, A.n, cnt, t.stride(1),
                     t.stride(0) if cnt > 1 else m * t.stride(1))
    if not isinstance(A, torch.Tensor) or not A.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if A.dtype == torch.float32:
        dt = TSK_F32
    elif A.dtype == torch.bfloat16:
        dt = TSK_BF16
    else:
        raise TypeError("expected float32 or bfloat16 slices")
    if A.dim() == 2:
        A = A.unsqueeze(0)
    if A.dim() != 3 or A.stride(2) != 1:
        raise ValueError("expected a (count, m, n) stack with unit column stride")
    cnt, m, n = A.shape
    return Stack(A.data_ptr(), dt, None, m, n, cnt, A.stride(1), A.stride(0) if cnt > 1 else m * A.stride(1))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """A captured batch (tsk_apply_multi_plan); `outs` are its problems'
    output dicts, `keep` holds the inputs it reads."""

    def __init__(self, ctx, h, outs, keep):
        self.ctx, self.h, self.outs, self.keep = ctx, h, outs, keep

    def launch(self):
        self.ctx.launch_plans([self])
        return self.outs

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tsk_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One libtsk context bound to a device; enqueues on torch's current stream."""

    def __init__(self, device: int = 0, tuning: str | None = "default"):
        """tuning: an autotuner cache to apply ("default": the package's
        tune_cache.json, measured on MI355X; None: no tuning entries)."""
        self.lib = load()
        self.device = device
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            st = self.lib.tsk_create(ctypes.byref(h), device, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        if st != TSK_OK:
            raise TskError(st, "tsk_create failed (no gfx950 device?)")
        self.h = h
        if tuning is not None:
            self.load_tuning(None if tuning == "default" else tuning)

    def close(self):
        if getattr(self, "h", None):
            self.lib.tsk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        self.lib.tsk_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, st: int, allow_noconv: bool = False) -> int:
        if st == TSK_OK or (allow_noconv and st == TSK_E_NOCONV):
            return st
        raise TskError(st, self.lib.tsk_last_error(self.h).decode())

    # --- entry points -----------------------------------------------------
    def stage(self, A: torch.Tensor, dtype: str = "bf16", norm2: bool = False):
        """Round an FP32 stack into a storage format ("bf16", "e4m3", or
        "mxe4m3": e4m3 with a scale per 32 elements of a row); returns a
        Staged stack (and ||A_d||^2 of the source when norm2; not for
        mxe4m3)."""
        self._sync_stream()
        s = _stack(A)
        if s.dtype != TSK_F32:
            raise TypeError("stage() takes an FP32 stack")
        # rows start on 128-byte cache lines: with a stride that is only a
        # multiple of 16 bytes, a 256-byte row segment spans three lines and
        # the streaming kernels lose about a quarter of their read rate
        per128 = 64 if dtype == "bf16" else 128
        ld = (s.n + per128 - 1) // per128 * per128
        tdt = torch.bfloat16 if dtype == "bf16" else torch.uint8
        dev = A.device
        out = torch.empty((s.count, s.m, ld), dtype=tdt, device=dev)
        if dtype == "mxe4m3":
            if norm2:
                raise ValueError("norm2 is not available for mxe4m3 staging")
            bs = torch.empty((s.count, s.m, (s.n + 31) // 32), dtype=torch.uint8, device=dev)
            self._check(self.lib.tsk_stage_mx(self.h, ctypes.byref(s), _ptr(out), ld, s.m * ld, _ptr(bs)))
            return Staged(out, s.n, dtype, bs)
        scale = torch.empty(s.count, dtype=torch.float32, device=dev) if dtype == "e4m3" else None
        nrm = torch.empty(s.count, dtype=torch.float64, device=dev) if norm2 else None
        self._check(self.lib.tsk_stage(self.h, ctypes.byref(s), _DTYPES[dtype], _ptr(out), ld, s.m * ld,
                                       _ptr(scale), _ptr(nrm)))
        st = Staged(out, s.n, dtype, scale)
        return (st, nrm) if norm2 else st

    def gram(self, A, G: torch.Tensor | None = None, compute: str = "f32") -> torch.Tensor:
        self._sync_stream()
        s = _stack(A)
        dev = (A.data if isinstance(A, Staged) else A).device
        if G is None:
            G = torch.empty((s.m, s.m), dtype=torch.float64, device=dev)
        self._check(self.lib.tsk_gram(self.h, ctypes.byref(s), _DTYPES[compute], _ptr(G)))
        return G

    def eig_topk(self, G: torch.Tensor, k: int, S: torch.Tensor | None = None, allow_noconv: bool = False):
        self._sync_stream()
        m = G.shape[0]
        if G.dtype != torch.float64 or G.shape != (m, m) or not G.is_contiguous():
            raise ValueError("G must be a contiguous (m, m) float64 CUDA tensor")
        if S is None:
            S = torch.empty((k, m), dtype=torch.float32, device=G.device)
        lam = (ctypes.c_double * (k + 1))()
        it = ctypes.c_int32(0)
        st = self._check(self.lib.tsk_eig_topk(self.h, _ptr(G), m, k, _ptr(S), lam, ctypes.byref(it)), allow_noconv)
        return S, list(lam), it.value, st

    def train(self, A, k: int, S: torch.Tensor | None = None, allow_noconv: bool = False, compute: str = "f32"):
        self._sync_stream()
        s = _stack(A)
        dev = (A.data if isinstance(A, Staged) else A).device
        if S is None:
            S = torch.empty((k, s.m), dtype=torch.float32, device=dev)
        lam = (ctypes.c_double * (k + 1))()
        it = ctypes.c_int32(0)
        st = self._check(self.lib.tsk_train(self.h, ctypes.byref(s), k, _DTYPES[compute], _ptr(S), lam,
                                            ctypes.byref(it)), allow_noconv)
        return S, list(lam), it.value, st

    def random_sketch(self, kind: str, k: int, m: int, seed: int = 0) -> torch.Tensor:
        """Data-free k x m sketch ("gaussian", "sign" or "sparse") of the SCW
        baseline, generated on the GPU (tsk_random_sketch)."""
        self._sync_stream()
        S = torch.empty((k, m), dtype=torch.float32, device=f"cuda:{self.device}")
        self._check(self.lib.tsk_random_sketch(self.h, SKETCH_KINDS[kind], k, m, seed, _ptr(S)))
        return S

    def apply(self, S: torch.Tensor, A, r: int, out: dict | None = None, relerr: bool = True,
              flags: bool = True, noalloc: bool = False) -> dict:
        """SCW on every slice; the arithmetic follows the stack's format
        (FP32 tensor, bfloat16 tensor or a Staged stack).  noalloc: through
        tsk_apply_noalloc (the library's fixed scratch, no device allocation
        by the library; the outputs here are still torch tensors unless
        `out` supplies them)."""
        self._sync_stream()
        s = _stack(A)
        k = S.shape[0]
        if S.dtype != torch.float32 or not S.is_contiguous() or S.shape[1] != s.m:
            raise ValueError("S must be a contiguous (k, m) float32 CUDA tensor")
        dev = S.device
        o = out if out is not None else {}
        if "L" not in o:
            o["L"] = torch.empty((s.count, s.m, r), dtype=torch.float32, device=dev)
            o["R"] = torch.empty((s.count, s.n, r), dtype=torch.float32, device=dev)
            o["sigma"] = torch.empty((s.count, r), dtype=torch.float32, device=dev)
            o["relerr"] = torch.empty(s.count, dtype=torch.float64, device=dev) if relerr else None
            o["flags"] = torch.empty(s.count, dtype=torch.int32, device=dev) if flags else None
        fn = self.lib.tsk_apply_noalloc if noalloc else self.lib.tsk_apply
        self._check(fn(self.h, _ptr(S), k, ctypes.byref(s), r, s.dtype, _ptr(o["L"]), _ptr(o["R"]),
                       _ptr(o["sigma"]), _ptr(o.get("relerr")), _ptr(o.get("flags"))))
        return o

    @staticmethod
    def _outputs(s, r, dev, relerr=True, flags=True):
        return {"L": torch.empty((s.count, s.m, r), dtype=torch.float32, device=dev),
                "R": torch.empty((s.count, s.n, r), dtype=torch.float32, device=dev),
                "sigma": torch.empty((s.count, r), dtype=torch.float32, device=dev),
                "relerr": torch.empty(s.count, dtype=torch.float64, device=dev) if relerr else None,
                "flags": torch.empty(s.count, dtype=torch.int32, device=dev) if flags else None}

    def _problem_array(self, problems, outs):
        n = len(problems)
        arr = (Problem * n)()
        res, keep, dts = [], [], set()
        for i, (S, A, r) in enumerate(problems):
            s = _stack(A)
            dts.add(s.dtype)
            if S.dtype != torch.float32 or not S.is_contiguous() or S.shape[1] != s.m:
                raise ValueError("S must be a contiguous (k, m) float32 CUDA tensor")
            o = outs[i] if outs is not None else self._outputs(s, r, S.device)
            opt = [o[key].data_ptr() if o.get(key) is not None else None for key in ("relerr", "flags")]
            arr[i] = Problem(s, S.data_ptr(), S.shape[0], r, o["L"].data_ptr(), o["R"].data_ptr(),
                             o["sigma"].data_ptr(), opt[0], opt[1])
            res.append(o)
            keep.append((S, A))
        if len(dts) != 1:
            raise ValueError("all problems of a batch must have the same format")
        return arr, res, keep, dts.pop()

    def plan_multi(self, problems, outs: list | None = None) -> "Plan":
        """Captured batch (tsk_apply_multi_plan): runs the batch once and
        returns a Plan whose launch() replays it on the same buffers."""
        self._sync_stream()
        arr, res, keep, dt = self._problem_array(problems, outs)
        h = ctypes.c_void_p()
        self._check(self.lib.tsk_apply_multi_plan(self.h, arr, len(problems), dt, ctypes.byref(h)))
        return Plan(self, h, res, keep)

    def launch_plans(self, plans):
        """Replay several plans together (tsk_plan_launch)."""
        self._sync_stream()
        arr = (ctypes.c_void_p * len(plans))(*[p.h for p in plans])
        self._check(self.lib.tsk_plan_launch(self.h, arr, len(plans)))

    def apply_multi(self, problems, outs: list | None = None) -> list:
        """SCW on a batch of problems [(S, A, r), ...] of different shapes
        (tsk_apply_multi); every A must have the same format.  Returns one
        output dict per problem (reusing `outs` when given)."""
        self._sync_stream()
        n = len(problems)
        arr = (Problem * n)()
        res, keep, dts = [], [], set()
        for i, (S, A, r) in enumerate(problems):
            s = _stack(A)
            dts.add(s.dtype)
            if S.dtype != torch.float32 or not S.is_contiguous() or S.shape[1] != s.m:
                raise ValueError("S must be a contiguous (k, m) float32 CUDA tensor")
            o = outs[i] if outs is not None else self._outputs(s, r, S.device)
            opt = [o[key].data_ptr() if o.get(key) is not None else None for key in ("relerr", "flags")]
            arr[i] = Problem(s, S.data_ptr(), S.shape[0], r, o["L"].data_ptr(), o["R"].data_ptr(),
                             o["sigma"].data_ptr(), opt[0], opt[1])
            res.append(o)
            keep.append((S, A))
        if len(dts) != 1:
            raise ValueError("all problems of a batch must have the same format")
        self._check(self.lib.tsk_apply_multi(self.h, arr, n, dts.pop()))
        return res

    def error(self, A: torch.Tensor, L: torch.Tensor, R: torch.Tensor, relerr: torch.Tensor | None = None):
        self._sync_stream()
        s = _stack(A)
        r = L.shape[-1]
        if relerr is None:
            relerr = torch.empty(s.count, dtype=torch.float64, device=A.device)
        self._check(self.lib.tsk_error(self.h, ctypes.byref(s), _ptr(L), _ptr(R), r, _ptr(relerr)))
        return relerr

    def opt_tail(self, A, r: int):
        """||A_d - [A_d]_r||_F and ||A_d||_F of every slice (numpy arrays),
        for metric (4.1)."""
        import numpy as np
        self._sync_stream()
        s = _stack(A)
        tail = np.empty(s.count)
        fro = np.empty(s.count)
        self._check(self.lib.tsk_opt_tail(self.h, ctypes.byref(s), r, tail.ctypes.data_as(ctypes.c_void_p),
                                          fro.ctypes.data_as(ctypes.c_void_p)))
        return tail, fro

    def train2(self, A: torch.Tensor, k: int, l: int, max_sweeps: int = 50, tol: float = 1e-10):
        """Two-sided training (tsk_train2): (S, W, core2 per sweep, sweeps)."""
        import numpy as np
        self._sync_stream()
        s = _stack(A)
        S = torch.empty((k, s.m), dtype=torch.float32, device=A.device)
        W = torch.empty((l, s.n), dtype=torch.float32, device=A.device)
        core2 = np.zeros(max(max_sweeps, 1))
        sw = ctypes.c_int32(0)
        self._check(self.lib.tsk_train2(self.h, ctypes.byref(s), k, l, max_sweeps, tol, _ptr(S), _ptr(W),
                                        core2.ctypes.data_as(ctypes.c_void_p), ctypes.byref(sw)))
        return S, W, core2[:sw.value], sw.value

    def apply2(self, S: torch.Tensor, W: torch.Tensor, A, r: int, out: dict | None = None) -> dict:
        """Two-sided SCW on every slice (tsk_apply2)."""
        self._sync_stream()
        s = _stack(A)
        for X, dim in ((S, s.m), (W, s.n)):
            if X.dtype != torch.float32 or not X.is_contiguous() or X.shape[1] != dim:
                raise ValueError("S (k x m) and W (l x n) must be contiguous float32 CUDA tensors")
        o = out if out is not None else self._outputs(s, r, S.device)
        self._check(self.lib.tsk_apply2(self.h, _ptr(S), S.shape[0], _ptr(W), W.shape[0], ctypes.byref(s), r, s.dtype,
                                        _ptr(o["L"]), _ptr(o["R"]), _ptr(o["sigma"]), _ptr(o.get("relerr")),
                                        _ptr(o.get("flags"))))
        return o

    def set_tuning(self, m: int, n: int, k: int, dtype: str, groups: int = 0, pj_cols: int = 0):
        """Tuning entry of one shape class (tsk_set_tuning)."""
        self._check(self.lib.tsk_set_tuning(self.h, m, n, k, _DTYPES[dtype], groups, pj_cols))

    def load_tuning(self, path: str | None = None) -> int:
        """Apply every entry of an autotuner cache (JSON, see autotune.py);
        returns the number of entries applied (0 when the file is absent)."""
        from . import autotune
        return autotune.apply_cache(self, path)

    def set_eig_params(self, block: int = 0, max_iter: int = 0, tol: float = 0.0, check: int = 0):
        self._check(self.lib.tsk_set_eig_params(self.h, block, max_iter, tol, check))

    def timing(self, on=True):
        """True: time every kernel class; False: off; or an iterable of class
        names (see KERNELS) to time only those."""
        if on is True:
            mask = -1
        elif not on:
            mask = 0
        else:
            mask = 0
            for name in on:
                mask |= 1 << KERNELS.index(name)
        self._check(self.lib.tsk_timing_enable(self.h, mask))

    def timing_read(self, reset: bool = True) -> dict:
        n = len(KERNELS)
        la = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        self._check(self.lib.tsk_timing_read(self.h, 1 if reset else 0, la, ms))
        return {KERNELS[i]: (la[i], ms[i]) for i in range(n)}
