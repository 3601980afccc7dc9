"""C-ABI checks that need no GPU: the library builds and loads, and it exports
every entry point include/tsk.h declares (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsk.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tsk_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["tsk_train", "tsk_apply", "tsk_error", "tsk_create", "tsk_destroy", "tsk_gram", "tsk_eig_topk"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2209_14637_amd import tsk
    lib = tsk.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) == set(tsk.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", tsk.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(tsk_[a-z0-9_]+)\b", out))
    assert set(declared_symbols()) <= exported


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2209_14637_amd import tsk
    lib = tsk.load()
    h = ctypes.c_void_p()
    st = lib.tsk_create(ctypes.byref(h), 0, None)
    assert st != tsk.TSK_OK and not h.value


def test_null_context_is_rejected():
    from paper_2209_14637_amd import tsk
    lib = tsk.load()
    assert lib.tsk_train(None, None, 4, tsk.TSK_F32, None, None, None) == tsk.TSK_E_ARG
    assert lib.tsk_apply(None, None, 4, None, 2, tsk.TSK_F32, None, None, None, None, None) == tsk.TSK_E_ARG
    assert lib.tsk_error(None, None, None, None, 2, None) == tsk.TSK_E_ARG
    assert lib.tsk_last_error(None) == b"null context"


def test_autotune_cache_keys():
    from paper_2209_14637_amd import autotune
    key = autotune.class_key(1920, 1080, 40, "bf16")
    assert key == "1920x1080:kp48:bf16"
    assert autotune.parse_key(key) == (1920, 1080, 48, "bf16")
