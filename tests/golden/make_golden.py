"""Writes the oracle's reference values for the full-size workloads to JSON.

Calls only the FP64 CPU oracle (oracle/) and the seeded stream generator; no
value here comes from the GPU path.  Usage:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle  # noqa: E402
from paper_2209_14637_amd import synth  # noqa: E402


def golden_stream(spec, name, n_err=64, n_opt=16):
    st = synth.Stream(spec)
    t0 = time.time()
    tr = st.train()
    S, lam, fro2 = oracle.train(tr, spec.k, return_fro2=True)
    t_train = time.time() - t0
    del tr
    te = st.test(n_err)
    res = oracle.apply(te, S, spec.r)
    e = res["relerr"]
    if n_opt:
        tail, fro = oracle.opt_tail(te[:n_opt], spec.r)
    else:
        tail = fro = np.zeros(0)
    out = {
        "workload": name,
        "spec": {k: v for k, v in spec.__dict__.items()},
        "source": "oracle/tsko.c via tests/golden/make_golden.py",
        "lambda": lam.tolist(),
        "train_fro2": fro2,
        "relerr": e.tolist(),
        "flags": res["flags"].tolist(),
        "opt_tail": tail.tolist(),
        "fro": fro.tolist(),
        "metric_4_1": ((e[:n_opt] * fro - tail) / tail).tolist(),
        "oracle_train_seconds": t_train,
        "threads": oracle.threads(),
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "lambda_1..3", lam[:3], "e[:3]", e[:3], f"train {t_train:.1f}s")


def golden_batch(name, n_train=100, n_err=4):
    """The uneven-shape batch workload: per stream, the oracle's sketch from
    its training slices and the errors of its first n_err test matrices."""
    out = {"workload": name, "source": "oracle/tsko.c via tests/golden/make_golden.py", "streams": []}
    t0 = time.time()
    for s in range(len(synth.BATCH_SHAPES)):
        spec = synth.spec_batch_stream(s, n_train=n_train)
        st = synth.Stream(spec)
        S, lam = oracle.train(st.train(), spec.k)
        res = oracle.apply(st.test(n_err), S, spec.r)
        out["streams"].append({"spec": {k: v for k, v in spec.__dict__.items()}, "lambda": lam.tolist(),
                               "relerr": res["relerr"].tolist(), "flags": res["flags"].tolist()})
        print(name, "stream", s, spec.m, spec.n, "e[:2]", res["relerr"][:2], flush=True)
    out["oracle_seconds"] = time.time() - t0
    out["threads"] = oracle.threads()
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


WORKLOADS = {
    "batch_8streams_k10-40": lambda: golden_batch("batch_8streams_k10-40"),
    "hsi_1024x768_k20_r10": lambda: golden_stream(synth.spec_hsi_fp32(), "hsi_1024x768_k20_r10"),
    # the precision form's stream: 1000 training slices of 1920 x 1080; the
    # oracle's reference is on the FP32 values (the reduced-precision paths
    # are gated against it at 1e-3)
    "stream_1920x1080_k40_r20": lambda: golden_stream(synth.spec_bf16_1920(), "stream_1920x1080_k40_r20",
                                                      n_err=32, n_opt=0),
    # the e4m3 form's stream: 4000 training slices, Student-t(3) noise at 1e-2
    "t3stream_1920x1080_k40_r20": lambda: golden_stream(synth.spec_fp8_1920(), "t3stream_1920x1080_k40_r20",
                                                        n_err=32, n_opt=0),
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    for nm in names:
        WORKLOADS[nm]()
