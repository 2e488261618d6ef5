"""GEMM launch-shape autotuner.

Every GEMM of the library (the FP64 and FP32 complex GEMMs, the split
16-bit GEMMs of the mixed form) picks its workgroup tile and its split-K
factor by a rule of the output shape.  This module measures instead: it
records the GEMM shapes a workload launches (per-shape event timing of one
step), ranks them by the time they took, and has the library time every
candidate tile and split factor of the heaviest ones
(``tt.gemm_autotune``), which keeps the fastest in the process-wide table
that every later GEMM of that exact shape consults.  Tables can be saved as
JSON and loaded back, so a tuned workload replays the same choices.
"""
import json
import re

from . import tt

_SHAPE = re.compile(r"^(zgemm|zgemm_fp32|zgemm_fp16x3|zgemm_bf16x3):([NTC])([NTC]):(\d+)x(\d+)x(\d+)x(\d+)$")
_PREC = {"zgemm": tt.TT_PREC_FP64, "zgemm_bf16x3": tt.TT_PREC_BF16X3, "zgemm_fp16x3": tt.TT_PREC_FP16X3,
         "zgemm_fp32": tt.TT_PREC_FP32}
_OPS = {"N": 0, "T": 1, "C": 2}


def gemm_shapes(stats, into=None):
    """{(precision, opA, opB, M, N, K, batch): milliseconds} from the stats of
    a context profiled with shapes on (``Context.set_profiling(True,
    shapes=True)``); ``into`` accumulates over several contexts."""
    out = {} if into is None else into
    for key, v in stats.items():
        m = _SHAPE.match(key)
        if not m:
            continue
        k = (_PREC[m[1]], _OPS[m[2]], _OPS[m[3]], int(m[4]), int(m[5]), int(m[6]), int(m[7]))
        out[k] = out.get(k, 0.0) + float(v["ms"])
    return out


def profile_shapes(ctx, run):
    """Shapes and times of the GEMMs that ``run()`` launches on ``ctx``."""
    ctx.reset_stats()
    ctx.set_profiling(True, shapes=True)
    try:
        run()
    finally:
        stats = ctx.dump_stats()
        ctx.set_profiling(False)
        ctx.reset_stats()
    return gemm_shapes(stats)


def tune(ctx, shapes_ms, top=48):
    """Tune the ``top`` shapes with the most time; returns a list of
    (shape, choice, microseconds)."""
    ranked = sorted(shapes_ms.items(), key=lambda kv: -kv[1])
    out = []
    for shape, _ in ranked[:top]:
        prec, oa, ob, m, n, k, b = shape
        if k == 0:
            continue
        choice, us = tt.gemm_autotune(ctx, prec, oa, ob, m, n, k, b)
        out.append((shape, choice, us))
    return out


def save(path):
    with open(path, "w") as fh:
        json.dump({"gemm_table": tt.gemm_table()}, fh)


def load(path):
    with open(path) as fh:
        tt.gemm_table_set(json.load(fh)["gemm_table"])
