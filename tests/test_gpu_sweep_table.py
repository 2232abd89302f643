"""Per-shape error table: every variant's relative Frobenius error against the full FP64 oracle
on the square sweep N in {128, ..., 8192} (normal(0,1), seed 1000 + log2 N) and on
ill-conditioned operands (normal(0,1) * 2^u, u per entry in [-20, 20]).  Each entry must be
within the variant's stated bound; the table is printed and, when CMP_RESULTS_DIR names a
directory, also written there as error_table.md."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
VARIANTS = ["f32_simt", "bf16x3", "fp8r", "bf16", "fp6x3"]
BOUND = {"f32_simt": 1e-5, "bf16x3": 1e-5, "fp8r": 1e-3, "bf16": 1e-2, "fp6x3": 1e-2}


def _errors(cx, A, B):
    import torch
    ref = oracle.gemm(A, B)
    dA, dB = dev(A), dev(B)
    out = {}
    for name in VARIANTS:
        dC = torch.zeros((A.shape[0], B.shape[1]), device="cuda")
        cx.gemm_variant(cx.variant_find(name), dA, dB, dC)
        out[name] = oracle.relfro(host(dC), ref)
    return out


def test_error_table():
    import paper_2311_03543_amd as pa
    cx = pa.Compar(0)
    cx.register_builtin("fp6x3")
    rows = []
    try:
        for n in synth.square_sweep_sizes():
            say(f"  error table normal N={n}")
            A, B = synth.gemm_operands(n, n, n, seed=synth.square_sweep_seed(n))
            rows.append(("normal(0,1)", n, _errors(cx, A, B)))
        for n in (256, 1024, 4096):
            say(f"  error table ill-conditioned N={n}")
            A = synth.ill_conditioned_matrix(n, n, 40 + n)
            B = synth.ill_conditioned_matrix(n, n, 41 + n)
            rows.append(("normal*2^u", n, _errors(cx, A, B)))
    finally:
        cx.close()
    lines = ["| inputs | N | " + " | ".join(VARIANTS) + " |", "|---|---|" + "---|" * len(VARIANTS)]
    for dist, n, e in rows:
        lines.append(f"| {dist} | {n} | " + " | ".join(f"{e[v]:.2e}" for v in VARIANTS) + " |")
    lines.append("| stated bound | | " + " | ".join(f"{BOUND[v]:.0e}" for v in VARIANTS) + " |")
    text = "\n".join(lines) + "\n"
    out_dir = os.environ.get("CMP_RESULTS_DIR")
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "error_table.md"), "w") as f:
            f.write(text)
    print(text, flush=True)
    for dist, n, e in rows:
        for v in VARIANTS:
            assert e[v] <= BOUND[v], (dist, n, v, e[v])
