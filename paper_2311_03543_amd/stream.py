"""Request-stream driver: many gemm requests of recurring shapes, each with its own tolerance,
served one by one (selection by context, then execution), with the FP64 residual probe
switched on for requests whose operands are ill-conditioned.  `run_stream_native` hands the
whole list to the library's executor (cmp_gemm_stream: the loop, the selection, the waits and
the latency clock are native); `run_stream` calls cmp_gemm once per request from Python.

The stream: `nshapes` shapes with M, N, K log-uniform in [lo, hi] (rank = draw order);
`nreq` requests whose shape rank follows a finite Zipf(s) law; tolerance uniform over the
three classes; a fraction `ill_frac` of requests use ill-conditioned operands
(normal(0,1) * 2^u, u uniform integer in [-20, 20] per entry).  Every shape has a pool of
two well-conditioned and two ill-conditioned operand pairs on the device.
"""
from __future__ import annotations

import time

import numpy as np

import synth


def make_stream(nshapes=50, nreq=10000, lo=64, hi=4096, s=1.1, ill_frac=0.2, seed=5):
    shapes = synth.log_uniform_shapes(nshapes, lo, hi, seed)
    ranks = synth.zipf_ranks(nreq, s, nshapes, seed + 1)
    tols = synth.tol_classes(nreq, seed + 2)
    ill = synth.rng(seed + 3).random(nreq) < ill_frac
    return dict(shapes=shapes, ranks=ranks, tols=tols, ill=ill)


def build_pool(shapes, seed=9, host_arrays=False, device_gen=False):
    """Per shape: {"well": [(A, B)] * 2, "ill": [(A, B)] * 2, "C": C} as device tensors
    (and the host copies when host_arrays, for checking).  device_gen draws the operands
    with torch's seeded generator on the device instead (faster for large pools)."""
    import torch
    pool = []
    g = torch.Generator(device="cuda").manual_seed(seed) if device_gen else None

    def dev_ill(r, c):
        x = torch.randn((r, c), device="cuda", generator=g)
        u = torch.randint(-20, 21, (r, c), device="cuda", generator=g).to(torch.float32)
        return x * torch.exp2(u)

    for i, (M, N, K) in enumerate(shapes):
        M, N, K = int(M), int(N), int(K)
        ent = {"well": [], "ill": [], "host": {"well": [], "ill": []}}
        if device_gen:
            for j in range(2):
                ent["well"].append((torch.randn((M, K), device="cuda", generator=g),
                                    torch.randn((K, N), device="cuda", generator=g)))
                ent["ill"].append((dev_ill(M, K), dev_ill(K, N)))
            ent["C"] = torch.zeros((M, N), dtype=torch.float32, device="cuda")
            pool.append(ent)
            continue
        for j in range(2):
            A, B = synth.gemm_operands(M, N, K, seed=seed * 100000 + 4 * i + j)
            Ai = synth.ill_conditioned_matrix(M, K, seed * 100000 + 4 * i + 2 + 10 * j)
            Bi = synth.ill_conditioned_matrix(K, N, seed * 100000 + 4 * i + 3 + 10 * j)
            ent["well"].append((torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()))
            ent["ill"].append((torch.from_numpy(Ai).cuda(), torch.from_numpy(Bi).cuda()))
            if host_arrays:
                ent["host"]["well"].append((A, B))
                ent["host"]["ill"].append((Ai, Bi))
        ent["C"] = torch.zeros((M, N), dtype=torch.float32, device="cuda")
        pool.append(ent)
    return pool


def requests_of(stream, pool, outputs=None):
    """(A, B, C) per request in stream order; C is the shape's shared output unless
    `outputs` gives one tensor per request."""
    reqs = []
    for i in range(len(stream["ranks"])):
        sh = int(stream["ranks"][i]) - 1
        kind = "ill" if stream["ill"][i] else "well"
        A, B = pool[sh][kind][i % 2]
        reqs.append((A, B, pool[sh]["C"] if outputs is None else outputs[i]))
    return reqs


def run_stream_native(cx, stream, pool, verify_ill=True, outputs=None):
    """Serve every request through cmp_gemm_stream, each complete before the next; returns
    per-request latency (us, host submit to completion, measured by the library), chosen
    variant ids and the context's verify-mode fallback count."""
    reqs = requests_of(stream, pool, outputs)
    verify = np.asarray(stream["ill"], dtype=bool) & bool(verify_ill)
    chosen, lat = cx.gemm_stream(reqs, np.asarray(stream["tols"], dtype=np.float64), verify=verify,
                                 sync=True)
    return lat, chosen, cx.last_verify()[1]


def run_stream(cx, stream, pool, verify_ill=True, on_result=None):
    """Serve every request synchronously; returns per-request latency (us, host submit to
    completion), chosen variant ids and the verify-mode fallback count.  `on_result(i, C)`
    is called after request i completes (C is that shape's output tensor)."""
    import torch
    import paper_2311_03543_amd as pa
    n = len(stream["ranks"])
    lat = np.empty(n)
    chosen = np.empty(n, dtype=np.int64)
    dev_stream = torch.cuda.current_stream()
    for i in range(n):
        sh = int(stream["ranks"][i]) - 1
        kind = "ill" if stream["ill"][i] else "well"
        A, B = pool[sh][kind][i % 2]
        C = pool[sh]["C"]
        cx.set_flags(pa.CMP_FLAG_VERIFY if (verify_ill and stream["ill"][i]) else 0)
        t0 = time.perf_counter()
        chosen[i] = cx.gemm(A, B, C, tol=float(stream["tols"][i]))
        dev_stream.synchronize()
        lat[i] = (time.perf_counter() - t0) * 1e6
        if on_result is not None:
            on_result(i, C)
    cx.set_flags(0)
    return lat, chosen, cx.last_verify()[1]
