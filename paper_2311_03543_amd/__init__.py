"""Python binding of libcompar: runtime selection of GEMM implementation variants on MI355X.

``Compar`` wraps one ``cmp_ctx`` and mirrors the C entry points of
``include/compar.h`` one to one.  Device matrices are torch tensors on a ROCm
device (row-major, unit column stride); torch only supplies device memory and
the current HIP stream.  All arithmetic runs in libcompar.so.
"""
from __future__ import annotations

import ctypes as C
from typing import Callable, Sequence

from . import _lib
from ._lib import (CMP_EDUP, CMP_EHIP, CMP_EINVAL, CMP_ENODATA, CMP_ENOMEM, CMP_ENOTFOUND,  # noqa: F401
                   CMP_ENOVARIANT, CMP_ESIG, CMP_EUNSUPPORTED, CMP_ECHECK, CMP_OK, CMP_F32,
                   CMP_F64, CMP_I32, CMP_I64, CMP_BF16, CMP_F8E4M3, CMP_READ, CMP_WRITE,
                   CMP_READWRITE, CMP_SEL_MLP, CMP_SEL_NN, CMP_SEL_STATIC, CMP_TARGET_HIP,
                   CMP_TARGET_HOST, CMP_FLAG_VERIFY, CMP_FLAG_LOG, ComparError, cmp_context, cmp_gemm_args,
                   cmp_param_desc)

GEMM = b"gemm"
BUILTIN_VARIANTS = ("f32_simt", "bf16x3", "fp8r", "bf16")
# optional built-ins, registered on request (Compar.register_builtin)
OPTIONAL_VARIANTS = ("fp6x3", "host_f32")


def library():
    return _lib.load()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _mat(t, name):
    """(pointer, rows, cols, leading dimension) of a row-major device matrix."""
    if t is None:
        return None, 0, 0, 1
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.numel() == 0:
        return t.data_ptr(), t.shape[0], t.shape[1], max(t.shape[1], 1)
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    ld = max(t.stride(0), t.shape[1], 1)
    return t.data_ptr(), t.shape[0], t.shape[1], ld


def gemm_args(A, B, C_, alpha=1.0, beta=0.0) -> cmp_gemm_args:
    pa, M, K, lda = _mat(A, "A")
    pb, K2, N, ldb = _mat(B, "B")
    pc, M2, N2, ldc = _mat(C_, "C")
    if (M, N) != (M2, N2) or K != K2:
        raise ValueError(f"shape mismatch A {M}x{K}, B {K2}x{N}, C {M2}x{N2}")
    return cmp_gemm_args(M, N, K, lda, ldb, ldc, alpha, beta, pa, pb, pc)


def param(name: str, dtype: int, extents: Sequence[str] = (), mode: int = CMP_READ) -> cmp_param_desc:
    ext = (C.c_char_p * 4)(*[e.encode() for e in extents], *([None] * (4 - len(extents))))
    return cmp_param_desc(name.encode(), dtype, len(extents), ext, mode)


class Compar:
    """One libcompar context (``cmp_init`` / ``cmp_terminate``)."""

    def __init__(self, device: int = 0):
        self.L = _lib.load()
        self.ctx = C.c_void_p()
        st = self.L.cmp_init(device, C.byref(self.ctx))
        if st != CMP_OK:
            raise ComparError(st, f"cmp_init(device={device}) failed")
        self._keep = []      # ctypes callbacks registered with the library

    # ---- lifetime -----------------------------------------------------------
    def close(self):
        if self.ctx:
            self.L.cmp_terminate(self.ctx)
            self.ctx = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != CMP_OK:
            raise ComparError(st, self.L.cmp_last_error(self.ctx).decode())
        return st

    def last_error(self) -> str:
        return self.L.cmp_last_error(self.ctx).decode()

    def device(self):
        dev, cus, clk = C.c_int(), C.c_int(), C.c_int()
        arch = C.create_string_buffer(64)
        self._check(self.L.cmp_device(self.ctx, C.byref(dev), arch, 64, C.byref(cus), C.byref(clk)))
        return dict(device=dev.value, arch=arch.value.decode(), cus=cus.value, clock_khz=clk.value)

    # ---- registry -----------------------------------------------------------
    def interface_declare(self, iface: str, params: Sequence[cmp_param_desc]) -> int:
        arr = (cmp_param_desc * len(params))(*params) if params else None
        return self.L.cmp_interface_declare(self.ctx, iface.encode(), len(params), arr)

    def variant_register(self, iface: str, name: str, target: int, fn: Callable, bound: float,
                         params: Sequence[cmp_param_desc] | None = None,
                         ws: Callable | None = None, user=None):
        """Register a variant; returns (status, id).  ``fn(args_ptr, ws_ptr, ws_bytes, stream,
        user) -> status`` is wrapped in a ctypes callback kept alive by this object."""
        cfn = _lib.cmp_variant_fn(fn)
        cws = _lib.cmp_ws_fn(ws) if ws is not None else C.cast(None, _lib.cmp_ws_fn)
        self._keep += [cfn, cws]
        arr = (cmp_param_desc * len(params))(*params) if params else None
        vid = C.c_int(-1)
        st = self.L.cmp_variant_register(self.ctx, iface.encode(), name.encode(), target,
                                         len(params) if params else 0, arr, cfn, cws, bound,
                                         user, C.byref(vid))
        return st, vid.value

    def variant_count(self, iface: str = "gemm") -> int:
        n = C.c_int()
        self._check(self.L.cmp_variant_count(self.ctx, iface.encode(), C.byref(n)))
        return n.value

    def variant_info(self, vid: int, iface: str = "gemm"):
        name, target, bound = C.c_char_p(), C.c_int(), C.c_double()
        self._check(self.L.cmp_variant_info(self.ctx, iface.encode(), vid, C.byref(name),
                                            C.byref(target), C.byref(bound)))
        return name.value.decode(), target.value, bound.value

    def variant_find(self, name: str, iface: str = "gemm") -> int:
        vid = C.c_int()
        self._check(self.L.cmp_variant_find(self.ctx, iface.encode(), name.encode(), C.byref(vid)))
        return vid.value

    def set_variant_mask(self, mask: int, iface: str = "gemm"):
        self._check(self.L.cmp_set_variant_mask(self.ctx, iface.encode(), mask))

    def force_variant(self, vid: int, iface: str = "gemm"):
        self._check(self.L.cmp_force_variant(self.ctx, iface.encode(), vid))

    # ---- selection ----------------------------------------------------------
    def selector_set(self, kind: int):
        self._check(self.L.cmp_selector_set(self.ctx, kind))

    def set_flags(self, flags: int):
        self._check(self.L.cmp_set_flags(self.ctx, flags))

    def set_log_file(self, path: str | None):
        self._check(self.L.cmp_set_log_file(self.ctx, path.encode() if path else None))

    def log_flush(self):
        self._check(self.L.cmp_log_flush(self.ctx))

    def reserve(self, M: int, N: int, K: int):
        self._check(self.L.cmp_reserve(self.ctx, M, N, K))

    def register_builtin(self, name: str) -> int:
        """Register an optional built-in variant ("fp6x3" or "host_f32"); returns its id."""
        vid = C.c_int(-1)
        self._check(self.L.cmp_register_builtin(self.ctx, name.encode(), C.byref(vid)))
        return vid.value

    def set_split_k(self, splits: int):
        """0: the cost model picks the split-K slice count per call; n >= 1 forces n."""
        self._check(self.L.cmp_set_split_k(self.ctx, splits))

    def split_k(self, vid: int, M: int, N: int, K: int) -> int:
        n = C.c_int()
        self._check(self.L.cmp_split_k(self.ctx, vid, M, N, K, C.byref(n)))
        return n.value

    def admissible(self, M, N, K, tol, iface: str = "gemm") -> int:
        q = cmp_context(M, N, K, CMP_F32, tol)
        m = C.c_uint64()
        self._check(self.L.cmp_admissible(self.ctx, iface.encode(), C.byref(q), C.byref(m)))
        return m.value

    def select(self, M, N, K, tol, iface: str = "gemm") -> int:
        q = cmp_context(M, N, K, CMP_F32, tol)
        vid = C.c_int()
        self._check(self.L.cmp_select(self.ctx, iface.encode(), C.byref(q), C.byref(vid)))
        return vid.value

    def select_batch(self, contexts, iface: str = "gemm") -> list[int]:
        n = len(contexts)
        arr = (cmp_context * n)(*[cmp_context(int(m), int(nn), int(k), CMP_F32, float(t))
                                  for m, nn, k, t in contexts])
        out = (C.c_int * n)()
        self._check(self.L.cmp_select_batch(self.ctx, iface.encode(), n, arr, out))
        return list(out)

    # ---- execution ----------------------------------------------------------
    def gemm(self, A, B, C_, alpha=1.0, beta=0.0, tol=1e-5, stream=None) -> int:
        """C_ = alpha A B + beta C_ with the variant selected for tol; returns its id."""
        a = gemm_args(A, B, C_, alpha, beta)
        chosen = C.c_int(-1)
        self._check(self.L.cmp_gemm(self.ctx, C.byref(a), tol, _stream_ptr(stream), C.byref(chosen)))
        return chosen.value

    def gemm_variant(self, vid: int, A, B, C_, alpha=1.0, beta=0.0, stream=None):
        a = gemm_args(A, B, C_, alpha, beta)
        self._check(self.L.cmp_gemm_variant(self.ctx, vid, C.byref(a), _stream_ptr(stream)))

    def gemm_variant_static(self, vid: int, A, B, C_, alpha=1.0, beta=0.0, stream=None):
        """gemm_variant with the workspace taken from the library's fixed device array
        (cmp_gemm_variant_static: no allocation)."""
        a = gemm_args(A, B, C_, alpha, beta)
        self._check(self.L.cmp_gemm_variant_static(self.ctx, vid, C.byref(a), _stream_ptr(stream)))

    def gemm_raw(self, args: cmp_gemm_args, tol: float, stream=None) -> tuple[int, int]:
        chosen = C.c_int(-1)
        st = self.L.cmp_gemm(self.ctx, C.byref(args), tol, _stream_ptr(stream), C.byref(chosen))
        return st, chosen.value

    def gemm_stream_raw(self, args, tols, verify=None, sync=True, stream=None):
        """cmp_gemm_stream over a list of cmp_gemm_args: returns (status, requests served,
        chosen ids, latencies in us or None)."""
        import numpy as np
        n = len(args)
        arr = (cmp_gemm_args * max(n, 1))(*args)
        t = np.ascontiguousarray(tols, dtype=np.float64)
        if t.shape != (n,):
            raise ValueError("one tolerance per request")
        fl = None
        if verify is not None:
            fl = np.where(np.asarray(verify, dtype=bool), CMP_FLAG_VERIFY, 0).astype(np.uint32)
            if fl.shape != (n,):
                raise ValueError("one verify flag per request")
        chosen = np.full(max(n, 1), -1, np.int32)
        lat = np.zeros(max(n, 1), np.float64)
        done = C.c_int(0)
        st = self.L.cmp_gemm_stream(self.ctx, n, arr, t.ctypes.data_as(C.POINTER(C.c_double)),
                                    None if fl is None else fl.ctypes.data_as(C.POINTER(C.c_uint32)),
                                    1 if sync else 0, _stream_ptr(stream),
                                    chosen.ctypes.data_as(C.POINTER(C.c_int)),
                                    lat.ctypes.data_as(C.POINTER(C.c_double)), C.byref(done))
        return st, done.value, chosen[:n].astype(np.int64), (lat[:n] if sync else None)

    def gemm_stream(self, requests, tols, verify=None, sync=True, stream=None):
        """Serve [(A, B, C[, alpha, beta]), ...] in order in the library (cmp_gemm_stream), each
        request selected by its own tolerance; verify: per-request booleans (None: the
        context's flags).  Returns (chosen ids, latencies in us, or None when sync is False)."""
        st, _, chosen, lat = self.gemm_stream_raw([gemm_args(*r) for r in requests], tols, verify,
                                                  sync, stream)
        self._check(st)
        return chosen, lat

    def call_host(self, iface: str, vid: int, args_ptr) -> int:
        return self.L.cmp_call_host(self.ctx, iface.encode(), vid, args_ptr)

    # ---- timing and history -------------------------------------------------
    def time_variant(self, vid: int, A, B, C_, warmup=3, reps=20, alpha=1.0, beta=0.0, stream=None):
        a = gemm_args(A, B, C_, alpha, beta)
        med, mn, mean = C.c_float(), C.c_float(), C.c_float()
        self._check(self.L.cmp_time_variant(self.ctx, vid, C.byref(a), warmup, reps,
                                            _stream_ptr(stream), C.byref(med), C.byref(mn), C.byref(mean)))
        return med.value, mn.value, mean.value

    def calibrate(self, shapes, A, B, C_, warmup=3, reps=20, stream=None):
        flat = [int(v) for s in shapes for v in s]
        arr = (C.c_int64 * len(flat))(*flat)
        self._check(self.L.cmp_calibrate(self.ctx, len(shapes), arr, A.data_ptr(), B.data_ptr(),
                                         C_.data_ptr(), warmup, reps, _stream_ptr(stream)))

    def history_add(self, M, N, K, vid, reps, med, mn=None, mean=None):
        self._check(self.L.cmp_history_add(self.ctx, M, N, K, vid, reps, med,
                                           med if mn is None else mn, med if mean is None else mean))

    def history(self):
        n = C.c_int()
        self._check(self.L.cmp_history_count(self.ctx, C.byref(n)))
        rows = []
        for r in range(n.value):
            mnk = (C.c_int64 * 3)()
            vid, reps = C.c_int(), C.c_int()
            med, mn, mean = C.c_float(), C.c_float(), C.c_float()
            self._check(self.L.cmp_history_get(self.ctx, r, mnk, C.byref(vid), C.byref(reps),
                                               C.byref(med), C.byref(mn), C.byref(mean)))
            rows.append((mnk[0], mnk[1], mnk[2], vid.value, reps.value, med.value, mn.value, mean.value))
        return rows

    def history_clear(self):
        self._check(self.L.cmp_history_clear(self.ctx))

    def history_save(self, path: str):
        self._check(self.L.cmp_history_save(self.ctx, path.encode()))

    def history_load(self, path: str, force: bool = False) -> int:
        return self.L.cmp_history_load(self.ctx, path.encode(), 1 if force else 0)

    # ---- learned selector ---------------------------------------------------
    @staticmethod
    def _fptr(a):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float32)
        return a, a.ctypes.data_as(C.POINTER(C.c_float))

    def mlp_set_params(self, p):
        a, ptr = self._fptr(p)
        self._check(self.L.cmp_mlp_set_params(self.ctx, ptr, a.size))

    def mlp_get_params(self):
        import numpy as np
        n = self.L.cmp_mlp_param_count()
        out = np.empty(n, np.float32)
        self._check(self.L.cmp_mlp_get_params(self.ctx, out.ctypes.data_as(C.POINTER(C.c_float)), n))
        return out

    def mlp_get_norm(self):
        import numpy as np
        arrs = [np.empty(4, np.float32) for _ in range(4)]
        self._check(self.L.cmp_mlp_get_norm(self.ctx, *[a.ctypes.data_as(C.POINTER(C.c_float)) for a in arrs]))
        return arrs

    def mlp_set_norm(self, mu_x, sd_x, mu_y, sd_y):
        arrs = [self._fptr(a) for a in (mu_x, sd_x, mu_y, sd_y)]
        self._check(self.L.cmp_mlp_set_norm(self.ctx, *[p for _, p in arrs]))

    def mlp_train(self, X, Y, steps, lr):
        import numpy as np
        x, px = self._fptr(X)
        y, py = self._fptr(Y)
        trace = np.empty(max(steps, 1), np.float32)
        self._check(self.L.cmp_mlp_train(self.ctx, x.shape[0], px, py, steps, lr,
                                         trace.ctypes.data_as(C.POINTER(C.c_float))))
        return trace[:steps]

    def mlp_grad(self, Xs, Ys):
        import numpy as np
        x, px = self._fptr(Xs)
        y, py = self._fptr(Ys)
        g = np.empty(self.L.cmp_mlp_param_count(), np.float32)
        loss = C.c_float()
        self._check(self.L.cmp_mlp_grad(self.ctx, x.shape[0], px, py, C.byref(loss),
                                        g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def mlp_infer(self, Xs):
        import numpy as np
        x, px = self._fptr(Xs)
        out = np.empty((x.shape[0], 4), np.float32)
        self._check(self.L.cmp_mlp_infer(self.ctx, x.shape[0], px, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def mlp_save(self, path: str):
        self._check(self.L.cmp_mlp_save(self.ctx, str(path).encode()))

    def mlp_load(self, path: str, force: bool = False):
        self._check(self.L.cmp_mlp_load(self.ctx, str(path).encode(), 1 if force else 0))

    def mlp_fit_history(self, steps=5000, lr=1e-3, seed=0) -> float:
        loss = C.c_float()
        self._check(self.L.cmp_mlp_fit_history(self.ctx, steps, lr, seed, C.byref(loss)))
        return loss.value

    # ---- verification and pre-pass -------------------------------------------
    def freivalds(self, A, B, C_, probe, alpha=1.0, beta=0.0, C0=None, stream=None) -> float:
        import numpy as np
        a = gemm_args(A, B, C_, alpha, beta)
        if C0 is not None:
            p0, m0, n0, ld0 = _mat(C0, "C0")
            if (m0, n0) != (a.M, a.N) or (a.M > 1 and ld0 != a.ldc):
                raise ValueError("C0 must have C's shape and leading dimension")
        x = np.ascontiguousarray(probe, dtype=np.float64)
        est = C.c_double()
        self._check(self.L.cmp_freivalds(self.ctx, C.byref(a), None if C0 is None else C0.data_ptr(),
                                         x.ctypes.data_as(C.POINTER(C.c_double)), _stream_ptr(stream),
                                         C.byref(est)))
        return est.value

    def last_verify(self):
        est, fb = C.c_double(), C.c_int()
        self._check(self.L.cmp_last_verify(self.ctx, C.byref(est), C.byref(fb)))
        return est.value, fb.value

    def split_bf16(self, X, hi, lo=None, stream=None):
        px, r, c, ld = _mat(X, "X")
        self._check(self.L.cmp_split_bf16(self.ctx, r, c, px, ld, hi.data_ptr(),
                                          None if lo is None else lo.data_ptr(), _stream_ptr(stream)))

    def quant_fp8(self, X, q, qscale, rq, rscale, stream=None):
        px, r, c, ld = _mat(X, "X")
        self._check(self.L.cmp_quant_fp8(self.ctx, r, c, px, ld, q.data_ptr(), qscale.data_ptr(),
                                         rq.data_ptr(), rscale.data_ptr(), _stream_ptr(stream)))

    def prepass_layout(self, vid: int, M: int, N: int, K: int) -> dict:
        L = _lib.cmp_image_layout()
        self._check(self.L.cmp_prepass_layout(self.ctx, vid, M, N, K, C.byref(L)))
        return dict(Mp=L.Mp, Np=L.Np, Kp=L.Kp, offset=list(L.offset[:L.count]),
                    bytes=list(L.bytes[:L.count]), total=L.total)

    def prepass_images(self, vid: int, A, B, out, stream=None) -> dict:
        """Run variant ``vid``'s own operand pre-pass on A and B into the uint8 device tensor
        ``out``; returns the layout (offsets of the images in ``out``)."""
        import torch
        pa, M, K, lda = _mat(A, "A")
        pb, K2, N, ldb = _mat(B, "B")
        if K != K2:
            raise ValueError("shape mismatch")
        lay = self.prepass_layout(vid, M, N, K)
        if out.dtype != torch.uint8 or not out.is_contiguous():
            raise ValueError("out must be a contiguous uint8 tensor")
        a = cmp_gemm_args(M, N, K, lda, ldb, N, 1.0, 0.0, pa, pb, None)
        self._check(self.L.cmp_prepass_images(self.ctx, vid, C.byref(a), out.data_ptr(), out.numel(),
                                              _stream_ptr(stream)))
        return lay

    def quant_mx6(self, X, q, qscale, rq, rscale, transpose=False, stream=None):
        px, r, c, ld = _mat(X, "X")
        self._check(self.L.cmp_quant_mx6(self.ctx, r, c, px, ld, 1 if transpose else 0, q.data_ptr(),
                                         qscale.data_ptr(), rq.data_ptr(), rscale.data_ptr(),
                                         _stream_ptr(stream)))

    # ---- per-kernel timing ------------------------------------------------------
    def kernel_timing(self, enable: bool):
        self._check(self.L.cmp_kernel_timing(self.ctx, 1 if enable else 0))

    def kernel_stats(self, reset: bool = False) -> dict:
        """{kernel name: (launches, total ms)} of the built-in variants' launches."""
        out = {}
        i = 0
        while True:
            name = C.create_string_buffer(64)
            n, ms = C.c_longlong(), C.c_double()
            st = self.L.cmp_kernel_stats(self.ctx, i, name, 64, C.byref(n), C.byref(ms))
            if st != CMP_OK:
                break
            out[name.value.decode()] = (n.value, ms.value)
            i += 1
        if reset:
            self.L.cmp_kernel_stats(self.ctx, -1, None, 0, None, None)
        return out

    # ---- grouped launches -----------------------------------------------------
    def grouped_plan(self, problems, config: int = -1, reps: int = 5, stream=None) -> "GroupedPlan":
        """problems: list of (A, B, C[, alpha, beta]) device-tensor tuples."""
        args = [gemm_args(*p) for p in problems]
        arr = (cmp_gemm_args * len(args))(*args)
        plan = C.c_void_p()
        self._check(self.L.cmp_grouped_plan_create(self.ctx, len(args), arr, config, reps,
                                                   _stream_ptr(stream), C.byref(plan)))
        return GroupedPlan(self, plan)


def grouped_configs():
    L = _lib.load()
    out = []
    for i in range(L.cmp_grouped_config_count()):
        bm, bn, bk = C.c_int(), C.c_int(), C.c_int()
        L.cmp_grouped_config_info(i, C.byref(bm), C.byref(bn), C.byref(bk))
        out.append((bm.value, bn.value, bk.value))
    return out


def grouped_config_variant(config: int) -> int:
    """Built-in variant id (0 f32_simt, 1 bf16x3) whose per-problem results a grouped
    configuration reproduces bit for bit."""
    v = C.c_int()
    st = _lib.load().cmp_grouped_config_variant(config, C.byref(v))
    if st:
        raise ComparError(st, f"unknown grouped configuration {config}")
    return v.value


class GroupedPlan:
    """A grouped launch plan (cmp_grouped_plan_*); destroy before its context."""

    def __init__(self, cx: Compar, handle):
        self.cx, self.h = cx, handle

    def info(self):
        import math
        n = self.cx.L.cmp_grouped_config_count()
        cfg, probs, tiles, grid = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        ms = (C.c_float * n)()
        self.cx._check(self.cx.L.cmp_grouped_plan_info(self.h, C.byref(cfg), C.byref(probs), C.byref(tiles),
                                                       C.byref(grid), ms))
        return dict(config=cfg.value, problems=probs.value, tiles=tiles.value, grid=grid.value,
                    config_ms=[None if math.isnan(v) else v for v in ms])

    def launch(self, stream=None):
        self.cx._check(self.cx.L.cmp_grouped_launch(self.h, _stream_ptr(stream)))

    def graph_launch(self, stream=None):
        self.cx._check(self.cx.L.cmp_grouped_graph_launch(self.h, _stream_ptr(stream)))

    def destroy(self):
        if self.h:
            self.cx.L.cmp_grouped_plan_destroy(self.h)
            self.h = C.c_void_p()
