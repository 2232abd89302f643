"""The C-ABI library on the CPU: exports, registry semantics, selection rules and history.

No GPU is touched: contexts are host-only (device -1) and the variants are
host functions registered through the ABI, as the runtime allows for any
interface.  Selection results are compared one by one with the oracle's plain
rules (oracle.selection), which are index results and must agree exactly.
"""
import ctypes as C
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import synth
from oracle import selection as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "compar.h")

pa = pytest.importorskip("paper_2311_03543_amd")
from paper_2311_03543_amd import _lib  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmp_[a-z0-9_]+)\s*\(", text)) - {"cmp_variant_fn", "cmp_ws_fn"})


def test_every_declared_symbol_is_exported():
    L = _lib.load()
    names = declared_functions()
    assert len(names) >= 40
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares exactly that set
    assert set(_lib.SIGNATURES) == set(names)


def test_version_and_status_strings():
    L = _lib.load()
    assert L.cmp_version().decode().startswith("compar-mi355x")
    assert L.cmp_status_string(-2).decode() == "CMP_EDUP"


def host_ctx():
    return pa.Compar(device=-1)


def _noop(args, ws, wsb, stream, user):
    return 0


def test_host_context_has_gemm_interface_and_no_gpu_variants():
    c = host_ctx()
    assert c.variant_count("gemm") == 0
    assert c.device()["arch"] == "host"
    st = c.L.cmp_gemm_variant(c.ctx, 0, None, None)
    assert st == pa.CMP_EINVAL


def test_registry_errors():
    c = host_ctx()
    P = [pa.param("arr", pa.CMP_F32, ["n"], pa.CMP_READWRITE), pa.param("n", pa.CMP_I32)]
    assert c.interface_declare("sort", P) == 0
    assert c.interface_declare("sort", P) == pa.CMP_EDUP                     # duplicate interface
    dup = [pa.param("x", pa.CMP_F32), pa.param("x", pa.CMP_F32)]
    assert c.interface_declare("other", dup) == pa.CMP_EDUP                  # duplicate parameter
    bad = [pa.param("a", pa.CMP_F32, ["nope"])]
    assert c.interface_declare("bad", bad) == pa.CMP_EINVAL                  # extent names nothing
    st, i0 = c.variant_register("sort", "bubble", pa.CMP_TARGET_HOST, _noop, 1e-5)
    assert st == 0 and i0 == 0                                               # shares the signature
    st, _ = c.variant_register("sort", "bubble", pa.CMP_TARGET_HOST, _noop, 1e-5)
    assert st == pa.CMP_EDUP                                                 # duplicate variant
    wrong = [pa.param("arr", pa.CMP_F64, ["n"], pa.CMP_READWRITE), pa.param("n", pa.CMP_I32)]
    st, _ = c.variant_register("sort", "merge", pa.CMP_TARGET_HOST, _noop, 1e-5, params=wrong)
    assert st == pa.CMP_ESIG                                                 # signature mismatch
    st, i1 = c.variant_register("sort", "merge", pa.CMP_TARGET_HOST, _noop, 1e-5, params=P)
    assert st == 0 and i1 == 1                                               # identical list is fine
    st, _ = c.variant_register("nosuch", "v", pa.CMP_TARGET_HOST, _noop, 1e-5)
    assert st == pa.CMP_ENOTFOUND                                            # undeclared, no params
    st, _ = c.variant_register("sort", "gpu", pa.CMP_TARGET_HIP, _noop, 1e-5)
    assert st == pa.CMP_EUNSUPPORTED                                         # HIP variant, no GPU
    st, _ = c.variant_register("sort", "neg", pa.CMP_TARGET_HOST, _noop, 0.0)
    assert st == pa.CMP_EINVAL                                               # bound must be > 0
    # a first variant may declare the interface itself
    st, j = c.variant_register("scale", "seq", pa.CMP_TARGET_HOST, _noop, 1e-5,
                               params=[pa.param("v", pa.CMP_F64, ["m"], pa.CMP_READWRITE),
                                       pa.param("m", pa.CMP_I64)])
    assert st == 0 and j == 0
    assert c.variant_info(1, "sort") == ("merge", pa.CMP_TARGET_HOST, 1e-5)
    assert c.variant_find("merge", "sort") == 1


def register_fakes(c, names=("f32_simt", "bf16x3", "fp8r", "bf16"), bounds=(1e-5, 1e-5, 1e-3, 1e-2)):
    calls = []

    def make(i):
        def fn(args, ws, wsb, stream, user):
            calls.append(i)
            return 0
        return fn
    for i, (n, b) in enumerate(zip(names, bounds)):
        st, vid = c.variant_register("gemm", n, pa.CMP_TARGET_HOST, make(i), b)
        assert st == 0 and vid == i
    return calls


def test_admissibility_masks():
    c = host_ctx()
    register_fakes(c)
    assert c.admissible(64, 64, 64, 1e-5) == 0b0011
    assert c.admissible(64, 64, 64, 1e-3) == 0b0111
    assert c.admissible(64, 64, 64, 1e-2) == 0b1111
    with pytest.raises(pa.ComparError) as e:
        c.select(64, 64, 64, 1e-8)
    assert e.value.status == pa.CMP_ENOVARIANT
    with pytest.raises(pa.ComparError) as e:
        c.select(64, 64, 64, 0.0)
    assert e.value.status == pa.CMP_EINVAL


BOUNDS = [1e-5, 1e-5, 1e-3, 1e-2]


def _table(nshapes, seed):
    shapes = synth.log_uniform_shapes(nshapes, 64, 8192, seed)
    g = synth.rng(seed + 1)
    T = g.uniform(0.01, 5.0, (nshapes, 4)).astype(np.float32).astype(np.float64)
    return shapes, T


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_nn_selector_matches_oracle(seed):
    c = host_ctx()
    register_fakes(c)
    shapes, T = _table(300, seed)
    for s, (m, n, k) in enumerate(shapes):
        for v in range(4):
            c.history_add(int(m), int(n), int(k), v, 20, float(T[s, v]))
    c.selector_set(pa.CMP_SEL_NN)
    q = synth.log_uniform_shapes(200, 32, 16384, seed + 50)
    tols = synth.tol_classes(200, seed + 60)
    got = c.select_batch([(m, n, k, t) for (m, n, k), t in zip(q, tols)])
    ref = [S.nn_select(shapes, T, BOUNDS, int(m), int(n), int(k), t) for (m, n, k), t in zip(q, tols)]
    assert got == ref
    # one-at-a-time selection agrees with the batch (and the decision cache)
    for i in range(0, 200, 17):
        assert c.select(int(q[i][0]), int(q[i][1]), int(q[i][2]), float(tols[i])) == ref[i]


def test_static_selector_matches_oracle():
    c = host_ctx()
    register_fakes(c)
    shapes, T = _table(100, 9)
    for s, (m, n, k) in enumerate(shapes):
        for v in range(4):
            c.history_add(int(m), int(n), int(k), v, 20, float(T[s, v]))
    c.selector_set(pa.CMP_SEL_STATIC)
    for tol in synth.TOL_CLASSES:
        ref = S.static_choice(T, BOUNDS, tol)
        assert c.select(100, 200, 300, tol) == ref


def test_nn_on_recorded_shapes_is_exhaustive_best():
    c = host_ctx()
    register_fakes(c)
    shapes, T = _table(80, 4)
    for s, (m, n, k) in enumerate(shapes):
        for v in range(4):
            c.history_add(int(m), int(n), int(k), v, 20, float(T[s, v]))
    tols = synth.tol_classes(80, 5)
    got = c.select_batch([(m, n, k, t) for (m, n, k), t in zip(shapes, tols)])
    assert S.regret(T, got, tols, BOUNDS)["aggregate"] == 0.0


def test_no_history_falls_back_to_static_order():
    c = host_ctx()
    register_fakes(c)
    # no data: tightest bound, then lowest id
    assert c.select(128, 128, 128, 1e-2) == 0
    assert c.select(128, 128, 128, 1e-3) == 0


def test_mask_and_force():
    c = host_ctx()
    register_fakes(c)
    c.set_variant_mask(0b1100)
    assert c.admissible(8, 8, 8, 1e-2) == 0b1100
    with pytest.raises(pa.ComparError):
        c.select(8, 8, 8, 1e-5)
    c.set_variant_mask(~0 & 0xFFFFFFFFFFFFFFFF)
    c.force_variant(3)
    assert c.select(8, 8, 8, 1e-2) == 3
    with pytest.raises(pa.ComparError):
        c.select(8, 8, 8, 1e-3)        # forced variant does not meet the tolerance
    c.force_variant(-1)
    assert c.select(8, 8, 8, 1e-3) == 0


def _host_gemm_args(A, B, Cm, alpha=1.0, beta=0.0):
    M, K = A.shape
    N = B.shape[1]
    return pa.cmp_gemm_args(M, N, K, K, N, N, alpha, beta, A.ctypes.data, B.ctypes.data, Cm.ctypes.data)


def test_gemm_dispatch_to_host_variants_and_fallback():
    c = host_ctx()
    ran = []

    def matmul(i, fail=False):
        def fn(args, ws, wsb, stream, user):
            a = pa.cmp_gemm_args.from_address(args)
            ran.append(i)
            if fail:
                return pa.CMP_EHIP
            A = np.ctypeslib.as_array(C.cast(a.A, C.POINTER(C.c_float)), (a.M, a.lda))
            B = np.ctypeslib.as_array(C.cast(a.B, C.POINTER(C.c_float)), (a.K, a.ldb))
            Cm = np.ctypeslib.as_array(C.cast(a.C, C.POINTER(C.c_float)), (a.M, a.ldc))
            Cm[:, :a.N] = a.alpha * (A[:, :a.K] @ B[:, :a.N]) + (a.beta * Cm[:, :a.N] if a.beta else 0)
            return 0
        return fn
    assert c.variant_register("gemm", "exact", pa.CMP_TARGET_HOST, matmul(0), 1e-5)[0] == 0
    assert c.variant_register("gemm", "broken", pa.CMP_TARGET_HOST, matmul(1, fail=True), 1e-3)[0] == 0
    c.history_add(16, 16, 16, 0, 1, 5.0)
    c.history_add(16, 16, 16, 1, 1, 1.0)          # broken is "faster"
    A, B = synth.gemm_operands(16, 16, 16, seed=1)
    Cm = np.zeros((16, 16), np.float32)
    st, chosen = c.gemm_raw(_host_gemm_args(A, B, Cm), 1e-3, stream=0)
    assert st == 0 and chosen == 0 and ran == [1, 0]  # tried the broken one, fell back once
    assert np.allclose(Cm, A @ B, rtol=1e-5, atol=1e-5)
    st, chosen = c.gemm_raw(_host_gemm_args(A, B, Cm), 1e-5, stream=0)
    assert st == 0 and chosen == 0


def test_request_stream_selects_per_request_and_stops_at_a_failure():
    """cmp_gemm_stream serves requests in order, each selected by its own tolerance exactly as
    cmp_select chooses it; a request no variant admits ends the stream with its status and the
    count of requests served before it."""
    c = host_ctx()
    ran = []

    def matmul(i):
        def fn(args, ws, wsb, stream, user):
            a = pa.cmp_gemm_args.from_address(args)
            ran.append(i)
            A = np.ctypeslib.as_array(C.cast(a.A, C.POINTER(C.c_float)), (a.M, a.lda))
            B = np.ctypeslib.as_array(C.cast(a.B, C.POINTER(C.c_float)), (a.K, a.ldb))
            Cm = np.ctypeslib.as_array(C.cast(a.C, C.POINTER(C.c_float)), (a.M, a.ldc))
            Cm[:, :a.N] = a.alpha * (A[:, :a.K] @ B[:, :a.N]) + (a.beta * Cm[:, :a.N] if a.beta else 0)
            return 0
        return fn
    assert c.variant_register("gemm", "exact", pa.CMP_TARGET_HOST, matmul(0), 1e-5)[:2] == (0, 0)
    assert c.variant_register("gemm", "quick", pa.CMP_TARGET_HOST, matmul(1), 1e-2)[:2] == (0, 1)
    c.history_add(16, 24, 8, 0, 1, 5.0)
    c.history_add(16, 24, 8, 1, 1, 1.0)
    tols = [1e-5, 1e-2, 1e-3, 1e-2, 1e-5, 0.5]
    ops = [synth.gemm_operands(16, 24, 8, seed=40 + i) for i in range(len(tols))]
    outs = [np.zeros((16, 24), np.float32) for _ in tols]
    args = [_host_gemm_args(A, B, Cm) for (A, B), Cm in zip(ops, outs)]
    st, done, chosen, lat = c.gemm_stream_raw(args, tols, sync=True, stream=0)
    assert st == 0 and done == len(tols)
    assert list(chosen) == [c.select(16, 24, 8, t) for t in tols] == [0, 1, 0, 1, 0, 1]
    assert ran == list(chosen)
    assert np.all(lat >= 0)
    for (A, B), Cm in zip(ops, outs):
        assert np.allclose(Cm, A @ B, rtol=1e-5, atol=1e-5)
    # the third request asks for 1e-9, which no variant meets
    ran.clear()
    st, done, chosen, _ = c.gemm_stream_raw(args[:5], [1e-2, 1e-5, 1e-9, 1e-2, 1e-2], sync=False, stream=0)
    assert st == pa.CMP_ENOVARIANT and done == 2 and ran == [1, 0]
    assert list(chosen[:2]) == [1, 0]
    st, done, _, _ = c.gemm_stream_raw([], [], stream=0)
    assert st == 0 and done == 0
    with pytest.raises(ValueError):
        c.gemm_stream_raw(args[:2], [1e-2], stream=0)


def test_gemm_argument_validation():
    c = host_ctx()
    register_fakes(c)
    A = np.zeros((4, 4), np.float32)
    a = _host_gemm_args(A, A, A)
    a.lda = 2
    assert c.gemm_raw(a, 1e-2, stream=0)[0] == pa.CMP_EINVAL
    a = _host_gemm_args(A, A, A)
    a.M = -1
    assert c.gemm_raw(a, 1e-2, stream=0)[0] == pa.CMP_EINVAL
    a = _host_gemm_args(A, A, A)
    assert c.gemm_raw(a, -1.0, stream=0)[0] == pa.CMP_EINVAL
    a = _host_gemm_args(A, A, A)
    a.A = None
    assert c.gemm_raw(a, 1e-2, stream=0)[0] == pa.CMP_EINVAL
    a.alpha = 0.0                                          # alpha == 0 never reads A or B
    assert c.gemm_raw(a, 1e-2, stream=0)[0] == 0


def test_host_timing():
    c = host_ctx()
    register_fakes(c)
    A = np.zeros((4, 4), np.float32)
    a = _host_gemm_args(A, A, A)
    med, mn, mean = C.c_float(), C.c_float(), C.c_float()
    st = c.L.cmp_time_variant(c.ctx, 2, C.byref(a), 1, 5, None, C.byref(med), C.byref(mn), C.byref(mean))
    assert st == 0 and 0 <= mn.value <= med.value


def test_history_roundtrip_and_signature(tmp_path):
    c = host_ctx()
    register_fakes(c)
    shapes, T = _table(20, 3)
    for s, (m, n, k) in enumerate(shapes):
        for v in range(4):
            c.history_add(int(m), int(n), int(k), v, 20, float(T[s, v]), float(T[s, v]) * 0.9, float(T[s, v]) * 1.1)
    p = str(tmp_path / "hist.txt")
    c.history_save(p)
    d = host_ctx()
    register_fakes(d)
    assert d.history_load(p) == 0
    assert d.history() == c.history()
    text = open(p).read().replace("arch=host", "arch=gfx950")
    q = str(tmp_path / "other.txt")
    open(q, "w").write(text)
    e = host_ctx()
    register_fakes(e)
    assert e.history_load(q) == pa.CMP_EINVAL          # recorded on another device
    assert e.history_load(q, force=True) == 0
    open(q, "w").write("garbage\n")
    assert e.history_load(q) == pa.CMP_EINVAL
    # rows that cmp_history_add would refuse are refused on load too, and nothing is added
    lines = open(p).read().splitlines()
    first = next(i for i, l in enumerate(lines) if l and not l.startswith("#"))
    for bad in ("0", "-5"):
        f = lines[:first] + [re.sub(r"^\S+", bad, lines[first])] + lines[first + 1:]
        open(q, "w").write("\n".join(f) + "\n")
        g = host_ctx()
        register_fakes(g)
        assert g.history_load(q) == pa.CMP_EINVAL
        assert g.history() == []
    for med in ("nan", "-1", "0", "inf"):
        cols = lines[first].split()
        cols[5] = med
        f = lines[:first] + [" ".join(cols)] + lines[first + 1:]
        open(q, "w").write("\n".join(f) + "\n")
        g = host_ctx()
        register_fakes(g)
        assert g.history_load(q) == pa.CMP_EINVAL, med
        assert g.history() == []


def test_mlp_checkpoint_roundtrip_and_errors(tmp_path):
    """The selector network and its normalisation statistics survive a save and a load bit for
    bit (Section 3.2 trains the network once and reuses it); a file from another device, a
    malformed file, one with a non-finite value or one with the wrong parameter count is refused
    and changes nothing."""
    rng = np.random.default_rng(7)
    c = host_ctx()
    p = str(tmp_path / "net.txt")
    with pytest.raises(pa.ComparError) as e:
        c.mlp_save(p)                                   # nothing trained or set yet
    assert e.value.status == pa.CMP_ENODATA
    n = _lib.load().cmp_mlp_param_count()
    params = (rng.standard_normal(n) * 10.0 ** rng.integers(-8, 8, n)).astype(np.float32)
    params[:3] = [np.float32(1) / 3, -0.0, np.finfo(np.float32).tiny]
    norm = [rng.standard_normal(4).astype(np.float32), rng.uniform(0.1, 9, 4).astype(np.float32),
            rng.standard_normal(4).astype(np.float32), rng.uniform(0.1, 9, 4).astype(np.float32)]
    c.mlp_set_params(params)
    c.mlp_set_norm(*norm)
    c.mlp_save(p)

    d = host_ctx()
    d.mlp_load(p)
    assert d.mlp_get_params().tobytes() == params.tobytes()
    for got, want in zip(d.mlp_get_norm(), norm):
        assert got.tobytes() == want.tobytes()

    text = open(p).read()
    q = str(tmp_path / "other.txt")
    open(q, "w").write(re.sub(r"(?m)^# device .*$", "# device arch=gfx950 cus=256", text))
    e = host_ctx()
    with pytest.raises(pa.ComparError) as err:
        e.mlp_load(q)                                   # saved on another device
    assert err.value.status == pa.CMP_EINVAL
    e.mlp_load(q, force=True)
    assert e.mlp_get_params().tobytes() == params.tobytes()

    bad = {
        "short": re.sub(r"(?m)^(params(?: \S+){%d}).*$" % (n - 1), r"\1", text),
        "value": text.replace("sd_x ", "sd_x x", 1),
        "sd": re.sub(r"(?m)^sd_y \S+", "sd_y 0", text),
        "nan": re.sub(r"(?m)^(params(?: \S+){5}) \S+", r"\1 nan", text),
        "inf": re.sub(r"(?m)^mu_x \S+", "mu_x inf", text),
        "header": "\n".join(l for l in text.splitlines() if not l.startswith("# compar-mlp")),
        "garbage": "garbage\n",
    }
    for name, body in bad.items():
        f = str(tmp_path / f"bad_{name}.txt")
        open(f, "w").write(body)
        g = host_ctx()
        g.mlp_set_params(np.zeros(n, np.float32))
        with pytest.raises(pa.ComparError) as err:
            g.mlp_load(f, force=True)
        assert err.value.status == pa.CMP_EINVAL, name
        assert not g.mlp_get_params().any(), name      # a refused file leaves the network alone


def test_env_restriction_in_subprocess():
    code = r"""
import paper_2311_03543_amd as pa
c = pa.Compar(-1)
for i, n in enumerate(["f32_simt", "bf16x3", "fp8r", "bf16"]):
    c.variant_register("gemm", n, pa.CMP_TARGET_HOST, lambda *a: 0, [1e-5, 1e-5, 1e-3, 1e-2][i])
print(c.admissible(8, 8, 8, 1e-2))
"""
    env = dict(os.environ, COMPAR_VARIANTS="bf16,fp8r", PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "12"        # fp8r (bit 2) and bf16 (bit 3) only


def test_split_k_and_optional_builtin_argument_checks():
    c = host_ctx()
    L, ctx = c.L, c.ctx
    # forcing knob: 0 (automatic) and 1..64 accepted, anything else refused
    assert L.cmp_set_split_k(ctx, 0) == pa.CMP_OK
    assert L.cmp_set_split_k(ctx, 64) == pa.CMP_OK
    assert L.cmp_set_split_k(ctx, 65) == pa.CMP_EINVAL
    assert L.cmp_set_split_k(ctx, -1) == pa.CMP_EINVAL
    assert L.cmp_set_split_k(None, 0) == pa.CMP_EINVAL
    n = C.c_int(-7)
    # the host context has no built-in variants: every id is out of range
    assert L.cmp_split_k(ctx, 0, 512, 512, 8192, C.byref(n)) == pa.CMP_EINVAL
    assert L.cmp_split_k(ctx, 0, -1, 512, 8192, C.byref(n)) == pa.CMP_EINVAL
    assert L.cmp_split_k(ctx, 0, 512, 512, 8192, None) == pa.CMP_EINVAL
    # a host variant reports no split
    st, vid = c.variant_register("gemm", "host_fake", pa.CMP_TARGET_HOST, _noop, 1e-5)
    assert st == pa.CMP_OK
    assert L.cmp_split_k(ctx, vid, 512, 512, 8192, C.byref(n)) == pa.CMP_OK and n.value == 1
    # fp6x3 needs a GPU context, host_f32 does not; unknown names and null pointers are refused
    vid = C.c_int(-1)
    assert L.cmp_register_builtin(ctx, b"fp6x3", C.byref(vid)) == pa.CMP_EUNSUPPORTED
    assert L.cmp_register_builtin(ctx, b"host_f32", C.byref(vid)) == pa.CMP_OK and vid.value >= 0
    assert L.cmp_register_builtin(ctx, b"host_f32", C.byref(vid)) == pa.CMP_EDUP
    assert L.cmp_register_builtin(ctx, b"fp4", C.byref(vid)) == pa.CMP_ENOTFOUND
    assert L.cmp_register_builtin(ctx, None, C.byref(vid)) == pa.CMP_EINVAL
    assert L.cmp_register_builtin(None, b"fp6x3", C.byref(vid)) == pa.CMP_EINVAL
    # workspace reservation needs a GPU context; negative sizes are refused
    assert L.cmp_reserve(ctx, 64, 64, 64) == pa.CMP_EUNSUPPORTED
    assert L.cmp_reserve(ctx, -1, 64, 64) == pa.CMP_EINVAL
    assert L.cmp_reserve(None, 1, 1, 1) == pa.CMP_EINVAL
    # the MX FP6 quantisation entry needs a GPU context
    assert L.cmp_quant_mx6(ctx, 4, 4, None, 4, 0, None, None, None, None, None) == pa.CMP_EUNSUPPORTED
    c.close()


def test_call_log_records(tmp_path):
    """CMP_FLAG_LOG: one JSON line per cmp_gemm with the context, the choice, the selector's
    predicted time (the recorded median at the nearest timed shape), the measured time of the
    run that produced C, and null residual without verify mode; unknown flag bits refused."""
    import json
    c = host_ctx()
    L, ctx = c.L, c.ctx
    assert L.cmp_set_flags(ctx, 4) == pa.CMP_EINVAL
    vid = c.register_builtin("host_f32")
    st, fake = c.variant_register("gemm", "fake_fast", pa.CMP_TARGET_HOST, _noop, 1e-2)
    assert st == 0
    c.history_add(32, 32, 32, vid, 5, 0.25)      # ms -> 250 us
    c.history_add(32, 32, 32, fake, 5, 0.5)
    c.history_add(64, 64, 64, vid, 5, 1.5)
    path = str(tmp_path / "calls.jsonl")
    assert c.set_log_file(path) is None
    c.set_flags(pa.CMP_FLAG_LOG)
    A, B = synth.gemm_operands(33, 31, 30, seed=3)
    Cm = np.zeros((33, 31), np.float32)
    assert c.gemm_raw(_host_gemm_args(A, B, Cm), 1e-2, stream=0) == (0, vid)   # nearest: 32^3
    assert c.gemm_raw(_host_gemm_args(A, B, Cm), 1e-5, stream=0) == (0, vid)   # only host_f32
    c.force_variant(fake)
    assert c.gemm_raw(_host_gemm_args(A, B, Cm), 1e-2, stream=0) == (0, fake)
    c.force_variant(-1)
    c.set_flags(0)
    assert c.gemm_raw(_host_gemm_args(A, B, Cm), 1e-2, stream=0)[0] == 0     # not logged
    c.log_flush()
    recs = [json.loads(l) for l in open(path).read().splitlines()]
    assert [r["call"] for r in recs] == [1, 2, 3]
    r0, r1, r2 = recs
    assert (r0["M"], r0["N"], r0["K"], r0["tol"]) == (33, 31, 30, 1e-2)
    assert r0["selector"] == "nn" and r0["variant"] == "host_f32" and r0["id"] == vid
    assert r0["predicted_us"] == pytest.approx(250.0)
    assert r0["measured_us"] > 0 and r0["residual"] is None and r0["fallbacks"] == 0
    assert r1["selector"] == "only" and r1["predicted_us"] is None and r1["tol"] == 1e-5
    assert r2["selector"] == "forced" and r2["variant"] == "fake_fast" and r2["measured_us"] >= 0
    # a new sink: later records go there, the old file is left as it was
    path2 = str(tmp_path / "more.jsonl")
    c.set_log_file(path2)
    c.set_flags(pa.CMP_FLAG_LOG)
    c.gemm_raw(_host_gemm_args(A, B, Cm), 1e-2, stream=0)
    c.close()                                     # terminate writes what is pending
    assert len(open(path).read().splitlines()) == 3
    assert [json.loads(l)["call"] for l in open(path2).read().splitlines()] == [4]
    d = host_ctx()
    assert d.L.cmp_set_log_file(d.ctx, str(tmp_path / "no" / "such" / "dir.jsonl").encode()) == pa.CMP_EINVAL
    d.close()


def test_call_log_from_environment(tmp_path):
    path = str(tmp_path / "env.jsonl")
    code = r"""
import numpy as np, paper_2311_03543_amd as pa, synth
c = pa.Compar(-1)
vid = c.register_builtin("host_f32")
A, B = synth.gemm_operands(8, 8, 8, seed=0)
Cm = np.zeros((8, 8), np.float32)
a = pa.cmp_gemm_args(8, 8, 8, 8, 8, 8, 1.0, 0.0, A.ctypes.data, B.ctypes.data, Cm.ctypes.data)
print(c.gemm_raw(a, 1e-3, stream=0))
c.close()
"""
    env = dict(os.environ, COMPAR_LOG=path, PYTHONPATH=ROOT)
    subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    import json
    recs = [json.loads(l) for l in open(path).read().splitlines()]
    assert len(recs) == 1 and recs[0]["variant"] == "host_f32" and recs[0]["M"] == 8


def test_grouped_configuration_table():
    """The grouped configurations (no GPU needed): the FP32 SIMT tiles reproduce f32_simt
    (variant 0), the last one bf16x3 (variant 1) with the 256 x 256 MFMA tile and a 32-value
    K block; out-of-range indices and a null output are refused."""
    L = _lib.load()
    n = L.cmp_grouped_config_count()
    assert n >= 2
    v = C.c_int()
    variants = []
    for i in range(n):
        assert L.cmp_grouped_config_variant(i, C.byref(v)) == pa.CMP_OK
        variants.append(v.value)
    assert variants == [0] * (n - 1) + [1]
    bm, bn, bk = C.c_int(), C.c_int(), C.c_int()
    assert L.cmp_grouped_config_info(n - 1, C.byref(bm), C.byref(bn), C.byref(bk)) == pa.CMP_OK
    assert (bm.value, bn.value, bk.value) == (256, 256, 32)
    for bad in (-1, n):
        assert L.cmp_grouped_config_variant(bad, C.byref(v)) == pa.CMP_EINVAL
        assert L.cmp_grouped_config_info(bad, C.byref(bm), C.byref(bn), C.byref(bk)) == pa.CMP_EINVAL
    assert L.cmp_grouped_config_variant(0, None) == pa.CMP_EINVAL
    assert [pa.grouped_config_variant(i) for i in range(n)] == variants
