"""The C-ABI library loads and exports every entry point the header declares;
host-only entry points (validation, working-set size, status strings) behave.
No GPU needed."""
import ctypes
import os
import re

import pytest

from paper_2012_07620_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "rerank.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rerank_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.library()
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(binding.EXPORTS)


def test_params_struct_matches_header():
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} rerank_params;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b([a-z_0-9]+)\s*[;,]", body)
    assert fields == [f for f, _ in binding.Params._fields_]


def _p(**kw):
    base = dict(n=1000, n_query=100, dim=128, k1=10, k2=3, layers=1)
    base.update(kw)
    return binding.make_params(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(), binding.OK),
    (dict(n=1), binding.E_INVALID),
    (dict(n_query=0), binding.E_INVALID),
    (dict(n_query=1000), binding.E_INVALID),
    (dict(dim=0), binding.E_INVALID),
    (dict(k1=0), binding.E_INVALID),
    (dict(k1=1001), binding.E_INVALID),
    (dict(k2=11), binding.E_INVALID),
    (dict(k2=0), binding.E_INVALID),
    (dict(layers=-1), binding.E_INVALID),
    (dict(layers=257), binding.E_INVALID),
    (dict(alpha=9), binding.E_INVALID),
    (dict(alpha=-1), binding.E_INVALID),
    (dict(k1=257, n=5000), binding.E_UNSUPPORTED),
    (dict(sim_prec="bf16", extra_cand=0), binding.E_INVALID),
    (dict(k1=1000, k2=1000, n=1000), binding.E_UNSUPPORTED),
    (dict(k1=256, k2=7, n=300), binding.OK),
    (dict(aggregator="mean"), binding.OK),
    (dict(aggregator="max", node="adj_raw"), binding.OK),
])
def test_validation(kw, status):
    assert binding.validate(_p(**kw)) == status
    if status != binding.OK:
        assert binding.library().rerank_last_error().decode()


def test_workspace_bytes_scales_with_n_squared():
    a = binding.workspace_bytes(_p())
    b = binding.workspace_bytes(_p(n=2000))
    c = binding.workspace_bytes(_p(layers=0))
    assert a > 2 * 4 * 1000 * 1000  # at least the two N x N float buffers
    assert 3.5 < b / a < 4.5
    assert c < a
    mid = binding.workspace_bytes(binding.make_params(19281, 3368, 2048, 26, 7, 1))
    assert 2 * 4 * 19281 * 19281 < mid < 3.5e9


def test_null_arguments_are_rejected_without_a_device():
    lib = binding.library()
    p = _p()
    assert lib.rerank_workspace_bytes(ctypes.byref(p), None) == binding.E_INVALID
    assert lib.rerank_validate(None) == binding.E_INVALID
    assert lib.rerank_run(None, ctypes.byref(p), None, 0, None, None, None, None) == binding.E_INVALID
    assert lib.rerank_run_static(None, ctypes.byref(p), None, 0, None, None, None, None) == binding.E_INVALID
    assert lib.rerank_create(None, 0, 0, 0) == binding.E_INVALID
    for s in range(8):
        assert lib.rerank_status_str(s)


def test_unknown_enums_rejected():
    lib = binding.library()
    for field, bad in (("aggregator", 3), ("node", 3), ("sim_prec", 3), ("final_prec", 4), ("final_prec", -1)):
        p = _p()
        setattr(p, field, bad)
        assert lib.rerank_validate(ctypes.byref(p)) == binding.E_INVALID, field


def test_sparse_final_needs_adjacency_features():
    lib = binding.library()
    for node, want in (("adj", binding.OK), ("adj_raw", binding.OK), ("raw", binding.E_INVALID)):
        p = binding.make_params(1000, 100, 64, 20, 6, 1, node=node, final_prec="sparse")
        assert lib.rerank_validate(ctypes.byref(p)) == want, node


def test_sparse_final_workspace_holds_both_feature_buffers_and_counters():
    # zero layers: the sparse product still needs the second N x N buffer for its compacted rows
    lib = binding.library()
    n = 1000
    dense = binding.workspace_bytes(binding.make_params(n, 100, 64, 20, 6, 0))
    sparse = binding.workspace_bytes(binding.make_params(n, 100, 64, 20, 6, 0, final_prec="sparse"))
    ldn = (n + 63) // 64 * 64
    assert sparse - dense >= n * ldn * 4 + (2 * n + 3 * ldn + 4) * 4


def test_context_flags_checked_before_any_device_call():
    # the flag check needs no GPU: unknown bits are rejected, known ones pass it
    lib = binding.library()
    h = ctypes.c_void_p()
    assert lib.rerank_create(ctypes.byref(h), 0, 0, 8) == binding.E_INVALID
    assert lib.rerank_create(ctypes.byref(h), 0, 0, 1 << 31) == binding.E_INVALID
    assert binding.CTX_STAGE_TIMING == 1 and binding.CTX_DENSE_LAYERS == 2 and binding.CTX_FUSED_KNN == 4
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "rerank.h")).read()
    assert "#define RERANK_CTX_STAGE_TIMING 1u" in hdr and "#define RERANK_CTX_DENSE_LAYERS 2u" in hdr
    assert "#define RERANK_CTX_FUSED_KNN 4u" in hdr
    # every known bit passes the flag check (what follows needs a device, absent here or not)
    for flags in (1, 2, 4, 7):
        st = lib.rerank_create(ctypes.byref(h), 0, 0, flags)
        assert st != binding.E_INVALID, flags
        if st == binding.OK:
            assert lib.rerank_destroy(h) == binding.OK


def test_evaluate_rejects_bad_arguments_before_any_device_call():
    lib = binding.library()
    buf = (ctypes.c_double * 8)()
    p = ctypes.addressof(buf)  # 8-byte aligned stand-in, never dereferenced on these paths
    ks = (ctypes.c_int32 * 2)(1, 5)
    bad_k = (ctypes.c_int32 * 2)(1, 0)
    assert lib.rerank_evaluate(None, p, 2, 3, 3, p, p, ks, 2, p, p, p, None) == binding.E_INVALID
    assert lib.rerank_evaluate(p, None, 2, 3, 3, p, p, ks, 2, p, p, p, None) == binding.E_INVALID
    assert lib.rerank_evaluate(p, p, 2, 3, 3, p, p, ks, 2, p + 4, p, p, None) == binding.E_INVALID  # ap misaligned
    assert lib.rerank_evaluate(p, p, 0, 3, 3, p, p, ks, 2, p, p, p, None) == binding.E_INVALID
    assert lib.rerank_evaluate(p, p, 2, 3, 2, p, p, ks, 2, p, p, p, None) == binding.E_INVALID  # ld < g
    assert lib.rerank_evaluate(p, p, 2, 3, 3, p, p, ks, 0, p, p, p, None) == binding.E_INVALID
    assert lib.rerank_evaluate(p, p, 2, 3, 3, p, p, ks, 17, p, p, p, None) == binding.E_INVALID
    assert lib.rerank_evaluate(p, p, 2, 3, 3, p, p, bad_k, 2, p, p, p, None) == binding.E_INVALID


def _fused_scratch(n, K, sbytes):
    """The fused path's scratch as the library sizes it: a stored sample of
    P panels of 128 columns per row and C candidate slots per row, with
    f = 1 + 6 / sqrt(K) slots per expected key and P balancing the two."""
    import math
    T = (n + 127) // 128
    f = 1.0 + 6.0 / math.sqrt(K)
    P = min(T, max(8, math.ceil(math.sqrt(8.0 * f * K * n / sbytes) / 128.0)))
    m = P * 128
    C = min(n, math.ceil(f * K * n / min(m, n)) + 128)
    up = lambda b: (b + 255) // 256 * 256
    return up(n * m * sbytes) + up(n * C * 8) + up(n * 4) + up(n * 4) + up(T * 4)


def test_knn_workspace_of_the_fused_path_has_no_n_by_n_buffer():
    n, d = 19281, 2048
    ldn = (n + 63) // 64 * 64
    p = binding.make_params(n, 1, d, 26, 1, 0)
    plain = binding.knn_workspace_bytes(p)
    fused = binding.knn_workspace_bytes(p, fused_knn=True)
    assert plain >= n * ldn * 4  # the N x N similarity buffer
    # the S buffer is replaced by the sample and candidate scratch (26 + 8 candidates, FP32 sample)
    # the unfused plan also holds the block maxima of S for its pruned selection
    # (34 candidates against 151 column blocks), the fused one the sample and slots
    bm = 4 * n * ((n + 127) // 128)
    assert abs(fused - (plain - n * ldn * 4 - bm + _fused_scratch(n, 34, 4))) < (1 << 20)
    assert fused < plain / 3
    # the scratch grows as N^1.5: twice the rows, about 2.8 times the scratch
    s1, s2 = _fused_scratch(n, 34, 4), _fused_scratch(2 * n, 34, 4)
    assert 2.5 < s2 / s1 < 3.1
    f2 = binding.knn_workspace_bytes(binding.make_params(2 * n, 1, d, 26, 1, 0), fused_knn=True)
    assert abs((f2 - fused) - (s2 - s1) - (plain - n * ldn * 4 - bm)) < (4 << 20)
    # N = 300000, d = 512, BF16: S alone would be 180 GB; the fused k-NN graph needs about 12 GB
    big = binding.make_params(300000, 1, 512, 20, 1, 0, sim_prec="bf16")
    assert binding.knn_workspace_bytes(big) > 300000 * 300032 * 2
    assert binding.knn_workspace_bytes(big, fused_knn=True) < 14e9


def test_kernel_names_do_not_depend_on_unnamed_types():
    """A kernel whose signature mentions a type built from an unnamed enum or
    lambda is mangled with a per-pass number ($_N) that the host and device
    compilations can assign differently; the host then registers a name the
    device code object lacks and the launch aborts. No such name may exist."""
    lib = binding.library()
    path = lib._name
    blob = open(path, "rb").read()
    names = set(re.findall(rb"_ZN2rr[A-Za-z0-9_$]+", blob))
    assert names, "no kernel names found in the library"
    bad = sorted(n.decode() for n in names if b"$_" in n)
    assert not bad, bad[:5]


def test_knn_workspace_checks():
    lib = binding.library()
    p = binding.make_params(1000, 1, 64, 60, 1, 0)  # 60 + 8 candidates
    assert binding.knn_workspace_bytes(p) > 0
    with pytest.raises(binding.RerankError) as e:
        binding.knn_workspace_bytes(p, fused_knn=True)
    assert e.value.status == binding.E_UNSUPPORTED
    out = ctypes.c_size_t(0)
    q = binding.make_params(1000, 1, 64, 10, 1, 0)
    assert lib.rerank_knn_workspace_bytes(ctypes.byref(q), 8, ctypes.byref(out)) == binding.E_INVALID
    assert lib.rerank_knn_workspace_bytes(ctypes.byref(q), 4, None) == binding.E_INVALID
    bad = binding.make_params(1000, 1, 64, 10, 20, 0)  # k2 > k1
    assert lib.rerank_knn_workspace_bytes(ctypes.byref(bad), 0, ctypes.byref(out)) == binding.E_INVALID


def test_static_array_size_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define RERANK_STATIC_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == binding.STATIC_BYTES


def test_block_maxima_buffer_follows_the_pruning_rule():
    """The similarity product records per-row block maxima (row stride padded
    to 64 columns) only when the selection is pruned: 4 (K - 1) <= blocks and
    K <= 128. Between K = 38 and K = 39 at N = 19281 (151 blocks) the knn
    working set drops the maxima and gains one candidate column in each of the
    two candidate arrays; above K = 128 nothing is pruned even at 512 blocks."""
    n, d, k1 = 19281, 64, 26
    ldn, tb = 19328, 151

    def ws(n_, k1_, extra):
        return binding.knn_workspace_bytes(binding.make_params(n_, 1, d, k1_, 1, 0, extra_cand=extra))

    def up(v):
        return (v + 255) // 256 * 256

    pruned, streaming = ws(n, k1, 12), ws(n, k1, 13)  # K = 38 and 39
    assert pruned - streaming == up(tb * ldn * 4) - 2 * (up(n * 39 * 4) - up(n * 38 * 4))
    # K = 128 prunes at N = 65536 (4 * 127 <= 512 blocks), K = 129 does not
    big = 65536
    assert ws(big, 128, 0) - ws(big, 129, 0) == up(512 * big * 4) - 4 * (up(big * 129 * 4) - up(big * 128 * 4))
