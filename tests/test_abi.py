"""The C-ABI library loads and exports every function include/rcqr.h declares (no GPU needed).

Only host-side entry points are called here: workspace sizing, status strings, phase names and
argument validation that fails before any device work.
"""

import ctypes
import os

import pytest

import paper_2309_05868_amd as rc


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rc.LIB_PATH):
        from paper_2309_05868_amd import build
        build.build()
    return rc.lib()


def test_exports_every_declared_symbol(lib):
    names = rc.declared_functions()
    assert {"rcqr_plan", "rcqr_factor", "rcqr_destroy", "rcqr_workspace_bytes", "rcqr_info"} <= set(names)
    raw = ctypes.CDLL(rc.LIB_PATH)
    missing = [nm for nm in names if not hasattr(raw, nm)]
    assert not missing, missing
    assert set(names) == set(rc._SIGNATURES), "binding signatures out of sync with the header"


def test_workspace_bytes_and_shape_checks(lib):
    ws = rc.workspace_bytes(10_000, 16, 512, 64)
    assert ws > 512 * 16 * 8 and ws % 256 == 0
    # CSR CountSketch needs per-row index storage; the LDS path does not
    assert rc.workspace_bytes(2_000_000, 64, 8192, 256) > 2 * 4 * 2_000_000
    assert rc.workspace_bytes(10, 16, 8, 16) == 0       # s1 < s2
    assert rc.workspace_bytes(10, 16, 64, 8) == 0       # s2 < n
    assert rc.workspace_bytes(8, 16, 64, 32) == 0       # m < n
    assert rc.workspace_bytes(1000, 0, 64, 32) == 0     # n < 1
    assert rc.workspace_bytes(10_000, 100, 20_000, 400) > 0
    assert rc.workspace_bytes(10_000, 129, 40_000, 600) == 0  # n beyond the kernels
    assert rc.workspace_bytes(2**31, 8, 128, 32) == 0   # row index must fit 31 bits
    for flags in (rc.FLAG_SKETCH_FP32, rc.FLAG_SKETCH_FP32 | rc.FLAG_GEMM_BF16, rc.FLAG_REORTH, 7, rc.FLAG_SKETCH_AT_PLAN, 15):
        assert rc.workspace_bytes(10_000, 16, 512, 64, flags) == ws
    assert rc.workspace_bytes(10_000, 16, 512, 64, 16) == 0   # unknown flag bit
    assert rc.workspace_bytes(10_000, 16, 512, 64, rc.FLAG_GEMM_BF16) == 0


def test_status_strings_and_phase_names(lib):
    assert rc.status_string(rc.OK) == "ok"
    assert "Cholesky" in rc.status_string(rc.E_CHOL)
    assert "diagonal" in rc.status_string(rc.E_RANK)
    names = [lib.rcqr_phase_name(i).decode() for i in range(7)]
    assert names == ["countsketch", "gaussian", "householder", "trsm_gram", "cholesky", "reorth", "final"]
    assert lib.rcqr_phase_name(7).decode() == "?"


def test_plan_rejects_bad_arguments_on_host(lib):
    h = ctypes.c_void_p()
    # null workspace, bad shapes, nonzero flags and misaligned workspace fail before any HIP call
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 16, 512, 64, 0, 0, None, 0, None) == rc.E_INVALID
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 16, 8, 64, 0, 0, ctypes.c_void_p(256), 1 << 30, None) == rc.E_INVALID
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 129, 40_000, 600, 0, 0, ctypes.c_void_p(256), 1 << 30, None) == rc.E_UNSUPPORTED
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 16, 512, 64, 0, 16, ctypes.c_void_p(256), 1 << 30, None) == rc.E_INVALID
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 16, 512, 64, 0, rc.FLAG_GEMM_BF16, ctypes.c_void_p(256), 1 << 30,
                         None) == rc.E_INVALID  # BF16 product needs the FP32 sketch
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 16, 512, 64, 0, 0, ctypes.c_void_p(8), 1 << 30, None) == rc.E_INVALID
    assert lib.rcqr_plan(None, 1000, 16, 512, 64, 0, 0, ctypes.c_void_p(256), 1 << 30, None) == rc.E_INVALID
    # a plan with a fake (never touched) workspace pointer: I/O argument checks are host-side
    ws = rc.workspace_bytes(1000, 16, 512, 64)
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 16, 512, 64, 0, 0, ctypes.c_void_p(1 << 20), ws, None) == rc.OK
    try:
        p = ctypes.c_void_p(4096)
        assert lib.rcqr_factor(h, None, 16, p, 16, p, 16) == rc.E_INVALID
        assert lib.rcqr_factor(h, p, 15, p, 16, p, 16) == rc.E_INVALID       # ldv < n
        assert lib.rcqr_factor(h, p, 16, p, 32, p, 16) == rc.E_INVALID       # in place with ldq != ldv
        assert lib.rcqr_factor(h, p, 16, p, 16, p, 8) == rc.E_INVALID        # ldr < n
        assert lib.rcqr_sketch_hash(h, -1, 4, p, p) == rc.E_INVALID
        cnt = ctypes.c_int32()
        arr = (ctypes.c_float * 6)()
        assert lib.rcqr_phase_times(h, arr, 6, ctypes.byref(cnt)) == rc.E_INVALID  # timing never enabled
    finally:
        assert lib.rcqr_destroy(h) == rc.OK
    assert lib.rcqr_destroy(None) == rc.E_INVALID
    # graphs: argument checks are host-side; a plan on the legacy default stream cannot be captured
    g = ctypes.c_void_p()
    assert lib.rcqr_graph_create(None, 0, p, 16, p, 16, p, 16, ctypes.byref(g)) == rc.E_INVALID
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 16, 512, 64, 0, 0, ctypes.c_void_p(1 << 20), ws, None) == rc.OK
    try:
        assert lib.rcqr_graph_create(h, 0, p, 16, p, 16, p, 16, ctypes.byref(g)) == rc.E_INVALID
        assert lib.rcqr_graph_create(h, 7, p, 16, p, 16, p, 16, ctypes.byref(g)) == rc.E_INVALID
        assert lib.rcqr_graph_create(h, 0, p, 16, p, 16, p, 16, None) == rc.E_INVALID
        # tuning knobs: defaults, host-side validation, round trip; rcqr_tune refuses Q aliasing V
        mode, mult = ctypes.c_int32(), ctypes.c_int32()
        assert lib.rcqr_get_tuning(h, ctypes.byref(mode), ctypes.byref(mult)) == rc.OK
        assert (mode.value, mult.value) == (rc.FINAL_RECOMPUTE, 2)
        assert lib.rcqr_set_tuning(h, 2, 1) == rc.E_INVALID
        assert lib.rcqr_set_tuning(h, 1, 0) == rc.E_INVALID
        assert lib.rcqr_set_tuning(h, 1, 9) == rc.E_INVALID
        assert lib.rcqr_set_tuning(h, rc.FINAL_MATERIALIZE, 4) == rc.OK
        assert lib.rcqr_get_tuning(h, ctypes.byref(mode), ctypes.byref(mult)) == rc.OK
        assert (mode.value, mult.value) == (rc.FINAL_MATERIALIZE, 4)
        assert lib.rcqr_tune(h, p, 16, p, 16, p, 16, 3, None) == rc.E_INVALID
        assert lib.rcqr_tune(h, p, 16, ctypes.c_void_p(8192), 16, p, 16, 0, None) == rc.E_INVALID
    finally:
        assert lib.rcqr_destroy(h) == rc.OK
    assert lib.rcqr_graph_launch(None) == rc.E_INVALID
    assert lib.rcqr_graph_destroy(None) == rc.E_INVALID
    # batches: host-side argument checks (no plan on a capturable stream is needed for these)
    b = ctypes.c_void_p()
    P1 = (ctypes.c_void_p * 1)()
    ptrs = (ctypes.c_void_p * 1)(p.value)
    lds = (ctypes.c_int64 * 1)(16)
    assert lib.rcqr_batch_create(0, P1, 0, ptrs, lds, ptrs, lds, ptrs, lds, ctypes.byref(b)) == rc.E_INVALID
    assert lib.rcqr_batch_create(1, None, 0, ptrs, lds, ptrs, lds, ptrs, lds, ctypes.byref(b)) == rc.E_INVALID
    assert lib.rcqr_batch_create(1, P1, 0, ptrs, lds, ptrs, lds, ptrs, lds, None) == rc.E_INVALID
    assert lib.rcqr_plan(ctypes.byref(h), 1000, 16, 512, 64, 0, 0, ctypes.c_void_p(1 << 20), ws, None) == rc.OK
    try:
        P1[0] = h.value
        assert lib.rcqr_batch_create(1, P1, 0, ptrs, lds, ptrs, lds, ptrs, lds, ctypes.byref(b)) == rc.E_INVALID  # default stream
        assert lib.rcqr_batch_create(1, P1, 5, ptrs, lds, ptrs, lds, ptrs, lds, ctypes.byref(b)) == rc.E_INVALID  # method
    finally:
        assert lib.rcqr_destroy(h) == rc.OK
    assert lib.rcqr_batch_launch(None) == rc.E_INVALID
    assert lib.rcqr_batch_destroy(None) == rc.E_INVALID
    # same-shaped batches: capacity, strides and support are checked before any device work
    m, n = 1000, 16
    ws1 = rc.workspace_bytes(m, n, 512, 64)
    assert lib.rcqr_plan(ctypes.byref(h), m, n, 512, 64, 0, 0, ctypes.c_void_p(1 << 20), 2 * ws1, None) == rc.OK
    try:
        V, Q, R = ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 31), ctypes.c_void_p(1 << 32)
        assert lib.rcqr_factor_batch(h, 3, V, n, m * n, Q, n, m * n, R, n, n * n, None) == rc.E_INVALID      # 3 > workspace for 2
        assert lib.rcqr_factor_batch(h, 0, V, n, m * n, Q, n, m * n, R, n, n * n, None) == rc.E_INVALID      # count < 1
        assert lib.rcqr_factor_batch(h, 2, V, n, m * n - 1, Q, n, m * n, R, n, n * n, None) == rc.E_INVALID  # members overlap
        assert lib.rcqr_factor_batch(h, 2, V, n, m * n, V, n, 2 * m * n, R, n, n * n, None) == rc.E_INVALID  # Q = V, other stride
        assert lib.rcqr_factor_batch(None, 2, V, n, m * n, Q, n, m * n, R, n, n * n, None) == rc.E_INVALID
        st, col = ctypes.c_int32(), ctypes.c_int32()
        assert lib.rcqr_info_member(h, 2, ctypes.byref(st), ctypes.byref(col)) == rc.E_INVALID        # no member 2
        assert lib.rcqr_info_member(h, -1, ctypes.byref(st), ctypes.byref(col)) == rc.E_INVALID
    finally:
        assert lib.rcqr_destroy(h) == rc.OK
    # batches run the plain FP64 method: a plan with flags is refused before anything is launched
    ws2 = rc.workspace_bytes(m, 100, 2000, 200)
    assert lib.rcqr_plan(ctypes.byref(h), m, 100, 2000, 200, 0, rc.FLAG_REORTH, ctypes.c_void_p(1 << 20), ws2, None) == rc.OK
    try:
        V, Q, R = ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 31), ctypes.c_void_p(1 << 32)
        assert lib.rcqr_factor_batch(h, 1, V, 100, m * 100, Q, 100, m * 100, R, 100, 100 * 100, None) == rc.E_UNSUPPORTED
        one = (rc._RaggedMember * 1)(rc._RaggedMember(1 << 30, 1 << 31, 1 << 32, m, 100, 100, 100, 7))
        assert lib.rcqr_factor_ragged(h, 1, one) == rc.E_UNSUPPORTED
    finally:
        assert lib.rcqr_destroy(h) == rc.OK


def test_ragged_argument_errors_need_no_device():
    # every rejection happens on the host, before the member table is copied or a kernel launched
    lib = rc.lib()
    h = ctypes.c_void_p()
    m, n = 1000, 16
    ws1 = rc.workspace_bytes(m, n, 512, 64)
    assert lib.rcqr_plan(ctypes.byref(h), m, n, 512, 64, 0, 0, ctypes.c_void_p(1 << 20), 2 * ws1, None) == rc.OK
    try:
        def member(mm=500, ldv=n, ldq=n, ldr=n, V=1 << 30, Q=1 << 31, R=1 << 32):
            return rc._RaggedMember(V, Q, R, mm, ldv, ldq, ldr, 3)

        def call(*members):
            t = (rc._RaggedMember * len(members))(*members)
            return lib.rcqr_factor_ragged(h, len(members), t)

        assert call(member(), member(), member()) == rc.E_INVALID      # 3 members, workspace for 2
        assert lib.rcqr_factor_ragged(h, 0, None) == rc.E_INVALID
        assert lib.rcqr_factor_ragged(None, 1, (rc._RaggedMember * 1)(member())) == rc.E_INVALID
        assert call(member(mm=m + 1)) == rc.E_INVALID                    # more rows than the plan
        assert call(member(mm=n - 1)) == rc.E_INVALID                    # fewer rows than columns
        assert call(member(ldv=n - 1)) == rc.E_INVALID
        assert call(member(ldr=n - 1)) == rc.E_INVALID
        assert call(member(V=0)) == rc.E_INVALID                         # null buffers
        assert call(member(Q=1 << 30, ldq=n + 1)) == rc.E_INVALID       # Q = V with another leading dimension
    finally:
        assert lib.rcqr_destroy(h) == rc.OK


def test_binding_refuses_cpu_tensors(lib):
    import torch
    V = torch.zeros((100, 16), dtype=torch.float64)
    with pytest.raises((TypeError, RuntimeError, AssertionError)):
        p = rc.Plan.__new__(rc.Plan)
        p.m, p.n = 100, 16
        rc._check_matrix(V, 100, 16, "V")
