"""CPU tests of the C ABI: the library loads, exports every declared symbol,
builds the 1D operators on the host, and rejects invalid arguments before any
device work (so none of these needs a GPU)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "adr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adr_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(adr):
    names = _declared()
    assert "adr_step" in names and "adr_precompute_phi" in names
    lib = ctypes.CDLL(adr.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(adr.EXPORTED)


@pytest.mark.parametrize("n,a,b,diff,vel", [(3, 0.0, 1.0, 1.0, 0.0), (64, 0.0, 1.0, 10.0, 0.0),
                                            (257, 0.0, math.pi, 0.02, 0.1), (31, -2.0, 5.0, 3.0, -0.7)])
def test_build_1d_ops_matches_oracle_operator(adr, n, a, b, diff, vel):
    A, band = adr.adr_build_1d_ops(n, a, b, diff, vel)
    ref = O.operator_1d(n, a, b, diff, vel)
    assert np.abs(A - ref).max() <= 1e-15 * np.abs(ref).max()
    # band layout: sub, diag, super
    assert band[0, 0] == 0.0 and band[2, n - 1] == 0.0
    for i in range(n):
        assert band[1, i] == A[i, i]
        if i > 0:
            assert band[0, i] == A[i, i - 1]
        if i < n - 1:
            assert band[2, i] == A[i, i + 1]


def test_build_1d_ops_rejects_bad_input(adr):
    lib = adr._lib
    buf = np.zeros(16)
    p = buf.ctypes.data
    assert lib.adr_build_1d_ops(2, 0.0, 1.0, 1.0, 0.0, 0, p, None) == adr.ADR_EINVAL
    assert lib.adr_build_1d_ops(4, 1.0, 1.0, 1.0, 0.0, 0, p, None) == adr.ADR_EINVAL
    assert lib.adr_build_1d_ops(4, 0.0, 1.0, float("nan"), 0.0, 0, p, None) == adr.ADR_EINVAL
    assert lib.adr_build_1d_ops(4, 0.0, 1.0, 1.0, 0.0, 7, p, None) == adr.ADR_EINVAL
    assert lib.adr_build_1d_ops(4, 0.0, 1.0, 1.0, 0.0, 0, None, None) == adr.ADR_EINVAL


def _problem(adr, d=3, n=(8, 8, 8)):
    p = adr.AdrProblem()
    p.d = d
    for mu in range(3):
        p.n[mu] = n[mu] if mu < d else 1
    p.model = adr.ADR_BRUSSELATOR
    p.scheme = adr.ADR_ETD2RKDS
    p.precision = adr.ADR_F64
    p.tau = 1e-3
    p.params[0], p.params[1] = 1.0, 3.0
    fake = 4096  # never dereferenced: every case below fails validation first
    for c in range(2):
        for mu in range(d):
            for j in range(3):
                p.phi[c][j][mu] = fake
            p.band[c][mu] = fake
    return p


def test_workspace_bytes(adr):
    p = _problem(adr)
    nb = adr.adr_workspace_bytes(p)
    assert nb >= 6 * 8 ** 3 * 8
    p.scheme = adr.ADR_LAWSON2B
    assert adr.adr_workspace_bytes(p) >= 10 * 8 ** 3 * 8
    p.precision = adr.ADR_F32
    assert adr.adr_workspace_bytes(p) < 10 * 8 ** 3 * 8


@pytest.mark.parametrize("field,value", [("d", 0), ("d", 4), ("model", 9), ("scheme", 5),
                                         ("precision", 7), ("flags", 1), ("tau", 0.0),
                                         ("tau", float("inf")), ("tau", -1e-3)])
def test_invalid_problem_rejected_without_device_work(adr, field, value):
    p = _problem(adr)
    setattr(p, field, value)
    lib = adr._lib
    assert lib.adr_workspace_bytes(ctypes.byref(p)) == 0
    st = lib.adr_step(ctypes.byref(p), 4096, 4096, 4096, 1 << 30, None)
    assert st == adr.ADR_EINVAL


def test_invalid_sizes_and_pointers_rejected(adr):
    lib = adr._lib
    p = _problem(adr)
    p.n[1] = 2
    assert lib.adr_step(ctypes.byref(p), 4096, 4096, 4096, 1 << 30, None) == adr.ADR_EINVAL
    p = _problem(adr)
    p.phi[1][2][0] = None
    assert lib.adr_step(ctypes.byref(p), 4096, 4096, 4096, 1 << 30, None) == adr.ADR_EINVAL
    p = _problem(adr)
    p.band[0][1] = None   # and no dense matrix either
    assert lib.adr_step(ctypes.byref(p), 4096, 4096, 4096, 1 << 30, None) == adr.ADR_EINVAL
    p = _problem(adr)
    assert lib.adr_step(ctypes.byref(p), None, 4096, 4096, 1 << 30, None) == adr.ADR_EINVAL
    assert lib.adr_solve(ctypes.byref(p), 4096, 4096, -1, 4096, 1 << 30, None) == adr.ADR_EINVAL
    # workspace too small
    assert lib.adr_step(ctypes.byref(p), 4096, 4096, 4096, 64, None) == adr.ADR_ENOMEM
    # misaligned workspace
    assert lib.adr_step(ctypes.byref(p), 4096, 4096, 4097, 1 << 30, None) == adr.ADR_EINVAL
    # reduced precision with a dense (non-banded) operator is not supported
    p = _problem(adr)
    p.precision = adr.ADR_F32
    p.band[0][0] = None
    p.dense[0][0] = 4096
    assert lib.adr_step(ctypes.byref(p), 4096, 4096, 4096, 1 << 30, None) == adr.ADR_ENOTSUP


def test_other_entry_points_validate(adr):
    lib = adr._lib
    n3 = (ctypes.c_int32 * 3)(4, 4, 4)
    assert lib.adr_precompute_phi(0, 4096, 1e-3, 4096, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi(8, None, 1e-3, 4096, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi(8, 4096, float("nan"), 4096, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi(8, 4096, 1e-3, None, None, None, None) == adr.ADR_EINVAL
    # the batched variant: count, sizes, steps and outputs are checked before device work
    n2 = (ctypes.c_int32 * 2)(8, 8)
    a2 = (ctypes.c_void_p * 2)(4096, 4096)
    t2 = (ctypes.c_double * 2)(1e-3, 1e-3)
    o2 = (ctypes.c_void_p * 2)(4096, 4096)
    nul2 = (ctypes.c_void_p * 2)(4096, None)
    assert lib.adr_precompute_phi_batch(0, n2, a2, t2, o2, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi_batch(4097, n2, a2, t2, o2, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi_batch(2, None, a2, t2, o2, None, None, None) == adr.ADR_EINVAL
    bad_n = (ctypes.c_int32 * 2)(8, 0)
    assert lib.adr_precompute_phi_batch(2, bad_n, a2, t2, o2, None, None, None) == adr.ADR_EINVAL
    bad_t = (ctypes.c_double * 2)(1e-3, float("inf"))
    assert lib.adr_precompute_phi_batch(2, n2, a2, bad_t, o2, None, None, None) == adr.ADR_EINVAL
    # the second matrix asks for no output at all
    assert lib.adr_precompute_phi_batch(2, n2, a2, t2, nul2, None, None, None) == adr.ADR_EINVAL
    # the no-allocation variant: same checks, and sizes beyond its fixed work area
    nmax = adr.ADR_PHI_NOALLOC_MAX_N
    assert lib.adr_precompute_phi_noalloc(0, 4096, 1e-3, 4096, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi_noalloc(8, None, 1e-3, 4096, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi_noalloc(8, 4096, 0.0, 4096, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi_noalloc(8, 4096, 1e-3, None, None, None, None) == adr.ADR_EINVAL
    assert lib.adr_precompute_phi_noalloc(nmax + 1, 4096, 1e-3, 4096, None, None, None) == adr.ADR_ENOMEM
    assert lib.adr_mode_product(3, n3, 3, 4096, 4096, 8192, 1.0, 0.0, None, None) == adr.ADR_EINVAL
    assert lib.adr_mode_product(3, n3, 0, 4096, 4096, 4096, 1.0, 0.0, None, None) == adr.ADR_EINVAL
    assert lib.adr_mode_product(4, n3, 0, 4096, 4096, 8192, 1.0, 0.0, None, None) == adr.ADR_EINVAL
    Ms = (ctypes.c_void_p * 3)(4096, 4096, 4096)
    assert lib.adr_tucker(3, n3, Ms, 4096, 8192, 1.0, 0.0, None, None, 0, None) == adr.ADR_ENOMEM
    assert lib.adr_tucker(3, n3, Ms, 4096, 4096, 1.0, 0.0, None, 4096, 1 << 20, None) == adr.ADR_EINVAL
    assert adr.adr_tucker_workspace_bytes((4, 4, 4)) >= 2 * 64 * 8
    assert lib.adr_device_copy(None, 4096, 8, None) == adr.ADR_EINVAL
    assert lib.adr_timing_enable(-1) == adr.ADR_EINVAL
    assert lib.adr_timing_enable(0) == adr.ADR_OK
    # timing classes 0..3 (3: products whose epilogue also computes a stage)
    cnt, tot = ctypes.c_int(-1), ctypes.c_double(-1.0)
    for kind in range(4):
        assert lib.adr_timing_read(kind, ctypes.byref(cnt), ctypes.byref(tot)) == adr.ADR_OK
        assert cnt.value == 0 and tot.value == 0.0
    assert lib.adr_timing_read(5, ctypes.byref(cnt), ctypes.byref(tot)) == adr.ADR_EINVAL
    assert lib.adr_timing_read(4, ctypes.byref(cnt), ctypes.byref(tot)) == adr.ADR_OK
    assert lib.adr_timing_read(-1, ctypes.byref(cnt), ctypes.byref(tot)) == adr.ADR_EINVAL


def test_strerror_covers_all_codes(adr):
    texts = {adr.adr_strerror(s) for s in (0, -1, -2, -3, -4, -5)}
    assert len(texts) == 6
    assert adr.adr_strerror(-99) == "unknown status"


def _batch_create(adr, probs, work=4096, work_bytes=1 << 30, flags=0, U=4096):
    lib = adr._lib
    count = len(probs)
    arr = (adr.AdrProblem * max(count, 1))(*probs)
    ptrs = lambda v: (ctypes.c_void_p * max(count, 1))(*([v] * max(count, 1)))
    sizes = (ctypes.c_size_t * max(count, 1))(*([work_bytes] * max(count, 1)))
    plan = ctypes.c_void_p(None)
    st = lib.adr_batch_create(count, arr, ptrs(U), ptrs(4096), ptrs(work), sizes, flags, None,
                              ctypes.byref(plan))
    assert plan.value is None  # no plan on failure
    return st


def test_batch_create_validates_before_device_work(adr):
    ok = _problem(adr)
    assert _batch_create(adr, []) == adr.ADR_EINVAL
    assert _batch_create(adr, [ok], flags=8) == adr.ADR_EINVAL
    assert _batch_create(adr, [ok], flags=adr.ADR_BATCH_TILE(5)) == adr.ADR_EINVAL
    assert _batch_create(adr, [ok], U=None) == adr.ADR_EINVAL
    assert _batch_create(adr, [ok], work=4097) == adr.ADR_EINVAL
    assert _batch_create(adr, [ok, ok], work_bytes=64) == adr.ADR_ENOMEM
    bad = _problem(adr)
    bad.tau = 0.0
    assert _batch_create(adr, [ok, bad]) == adr.ADR_EINVAL
    law = _problem(adr)
    law.scheme = adr.ADR_LAWSON2B
    assert _batch_create(adr, [ok, law]) == adr.ADR_ENOTSUP
    f32 = _problem(adr)
    f32.precision = adr.ADR_F32
    assert _batch_create(adr, [ok, f32]) == adr.ADR_ENOTSUP   # mixed precisions
    b3 = _problem(adr)
    b3.precision = adr.ADR_BF16X3
    assert _batch_create(adr, [b3]) == adr.ADR_ENOTSUP
    dense = _problem(adr)
    dense.band[1][2] = None
    dense.dense[1][2] = 4096
    assert _batch_create(adr, [dense]) == adr.ADR_ENOTSUP
    lib = adr._lib
    assert lib.adr_batch_run(None, 1, None) == adr.ADR_EINVAL
    assert lib.adr_batch_info(None, None, 0, None) == adr.ADR_EINVAL
    assert lib.adr_batch_destroy(None) == adr.ADR_EINVAL
    assert lib.adr_batch_create(1, None, None, None, None, None, 0, None, None) == adr.ADR_EINVAL


def test_indicator_entry_points_validate(adr):
    lib = adr._lib
    n3 = (ctypes.c_int32 * 3)(4, 4, 4)
    wb = adr.adr_indicators_workspace_bytes((4, 4, 4))
    assert wb >= 5 * 8
    assert lib.adr_indicators(0, n3, 4096, 4096, None, None, 4096, 4096, wb, None) == adr.ADR_EINVAL
    assert lib.adr_indicators(3, n3, None, 4096, None, None, 4096, 4096, wb, None) == adr.ADR_EINVAL
    # both previous states or neither
    assert lib.adr_indicators(3, n3, 4096, 4096, 4096, None, 4096, 4096, wb, None) == adr.ADR_EINVAL
    assert lib.adr_indicators(3, n3, 4096, 4096, None, None, 4096, 4096, 8, None) == adr.ADR_ENOMEM
    p = _problem(adr)
    mb = adr.adr_monitor_workspace_bytes(p)
    assert mb >= 2 * 8 ** 3 * 8
    st = lib.adr_solve_monitored(ctypes.byref(p), 4096, 4096, 4, 0, 4096, 4096, 1 << 30, 4096,
                                 mb, None)
    assert st == adr.ADR_EINVAL                      # every < 1
    st = lib.adr_solve_monitored(ctypes.byref(p), 4096, 4096, 4, 1, None, 4096, 1 << 30, 4096,
                                 mb, None)
    assert st == adr.ADR_EINVAL                      # no record buffer
    st = lib.adr_solve_monitored(ctypes.byref(p), 4096, 4096, 4, 1, 4096, 4096, 1 << 30, 4096,
                                 mb - 8, None)
    assert st == adr.ADR_ENOMEM
    st = lib.adr_solve_monitored(ctypes.byref(p), 4096, 4096, 4, 1, 4096, 4096, 1 << 30, 4097,
                                 mb, None)
    assert st == adr.ADR_EINVAL                      # misaligned monitor workspace
