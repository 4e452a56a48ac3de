"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol the header declares, validates arguments, and its planner reproduces
the structure counts of App. B."""
import ctypes
import math
import os
import re

import pytest
import torch

from paper_2303_08879_amd import fockdiag as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "fockdiag.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:fd_status|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = F.lib()
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(F.EXPORTS)


def test_plan_create_rejects_bad_arguments():
    L = F.lib()
    h = ctypes.c_void_p()
    cut = (ctypes.c_int * 2)(4, 4)
    assert L.fd_plan_create(0, cut, 0b11, 0, 0, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    assert L.fd_plan_create(2, cut, 0b111, 0, 0, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    assert L.fd_plan_create(2, cut, 0b11, 7, 0, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    assert L.fd_plan_create(2, cut, 0b11, 0, 9, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    bad = (ctypes.c_int * 2)(0, 4)
    assert L.fd_plan_create(2, bad, 0b11, 0, 0, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    nine = (ctypes.c_int * 9)(*([3] * 9))
    assert L.fd_plan_create(9, nine, 0x1FF, 0, 0, ctypes.byref(h)) == F.FD_ERR_UNSUPPORTED
    four_u = (ctypes.c_int * 4)(3, 3, 3, 3)
    assert L.fd_plan_create(4, four_u, 0, 0, 0, ctypes.byref(h)) == F.FD_ERR_UNSUPPORTED
    assert "undetected" in F.fd_last_error()
    # two undetected modes at cutoff 17: a block of 83521 entries
    big2 = (ctypes.c_int * 3)(17, 17, 3)
    assert L.fd_plan_create(3, big2, 0b100, 0, 0, ctypes.byref(h)) == F.FD_ERR_UNSUPPORTED
    assert "65536" in F.fd_last_error()


@pytest.mark.parametrize("cut,mask,dtype", [
    ((3, 3, 3), 0, 0), ((4, 4, 4, 3), 0b1000, 0), ((3, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3), 0b11111111000, 0),
    ((9, 9, 3), 0b100, 0), ((9, 9, 3, 3, 3, 3, 3), 0b1111100, 0), ((9, 9, 3, 3, 3, 3, 3, 3), 0b11111100, 1),
    ((9, 9, 3, 3, 3, 3, 3, 3), 0b11111100, 0), ((12, 12, 3), 0b100, 0), ((5, 5, 5, 2), 0b1000, 0),
    ((16, 16, 2), 0b100, 1)])
def test_plan_create_three_undetected_modes_and_large_blocks(cut, mask, dtype):
    # three undetected modes, and blocks of up to 65536 entries: rows that do
    # not fit the LDS staging stream from HBM
    L = F.lib()
    h = ctypes.c_void_p()
    arr = (ctypes.c_int * len(cut))(*cut)
    assert L.fd_plan_create(len(cut), arr, mask, dtype, 0, ctypes.byref(h)) == F.FD_OK, F.fd_last_error()
    assert L.fd_plan_destroy(h) == F.FD_OK


def test_streamed_rows_workspace_sizes():
    # a plan whose forward rows stream keeps one bridge-pivot slot per
    # streaming workgroup (1024) after the prep block, in every workspace that
    # holds a prep block: two undetected modes at cutoff 12 with two detected
    # modes (MD = 2, R0 = 1728, RC = 1: 1024 x 2 x 2 x 1728 entries)
    import torch
    big = F.Plan([12, 12, 2, 2], 0b1100, torch.complex128, "general")
    eb, B, nodes = 16, 12 ** 4, 4
    al = lambda x: (x + 255) // 256 * 256
    slots = al(1024 * 2 * 2 * 1728 * eb)
    fwd, _ = big.workspace(False)
    assert fwd >= slots + al(nodes * B * eb)
    vjp, saved = big.workspace(True)
    assert vjp >= slots and saved >= nodes * B * eb


def test_calls_reject_null_plan_and_pointers():
    L = F.lib()
    assert L.fock_diag_fwd(None, None, None, None, None, None, 0, None, 0, None) == F.FD_ERR_INVALID_ARG
    p = F.Plan([4, 4], 0b11)
    assert L.fock_diag_fwd(p.handle, None, None, None, None, None, 0, None, 0, None) == F.FD_ERR_INVALID_ARG
    # detection_probs needs every mode detected
    q = F.Plan([4, 4], 0b10)
    assert L.detection_probs(q.handle, 16, 16, 16, 16, 256, 1 << 20, None) == F.FD_ERR_INVALID_ARG


def pivots_formula(C):
    # App. B.1
    M = len(C)
    prod = lambda xs: 1 if not xs else __import__("math").prod(xs)
    return (C[0] - 1) * prod(C[1:]) + sum((C[K] - 1) * prod(C[K + 1:]) for K in range(M))


def written_formula(M, C):
    # App. B.3 (equal cutoffs)
    t1 = (C - 1) * C ** (M - 1) + (C - 2) * C ** (M - 1) + (2 * M - 2) * (C - 1) ** 2 * C ** (M - 2)
    t2 = (C - 2) * sum(C ** (M - K - 1) for K in range(M))
    t10 = (C - 1) ** 2 * sum((M - K - 1) * C ** (M - K - 2) for K in range(M - 1))
    return C ** M, t1, t2, t10


@pytest.mark.parametrize("M,C", [(2, 4), (3, 5), (4, 10), (5, 6), (8, 8)])
def test_planner_counts_match_appendix_b(M, C):
    p = F.Plan([C] * M, (1 << M) - 1)
    t0, t1, t2, t10 = written_formula(M, C)
    assert p.query(F.FD_Q_NODES_F0) == t0
    assert p.query(F.FD_Q_NODES_F1) == t1
    assert p.query(F.FD_Q_NODES_F2) == t2
    assert p.query(F.FD_Q_NODES_F1010) == t10
    assert p.query(F.FD_Q_NODES_F1001) == t10
    assert p.query(F.FD_Q_PIVOTS) == 2 * C ** M - C ** (M - 1) - 1
    assert p.query(F.FD_Q_LEVELS) == M * (C - 1) + 1


def test_planner_figure11_and_figure7():
    p = F.Plan([4, 3, 3], 0b111)
    assert p.query(F.FD_Q_PIVOTS) == pivots_formula([4, 3, 3]) == 62
    assert p.query(F.FD_Q_STORED_NODES) == 255
    q = F.Plan([4, 4], 0b11)
    assert q.query(F.FD_Q_PIVOTS) == 27 and q.query(F.FD_Q_STORED_NODES) == 82


def test_planner_shapes_and_workspace():
    p = F.Plan([30, 12, 12, 12], 0b1110)
    assert p.out_shape == (30, 30, 12, 12, 12)
    assert p.query(F.FD_Q_OUT_ELEMS) == 30 * 30 * 12 ** 3
    assert p.query(F.FD_Q_BLOCK) == 900
    ws, saved = p.workspace(False)
    assert ws > 0 and saved == 0
    ws2, saved2 = p.workspace(True)
    assert saved2 > ws and ws2 > 0
    # cutoff-1 modes are dropped but keep their output axis
    r = F.Plan([1, 5, 1], 0b101)
    assert r.out_shape == (5, 5, 1, 1)
    assert r.query(F.FD_Q_BLOCK) == 25


def test_batch_rejects_bad_arguments_on_the_host():
    L = F.lib()
    assert L.fock_diag_fwd_batch(0, None, None, None, None, None, None, None, None) == F.FD_OK
    assert L.fock_diag_fwd_batch(-1, None, None, None, None, None, None, None, None) == F.FD_ERR_INVALID_ARG
    assert L.fock_diag_fwd_batch(2, None, None, None, None, None, None, None, None) == F.FD_ERR_INVALID_ARG
    p = F.Plan([3, 3], 0b11)
    q = F.Plan([3, 3], 0b11, dtype=__import__("torch").complex64)
    n = 2
    P = (ctypes.c_void_p * n)(p.handle.value, q.handle.value)
    ptr = (ctypes.c_void_p * n)(256, 512)
    sizes = (ctypes.c_size_t * n)(1 << 20, 1 << 20)
    # mixed dtypes are refused before any device work
    assert L.fock_diag_fwd_batch(n, P, ptr, ptr, ptr, ptr, ptr, sizes, None) == F.FD_ERR_INVALID_ARG
    assert "dtype" in F.fd_last_error()
    Pn = (ctypes.c_void_p * n)(p.handle.value, None)
    assert L.fock_diag_fwd_batch(n, Pn, ptr, ptr, ptr, ptr, ptr, sizes, None) == F.FD_ERR_INVALID_ARG


def test_batch_tuning_round_trip_and_range_checks():
    old = F.fd_batch_get_tuning()
    assert old == (2, 64, 4, 2048, 0)
    try:
        F.fd_batch_set_tuning(3, 128, 5)
        assert F.fd_batch_get_tuning() == (3, 128, 5, 2048, 0)
        F.fd_batch_set_tuning(3, 128, 5, 512, 1)
        assert F.fd_batch_get_tuning() == (3, 128, 5, 512, 1)
        for bad in [(0, 64, 2), (2, 0, 2), (2, 64, 0), (-4, 64, 2), (2, 64, 2, 0), (2, 64, 2, 2048, 2),
                    (2, 64, 2, 2048, -1)]:
            with pytest.raises(F.FockDiagError) as e:
                F.fd_batch_set_tuning(*bad)
            assert e.value.status == F.FD_ERR_INVALID_ARG
        assert F.fd_batch_get_tuning() == (3, 128, 5, 512, 1)
    finally:
        F.fd_batch_set_tuning(*old)


def test_exact_reciprocal_coordinate_split():
    # the device splits an undetected-block entry index into coordinates with
    # trunc((rem + 0.5) * (1 / stride)) in double precision instead of an
    # integer division; exhaustively equal to floor division on its range
    import numpy as np
    rem = np.arange(16384, dtype=np.float64)
    ref = np.arange(16384)
    for d in range(1, 16385):
        q = ((rem + 0.5) * (1.0 / d)).astype(np.int64)
        assert np.array_equal(q, ref // d), d


def test_state_plan_host_checks():
    L = F.lib()
    h = ctypes.c_void_p()
    cut = (ctypes.c_int * 3)(4, 1, 5)
    assert L.fd_state_plan_create(0, cut, 0, 0, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    assert L.fd_state_plan_create(3, cut, 0, 9, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    assert L.fd_state_plan_create(3, cut, 5, 0, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    bad = (ctypes.c_int * 2)(65, 4)
    assert L.fd_state_plan_create(2, bad, 0, 0, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    nine = (ctypes.c_int * 9)(*([2] * 9))
    assert L.fd_state_plan_create(9, nine, 0, 0, ctypes.byref(h)) == F.FD_ERR_UNSUPPORTED
    p = F.StatePlan([4, 1, 5], b_mode="general")
    assert p.out_shape == (4, 1, 5)
    # amplitudes in level order (20 x 16 B, 256-aligned) + A and b of the 2 kept modes
    assert p.workspace() == 512 + 256
    assert L.fock_state_fwd(None, None, None, None, None, None, 0, None) == F.FD_ERR_INVALID_ARG
    assert L.fock_state_fwd(p.handle, None, 16, 16, 16, 256, 1 << 20, None) == F.FD_ERR_INVALID_ARG
    assert L.fock_state_fwd(p.handle, 16, 16, 16, 16, 256 + 16, 1 << 20, None) == F.FD_ERR_INVALID_ARG
    assert L.fock_state_fwd(p.handle, 16, 16, 16, 16, 256, 512, None) == F.FD_ERR_WORKSPACE
    assert L.fd_state_plan_destroy(None) == F.FD_OK


def test_density_jvp_host_checks():
    # fock_diag_jvp: argument checks and unsupported plans are rejected on the
    # host, before any device work
    import torch
    L = F.lib()
    p = F.Plan([4, 3], 0b11, torch.complex128, "general")
    half = (p.workspace(False)[0] + 255) // 256 * 256
    assert p.jvp_workspace() == 2 * half
    ws = p.jvp_workspace()
    ptrs = [16] * 8
    assert L.fock_diag_jvp(None, *ptrs, 256, ws, None) == F.FD_ERR_INVALID_ARG
    assert L.fock_diag_jvp(p.handle, *ptrs[:7], None, 256, ws, None) == F.FD_ERR_INVALID_ARG
    assert L.fock_diag_jvp(p.handle, *ptrs, 256 + 16, ws, None) == F.FD_ERR_INVALID_ARG
    assert L.fock_diag_jvp(p.handle, *ptrs, 256, ws - 1, None) == F.FD_ERR_WORKSPACE
    # the b = 0 schedule skips the odd levels a non-zero db reaches
    pz = F.Plan([4, 3], 0b11, torch.complex128, "zero")
    assert L.fock_diag_jvp(pz.handle, *ptrs, 256, 1 << 30, None) == F.FD_ERR_UNSUPPORTED
    # undetected blocks whose values and tangents exceed the LDS staging:
    # two undetected modes at cutoff 9 with five detected modes (the forward
    # alone fits)
    pu = F.Plan([9, 9, 3, 3, 3, 3, 3], 0b1111100, torch.complex128, "general")
    assert L.fock_diag_jvp(pu.handle, *ptrs, 256, 1 << 40, None) == F.FD_ERR_UNSUPPORTED
    assert "LDS" in F.fd_last_error()


def test_exact_reciprocal_digit_split_of_cindex():
    # The permutations between C order and node order split a C-order index
    # x < 2^31 into digits with trunc((x + 0.5) * (1 / C)), C <= 64, in double
    # precision (same arithmetic as the device).  Checked against integer
    # division at every residue near the top of the range, around powers of
    # two, and on random indices.
    import numpy as np
    rng = np.random.default_rng(0)
    top = (1 << 31) - 1
    xs = [np.arange(top - 4096, top + 1, dtype=np.int64)]
    for k in range(1, 31):
        xs.append(np.arange(max(0, (1 << k) - 130), (1 << k) + 130, dtype=np.int64))
    xs.append(rng.integers(0, top, size=200000, dtype=np.int64))
    x = np.concatenate(xs)
    for C in range(2, 65):
        q = ((x + 0.5) * (1.0 / C)).astype(np.int64)
        assert np.array_equal(q, x // C), C


def test_total_cutoff_plan_counts_and_offsets():
    import itertools
    L = F.lib()
    h = ctypes.c_void_p()
    cut = (ctypes.c_int * 2)(4, 4)
    assert L.fd_plan_create_total(2, cut, -1, 0, 0, ctypes.byref(h)) == F.FD_ERR_INVALID_ARG
    # a cap at or above the box's top level changes nothing: the counts are App. B's
    for C in ([4, 3, 5], [6, 6], [3, 3, 3, 3]):
        box = F.Plan(C, (1 << len(C)) - 1)
        cap = F.Plan(C, 0, total_cutoff=sum(c - 1 for c in C) + 2)
        for q in (F.FD_Q_OUT_ELEMS, F.FD_Q_LEVELS, F.FD_Q_PIVOTS, F.FD_Q_NODES_F0, F.FD_Q_NODES_F1,
                  F.FD_Q_NODES_F2, F.FD_Q_NODES_F1010, F.FD_Q_NODES_F1001):
            assert cap.query(q) == box.query(q), (C, q)
    # below it: the points with |n| <= N, level offsets as counted by brute force
    C, N = [5, 1, 4, 6], 6
    p = F.Plan(C, 0, total_cutoff=N)
    pts = [n for n in itertools.product(*[range(c) for c in C]) if sum(n) <= N]
    assert p.query(F.FD_Q_OUT_ELEMS) == len(pts) and p.out_shape == (len(pts),)
    assert p.query(F.FD_Q_LEVELS) == N + 1
    offs = p.level_offsets()
    assert offs == [sum(1 for n in pts if sum(n) < S) for S in range(N + 2)]
    # F2(K) nodes: n_<K = 0, n_K <= C_K - 3, |n| <= N (kept modes 5, 4, 6)
    K = [5, 4, 6]
    f2 = sum(1 for K0 in range(3) for n in itertools.product(*[range(c) for c in K])
             if sum(n) <= N and all(n[d] == 0 for d in range(K0)) and n[K0] <= K[K0] - 3)
    assert p.query(F.FD_Q_NODES_F2) == f2
    # a box product beyond 2^31 is fine below a total cutoff
    big = F.Plan([64] * 8, 0, total_cutoff=10)
    assert big.query(F.FD_Q_OUT_ELEMS) == math.comb(18, 8)
    # host-side argument checks of the stopping call
    assert L.detection_probs_until(p.handle, 16, 16, 16, 16, 1.5, ctypes.byref(ctypes.c_int()),
                                   ctypes.byref(ctypes.c_double()), 256, 1 << 20, None) == F.FD_ERR_INVALID_ARG
    assert L.detection_probs_until(p.handle, 16, 16, 16, 16, 1e-3, None, None, 256, 1 << 20, None) == \
        F.FD_ERR_INVALID_ARG


@pytest.mark.parametrize("M,Nmax", [(3, 6), (4, 5), (2, 9)])
def test_total_cutoff_pivot_count_app_b1(M, Nmax):
    # App. B.1, global cutoff w < 2 N_max (|n| <= N_max - 1): per level N the
    # diagonal pivots C(N+M-1, N) plus the K-pivots sum_K C(N+M-K, N) =
    # C(N+M, N+1); per-mode cutoffs large enough not to bind
    p = F.Plan([64] * M, 0, total_cutoff=Nmax - 1)
    expect = sum(math.comb(N + M - 1, N) + math.comb(N + M, N + 1) for N in range(Nmax))
    assert p.query(F.FD_Q_PIVOTS) == expect
    assert p.query(F.FD_Q_OUT_ELEMS) == math.comb(Nmax - 1 + M, M)


def test_checkpoint_setting_and_memory():
    L = F.lib()
    plan = F.Plan([8] * 8, 0xFF, torch.complex128, "zero")
    ws0, sv0 = plan.workspace(True)
    assert L.fd_plan_set_checkpoint(plan.handle, -1) == F.FD_ERR_INVALID_ARG
    F.fd_plan_set_checkpoint(plan, 8)
    ws8, sv8 = plan.workspace(True)
    # F0 (the output, 16.8M entries) plus 6 checkpoints of one level of every
    # family, against every level of every family
    out = 16 * 8 ** 8
    assert out < sv8 < 0.3 * sv0
    assert ws8 > ws0                      # the segment buffer of 9 levels
    F.fd_plan_set_checkpoint(plan, 0)
    assert plan.workspace(True) == (ws0, sv0)
    with pytest.raises(F.FockDiagError):
        F.fd_plan_set_checkpoint(type("P", (), {"handle": None})(), 2)


def test_write_counter_arguments():
    # host-side checks of the debug write-counter mode (no device access: the
    # counter pointer is only stored by the call)
    L = F.lib()
    plan = F.Plan([4, 3, 3], 0b111, torch.complex128, "zero")
    _, sv = plan.workspace(True)
    need = sv // 16
    fake = ctypes.c_void_p(0x1000)
    assert L.fd_plan_set_write_counters(None, fake, need) == F.FD_ERR_INVALID_ARG
    assert L.fd_plan_set_write_counters(plan.handle, fake, need - 1) == F.FD_ERR_INVALID_ARG
    assert L.fd_plan_set_write_counters(plan.handle, None, 5) == F.FD_ERR_INVALID_ARG
    assert L.fd_plan_set_write_counters(plan.handle, fake, need) == F.FD_OK
    assert L.fd_plan_set_write_counters(plan.handle, None, 0) == F.FD_OK
    F.fd_plan_set_checkpoint(plan, 2)   # a checkpointed saved buffer does not hold every amplitude
    assert L.fd_plan_set_write_counters(plan.handle, fake, need) == F.FD_ERR_UNSUPPORTED
