"""Batched persistent forward (one sweep launch over many circuits of uneven
shape) against the per-circuit path and the FP64 oracle.  The batched sweep
runs the same per-unit device code as the per-circuit level kernels, so its
outputs must equal theirs bit for bit; the oracle bar is the usual 1e-10
normwise relative error in complex128."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from parity import assert_close, assert_grad_close  # noqa: F401
from paper_2303_08879_amd import fockdiag as F
from paper_2303_08879_amd import ops
from paper_2303_08879_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


def small_batch(seed, n, b_general=False, max_entries=400_000):
    """Circuits drawn like the uneven batch workload (M~U{3..6}, one undetected
    mode with probability 1/2, Haar, loss), at cutoffs small enough for the
    oracle's full density matrix (prod C_i^2 <= max_entries)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        M = int(rng.integers(3, 7))
        cut = [int(x) for x in rng.integers(2, 5, size=M)]
        mask = (1 << M) - 1
        if rng.random() < 0.5:
            u = int(rng.integers(0, M))
            cut[u] = int(rng.integers(3, 7))
            mask &= ~(1 << u)
        if math.prod(c * c for c in cut) > max_entries:
            continue
        circ = W._circuit(rng, M, 0.1, 1.2, lambda g, MM: g.uniform(0.7, 1.0, size=MM), cut, mask,
                          alpha_var=0.1 if b_general else 0.0)
        out.append(circ)
    return out


def run_batch(circs, dtype=torch.complex128, b_mode="zero"):
    print(f"[gpu] batch n={len(circs)} dtype={dtype} b_mode={b_mode}", flush=True)
    rho = ops.fock_diag_batch([(c.A, c.b, c.c) for c in circs], [(c.cutoffs, c.detected_mask) for c in circs],
                              dtype=dtype, b_mode=b_mode)
    torch.cuda.synchronize()
    for c in circs:
        F.fd_device_status(ops.get_plan(c.cutoffs, c.detected_mask, dtype, b_mode))
    return [r.cpu().numpy() for r in rho]


def run_single(c, dtype=torch.complex128, b_mode="zero"):
    out = ops.fock_diag(c.A, c.b, c.c, c.cutoffs, c.detected_mask, dtype=dtype, b_mode=b_mode)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("b_general", [False, True])
def test_small_batch_matches_single_and_oracle(b_general):
    circs = small_batch(301 + b_general, 24, b_general)
    mode = "general" if b_general else "zero"
    outs = run_batch(circs, b_mode=mode)
    for c, out in zip(circs, outs):
        assert out.shape == c.out_shape
        np.testing.assert_array_equal(out, run_single(c, b_mode=mode))
        ref = O.fock_diag(c.A, c.b, c.c, c.cutoffs, c.detected_mask)
        assert_close(out, ref, label=str((c.cutoffs, bin(c.detected_mask))))


def test_batch_repeated_calls_and_new_pointers():
    circs = small_batch(311, 10)
    first = run_batch(circs)
    second = run_batch(circs)          # new buffers: a second schedule
    plans = [ops.get_plan(c.cutoffs, c.detected_mask, torch.complex128, "zero") for c in circs]
    ins = [ops._as_inputs(c.A, c.b, c.c, torch.complex128, "cuda") for c in circs]
    ws = [ops._workspace(p.workspace(False)[0], "cuda") for p in plans]
    rho = [torch.empty(p.out_shape, dtype=torch.complex128, device="cuda") for p in plans]
    for rep in range(3):               # same pointers: the cached schedule, counters cleared each call
        for r in rho:
            r.fill_(float("nan"))
        F.fock_diag_fwd_batch(plans, [x[0] for x in ins], [x[1] for x in ins], [x[2] for x in ins], rho, ws)
        torch.cuda.synchronize()
        for a, b, r in zip(first, second, rho):
            np.testing.assert_array_equal(a, b)
            np.testing.assert_array_equal(a, r.cpu().numpy())


def test_batch_wide_and_degenerate_members():
    rng = np.random.default_rng(321)
    circs = [
        W._circuit(rng, 8, 0.3, 0.8, lambda g, M: g.uniform(0.8, 0.95, size=M), [3, 2, 3, 2, 2, 3, 2, 2], 0xFF),
        W._circuit(rng, 2, 0.3, 0.8, lambda g, M: g.uniform(0.8, 0.95, size=M), [5, 4], 0b00),   # nothing detected
        W._circuit(rng, 3, 0.3, 0.8, lambda g, M: g.uniform(0.8, 0.95, size=M), [1, 5, 4], 0b110),  # cutoff-1 mode
        W._circuit(rng, 1, 0.3, 0.8, lambda g, M: g.uniform(0.8, 0.95, size=M), [9], 0b1),
        W._circuit(rng, 4, 0.3, 0.8, lambda g, M: g.uniform(0.8, 0.95, size=M), [4, 3, 5, 3], 0b1011),
    ]
    outs = run_batch(circs)            # MD = 8 present: the wide sweep build
    for c, out in zip(circs, outs):
        np.testing.assert_array_equal(out, run_single(c))
        ref = O.fock_diag(c.A, c.b, c.c, c.cutoffs, c.detected_mask)
        assert_close(out, ref, label=str(c.cutoffs))


def test_batch_with_three_undetected_modes_and_large_blocks():
    # members the persistent sweep does not stage (six block coordinates; a
    # 6561-entry block; a 20736-entry block whose rows stream from HBM) run
    # their own level launches inside the batched call, beside sweep members
    rng = np.random.default_rng(322)
    mk = lambda M, cut, mask: W._circuit(rng, M, 0.3, 0.8, lambda g, MM: g.uniform(0.8, 0.95, size=MM), cut, mask)
    circs = [mk(4, [3, 2, 3, 3], 0b1000), mk(3, [9, 9, 3], 0b100), mk(3, [4, 3, 3], 0b110), mk(4, [3, 3, 3, 3], 0xF),
             mk(5, [2, 3, 2, 3, 3], 0b11000), mk(4, [12, 12, 2, 2], 0b1100)]
    outs = run_batch(circs)
    for c, out in zip(circs, outs):
        np.testing.assert_array_equal(out, run_single(c))
        ref = O.fock_diag(c.A, c.b, c.c, c.cutoffs, c.detected_mask)
        assert_close(out, ref, label=f"{c.cutoffs} {bin(c.detected_mask)}")


def test_batch_c64_error_stated():
    circs = small_batch(331, 16)
    outs = run_batch(circs, dtype=torch.complex64)
    worst = 0.0
    for c, out in zip(circs, outs):
        np.testing.assert_array_equal(out, run_single(c, dtype=torch.complex64))
        ref = O.fock_diag(c.A, c.b, c.c, c.cutoffs, c.detected_mask)
        worst = max(worst, O.rel_err(out.astype(np.complex128), ref))
    print(f"[c64 batch] worst rel err {worst:.3e}")
    assert worst <= 1e-5


def test_uneven_batch_full_size_subset():
    # the 64 smallest circuits of the 256-circuit uneven batch at full cutoffs,
    # plus two of medium size: bitwise equal to the per-circuit path, and the
    # low corner of two of them against the oracle
    circs = W.config3()
    size = [math.prod(c.out_shape) for c in circs]
    order = np.argsort(size)
    pick = [circs[i] for i in order[:64]] + [circs[i] for i in order[128:130]]
    outs = run_batch(pick)
    for c, out in zip(pick, outs):
        np.testing.assert_array_equal(out, run_single(c))
    for k in (0, 65):
        c, out = pick[k], outs[k]
        corner = [min(x, 3) if (c.detected_mask >> j) & 1 else x for j, x in enumerate(c.cutoffs)]
        if math.prod(x * x for x in corner) > 3_000_000:
            corner = [min(x, 3) if (c.detected_mask >> j) & 1 else min(x, 8) for j, x in enumerate(c.cutoffs)]
        ref = O.fock_diag(c.A, c.b, c.c, corner, c.detected_mask)
        nU = sum(1 for j in range(c.M) if not (c.detected_mask >> j) & 1)
        sl = tuple(slice(0, s) for s in ref.shape)
        assert_close(out[sl], ref, label="gpu_batch:136")


def test_batch_rejects_overlapping_workspaces():
    circs = small_batch(341, 2)
    plans = [ops.get_plan(c.cutoffs, c.detected_mask, torch.complex128, "zero") for c in circs]
    ins = [ops._as_inputs(c.A, c.b, c.c, torch.complex128, "cuda") for c in circs]
    need = max(p.workspace(False)[0] for p in plans)
    ws = ops._workspace(2 * need, "cuda")
    rho = [torch.empty(p.out_shape, dtype=torch.complex128, device="cuda") for p in plans]
    with pytest.raises(F.FockDiagError) as e:
        F.fock_diag_fwd_batch(plans, [x[0] for x in ins], [x[1] for x in ins], [x[2] for x in ins], rho, [ws, ws])
    assert e.value.status == F.FD_ERR_INVALID_ARG


def test_batch_runner_memory_groups_and_autotune():
    from paper_2303_08879_amd import batching as Bt
    circs = small_batch(351, 12)
    runner = Bt.BatchRunner([(c.cutoffs, c.detected_mask) for c in circs], [(c.A, c.b, c.c) for c in circs],
                            budget_bytes=1)            # the largest circuit alone sets the group size
    assert len(runner.groups) > 1
    old = F.fd_batch_get_tuning()
    try:
        best, times = Bt.autotune(runner, candidates=[(2, 64, 4), (1, 64, 1), (2, 64, 4, 1), (2, 64, 4, 2048, 1)])
        assert best in times and F.fd_batch_get_tuning() == best
        assert (2, 64, 4, 1, 0) in times     # the routing threshold at its minimum
        got = {}
        runner.run(True, callback=lambda k, rho: got.update({i: r.cpu().numpy() for i, r in rho.items()}))
        runner.check_status()
        assert sorted(got) == list(range(len(circs)))
        for i, c in enumerate(circs):
            np.testing.assert_array_equal(got[i], run_single(c))
        # the staged search, then its cached winner for the same signature
        best2, times2 = Bt.autotune(runner, use_cache=False)
        assert len(times2) >= 6 and F.fd_batch_get_tuning() == best2
        best3, times3 = Bt.autotune(runner)
        assert best3 == best2 and times3 == {}
    finally:
        F.fd_batch_set_tuning(*old[:4], max(old[4], 0))


def test_batch_graph_replay_matches_eager_over_repeated_calls():
    # the whole batched call (level launches of the largest circuit, the
    # sweep's prep, sweep and permutation) captured once and replayed; eager
    # work and synchronisations between the replays; new input values between
    # calls; every replay equal to the eager call bit for bit
    rng = np.random.default_rng(352)
    circs = small_batch(352, 10)
    circs.append(W._circuit(rng, 5, 0.3, 0.8, lambda g, M: g.uniform(0.8, 0.95, size=M), [9, 8, 7, 6, 6], 0x1F))
    dt = torch.complex128
    plans = [ops.get_plan(c.cutoffs, c.detected_mask, dt, "zero") for c in circs]
    ins = [[torch.as_tensor(x, dtype=dt, device="cuda").reshape(-1 if k == 2 else x.shape).contiguous()
            for k, x in enumerate((c.A, c.b, np.asarray([c.c])))] for c in circs]
    ws = [torch.empty(max(p.workspace(False)[0], 256), dtype=torch.uint8, device="cuda") for p in plans]
    rho = [torch.empty(p.out_shape, dtype=dt, device="cuda") for p in plans]
    old = F.fd_batch_get_tuning()
    call = lambda: F.fock_diag_fwd_batch(plans, [x[0] for x in ins], [x[1] for x in ins], [x[2] for x in ins],
                                         rho, ws)
    c0 = [x[2].clone() for x in ins]
    scale = (1.0, 1.25, 0.5)

    def set_inputs(rep):
        for x, c in zip(ins, c0):
            x[2].copy_(c * scale[rep])

    try:
        # fill_waves = 4: the 5-mode circuit runs its own level launches
        F.fd_batch_set_tuning(2, 64, 4, 4, 0)
        refs = []
        for rep in range(3):
            set_inputs(rep)
            call()
            torch.cuda.synchronize()
            refs.append([r.cpu().numpy() for r in rho])
        F.fd_batch_set_tuning(2, 64, 4, 4, 1)
        for rep in range(3):
            set_inputs(rep)
            for r in rho:
                r.zero_()
            call()
            _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
            torch.cuda.synchronize()
            for r, ref in zip(rho, refs[rep]):
                np.testing.assert_array_equal(r.cpu().numpy(), ref)
        graph_state = F.fd_batch_get_tuning()[4]
        print(f"[batch graph] use_graph reads {graph_state}", flush=True)
        assert graph_state in (1, -1)
        for c, p in zip(circs, plans):
            F.fd_device_status(p)
    finally:
        F.fd_batch_set_tuning(*old[:4], max(old[4], 0))


def test_vjp_batch_matches_single_calls():
    circs = small_batch(361, 6, b_general=True)
    dt = torch.complex128
    plans = [ops.get_plan(c.cutoffs, c.detected_mask, dt, "general") for c in circs]
    ins = [ops._as_inputs(c.A, c.b, c.c, dt, "cuda") for c in circs]
    saved, ws, g, outs = [], [], [], []
    for k, (p, c) in enumerate(zip(plans, circs)):
        wb, sb = p.workspace(True)
        w = ops._workspace(wb + sb + 4096, "cuda")     # room to recompute when saved is None
        s = ops._workspace(sb, "cuda")
        rho = torch.empty(p.out_shape, dtype=dt, device="cuda")
        F.fock_diag_fwd(p, *ins[k], rho, ops._workspace(wb, "cuda"), s)
        saved.append(s if k % 2 == 0 else None)
        ws.append(w)
        g.append(torch.tensor(W.random_cotangent(p.out_shape, 50 + k), dtype=dt, device="cuda"))
    dA = [torch.empty_like(x[0]) for x in ins]
    db = [torch.empty_like(x[1]) for x in ins]
    dc = [torch.empty_like(x[2]) for x in ins]
    F.fock_diag_vjp_batch(plans, [x[0] for x in ins], [x[1] for x in ins], [x[2] for x in ins], saved, g,
                          dA, db, dc, ws)
    torch.cuda.synchronize()
    for k, (p, c) in enumerate(zip(plans, circs)):
        eA, eb, ec = torch.empty_like(dA[k]), torch.empty_like(db[k]), torch.empty_like(dc[k])
        F.fock_diag_vjp(p, *ins[k], saved[k], g[k], eA, eb, ec, ws[k])
        torch.cuda.synchronize()
        for got, exp in ((dA[k], eA), (db[k], eb), (dc[k], ec)):
            np.testing.assert_array_equal(got.cpu().numpy(), exp.cpu().numpy())
