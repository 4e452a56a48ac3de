"""Checkpointed reverse sweeps (fd_plan_set_checkpoint): the saved buffer keeps
F0 and one level of intermediates per segment of s levels, and the reverse
sweep recomputes each segment before using it.  The gradient and rho must be
bitwise those of the store-all sweep (same kernels on the same values), for
Algorithm 1 and 2 plans, b = 0 and b != 0, a total photon cutoff, both
precisions, several intervals (1, 2, ceil(sqrt L), L and more), and the
recompute-everything path (saved == NULL)."""
import math

import numpy as np
import pytest
import torch

from paper_2303_08879_amd import fockdiag as F
from paper_2303_08879_amd import workloads as W

pytestmark = pytest.mark.gpu


def rand_triple(rng, M, b_zero, scale=0.2):
    D = 2 * M
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    X = scale * (X + X.T)
    b = np.zeros(D, complex) if b_zero else 0.3 * (rng.standard_normal(D) + 1j * rng.standard_normal(D))
    return X, b, 0.8 + 0.1j


def run(plan, A, b, c, g, every, dtype, use_saved=True):
    print(f"[gpu ckpt] cut={plan.cutoffs} mask={bin(plan.detected_mask)} every={every} saved={use_saved}", flush=True)
    F.fd_plan_set_checkpoint(plan, every)
    T = lambda x: torch.tensor(np.asarray(x), dtype=dtype, device="cuda")
    At, bt, ct = T(A), T(b), T([c])
    wsb, svb = plan.workspace(True)
    rho = torch.empty(plan.out_shape, dtype=dtype, device="cuda")
    dA, db, dc = torch.empty_like(At), torch.empty_like(bt), torch.empty_like(ct)
    if use_saved:
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        saved = torch.empty(svb, dtype=torch.uint8, device="cuda")
        F.fock_diag_fwd(plan, At, bt, ct, rho, ws, saved)
        F.fock_diag_vjp(plan, At, bt, ct, saved, T(g), dA, db, dc, ws)
    else:
        ws = torch.empty(wsb + svb + 256, dtype=torch.uint8, device="cuda")
        F.fock_diag_vjp(plan, At, bt, ct, None, T(g), dA, db, dc, ws)
    torch.cuda.synchronize()
    F.fd_device_status(plan)
    return rho.cpu().numpy(), dA.cpu().numpy(), db.cpu().numpy(), dc.cpu().numpy(), svb


CASES = [
    (4, [4, 3, 3, 3], 0b1111, True), (4, [4, 3, 3, 3], 0b1111, False), (3, [6, 4, 3], 0b110, False),
    (3, [5, 3, 4], 0b011, True), (4, [3, 3, 3, 3], 0b1100, False), (6, [3, 3, 2, 2, 2, 2], 0b111111, True),
]


@pytest.mark.parametrize("M,cut,mask,bz", CASES)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_checkpointed_reverse_is_bitwise_store_all(M, cut, mask, bz, dtype):
    rng = np.random.default_rng(600 + M * 13 + mask)
    A, b, c = rand_triple(rng, M, bz)
    plan = F.Plan(cut, mask, dtype, "zero" if bz else "general")
    g = rng.standard_normal(plan.out_shape) + 1j * rng.standard_normal(plan.out_shape)
    ref = run(plan, A, b, c, g, 0, dtype)
    L = plan.query(F.FD_Q_LEVELS)
    for every in sorted({1, 2, math.ceil(math.sqrt(L)), L, L + 3}):
        got = run(plan, A, b, c, g, every, dtype)
        for x, r in zip(got[:4], ref[:4]):
            assert np.array_equal(x, r), every
    got = run(plan, A, b, c, g, 2, dtype, use_saved=False)
    for x, r in zip(got[:4], ref[:4]):
        assert np.array_equal(x, r)


def test_checkpointed_total_cutoff_plan():
    rng = np.random.default_rng(77)
    A, b, c = rand_triple(rng, 4, True)
    plan = F.Plan([6, 6, 6, 6], 0b1111, torch.complex128, "zero", total_cutoff=9)
    g = rng.standard_normal(plan.out_shape) + 1j * rng.standard_normal(plan.out_shape)
    ref = run(plan, A, b, c, g, 0, torch.complex128)
    for every in (1, 3, 4):
        got = run(plan, A, b, c, g, every, torch.complex128)
        for x, r in zip(got[:4], ref[:4]):
            assert np.array_equal(x, r), every


def test_checkpointed_eight_modes_full_size():
    # the 8-mode, cutoff-8 workload (57 levels): interval 8 keeps F0 and 7 levels
    # of intermediates instead of all 57
    circ = W.config5()
    plan = F.Plan(circ.cutoffs, circ.detected_mask, torch.complex128, "zero")
    g = W.random_cotangent(plan.out_shape, seed=9)
    ref = run(plan, circ.A, circ.b, circ.c, g, 0, torch.complex128)
    got = run(plan, circ.A, circ.b, circ.c, g, 8, torch.complex128)
    print(f"[ckpt] saved bytes: store-all {ref[4]}, every 8 levels {got[4]}")
    for x, r in zip(got[:4], ref[:4]):
        assert np.array_equal(x, r)
    assert got[4] < 0.3 * ref[4]
