"""Exactly-once writes of the forward sweep, counted on the device.

The buffer strategy of Sec. 3.1.4 rests on every stored amplitude being
written once and read once; App. B.3 counts the stored amplitudes.  With
fd_plan_set_write_counters each kernel write into the store-all saved buffer
adds one to that element's counter.  A correct schedule leaves every count at
0 (slots its family does not store) or 1, the sum equals the number of Eq.
recrel targets (the test-side schedule model's stored nodes times the block
size, less the seed G_0 = c, which the prep sets), and the outputs are those of
the same call without counters, bit for bit."""
import numpy as np
import pytest
import torch

from parity import assert_close
from schedule_model import Model
import oracle as O
from paper_2303_08879_amd import fockdiag as F
from paper_2303_08879_amd import workloads as W

pytestmark = pytest.mark.gpu

# (cutoffs, detected mask, b = 0): one to three undetected modes in first and
# later positions, an undetected block whose rows stream from HBM
CASES = [([4, 3, 3], 0b111, True), ([4, 3, 3], 0b111, False), ([3] * 6, 0x3F, True), ([5, 3, 3], 0b110, True),
         ([3, 4, 3], 0b101, False), ([3, 3, 3, 3], 0b1100, True), ([3, 2, 3], 0b100, True),
         ([12, 12, 2, 2], 0b1100, True)]


def counted_forward(circ, dtype, b_mode, total=None):
    print(f"[gpu] write counters {circ.cutoffs} {bin(circ.detected_mask)} {dtype} {b_mode} total={total}", flush=True)
    kw = {} if total is None else {"total_cutoff": total}
    plan = F.Plan(circ.cutoffs, circ.detected_mask, dtype, b_mode, **kw)
    wb, sb = plan.workspace(True)
    elem = 16 if dtype == torch.complex128 else 8
    dev = "cuda"
    ws = torch.empty(max(wb, 256), dtype=torch.uint8, device=dev)
    saved = torch.empty(sb, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(sb // elem, dtype=torch.int32, device=dev)
    T = lambda x: torch.tensor(np.asarray(x), dtype=dtype, device=dev)
    args = (T(circ.A), T(circ.b), T([circ.c]))
    rho = torch.empty(plan.out_shape, dtype=dtype, device=dev)
    F.fd_plan_set_write_counters(plan, cnt)
    F.fock_diag_fwd(plan, *args, rho, ws, saved)
    torch.cuda.synchronize()
    counts = cnt.cpu().numpy()
    F.fd_plan_set_write_counters(plan, None)
    rho2 = torch.empty_like(rho)
    F.fock_diag_fwd(plan, *args, rho2, ws, saved)
    torch.cuda.synchronize()
    F.fd_device_status(plan)
    targets = plan.query(F.FD_Q_TARGETS)
    return counts, targets, rho.cpu().numpy(), rho2.cpu().numpy()


@pytest.mark.parametrize("cut,mask,b_zero", CASES)
def test_every_stored_amplitude_written_once(cut, mask, b_zero):
    rng = np.random.default_rng(sum(cut) * 13 + mask)
    circ = W._circuit(rng, len(cut), 0.3, 0.8, lambda g, M: g.uniform(0.8, 0.95, size=M), cut, mask,
                      alpha_var=0.0 if b_zero else 0.1)
    counts, targets, rho, rho2 = counted_forward(circ, torch.complex128, "zero" if b_zero else "general")
    assert counts.max() <= 1, f"an amplitude written {counts.max()} times"
    model = Model(len(cut), cut, mask, b_zero)
    model.forward(circ.A, circ.b, circ.c)
    # every stored node is a block of B amplitudes, all written by Eq. recrel
    # except the seed G_0 = c (entry 0 of node 0), which the prep sets
    expect = sum(model.stored_counts().values()) * model.B - 1
    print(f"[counters] {cut} {bin(mask)} writes={int(counts.sum())} model={expect} targets={targets}", flush=True)
    assert int(counts.sum()) == expect == targets
    np.testing.assert_array_equal(rho, rho2)   # counting changes no value
    if np.prod([c * c for c in cut]) <= 400_000:
        assert_close(rho, O.fock_diag(circ.A, circ.b, circ.c, cut, mask), label="counted forward")


def test_write_counters_complex64_and_total_cutoff():
    rng = np.random.default_rng(77)
    circ = W._circuit(rng, 4, 0.3, 0.8, lambda g, M: g.uniform(0.8, 0.95, size=M), [4, 4, 3, 3], 0b1111)
    counts, targets, rho, rho2 = counted_forward(circ, torch.complex64, "zero")
    assert counts.max() <= 1 and int(counts.sum()) == targets
    np.testing.assert_array_equal(rho, rho2)
    # a total photon cutoff: only the levels up to N are swept and stored
    counts, targets, rho, rho2 = counted_forward(circ, torch.complex128, "zero", total=5)
    assert counts.max() <= 1 and int(counts.sum()) == targets
    np.testing.assert_array_equal(rho, rho2)
