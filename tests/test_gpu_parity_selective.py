"""GPU parity on every output of workloads beyond the Taylor box's reach,
against the selective CPU oracle (the paper's pivot schedules run as printed
in plain C, oracle/fock_selective.c): eight detected modes at cutoffs 4 and 5
(390625 probabilities), seven and six at cutoff 6, conditional states with one, two and three undetected modes, and a
block whose rows stream from HBM.  Bar (c128, tests/parity.py): 1e-10
normwise and entry by entry; complex64 errors are printed and bounded."""
import numpy as np
import pytest
import torch

from oracle import selective as S
from parity import assert_close, compare
from paper_2303_08879_amd import ops
from paper_2303_08879_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    # (modes, cutoffs, detected mask, displacement variance, b mode)
    (8, [4] * 8, 0xFF, 0.0, "zero"),
    (8, [4] * 8, 0xFF, 0.1, "general"),
    (8, [5] * 8, 0xFF, 0.0, "zero"),
    (7, [6] * 7, 0x7F, 0.1, "general"),
    (6, [6] * 6, 0x3F, 0.1, "general"),
    (4, [12, 6, 6, 6], 0b1110, 0.1, "general"),
    (5, [6, 6, 4, 4, 4], 0b11100, 0.0, "zero"),
    (5, [3, 3, 3, 4, 4], 0b11000, 0.1, "general"),
    (4, [12, 12, 2, 2], 0b1100, 0.1, "general"),
]


@pytest.mark.parametrize("M,cut,mask,av,b_mode", CASES)
def test_every_output_against_the_selective_oracle(M, cut, mask, av, b_mode):
    rng = np.random.default_rng(8000 + 13 * M + sum(cut) + mask)
    circ = W._circuit(rng, M, 0.2, 0.8, lambda g, MM: g.uniform(0.8, 0.95, size=MM), cut, mask, alpha_var=av)
    ref, piv = S.fock_diag_selective(circ.A, circ.b, circ.c, cut, mask, nthreads=16)
    print(f"[gpu] cut={cut} mask={bin(mask)} b_mode={b_mode} outputs={ref.size} oracle pivots={piv}", flush=True)
    out = ops.fock_diag(circ.A, circ.b, circ.c, cut, mask, dtype=torch.complex128, b_mode=b_mode)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got.shape == ref.shape
    assert_close(got, ref, label=f"{cut} {bin(mask)}")
    o64 = ops.fock_diag(circ.A.astype(np.complex64), circ.b.astype(np.complex64), np.complex64(circ.c), cut, mask,
                        dtype=torch.complex64, b_mode=b_mode)
    torch.cuda.synchronize()
    e = compare(o64.cpu().numpy(), ref)
    print(f"[c64] {cut} {bin(mask)} normwise {e['normwise']:.2e} element-wise {e['elementwise_large']:.2e}", flush=True)
    assert e["normwise"] <= 1e-5
