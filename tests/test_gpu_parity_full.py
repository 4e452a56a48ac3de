"""Full-size parity at the workloads' real shapes, entry by entry, against
oracle references stored in tests/golden/ (written by
tests/golden/make_parity_refs.py, which calls only the oracle and the seeded
input generators).

* High detection patterns (Tier B: a pattern's block, and the adjoint of a
  cotangent supported on it, need only the box with detected cutoffs
  n_j + 1): forward blocks, and one reverse sweep whose cotangent is spread
  over every stored pattern, so levels far above the low corner carry
  cotangent through the reverse kernels.  The adjoint is linear in the
  cotangent: the reference is the sum of the per-pattern adjoints.
* The 8-mode, cutoff-8 state without loss: the adjoint of a dense cotangent
  over all 8^8 detection probabilities (every level of the reverse sweep).
* Every circuit of the 256-circuit uneven batch on sampled patterns, through
  the batched launch, in complex128 (bar 1e-10) and complex64 (error stated).
"""
import os

import numpy as np
import pytest
import torch

from parity import assert_close, assert_grad_close, compare
from paper_2303_08879_amd import batching as Bt
from paper_2303_08879_amd import fockdiag as F
from paper_2303_08879_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def circuit(name):
    return {"config2": W.config2, "config4": W.config4, "config5": W.config5,
            "config5b": lambda: W.config5b(n=1)[0]}[name]()


def fwd_vjp(circ, g, dtype=torch.complex128):
    b_mode = "zero" if not np.any(circ.b) else "general"
    print(f"[gpu] fwd+vjp cut={circ.cutoffs} mask={bin(circ.detected_mask)} b_mode={b_mode}", flush=True)
    plan = F.Plan(circ.cutoffs, circ.detected_mask, dtype, b_mode)
    T = lambda x: torch.tensor(np.asarray(x), dtype=dtype, device="cuda")
    A, b, c = T(circ.A), T(circ.b), T([circ.c])
    wsb, svb = plan.workspace(True)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    saved = torch.empty(svb, dtype=torch.uint8, device="cuda")
    rho = torch.empty(plan.out_shape, dtype=dtype, device="cuda")
    dA, db, dc = torch.empty_like(A), torch.empty_like(b), torch.empty_like(c)
    F.fock_diag_fwd(plan, A, b, c, rho, ws, saved)
    F.fock_diag_vjp(plan, A, b, c, saved, T(g), dA, db, dc, ws)
    torch.cuda.synchronize()
    F.fd_device_status(plan)
    out = rho.cpu().numpy(), (dA.cpu().numpy(), db.cpu().numpy(), complex(dc.cpu().numpy()[0]))
    plan.close()
    return out


@pytest.mark.parametrize("name", ["config2", "config4", "config5", "config5b"])
def test_high_patterns_forward_and_reverse(name):
    Z = np.load(os.path.join(GOLD, "parity_patterns.npz"))
    circ = circuit(name)
    ks = sorted(int(k.rsplit("_", 1)[1]) for k in Z.files if k.startswith(f"{name}_pattern_"))
    assert ks, name
    g = np.zeros(circ.out_shape, complex)
    rA, rb, rc = 0, 0, 0
    for k in ks:
        n = tuple(int(x) for x in Z[f"{name}_pattern_{k}"])
        g[(Ellipsis,) + n] = Z[f"{name}_g_{k}"]
        rA, rb, rc = rA + Z[f"{name}_dA_{k}"], rb + Z[f"{name}_db_{k}"], rc + Z[f"{name}_dc_{k}"][0]
    rho, grads = fwd_vjp(circ, g)
    for k in ks:
        n = tuple(int(x) for x in Z[f"{name}_pattern_{k}"])
        assert_close(rho[(Ellipsis,) + n], Z[f"{name}_rho_{k}"], label=f"{name} rho{n}")
    all_det = circ.detected_mask == (1 << circ.M) - 1
    zero = ("db",) if (all_det and not np.any(circ.b)) else ()
    assert_grad_close(grads, (rA, rb, rc), zero=zero, label=f"{name} grad over {len(ks)} patterns")


def test_pure_eight_modes_dense_cotangent_every_level():
    Z = np.load(os.path.join(GOLD, "parity_pure8.npz"))
    M, C = int(Z["M"]), int(Z["cut"])
    ci = W.pure_state(int(Z["seed"]), M, [C] * M, float(Z["r_lo"]), float(Z["r_hi"]))
    A, b, c = ci.params["rho_triple"]
    circ = W.Circuit(A, b, c, [C] * M, (1 << M) - 1)
    g = W.random_cotangent((C,) * M, seed=int(Z["cot_seed"]))
    rho, grads = fwd_vjp(circ, g)
    assert rho.shape == (C,) * M
    assert_grad_close(grads, (Z["dA"], Z["db"], Z["dc"][0]), zero=("db",), label="pure 8 modes, all outputs")


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_uneven_batch_every_circuit_sampled_patterns(dtype):
    Z = np.load(os.path.join(GOLD, "parity_batch.npz"))
    circs = W.config3()
    refs = {}
    for j, i in enumerate(Z["circ"]):
        n = tuple(int(x) for x in Z["pattern"][j] if x >= 0)
        refs.setdefault(int(i), []).append((n, Z["values"][Z["offsets"][j]:Z["offsets"][j + 1]]))
    assert sorted(refs) == list(range(len(circs)))
    print(f"[gpu] uneven batch of {len(circs)} circuits, dtype={dtype}", flush=True)
    runner = Bt.BatchRunner([(c.cutoffs, c.detected_mask) for c in circs], [(c.A, c.b, c.c) for c in circs],
                            dtype=dtype, budget_bytes=int(120e9))
    errs = {}

    def check_group(k, rho):
        torch.cuda.synchronize()
        for i, r in rho.items():
            got = np.concatenate([r[(Ellipsis,) + n].reshape(-1).cpu().numpy() for n, _ in refs[i]])
            ref = np.concatenate([v for _, v in refs[i]])
            if dtype == torch.complex128:
                assert_close(got, ref, label=f"circuit {i} {circs[i].cutoffs} {bin(circs[i].detected_mask)}")
            errs[i] = compare(got, ref)

    runner.run(True, check_group)
    runner.check_status()
    assert sorted(errs) == list(range(len(circs)))
    worst = max(e["normwise"] for e in errs.values())
    worst_el = max(e["elementwise_large"] for e in errs.values())
    print(f"[batch {dtype}] worst per-circuit normwise {worst:.3e}, element-wise {worst_el:.3e}", flush=True)
    if dtype == torch.complex64:
        assert worst <= 1e-4
    del runner
    torch.cuda.empty_cache()
