"""GPU parity of the total photon cutoff (plans from fd_plan_create_total,
p(n) for |n| <= N in level order) and of probability-sum stopping
(detection_probs_until) against the FP64 oracle, through the C ABI.  Bar
(c128): normwise relative error <= 1e-10; entries above the stopping level are
exactly zero."""
import itertools
import math

import numpy as np
import pytest
import torch

import oracle as O
from parity import assert_close, assert_grad_close  # noqa: F401
from paper_2303_08879_amd import fockdiag as F
from paper_2303_08879_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


def run_total(A, b, c, cut, N, b_mode="auto", eps=None):
    print(f"[gpu] total cut={cut} N={N} b_mode={b_mode} eps={eps}", flush=True)
    plan = F.Plan(cut, 0, torch.complex128, b_mode, total_cutoff=N)
    At = torch.tensor(A, dtype=torch.complex128, device="cuda")
    bt = torch.tensor(b, dtype=torch.complex128, device="cuda")
    ct = torch.tensor([c], dtype=torch.complex128, device="cuda")
    ws = torch.empty(max(plan.workspace(False)[0], 256), dtype=torch.uint8, device="cuda")
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    info = None
    if eps is None:
        F.detection_probs(plan, At, bt, ct, out, ws)
    else:
        info = F.detection_probs_until(plan, At, bt, ct, out, eps, ws)
    torch.cuda.synchronize()
    F.fd_device_status(plan)
    return out.cpu().numpy(), plan.level_offsets(), info


def lossy(seed, M, r=(0.3, 0.8), eta=0.8, alpha_var=0.0):
    rng = np.random.default_rng(seed)
    U = W.haar_unitary(rng, M)
    sd = math.sqrt(alpha_var / 2) if alpha_var else 0.0
    alpha = rng.normal(0, sd, M) + 1j * rng.normal(0, sd, M) if alpha_var else None
    sig, mu = W.gaussian_moments(rng.uniform(*r, size=M), U, np.full(M, eta), alpha)
    return W.bargmann_triple(sig, mu)


CASES = [([6, 5, 7], 5, 0.0), ([6, 5, 7], 5, 0.2), ([4, 1, 4, 3], 4, 0.1), ([9, 9], 12, 0.0),
         ([3, 3, 3, 3, 3, 3], 5, 0.1), ([5] * 8, 6, 0.0), ([4, 4, 4], 20, 0.2)]


@pytest.mark.parametrize("cut,N,alpha_var", CASES)
def test_total_cutoff_parity(cut, N, alpha_var):
    A, b, c = lossy(len(cut) * 13 + N, len(cut), alpha_var=alpha_var)
    p, offs, _ = run_total(A, b, c, cut, N)
    ref, roffs = O.probs_total(A, b, c, cut, N)
    assert offs == roffs
    assert_close(p, ref, label="gpu_total:58")


def test_large_box_small_simplex():
    # 8 modes with per-mode cutoff 40 (a box of 40^8 points) below a total
    # cutoff of 10 (43758 points): sampled entries of levels 3-4 against the
    # loop-hafnian expansion, and every entry with all n_j <= 1 against the
    # oracle's box of per-mode cutoff 2
    A, b, c = lossy(5, 8, eta=0.9, alpha_var=0.05)
    p, offs, _ = run_total(A, b, c, [40] * 8, 10)
    pts, roffs = O.level_points([40] * 8, 10)
    assert len(p) == len(pts) == math.comb(18, 8) and offs == roffs
    Ai, bi = O.to_interleaved(A, b)
    for k in range(offs[3], offs[5], 37):
        n = pts[k]
        kk = tuple(x for m in n for x in (m, m))
        ref = O.amplitude_bruteforce(Ai, bi, c, kk)
        assert abs(p[k] - ref) <= 1e-12 * abs(ref) + 1e-18, n
    where = {n: k for k, n in enumerate(pts)}
    corner = O.detection_probs(A, b, c, [2] * 8)
    got = np.array([p[where[n]] for n in itertools.product((0, 1), repeat=8)])
    assert_close(got, corner.reshape(-1), label="gpu_total:79")


@pytest.mark.parametrize("eps,expect", [(1e-2, 4), (1e-5, 10), (1e-8, None)])
def test_probability_sum_stopping(eps, expect):
    # levels 0..30 of a box with per-mode cutoff 12 hold 1 - 4.5e-7 of this
    # state's probability: the sum reaches 1 - eps at levels 4 and 10 (margins
    # > 1e-6), and never for eps = 1e-8 (every level is then returned)
    cut, N = [12, 12, 12], 30
    A, b, c = lossy(21, 3, r=(0.25, 0.45), eta=0.85)
    p, offs, (levels, mass) = run_total(A, b, c, cut, N, eps=eps)
    ref, roffs = O.probs_total(A, b, c, cut, N)
    lm = [np.real(ref[roffs[S]:roffs[S + 1]]).sum() for S in range(len(roffs) - 1)]
    assert O.stop_level(lm, eps) == expect
    assert levels == (expect + 1 if expect is not None else N + 1)
    assert abs(mass - sum(lm[:levels])) < 1e-12
    if expect is not None:
        assert mass >= 1 - eps
    cut_at = offs[levels]
    assert_close(p[:cut_at], ref[:cut_at], label="gpu_total:98")
    assert np.all(p[cut_at:] == 0)


def test_stopping_on_a_box_plan():
    # the stopping rule on an ordinary all-detected plan: rho in C order, zero above S*
    cut = [10, 10]
    A, b, c = lossy(8, 2, r=(0.4, 0.6), eta=0.9, alpha_var=0.1)
    plan = F.Plan(cut, 0b11, torch.complex128, "general")
    ws = torch.empty(plan.workspace(False)[0], dtype=torch.uint8, device="cuda")
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    levels, mass = F.detection_probs_until(plan, torch.tensor(A, device="cuda"), torch.tensor(b, device="cuda"),
                                           torch.tensor([c], dtype=torch.complex128, device="cuda"), out, 1e-3, ws)
    torch.cuda.synchronize()
    p = out.cpu().numpy()
    ref = O.detection_probs(A, b, c, cut)
    lm = [np.real(sum(ref[n] for n in itertools.product(range(10), range(10)) if sum(n) == S)) for S in range(19)]
    assert levels == O.stop_level(lm, 1e-3) + 1
    S = np.add.outer(np.arange(10), np.arange(10))
    assert np.all(p[S >= levels] == 0)
    assert_close(p[S < levels], ref[S < levels], label="gpu_total:118")


def test_total_cutoff_edges():
    A, b, c = lossy(3, 3, alpha_var=0.1)
    # N = 0: the vacuum only, p(0) = c
    p, offs, _ = run_total(A, b, c, [5, 5, 5], 0)
    assert offs == [0, 1] and len(p) == 1 and abs(p[0] - c) <= 1e-15 * abs(c)
    # every mode with cutoff 1: one point whatever N
    p, offs, _ = run_total(A, b, c, [1, 1, 1], 7)
    assert len(p) == 1 and abs(p[0] - c) <= 1e-15 * abs(c)
    # N above the box's top level: the whole box in level order
    p, offs, _ = run_total(A, b, c, [3, 2, 3], 50)
    ref, roffs = O.probs_total(A, b, c, [3, 2, 3], 50)
    assert offs == roffs
    assert_close(p, ref, label="total offsets")


def test_total_cutoff_c64():
    A, b, c = lossy(4, 4, alpha_var=0.1)
    cut, N = [6, 6, 6, 6], 7
    plan = F.Plan(cut, 0, torch.complex64, "general", total_cutoff=N)
    T = lambda x: torch.tensor(np.asarray(x), dtype=torch.complex64, device="cuda")
    ws = torch.empty(plan.workspace(False)[0], dtype=torch.uint8, device="cuda")
    out = torch.empty(plan.out_shape, dtype=torch.complex64, device="cuda")
    F.detection_probs(plan, T(A), T(b), T([c]), out, ws)
    torch.cuda.synchronize()
    ref, _ = O.probs_total(A, b, c, cut, N)
    assert O.rel_err(out.cpu().numpy().astype(np.complex128), ref) <= 1e-5


@pytest.mark.parametrize("cut,N", [([6, 5, 7], 5), ([4, 4, 4], 20), ([5, 1, 4, 3], 4), ([3, 3, 3, 3, 3], 6)])
def test_total_cutoff_vjp(cut, N):
    # gradient of sum_k conj(g_k) p(n_k) over the points below the cutoff; the
    # oracle differentiates the box of per-mode cutoffs min(C_j, N + 1) with
    # the cotangent placed on those points (zero elsewhere)
    print(f"[gpu] total vjp cut={cut} N={N}", flush=True)
    A, b, c = lossy(len(cut) * 5 + N, len(cut), alpha_var=0.1)
    dt, dev = torch.complex128, "cuda"
    plan = F.Plan(cut, 0, dt, "general", total_cutoff=N)
    wb, sb = plan.workspace(True)
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    sv = torch.empty(sb, dtype=torch.uint8, device=dev)
    T = lambda x: torch.tensor(np.asarray(x), dtype=dt, device=dev)
    At, bt, ct = T(A), T(b), T([c])
    out = torch.empty(plan.out_shape, dtype=dt, device=dev)
    F.fock_diag_fwd(plan, At, bt, ct, out, ws, sv)
    rng = np.random.default_rng(N)
    g = rng.standard_normal(out.shape[0]) + 1j * rng.standard_normal(out.shape[0])
    dA, db, dc = torch.empty_like(At), torch.empty_like(bt), torch.empty_like(ct)
    F.fock_diag_vjp(plan, At, bt, ct, sv, T(g), dA, db, dc, ws)
    torch.cuda.synchronize()
    dims = [min(C, N + 1) for C in cut]
    pts, _ = O.level_points(cut, N)
    gbox = np.zeros(dims, dtype=np.complex128)
    for k, n in enumerate(pts):
        gbox[n] = g[k]
    rA, rb, rc = O.fock_diag_vjp(A, b, c, dims, (1 << len(cut)) - 1, gbox)
    got = np.concatenate([dA.cpu().numpy().ravel(), db.cpu().numpy().ravel(), dc.cpu().numpy().ravel()])
    ref = np.concatenate([np.asarray(rA).ravel(), np.asarray(rb).ravel(), [rc]])
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= TOL
