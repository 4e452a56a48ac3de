"""GPU parity of the density-matrix forward mode (fock_diag_jvp: rho and its
derivative along a direction (dA, db, dc); every mode detected, or undetected
modes through the block units) against the oracle's tangent recurrences
(Sec. 2.5), through the C ABI.  Bar (c128, tests/parity.py): relative error
<= 1e-10 for rho and for drho, normwise and entry by entry."""
import numpy as np
import pytest
import torch

import oracle as O
from parity import assert_close, assert_grad_close  # noqa: F401
from paper_2303_08879_amd import fockdiag as F
from paper_2303_08879_amd import ops

pytestmark = pytest.mark.gpu
TOL = 1e-10


def rand_triple(rng, M, b_zero, scale=0.25):
    D = 2 * M
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    X = scale * (X + X.T)
    b = np.zeros(D, complex) if b_zero else 0.4 * (rng.standard_normal(D) + 1j * rng.standard_normal(D))
    return X, b, 0.8 + 0.1j


def rand_dir(rng, M):
    D = 2 * M
    dA = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    db = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    return dA, db, complex(rng.standard_normal(), rng.standard_normal())


def gpu_jvp(A, b, c, dA, db, dc, cut, dtype=torch.complex128, b_mode="general", total=None, mask=None):
    print(f"[gpu] jvp cut={cut} total={total} mask={mask} dtype={dtype} b_mode={b_mode}", flush=True)
    if mask is None:
        mask = 0 if total is not None else (1 << len(cut)) - 1
    plan = F.Plan(cut, mask, dtype, b_mode, total_cutoff=total)
    T = lambda x: torch.tensor(np.asarray(x), dtype=dtype, device="cuda")
    ws = torch.empty(plan.jvp_workspace(), dtype=torch.uint8, device="cuda")
    rho = torch.empty(plan.out_shape, dtype=dtype, device="cuda")
    drho = torch.empty_like(rho)
    F.fock_diag_jvp(plan, T(A), T(b), T([c]), T(dA), T(db), T([dc]), rho, drho, ws)
    torch.cuda.synchronize()
    F.fd_device_status(plan)
    return rho.cpu().numpy(), drho.cpu().numpy()


CASES = [(1, [9]), (2, [4, 4]), (2, [6, 3]), (3, [4, 3, 3]), (3, [3, 1, 4]), (4, [3, 3, 3, 3]),
         (4, [2, 4, 3, 2])]


@pytest.mark.parametrize("M,cut", CASES)
@pytest.mark.parametrize("bz", [False, True])
def test_jvp_small(M, cut, bz):
    # bz: b = 0 at the base point, db != 0 (the tangent reaches the odd levels)
    rng = np.random.default_rng(500 + 17 * M + sum(cut) + bz)
    A, b, c = rand_triple(rng, M, bz)
    dA, db, dc = rand_dir(rng, M)
    mask = (1 << M) - 1
    ref, dref = O.fock_diag_jvp(A, b, c, cut, mask, dA, db, dc)
    for b_mode in (["general", "auto"] if bz else ["general"]):
        rho, drho = gpu_jvp(A, b, c, dA, db, dc, cut, b_mode=b_mode)
        assert_close(rho, ref, label="gpu_jvp:61")
        assert_close(drho, dref, label="gpu_jvp:62")


# Algorithm 2 plans: one, two and three undetected modes (first or not),
# nothing detected, several row chunks per node
UNDET = [(2, [5, 4], 0b10), (2, [5, 4], 0b01), (3, [4, 3, 3], 0b110), (3, [3, 4, 3], 0b101),
         (3, [4, 3, 3], 0b100), (4, [3, 3, 3, 3], 0b1100), (4, [3, 2, 3, 3], 0b1000), (2, [4, 3], 0b00),
         (3, [12, 3, 3], 0b110), (4, [3, 1, 4, 3], 0b1010)]


@pytest.mark.parametrize("M,cut,mask", UNDET)
@pytest.mark.parametrize("bz", [False, True])
def test_jvp_undetected_modes(M, cut, mask, bz):
    rng = np.random.default_rng(600 + 19 * M + sum(cut) + mask + bz)
    A, b, c = rand_triple(rng, M, bz, scale=0.2)
    dA, db, dc = rand_dir(rng, M)
    ref, dref = O.fock_diag_jvp(A, b, c, cut, mask, dA, db, dc)
    for b_mode in (["general", "auto"] if bz else ["general"]):
        rho, drho = gpu_jvp(A, b, c, dA, db, dc, cut, b_mode=b_mode, mask=mask)
        assert rho.shape == ref.shape
        assert_close(rho, ref, label=f"rho {cut} {bin(mask)}")
        assert_close(drho, dref, label=f"drho {cut} {bin(mask)}")
    rho, drho = gpu_jvp(A.astype(np.complex64), b.astype(np.complex64), np.complex64(c), dA.astype(np.complex64),
                        db.astype(np.complex64), np.complex64(dc), cut, dtype=torch.complex64, mask=mask)
    err = O.rel_err(drho, dref)
    print(f"c64 jvp rel_err {cut} {bin(mask)}: rho {O.rel_err(rho, ref):.3e} drho {err:.3e}", flush=True)
    assert err < 1e-4


def test_jvp_config2_full_size_sampled_patterns():
    # the 4-mode conditional workload at full size (undetected cutoff 30,
    # detected cutoffs 12, b != 0): rho and drho at sampled patterns n, each
    # against the oracle's tangent recurrences on the box with detected
    # cutoffs n + 1 (amplitudes and tangents do not depend on the cutoffs)
    from paper_2303_08879_amd import workloads as W
    circ = W.config2()
    rng = np.random.default_rng(71)
    dA, db, dc = rand_dir(rng, circ.M)
    rho, drho = gpu_jvp(circ.A, circ.b, circ.c, dA, db, dc, circ.cutoffs, mask=circ.detected_mask)
    assert rho.shape == (30, 30, 12, 12, 12)
    for n in [(0, 0, 0), (1, 1, 1), (5, 0, 0), (0, 7, 0), (0, 0, 11), (2, 1, 1), (1, 0, 3)]:
        cut = [circ.cutoffs[0]] + [k + 1 for k in n]
        ref, dref = O.fock_diag_jvp(circ.A, circ.b, circ.c, cut, circ.detected_mask, dA, db, dc)
        idx = (slice(None), slice(None)) + n
        assert_close(rho[idx], ref[idx], label=f"config2 rho{n}")
        assert_close(drho[idx], dref[idx], label=f"config2 drho{n}")


def test_jvp_multi_tile_sampled():
    # 5 modes, levels of up to 578 points (three 256-thread tiles, ragged
    # tails): sampled entries against the oracle on the box each needs
    # (cutoffs n_j + 1), and the value side against the forward call
    rng = np.random.default_rng(77)
    M, cut = 5, [6, 5, 6, 5, 6]
    A, b, c = rand_triple(rng, M, False, scale=0.15)
    dA, db, dc = rand_dir(rng, M)
    rho, drho = gpu_jvp(A, b, c, dA, db, dc, cut)
    samples = [(2, 2, 2, 1, 1), (4, 2, 1, 1, 0), (0, 3, 1, 2, 2), (1, 1, 1, 4, 1), (2, 0, 3, 0, 3),
               (1, 2, 2, 2, 1), (3, 1, 1, 1, 2), (0, 0, 2, 4, 3), (5, 1, 0, 1, 1), (1, 4, 0, 0, 4)]
    got, ref = [], []
    for n in samples:
        _, d = O.fock_diag_jvp(A, b, c, [k + 1 for k in n], (1 << M) - 1, dA, db, dc)
        got.append(drho[n])
        ref.append(d[n])
    assert_close(np.array(got), np.array(ref), label="gpu_jvp:81")
    plan = F.Plan(cut, (1 << M) - 1, torch.complex128, "general")
    T = lambda x: torch.tensor(np.asarray(x), dtype=torch.complex128, device="cuda")
    ws = torch.empty(plan.workspace(False)[0], dtype=torch.uint8, device="cuda")
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    F.fock_diag_fwd(plan, T(A), T(b), T([c]), out, ws)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), rho)


def test_jvp_vjp_adjoint_identity():
    # sum_k conj(g_k) drho_k = <dA, dA_vjp> + <db, db_vjp> + dc conj(dc_vjp),
    # with the reverse sweep's gradient of the same plan (a property that holds
    # at any size; here 4 modes with cutoff 7, 2401 outputs)
    rng = np.random.default_rng(5)
    M, cut = 4, [7, 7, 7, 7]
    A, b, c = rand_triple(rng, M, False, scale=0.12)
    dA, db, dc = rand_dir(rng, M)
    _, drho = gpu_jvp(A, b, c, dA, db, dc, cut)
    g = rng.standard_normal(cut) + 1j * rng.standard_normal(cut)
    plan = F.Plan(cut, (1 << M) - 1, torch.complex128, "general")
    T = lambda x: torch.tensor(np.asarray(x), dtype=torch.complex128, device="cuda")
    wb, sb = plan.workspace(True)
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    sv = torch.empty(sb, dtype=torch.uint8, device="cuda")
    At, bt, ct = T(A), T(b), T([c])
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    F.fock_diag_fwd(plan, At, bt, ct, out, ws, sv)
    gA, gb, gc = torch.empty_like(At), torch.empty_like(bt), torch.empty_like(ct)
    F.fock_diag_vjp(plan, At, bt, ct, sv, T(g), gA, gb, gc, ws)
    torch.cuda.synchronize()
    lhs = np.sum(np.conj(g) * drho)
    rhs = (np.sum(dA * np.conj(gA.cpu().numpy())) + np.sum(db * np.conj(gb.cpu().numpy()))
           + dc * np.conj(gc.cpu().numpy()[0]))
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))


@pytest.mark.parametrize("cut,N", [([6, 5, 7], 5), ([4, 4, 4], 20), ([3, 3, 3, 3], 4)])
def test_jvp_total_cutoff(cut, N):
    # total photon cutoff: rho and drho in level order over |n| <= N, against
    # the oracle on the box of per-mode cutoffs min(C_j, N + 1)
    rng = np.random.default_rng(N + len(cut))
    M = len(cut)
    A, b, c = rand_triple(rng, M, False, scale=0.2)
    dA, db, dc = rand_dir(rng, M)
    rho, drho = gpu_jvp(A, b, c, dA, db, dc, cut, total=N)
    dims = [min(C, N + 1) for C in cut]
    ref, dref = O.fock_diag_jvp(A, b, c, dims, (1 << M) - 1, dA, db, dc)
    pts, _ = O.level_points(cut, N)
    assert_close(rho, np.array([ref[n] for n in pts]), label="gpu_jvp:130")
    assert_close(drho, np.array([dref[n] for n in pts]), label="gpu_jvp:131")


def test_jvp_c64():
    rng = np.random.default_rng(9)
    A, b, c = rand_triple(rng, 3, False)
    dA, db, dc = rand_dir(rng, 3)
    cut = [5, 4, 5]
    ref, dref = O.fock_diag_jvp(A, b, c, cut, 0b111, dA, db, dc)
    rho, drho = gpu_jvp(A, b, c, dA, db, dc, cut, dtype=torch.complex64)
    assert O.rel_err(rho.astype(np.complex128), ref) <= 1e-5
    assert O.rel_err(drho.astype(np.complex128), dref) <= 1e-5


def test_torch_forward_ad():
    # torch.autograd.forward_ad through FockDiagFunction (fock_diag_jvp)
    import torch.autograd.forward_ad as fwAD
    rng = np.random.default_rng(21)
    cut = [4, 3, 5]
    A, b, c = rand_triple(rng, 3, False)
    dA, db, dc = rand_dir(rng, 3)
    ref, dref = O.fock_diag_jvp(A, b, c, cut, 0b111, dA, db, dc)
    T = lambda x: torch.tensor(np.asarray(x), dtype=torch.complex128, device="cuda")
    print("[gpu] forward_ad cut=[4, 3, 5]", flush=True)
    with fwAD.dual_level():
        rho = ops.fock_diag_ad(fwAD.make_dual(T(A), T(dA)), fwAD.make_dual(T(b), T(db)),
                               fwAD.make_dual(T([c]), T([dc])), cut, 0b111, b_mode="general")
        p, t = fwAD.unpack_dual(rho)
        p, t = p.cpu().numpy(), t.cpu().numpy()
    assert_close(p, ref, label="gpu_jvp:160")
    assert_close(t, dref, label="gpu_jvp:161")


def test_jvp_edges():
    rng = np.random.default_rng(33)
    A, b, c = rand_triple(rng, 3, False)
    dA, db, dc = rand_dir(rng, 3)
    # every cutoff 1: no level to sweep, rho = c and drho = dc
    rho, drho = gpu_jvp(A, b, c, dA, db, dc, [1, 1, 1])
    assert rho.shape == (1, 1, 1) and abs(rho.item() - c) <= 1e-15 and abs(drho.item() - dc) <= 1e-15
    # total photon cutoff 0: the vacuum only
    rho, drho = gpu_jvp(A, b, c, dA, db, dc, [4, 4, 4], total=0)
    assert rho.shape == (1,) and abs(rho[0] - c) <= 1e-15 and abs(drho[0] - dc) <= 1e-15
    # the zero direction gives a zero tangent; a cutoff-1 mode among detected modes
    rho, drho = gpu_jvp(A, b, c, 0 * dA, 0 * db, 0j, [4, 1, 5])
    assert np.all(drho == 0)
    ref, dref = O.fock_diag_jvp(A, b, c, [4, 1, 5], 0b111, dA, db, dc)
    rho, drho = gpu_jvp(A, b, c, dA, db, dc, [4, 1, 5])
    assert_close(rho, ref, label="jvp rho")
    assert_close(drho, dref, label="jvp drho")


@pytest.mark.parametrize("M", [6, 7, 8])
def test_jvp_many_modes_sampled(M):
    # 6-8 detected modes (cutoff 3 each): seeded patterns with total <= 5
    # against the oracle on each pattern's own box (cutoffs n_j + 1)
    rng = np.random.default_rng(300 + M)
    cut = [3] * M
    A, b, c = rand_triple(rng, M, False, scale=0.12)
    dA, db, dc = rand_dir(rng, M)
    rho, drho = gpu_jvp(A, b, c, dA, db, dc, cut)
    pats = set()
    while len(pats) < 8:
        n = tuple(int(v) for v in rng.integers(0, 3, size=M))
        if 0 < sum(n) <= 5:
            pats.add(n)
    got_v, got_t, ref_v, ref_t = [], [], [], []
    for n in sorted(pats):
        r, d = O.fock_diag_jvp(A, b, c, [k + 1 for k in n], (1 << M) - 1, dA, db, dc)
        got_v.append(rho[n])
        got_t.append(drho[n])
        ref_v.append(r[n])
        ref_t.append(d[n])
    assert_close(np.array(got_v), np.array(ref_v), label="gpu_jvp:203")
    assert_close(np.array(got_t), np.array(ref_t), label="gpu_jvp:204")


def test_jvp_config5_full_size():
    # the bench workload (8 modes, cutoff 8, 16.8M outputs, b = 0 at the base
    # point, general schedule): rho equals the forward sweep's bit for bit,
    # sampled tangent entries match the oracle on each pattern's own box, and
    # the adjoint identity with the reverse sweep holds over all outputs
    from paper_2303_08879_amd import workloads as W
    circ = W.config5()
    M, dt, dev = circ.M, torch.complex128, "cuda"
    rng = np.random.default_rng(12)
    dA, db, dc = rand_dir(rng, M)
    print("[gpu] jvp config5 full size", flush=True)
    plan = F.Plan(circ.cutoffs, circ.detected_mask, dt, "general")
    T = lambda x: torch.tensor(np.asarray(x), dtype=dt, device=dev)
    At, bt, ct = T(circ.A), T(circ.b), T([circ.c])
    ws = torch.empty(plan.jvp_workspace(), dtype=torch.uint8, device=dev)
    rho = torch.empty(plan.out_shape, dtype=dt, device=dev)
    drho = torch.empty_like(rho)
    F.fock_diag_jvp(plan, At, bt, ct, T(dA), T(db), T([dc]), rho, drho, ws)
    del ws
    wb, sb = plan.workspace(True)
    wsv = torch.empty(wb, dtype=torch.uint8, device=dev)
    sv = torch.empty(sb, dtype=torch.uint8, device=dev)
    rf = torch.empty_like(rho)
    F.fock_diag_fwd(plan, At, bt, ct, rf, wsv, sv)
    torch.cuda.synchronize()
    assert torch.equal(rho, rf)
    pats = set()
    while len(pats) < 8:
        n = tuple(int(v) for v in rng.integers(0, 3, size=M))
        if 0 < sum(n) <= 6:
            pats.add(n)
    d_np = drho.cpu().numpy()
    got, ref = [], []
    for n in sorted(pats):
        _, d = O.fock_diag_jvp(circ.A, circ.b, circ.c, [k + 1 for k in n], (1 << M) - 1, dA, db, dc)
        got.append(d_np[n])
        ref.append(d[n])
    assert_close(np.array(got), np.array(ref), label="gpu_jvp:244")
    g = T(rng.standard_normal(plan.out_shape) + 1j * rng.standard_normal(plan.out_shape))
    gA, gb, gc = torch.empty_like(At), torch.empty_like(bt), torch.empty_like(ct)
    F.fock_diag_vjp(plan, At, bt, ct, sv, g, gA, gb, gc, wsv)
    torch.cuda.synchronize()
    lhs = complex(torch.sum(torch.conj(g) * drho).item())
    rhs = (np.sum(dA * np.conj(gA.cpu().numpy())) + np.sum(db * np.conj(gb.cpu().numpy()))
           + dc * np.conj(gc.cpu().numpy()[0]))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
