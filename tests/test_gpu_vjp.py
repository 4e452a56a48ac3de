"""GPU reverse sweep (fock_diag_vjp) against the oracle's closed-form adjoint
(derivatives of the generating function, evaluated on the full box or on the
smallest box that holds the cotangent's support), and against central finite
differences of the GPU forward.  Bar (c128, tests/parity.py): relative error
<= 1e-10 on (dA, db, dc), normwise and entry by entry."""
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


def rand_triple(rng, M, b_zero, scale=0.25):
    D = 2 * M
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    X = scale * (X + X.T)
    b = np.zeros(D, complex) if b_zero else 0.4 * (rng.standard_normal(D) + 1j * rng.standard_normal(D))
    return X, b, 0.8 + 0.1j


def gpu_vjp(A, b, c, cut, mask, g, dtype=torch.complex128, b_mode="auto", use_saved=True):
    print(f"[gpu vjp] cut={cut} mask={bin(mask)} dtype={dtype} b_mode={b_mode} saved={use_saved}", flush=True)
    plan = ops.get_plan(cut, mask, dtype, b_mode)
    dev = "cuda"
    At = torch.as_tensor(A, dtype=dtype, device=dev).contiguous()
    bt = torch.as_tensor(b, dtype=dtype, device=dev).contiguous()
    ct = torch.as_tensor([c], dtype=dtype, device=dev)
    gt = torch.as_tensor(g, dtype=dtype, device=dev).contiguous()
    ws_bytes, saved_bytes = plan.workspace(True)
    rho = torch.empty(plan.out_shape, dtype=dtype, device=dev)
    dA, db, dc = torch.empty_like(At), torch.empty_like(bt), torch.empty_like(ct)
    if use_saved:
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        saved = torch.empty(saved_bytes, dtype=torch.uint8, device=dev)
        F.fock_diag_fwd(plan, At, bt, ct, rho, ws, saved)
        F.fock_diag_vjp(plan, At, bt, ct, saved, gt, dA, db, dc, ws)
    else:
        ws = torch.empty(ws_bytes + saved_bytes + 256, dtype=torch.uint8, device=dev)
        F.fock_diag_vjp(plan, At, bt, ct, None, gt, dA, db, dc, ws)
    torch.cuda.synchronize()
    F.fd_device_status(plan)
    return dA.cpu().numpy(), db.cpu().numpy(), complex(dc.cpu().numpy()[0])


def check(got, ref, tol=TOL, zero=(), label=""):
    """Element-wise and normwise parity of (dA, db, dc) over the concatenated
    gradient (tests/parity.py); ``zero`` names components that vanish by
    construction (db when b = 0 and every output has even weight; dc for a
    loss invariant under scaling c): their reference is checked to be zero
    and they are held to the absolute floor like every other tiny entry."""
    return assert_grad_close(got, ref, tol, label=label, zero=zero)


SMALL = [
    (2, [4, 4], 0b11, True), (2, [4, 4], 0b11, False), (3, [4, 3, 3], 0b111, True),
    (3, [4, 3, 3], 0b111, False), (1, [9], 0b1, False), (4, [3, 3, 3, 3], 0b1111, True),
    (4, [2, 4, 3, 2], 0b1111, False), (2, [5, 4], 0b10, True), (2, [5, 4], 0b10, False),
    (3, [4, 3, 3], 0b110, False), (3, [3, 4, 3], 0b101, True), (3, [3, 3, 4], 0b100, False),
    (3, [1, 4, 3], 0b011, False), (2, [4, 3], 0b00, False), (4, [2, 3, 1, 3], 0b1110, False),
    (5, [2, 2, 2, 2, 2], 0b11111, False),
    # two undetected modes with two and three detected modes (block kernel, four coordinates)
    (4, [3, 3, 3, 3], 0b1100, False), (4, [3, 3, 3, 3], 0b1100, True), (5, [3, 3, 2, 2, 2], 0b11100, False),
    (4, [3, 2, 3, 3], 0b1010, False),
    # the point kernel at six and seven detected modes
    (6, [3, 3, 3, 2, 2, 2], 0b111111, True), (6, [3, 3, 3, 2, 2, 2], 0b111111, False),
    (7, [3, 3, 2, 2, 2, 2, 2], 0b1111111, True), (7, [3, 3, 2, 2, 2, 2, 2], 0b1111111, False),
    # one undetected mode with five detected modes (the gradient batch's shape)
    (6, [4, 2, 2, 2, 2, 2], 0b111110, True), (6, [4, 2, 2, 2, 2, 2], 0b111110, False),
]


@pytest.mark.parametrize("M,cut,mask,bz", SMALL)
def test_vjp_small_random(M, cut, mask, bz):
    rng = np.random.default_rng(2000 + M * 37 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz)
    shape = O.fock_diag(A, b, c, cut, mask).shape
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = O.fock_diag_vjp(A, b, c, cut, mask, g)
    check(gpu_vjp(A, b, c, cut, mask, g), ref)
    check(gpu_vjp(A, b, c, cut, mask, g, use_saved=False), ref)
    if bz:
        check(gpu_vjp(A, b, c, cut, mask, g, b_mode="zero"), ref)


# three undetected modes (six block coordinates) with zero to three detected
# modes, and a mixed-cutoff block of 1296 entries
THREE_U = [
    (3, [3, 3, 3], 0b000, False), (4, [3, 2, 3, 3], 0b1000, False), (4, [3, 2, 3, 3], 0b1000, True),
    (5, [2, 3, 2, 3, 3], 0b11000, False), (5, [3, 3, 3, 2, 2], 0b11000, True),
    (6, [2, 2, 2, 3, 2, 2], 0b111000, False), (4, [4, 3, 3, 2], 0b1000, False),
]


@pytest.mark.parametrize("M,cut,mask,bz", THREE_U)
def test_vjp_three_undetected_modes(M, cut, mask, bz):
    rng = np.random.default_rng(4000 + M * 43 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz, scale=0.2)
    shape = O.fock_diag(A, b, c, cut, mask).shape
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = O.fock_diag_vjp(A, b, c, cut, mask, g)
    check(gpu_vjp(A, b, c, cut, mask, g), ref, label=f"{cut} {bin(mask)}")
    check(gpu_vjp(A, b, c, cut, mask, g, use_saved=False), ref, label=f"{cut} {bin(mask)} recompute")
    if bz:
        check(gpu_vjp(A, b, c, cut, mask, g, b_mode="zero"), ref, label=f"{cut} {bin(mask)} b=0")


# one undetected mode at cutoff 23-40: several row chunks of several rows
# per node, the last one ragged (rows of the first block coordinate split
# unevenly); the units of one chunk span several wavefronts
TALL = [(3, [25, 3, 3], 0b110, True), (3, [25, 3, 3], 0b110, False), (4, [23, 3, 2, 3], 0b1110, False),
        (2, [40, 4], 0b10, False)]


@pytest.mark.parametrize("M,cut,mask,bz", TALL)
def test_vjp_tall_row_chunks(M, cut, mask, bz):
    rng = np.random.default_rng(4700 + M * 43 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz, scale=0.15)
    shape = O.fock_diag(A, b, c, cut, mask).shape
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = O.fock_diag_vjp(A, b, c, cut, mask, g)
    check(gpu_vjp(A, b, c, cut, mask, g), ref, label=f"{cut} {bin(mask)}")
    check(gpu_vjp(A, b, c, cut, mask, g, use_saved=False), ref, label=f"{cut} {bin(mask)} recompute")
    if bz:
        check(gpu_vjp(A, b, c, cut, mask, g, b_mode="zero"), ref, label=f"{cut} {bin(mask)} b=0")


STREAMED = [(3, [9, 9, 3], 0b100, False), (3, [12, 12, 3], 0b100, False), (4, [12, 12, 2, 2], 0b1100, False),
            (3, [16, 16, 2], 0b100, False),
            (4, [12, 12, 2, 2], 0b1100, True), (4, [5, 5, 5, 2], 0b1000, False)]


@pytest.mark.parametrize("M,cut,mask,bz", STREAMED)
def test_vjp_streamed_block_rows(M, cut, mask, bz):
    # blocks whose rows or fill do not fit the LDS staging: the reverse block
    # units read the forward pivot rows from HBM and keep the neighbour terms
    # in their private slots; the reverse fill accumulates in the workspace
    rng = np.random.default_rng(4500 + M * 43 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz, scale=0.15)
    shape = O.fock_diag(A, b, c, cut, mask).shape
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = O.fock_diag_vjp(A, b, c, cut, mask, g)
    check(gpu_vjp(A, b, c, cut, mask, g), ref, label=f"{cut} {bin(mask)}")
    check(gpu_vjp(A, b, c, cut, mask, g, use_saved=False), ref, label=f"{cut} {bin(mask)} recompute")
    if bz:
        check(gpu_vjp(A, b, c, cut, mask, g, b_mode="zero"), ref, label=f"{cut} {bin(mask)} b=0")


def test_vjp_block_complex64_two_undetected_at_cutoff_9():
    rng = np.random.default_rng(45)
    cut, mask = [9, 9, 3], 0b100
    A, b, c = rand_triple(rng, 3, False, scale=0.2)
    shape = O.fock_diag(A, b, c, cut, mask).shape
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = O.fock_diag_vjp(A, b, c, cut, mask, g)
    got = gpu_vjp(A.astype(np.complex64), b.astype(np.complex64), np.complex64(c), cut, mask, g,
                  dtype=torch.complex64)
    err = O.rel_err(np.concatenate([got[0].ravel(), got[1].ravel(), [got[2]]]),
                    np.concatenate([ref[0].ravel(), ref[1].ravel(), [ref[2]]]))
    print(f"c64 vjp rel_err {cut} {bin(mask)} = {err:.3e}", flush=True)
    assert err < 1e-4


def test_vjp_ragged_multi_tile():
    rng = np.random.default_rng(21)
    A, b, c = rand_triple(rng, 4, False, scale=0.2)
    cut = [7, 6, 5, 4]
    shape = (7, 6, 5, 4)
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    check(gpu_vjp(A, b, c, cut, 0b1111, g), O.fock_diag_vjp(A, b, c, cut, 0b1111, g))
    A, b, c = rand_triple(rng, 3, True, scale=0.2)
    cut = [17, 4, 4]
    shape = (17, 17, 4, 4)
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    check(gpu_vjp(A, b, c, cut, 0b110, g), O.fock_diag_vjp(A, b, c, cut, 0b110, g))


def test_vjp_config1_dense_cotangent_and_determinism():
    circ = W.config1()
    rng = np.random.default_rng(31)
    g = rng.standard_normal((10, 10)) + 1j * rng.standard_normal((10, 10))
    ref = O.fock_diag_vjp(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, g)
    got1 = gpu_vjp(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, g)
    got2 = gpu_vjp(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, g)
    check(got1, ref, zero=("db",), label="config1")
    assert np.array_equal(got1[0], got2[0]) and np.array_equal(got1[1], got2[1]) and got1[2] == got2[2]
    # b = 0 with every mode detected: every output has even weight, so db = 0 exactly
    assert np.all(got1[1] == 0)


def test_vjp_config1_complex64_error_stated():
    circ = W.config1()
    rng = np.random.default_rng(32)
    g = rng.standard_normal((10, 10)) + 1j * rng.standard_normal((10, 10))
    rA, rb, rc = O.fock_diag_vjp(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, g)
    dA, db, dc = gpu_vjp(circ.A.astype(np.complex64), circ.b.astype(np.complex64), np.complex64(circ.c),
                         circ.cutoffs, circ.detected_mask, g, dtype=torch.complex64)
    err = O.rel_err(dA, rA)
    print(f"c64 vjp rel_err config1 dA = {err:.3e}, dc = {abs(dc - rc) / abs(rc):.3e}")
    assert err < 1e-4 and abs(dc - rc) / abs(rc) < 1e-4


def test_vjp_config2_dense_cotangent_sampled_against_slabs():
    # dense cotangent supported on a low corner n <= (2,2,2): the closed-form
    # adjoint needs only the box with cutoffs (30, 3, 3, 3)
    circ = W.config2()
    rng = np.random.default_rng(33)
    g = np.zeros((30, 30, 12, 12, 12), complex)
    gc = rng.standard_normal((30, 30, 3, 3, 3)) + 1j * rng.standard_normal((30, 30, 3, 3, 3))
    g[:, :, :3, :3, :3] = gc
    ref = O.fock_diag_vjp(circ.A, circ.b, circ.c, [30, 3, 3, 3], circ.detected_mask, gc)
    check(gpu_vjp(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, g), ref)


def config4_loss_torch(rho_block, psi):
    X = rho_block / torch.diagonal(rho_block).sum()
    return 1 - torch.abs(torch.conj(psi) @ X @ psi)


def test_vjp_config4_loss_against_closed_form_and_finite_differences():
    circ = W.config4()
    psi = circ.params["psi_target"]
    n = circ.params["n_star"]
    # GPU: autograd through the library's forward and reverse sweeps
    dev = "cuda"
    A = torch.tensor(circ.A, device=dev, requires_grad=True)
    b = torch.tensor(circ.b, device=dev, requires_grad=True)
    c = torch.tensor([circ.c], dtype=torch.complex128, device=dev, requires_grad=True)
    psi_t = torch.tensor(psi, device=dev)
    rho = ops.fock_diag_ad(A, b, c, circ.cutoffs, circ.detected_mask)
    L = config4_loss_torch(rho[(slice(None), slice(None)) + n], psi_t)
    L.backward()
    gA, gb, gc = A.grad.cpu().numpy(), b.grad.cpu().numpy(), complex(c.grad.cpu().numpy()[0])
    # oracle: cotangent of the loss at rho[:, :, n*] (CPU torch on the oracle's block), then the
    # closed-form adjoint on the box with detected cutoffs n* + 1
    small = [40] + [k + 1 for k in n]
    blk = O.fock_diag(circ.A, circ.b, circ.c, small, circ.detected_mask)[(slice(None), slice(None)) + n]
    Xb = torch.tensor(blk, requires_grad=True)
    config4_loss_torch(Xb, torch.tensor(psi)).backward()
    G = np.zeros((40, 40) + tuple(k + 1 for k in n), complex)
    G[(slice(None), slice(None)) + n] = Xb.grad.numpy()
    ref = O.fock_diag_vjp(circ.A, circ.b, circ.c, small, circ.detected_mask, G)
    check((gA, gb, gc), ref, zero=("dc",), label="config4 loss")
    assert np.linalg.norm(gb) > 0          # odd-weight entries of the block carry cotangent
    # central finite differences of the GPU forward, 32 random directions
    rng = np.random.default_rng(44)
    h = 1e-6

    def loss_at(Av, bv, cv):
        with torch.no_grad():
            r = ops.fock_diag(Av, bv, cv, circ.cutoffs, circ.detected_mask)
            return float(config4_loss_torch(r[(slice(None), slice(None)) + n], psi_t))

    worst = 0.0
    for _ in range(32):
        EA = rng.standard_normal(circ.A.shape) + 1j * rng.standard_normal(circ.A.shape)
        EA = 0.5 * (EA + EA.T)
        Eb = rng.standard_normal(10) + 1j * rng.standard_normal(10)
        Ec = complex(rng.standard_normal(), rng.standard_normal())
        fd = (loss_at(circ.A + h * EA, circ.b + h * Eb, circ.c + h * Ec)
              - loss_at(circ.A - h * EA, circ.b - h * Eb, circ.c - h * Ec)) / (2 * h)
        pred = np.real(np.sum(np.conj(gA) * EA) + np.sum(np.conj(gb) * Eb) + np.conj(gc) * Ec)
        worst = max(worst, abs(fd - pred) / max(abs(pred), 1e-3))
    print(f"config4 finite-difference worst relative disagreement = {worst:.2e}")
    assert worst < 1e-5


def test_vjp_config5_sampled_cotangent():
    # dense cotangent on the corner n <= 1 of the 8-mode, cutoff-8 problem
    circ = W.config5()
    rng = np.random.default_rng(35)
    gc = rng.standard_normal((2,) * 8) + 1j * rng.standard_normal((2,) * 8)
    g = np.zeros((8,) * 8, complex)
    g[(slice(0, 2),) * 8] = gc
    ref = O.fock_diag_vjp(circ.A, circ.b, circ.c, [2] * 8, circ.detected_mask, gc)
    check(gpu_vjp(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, g, b_mode="zero"), ref,
          zero=("db",), label="config5 corner")
