"""GPU forward parity: the HIP sweep against the FP64 oracle, called through
the C ABI.  Bar (c128, tests/parity.py): relative error <= 1e-10 normwise and
entry by entry on every entry above 1e-6 of the largest (expected ~1e-15:
both sides sum the same Taylor coefficients by different routes in double
precision).  c64: the error is measured and bounded loosely
(single precision accumulates ~1e-7 per level)."""
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


def rand_triple(rng, M, b_zero, scale=0.25):
    D = 2 * M
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    X = scale * (X + X.T)
    b = np.zeros(D, complex) if b_zero else 0.4 * (rng.standard_normal(D) + 1j * rng.standard_normal(D))
    return X, b, 0.8 + 0.1j


def gpu(A, b, c, cut, mask, dtype=torch.complex128, b_mode="auto"):
    print(f"[gpu] cut={cut} mask={bin(mask)} dtype={dtype} b_mode={b_mode}", flush=True)
    out = ops.fock_diag(A, b, c, cut, mask, dtype=dtype, b_mode=b_mode)
    torch.cuda.synchronize()
    return out.cpu().numpy()


SMALL = [
    (2, [4, 4], 0b11, True), (2, [4, 4], 0b11, False), (3, [4, 3, 3], 0b111, True),
    (3, [4, 3, 3], 0b111, False), (1, [9], 0b1, False), (1, [9], 0b1, True),
    (4, [3, 3, 3, 3], 0b1111, True), (4, [2, 4, 3, 2], 0b1111, False),
    (2, [5, 4], 0b10, True), (2, [5, 4], 0b10, False), (3, [4, 3, 3], 0b110, False),
    (3, [3, 4, 3], 0b101, True), (3, [3, 3, 4], 0b011, False), (3, [3, 3, 4], 0b100, False),
    (3, [1, 4, 3], 0b011, False), (3, [3, 1, 3], 0b101, True), (2, [4, 3], 0b00, False),
    (4, [2, 3, 1, 3], 0b1110, False), (5, [2, 2, 2, 2, 2], 0b11111, False),
    (4, [3, 3, 3, 3], 0b1100, False), (5, [3, 3, 2, 2, 2], 0b11100, True), (4, [3, 2, 3, 3], 0b1010, False),
    (6, [3, 3, 3, 2, 2, 2], 0b111111, False), (7, [3, 3, 2, 2, 2, 2, 2], 0b1111111, True),
    (6, [4, 2, 2, 2, 2, 2], 0b111110, False),
]


@pytest.mark.parametrize("M,cut,mask,bz", SMALL)
def test_small_random_triples(M, cut, mask, bz):
    rng = np.random.default_rng(1000 + M * 37 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz)
    ref = O.fock_diag(A, b, c, cut, mask)
    for b_mode in (["auto", "zero"] if bz else ["auto", "general"]):
        out = gpu(A, b, c, cut, mask, b_mode=b_mode)
        assert out.shape == ref.shape
        assert_close(out, ref, label=str(b_mode))


# block shapes with four or more detected modes, or three with two undetected
# modes: the forward block unit fences its row and bridge iterations there;
# undetected cutoffs large enough for several row chunks
FENCED = [
    (5, [9, 4, 3, 3, 3], 0b11110), (6, [8, 3, 3, 2, 3, 3], 0b111110), (5, [5, 5, 4, 3, 3], 0b11100),
    (6, [4, 4, 3, 3, 2, 3], 0b111100), (7, [5, 2, 2, 3, 2, 2, 3], 0b1111110),
]


@pytest.mark.parametrize("M,cut,mask", FENCED)
@pytest.mark.parametrize("bz", [True, False])
def test_fenced_block_shapes(M, cut, mask, bz):
    rng = np.random.default_rng(2000 + M * 31 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz, scale=0.2)
    ref = O.fock_diag(A, b, c, cut, mask)
    for b_mode in (["auto", "zero"] if bz else ["general"]):
        out = gpu(A, b, c, cut, mask, b_mode=b_mode)
        assert_close(out, ref, label=str(b_mode))


# one undetected mode at cutoff 23-40: several row chunks of several rows
# per node, the last one ragged; one chunk's unit spans several wavefronts
TALL = [(3, [25, 3, 3], 0b110, True), (3, [25, 3, 3], 0b110, False), (4, [23, 3, 2, 3], 0b1110, False),
        (2, [40, 4], 0b10, False)]


@pytest.mark.parametrize("M,cut,mask,bz", TALL)
def test_tall_row_chunks(M, cut, mask, bz):
    rng = np.random.default_rng(2700 + M * 31 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz, scale=0.15)
    ref = O.fock_diag(A, b, c, cut, mask)
    for b_mode in (["auto", "zero"] if bz else ["general"]):
        out = gpu(A, b, c, cut, mask, b_mode=b_mode)
        assert_close(out, ref, label=f"{cut} {bin(mask)} {b_mode}")


# three undetected modes (six block coordinates), with zero to four detected
# modes; blocks of several row chunks; two undetected modes at cutoff 9 (6561
# entries per node, more than one LDS tile per row chunk)
THREE_U = [
    (3, [3, 3, 3], 0b000, False), (4, [3, 2, 3, 3], 0b1000, False), (4, [3, 2, 3, 3], 0b1000, True),
    (5, [2, 3, 2, 3, 3], 0b11000, False), (5, [3, 3, 3, 2, 2], 0b11000, True),
    (6, [2, 2, 2, 3, 2, 2], 0b111000, False), (7, [2, 2, 2, 2, 2, 2, 2], 0b1111000, True),
    (4, [4, 4, 4, 3], 0b1000, False), (4, [4, 3, 3, 3], 0b1000, False), (3, [9, 9, 3], 0b100, False),
]


# blocks whose rows do not fit the LDS staging stream from HBM: two
# undetected modes at cutoff 12 (20736 entries; the fill streams, and with two
# detected modes the block units too) and 16 (65536 entries), three at cutoff 5
STREAMED = [(3, [12, 12, 3], 0b100, False), (4, [12, 12, 2, 2], 0b1100, False), (4, [12, 12, 2, 2], 0b1100, True),
            (4, [5, 5, 5, 2], 0b1000, False), (3, [16, 16, 2], 0b100, False)]


@pytest.mark.parametrize("M,cut,mask,bz", STREAMED)
def test_streamed_block_rows(M, cut, mask, bz):
    rng = np.random.default_rng(3500 + M * 41 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz, scale=0.15)
    ref = O.fock_diag(A, b, c, cut, mask)
    for b_mode in (["auto", "zero"] if bz else ["general"]):
        out = gpu(A, b, c, cut, mask, b_mode=b_mode)
        assert out.shape == ref.shape
        assert_close(out, ref, label=f"{cut} {bin(mask)} {b_mode}")
    out = gpu(A.astype(np.complex64), b.astype(np.complex64), np.complex64(c), cut, mask, dtype=torch.complex64)
    err = O.rel_err(out, ref)
    print(f"c64 rel_err {cut} {bin(mask)} = {err:.3e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("M,cut,mask,bz", THREE_U)
def test_three_undetected_modes_and_large_blocks(M, cut, mask, bz):
    rng = np.random.default_rng(3000 + M * 41 + sum(cut) + mask)
    A, b, c = rand_triple(rng, M, bz, scale=0.2)
    ref = O.fock_diag(A, b, c, cut, mask)
    for b_mode in (["auto", "zero"] if bz else ["auto", "general"]):
        out = gpu(A, b, c, cut, mask, b_mode=b_mode)
        assert out.shape == ref.shape
        assert_close(out, ref, label=f"{cut} {bin(mask)} {b_mode}")
    if M == 4 and cut[0] == 3:
        out = gpu(A.astype(np.complex64), b.astype(np.complex64), np.complex64(c), cut, mask, dtype=torch.complex64)
        err = O.rel_err(out, ref)
        print(f"c64 rel_err {cut} {bin(mask)} = {err:.3e}", flush=True)
        assert err < 1e-5


def test_ragged_multi_tile_levels():
    # levels wider than one 256-thread tile, ragged tails, unequal cutoffs
    rng = np.random.default_rng(7)
    A, b, c = rand_triple(rng, 4, False, scale=0.2)
    cut = [9, 7, 6, 5]
    ref = O.fock_diag(A, b, c, cut, 0b1111)
    out = gpu(A, b, c, cut, 0b1111)
    assert_close(out, ref, label="gpu_forward:85")
    A, b, c = rand_triple(rng, 3, False, scale=0.2)
    cut = [17, 5, 4]           # undetected block 289 entries: more than one tile per node
    ref = O.fock_diag(A, b, c, cut, 0b110)
    out = gpu(A, b, c, cut, 0b110)
    assert_close(out, ref, label="gpu_forward:90")


def test_config1_against_full_density_matrix():
    circ = W.config1()
    ref = O.fock_diag(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask)
    out = gpu(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask)
    assert_close(out, ref, label="gpu_forward:97")
    assert np.max(np.abs(out.imag)) < 1e-15
    probs = ops.detection_probs(circ.A, circ.b, circ.c, circ.cutoffs).cpu().numpy()
    assert_close(probs, ref, label="gpu_forward:100")


def test_config1_complex64_error_stated():
    circ = W.config1()
    ref = O.fock_diag(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask)
    out = gpu(circ.A.astype(np.complex64), circ.b.astype(np.complex64), np.complex64(circ.c), circ.cutoffs,
              circ.detected_mask, dtype=torch.complex64)
    err = O.rel_err(out, ref)
    print(f"c64 rel_err config1 = {err:.3e}")
    assert err < 1e-5


def test_config2_sampled_patterns_and_corner():
    circ = W.config2()
    out = gpu(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask)
    assert out.shape == (30, 30, 12, 12, 12)
    # Tier B: the whole low corner n <= (2,2,2) from one box, then single patterns
    corner = O.fock_diag(circ.A, circ.b, circ.c, [30, 3, 3, 3], circ.detected_mask)
    assert_close(out[:, :, :3, :3, :3], corner, label="gpu_forward:119")
    for n in [(11, 0, 0), (0, 11, 0), (0, 0, 11), (4, 2, 1), (1, 5, 2), (2, 1, 6), (7, 3, 0)]:
        ref = O.fock_diag_pattern(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, n)
        assert_close(out[(slice(None), slice(None)) + n], ref, label=str(n))
    # conditional blocks are Hermitian
    blk = out[:, :, 2, 1, 3]
    assert np.max(np.abs(blk - blk.conj().T)) <= 1e-12 * np.max(np.abs(blk))


def test_config5_full_size_pure_variant():
    # config 5 without loss is a pure state: p(n) = |psi_n|^2 with psi from the
    # state-vector recurrence with A_psi = U diag(-tanh r) U^T (Sec. 2.1-2.2).
    circ = W.config5()
    r, U = circ.params["r"], circ.params["U"]
    sig, mu = W.gaussian_moments(r, U, 1.0)
    A, b, c = W.bargmann_triple(sig, mu)
    out = gpu(A, b, c, circ.cutoffs, circ.detected_mask, b_mode="zero")
    Apsi = U @ np.diag(-np.tanh(r)) @ U.T
    psi = O.taylor_box(Apsi, np.zeros(8), math.sqrt(np.prod(1 / np.cosh(r))), [8] * 8)
    ref = np.abs(psi) ** 2
    assert_close(out, ref, label="gpu_forward:139")
    # a lossless squeezed state has even total photon number only
    tot = np.indices(out.shape).sum(axis=0)
    assert np.max(np.abs(out[tot % 2 == 1])) <= 1e-13 * np.max(np.abs(out))


def test_config5_lossy_sampled_patterns():
    circ = W.config5()
    out = gpu(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, b_mode="zero")
    assert out.shape == (8,) * 8
    corner = O.fock_diag(circ.A, circ.b, circ.c, [2] * 8, circ.detected_mask)
    assert_close(out[(slice(0, 2),) * 8], corner, label="gpu_forward:150")
    rng = np.random.default_rng(55)
    for _ in range(12):
        n = [0] * 8
        for j in rng.choice(8, size=3, replace=False):
            n[j] = int(rng.integers(1, 8))
        ref = O.fock_diag_pattern(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask, tuple(n))
        assert abs(out[tuple(n)] - ref) <= TOL * max(abs(ref), 1e-300) + 1e-300, n
    assert np.max(np.abs(out.imag)) < 1e-14


def test_device_status_reports_bad_inputs():
    circ = W.config1()
    plan = ops.get_plan(circ.cutoffs, circ.detected_mask, torch.complex128, "zero")
    A = torch.as_tensor(circ.A, device="cuda")
    b = torch.full((4,), 0.1 + 0j, dtype=torch.complex128, device="cuda")
    c = torch.as_tensor([circ.c], dtype=torch.complex128, device="cuda")
    ws = torch.empty(plan.workspace(False)[0], dtype=torch.uint8, device="cuda")
    rho = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    F.fd_device_status(plan)
    F.fock_diag_fwd(plan, A, b, c, rho, ws)
    with pytest.raises(F.FockDiagError) as ei:
        F.fd_device_status(plan)
    assert ei.value.status == F.FD_ERR_INVALID_ARG
    b.zero_()
    A[0, 0] = float("nan")
    F.fock_diag_fwd(plan, A, b, c, rho, ws)
    with pytest.raises(F.FockDiagError) as ei:
        F.fd_device_status(plan)
    assert ei.value.status == F.FD_ERR_NONFINITE
    F.fd_device_status(plan)   # cleared


def test_workspace_too_small_is_rejected():
    circ = W.config1()
    plan = ops.get_plan(circ.cutoffs, circ.detected_mask, torch.complex128, "auto")
    A = torch.as_tensor(circ.A, device="cuda")
    b = torch.as_tensor(circ.b, device="cuda")
    c = torch.as_tensor([circ.c], dtype=torch.complex128, device="cuda")
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    rho = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(F.FockDiagError) as ei:
        F.fock_diag_fwd(plan, A, b, c, rho, ws)
    assert ei.value.status == F.FD_ERR_WORKSPACE
