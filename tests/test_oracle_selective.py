"""Pins of the selective CPU oracle (Tier D: the paper's pivot schedules run
as printed, oracle/fock_selective.c) -- CPU only.

* every selected amplitude equals the Taylor box's (Tier A) entry by entry,
  with and without displacement, one to three undetected modes, modes of
  cutoff 1, nothing detected;
* the schedules are self-sufficient (the oracle errors on a read before its
  write) and consistent (it errors when two writes of one amplitude differ);
* the number of pivots of Algorithm 1 is the count of App. B.1, and that of
  Algorithm 2 is the undetected block's entries (step 1) plus the block times
  the Algorithm 1 count over the detected modes (step 2);
* threads change nothing: the pivots of one weight are independent (Sec. 2.2).
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import selective as S


def rand_triple(rng, M, b_zero, scale=0.25):
    D = 2 * M
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    X = scale * (X + X.T)
    b = np.zeros(D, complex) if b_zero else 0.4 * (rng.standard_normal(D) + 1j * rng.standard_normal(D))
    return X, b, 0.8 + 0.1j


def alg1_pivots(C):
    # App. B.1: (C_1 - 1) prod_{j>1} C_j diagonal pivots, sum_K (C_K - 1) prod_{j>K} C_j off-diagonal ones
    return (C[0] - 1) * math.prod(C[1:]) + sum((C[K] - 1) * math.prod(C[K + 1:]) for K in range(len(C)))


SHAPES = [
    (2, [4, 4], 0b11, False), (2, [4, 4], 0b11, True), (3, [4, 3, 3], 0b111, False), (1, [9], 0b1, False),
    (4, [3, 3, 3, 3], 0b1111, True), (4, [2, 4, 3, 2], 0b1111, False), (2, [5, 4], 0b10, False),
    (2, [5, 4], 0b01, True), (3, [4, 3, 3], 0b110, False), (3, [3, 4, 3], 0b101, True), (3, [4, 3, 3], 0b100, False),
    (4, [3, 3, 3, 3], 0b1100, False), (4, [3, 2, 3, 3], 0b1000, False), (2, [4, 3], 0b00, False),
    (3, [1, 4, 3], 0b011, False), (4, [2, 3, 1, 3], 0b1110, True), (3, [3, 1, 3], 0b100, False),
]


@pytest.mark.parametrize("M,cut,mask,bz", SHAPES)
def test_selective_equals_taylor_box(M, cut, mask, bz):
    rng = np.random.default_rng(7000 + 31 * M + sum(cut) + mask + bz)
    A, b, c = rand_triple(rng, M, bz)
    ref = O.fock_diag(A, b, c, cut, mask)
    got, piv = S.fock_diag_selective(A, b, c, cut, mask)
    assert got.shape == ref.shape
    amax = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-13 * amax
    big = np.abs(ref) >= 1e-6 * amax
    assert np.max(np.abs(got - ref)[big] / np.abs(ref)[big]) <= 1e-12


@pytest.mark.parametrize("C", [[4, 4], [5, 3, 4], [3, 3, 3, 3], [2, 6, 2, 3, 2], [8] * 4])
def test_algorithm1_pivot_count_is_appendix_b1(C):
    rng = np.random.default_rng(11)
    A, b, c = rand_triple(rng, len(C), False, scale=0.1)
    _, piv = S.fock_diag_selective(A, b, c, C, (1 << len(C)) - 1)
    assert piv == alg1_pivots(C)


@pytest.mark.parametrize("cut,mask", [([5, 4, 3], 0b110), ([3, 4, 2, 3], 0b1100), ([3, 2, 3, 3], 0b1000)])
def test_algorithm2_pivot_count(cut, mask):
    rng = np.random.default_rng(12)
    M = len(cut)
    A, b, c = rand_triple(rng, M, False, scale=0.1)
    _, piv = S.fock_diag_selective(A, b, c, cut, mask)
    U = [cut[j] for j in range(M) if not (mask >> j) & 1]
    Dc = [cut[j] for j in range(M) if (mask >> j) & 1]
    block = math.prod(x * x for x in U)
    assert piv == block + block * alg1_pivots(Dc)


def test_threads_change_nothing():
    rng = np.random.default_rng(13)
    A, b, c = rand_triple(rng, 5, False, scale=0.15)
    one, p1 = S.fock_diag_selective(A, b, c, [4, 3, 4, 3, 4], 0b11110, nthreads=1)
    many, p8 = S.fock_diag_selective(A, b, c, [4, 3, 4, 3, 4], 0b11110, nthreads=8)
    assert p1 == p8 and np.array_equal(one, many)


def test_beyond_the_taylor_box_against_single_patterns():
    # eight detected modes at cutoff 4 (65536 probabilities; the Taylor box
    # would hold 4^16 entries): sampled patterns against Tier B, element-wise
    rng = np.random.default_rng(14)
    A, b, c = rand_triple(rng, 8, True, scale=0.12)
    cut = [4] * 8
    got, piv = S.fock_diag_selective(A, b, c, cut, 0xFF, nthreads=4)
    assert piv == alg1_pivots(cut)
    for n in [(0,) * 8, (1, 0, 2, 0, 0, 3, 0, 1), (3, 3, 0, 0, 0, 0, 0, 0), (0, 0, 0, 0, 0, 0, 2, 3), (1,) * 8]:
        ref = O.fock_diag_pattern(A, b, c, cut, 0xFF, n)
        assert abs(got[n] - ref) <= 1e-12 * max(abs(ref), 1e-300) + 1e-300, n
