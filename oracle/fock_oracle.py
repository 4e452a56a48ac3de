"""Plain float64 oracle for Fock amplitudes of mixed Gaussian states.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and ``bench.py``'s CPU-baseline leg, never by the GPU library.

What the selective GPU path computes has a plain definition.  For the
Bargmann triple (A, b, c) of a state (A complex symmetric D x D, D = 2M for a
density matrix, Eq. cases_D), the Fock amplitudes are the scaled Taylor
coefficients

    rho_k = d^k F(0) / sqrt(k!),      F(z) = c * exp(1/2 z^T A z + b^T z),

because d_i F = (b_i + (A z)_i) F turns into exactly the recurrence Eq. recrel
of Sec. 2.1.  Every amplitude therefore has one value, whatever cutoffs or
pivot route are used to reach it.  The selective algorithms (Algorithms 1 and
2, Sec. 3) return a subset of these numbers:

    rho[k_U, l_U, n_D] = <k_U, n_D| rho |l_U, n_D>

i.e. every ket/bra pair of the undetected modes U and the diagonal of every
detected mode D (Sec. 3.1 probability p(n) = G_{n1 n1 ... nM nM}; Sec. 3.2
conditional blocks).

This module writes that definition out in the most direct way:

* ``taylor_box`` (Tier A) fills the whole box 0 <= k < dims with Eq. recrel,
  taking as pivot direction the first non-zero axis of each index (the naive
  full density-matrix route of Sec. 3.1), vectorised over slabs.
* ``fock_diag`` / ``fock_diag_pattern`` select the returned entries; a
  pattern's entries only need the box with cutoffs n_j + 1 (Tier B).
* ``amplitude_bruteforce`` (Tier E) expands the generating function into loop
  hafnians: a different algorithm, used to pin Tier A.
* ``adjoint_closed_form`` differentiates the generating function directly;
  ``tangent_recurrences`` runs the paper's forward-mode recurrences
  (Eqs. recrel_dB and recrel_dA, Sec. 2.5) as a cross-check;
  ``fock_diag_jvp`` sums them along one direction (forward mode of rho).

Index convention: a density-matrix index is interleaved per mode,
[ket_1, bra_1, ket_2, bra_2, ...] (Sec. 2.1: each pair of consecutive indices
belongs to one mode).  The triple is handed over in block order
[ket_1..ket_M, bra_1..bra_M]; ``to_interleaved`` converts it.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

__all__ = [
    "to_interleaved",
    "from_interleaved",
    "taylor_box",
    "full_density_matrix",
    "state_vector",
    "select_outputs",
    "fock_diag",
    "fock_diag_pattern",
    "detection_probs",
    "level_points",
    "probs_total",
    "stop_level",
    "loop_hafnian",
    "amplitude_bruteforce",
    "adjoint_closed_form",
    "fock_diag_vjp",
    "tangent_recurrences",
    "fock_diag_jvp",
    "probs_vjp_pure",
    "rel_err",
]


# --------------------------------------------------------------------------
# index conventions
# --------------------------------------------------------------------------
def _perm_block_to_interleaved(M: int) -> np.ndarray:
    """perm[p] = block-order index of interleaved position p (ket_j -> 2j, bra_j -> 2j+1)."""
    perm = np.empty(2 * M, dtype=np.int64)
    perm[0::2] = np.arange(M)
    perm[1::2] = M + np.arange(M)
    return perm


def to_interleaved(A, b):
    """Block order [ket_1..ket_M, bra_1..bra_M] -> interleaved [ket_1, bra_1, ...]."""
    A = np.asarray(A, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    perm = _perm_block_to_interleaved(A.shape[0] // 2)
    return A[np.ix_(perm, perm)], b[perm]


def from_interleaved(Ai, bi):
    """Inverse of ``to_interleaved``."""
    Ai = np.asarray(Ai)
    bi = np.asarray(bi)
    perm = _perm_block_to_interleaved(Ai.shape[0] // 2)
    A = np.empty_like(Ai)
    A[np.ix_(perm, perm)] = Ai
    b = np.empty_like(bi)
    b[perm] = bi
    return A, b


# --------------------------------------------------------------------------
# Tier A: the definition, by Eq. recrel over the whole box
# --------------------------------------------------------------------------
def _shift_down(X: np.ndarray, axis: int) -> np.ndarray:
    """Y[..., i, ...] = X[..., i-1, ...] along ``axis`` (zero at i = 0)."""
    Y = np.zeros_like(X)
    src = [slice(None)] * X.ndim
    dst = [slice(None)] * X.ndim
    src[axis] = slice(0, X.shape[axis] - 1)
    dst[axis] = slice(1, None)
    Y[tuple(dst)] = X[tuple(src)]
    return Y


def _sqrt_index(n: int, axis: int, ndim: int) -> np.ndarray:
    shape = [1] * ndim
    shape[axis] = n
    return np.sqrt(np.arange(n, dtype=np.float64)).reshape(shape)


def taylor_box(A, b, c, dims):
    """All rho_k for 0 <= k < dims (any D = len(dims)), float64 complex.

    Eq. recrel with i = d, the first non-zero axis of the target:
        G_{k+1_d} = ( b_d G_k + sum_l sqrt(k_l) A_{d l} G_{k-1_l} ) / sqrt(k_d + 1).
    Entries whose first non-zero axis is d form the slabs k_d = 1, 2, ... of the
    sub-box whose axes before d are zero; slab k_d + 1 needs slabs k_d and
    k_d - 1 only, and inside a slab the terms with l > d are shifts along l.
    The sub-boxes are filled from the last axis to the first.
    """
    A = np.asarray(A, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    dims = tuple(int(x) for x in dims)
    D = len(dims)
    assert A.shape == (D, D) and b.shape == (D,)
    if D == 0:
        return np.array(complex(c))
    if min(dims) <= 0:
        return np.zeros(dims, dtype=np.complex128)
    G = np.zeros(dims, dtype=np.complex128)
    G[(0,) * D] = c
    for d in range(D - 1, -1, -1):
        sub = G[(0,) * d]          # view over axes d..D-1, leading axes fixed at 0
        nrest = D - d - 1
        roots = [_sqrt_index(dims[l], l - d - 1, nrest) for l in range(d + 1, D)]
        for k in range(dims[d] - 1):
            cur = sub[k]
            acc = b[d] * cur
            if k >= 1:
                acc = acc + math.sqrt(k) * A[d, d] * sub[k - 1]
            for l in range(d + 1, D):
                ax = l - d - 1
                acc = acc + A[d, l] * (roots[l - d - 1] * _shift_down(cur, ax))
            sub[k + 1] = acc / math.sqrt(k + 1)
    return G


def state_vector(A, b, c, cutoffs):
    """Tier A for a pure state: psi[n] = <n|psi> for 0 <= n < cutoffs, the
    Taylor box of the state's generating function with one index per mode
    (D = M, Sec. 2.1; the pure-state case of Sec. 2.2).  A is M x M, b has M
    entries."""
    return taylor_box(A, b, c, cutoffs)


def full_density_matrix(A, b, c, cutoffs):
    """Tier A for a density matrix: the whole box with interleaved dims
    (C_1, C_1, C_2, C_2, ...).  (A, b) in block order."""
    Ai, bi = to_interleaved(A, b)
    dims = []
    for C in cutoffs:
        dims += [C, C]
    return taylor_box(Ai, bi, c, dims)


def select_outputs(rho_full, detected_mask: int):
    """rho[k_U..., l_U..., n_D...] from a full interleaved box: the ket/bra
    block of the undetected modes and the diagonal of the detected modes."""
    M = rho_full.ndim // 2
    X = rho_full
    det = [j for j in range(M) if (detected_mask >> j) & 1]
    und = [j for j in range(M) if not (detected_mask >> j) & 1]
    # Highest detected mode first: removing its two axes does not move the
    # axes of lower modes (np.diagonal appends the diagonal as the last axis).
    for j in reversed(det):
        X = np.diagonal(X, axis1=2 * j, axis2=2 * j + 1)
    # Remaining leading axes: (k_u, l_u) pairs of the undetected modes in order;
    # trailing axes: diagonals of detected modes, highest mode first.
    nU = len(und)
    lead = list(range(2 * nU))
    trail = list(range(2 * nU, X.ndim))[::-1]
    order = lead[0::2] + lead[1::2] + trail
    return np.ascontiguousarray(np.transpose(X, order))


def fock_diag(A, b, c, cutoffs, detected_mask: int):
    """rho[k_U, l_U, n_D] for all k_U, l_U < C_U and n_D < C_D via the full box."""
    return select_outputs(full_density_matrix(A, b, c, cutoffs), detected_mask)


def detection_probs(A, b, c, cutoffs):
    """p(n) = G_{n1 n1 ... nM nM} for all n < cutoffs (all modes detected)."""
    return fock_diag(A, b, c, cutoffs, (1 << len(cutoffs)) - 1)


def fock_diag_pattern(A, b, c, cutoffs, detected_mask: int, pattern):
    """Tier B: rho[k_U, l_U] at one detection pattern n_D, from the smallest
    box that holds it (undetected cutoffs C_U, detected cutoffs n_j + 1)."""
    M = len(cutoffs)
    det = [j for j in range(M) if (detected_mask >> j) & 1]
    cut = list(cutoffs)
    for j, n in zip(det, pattern):
        cut[j] = int(n) + 1
    out = fock_diag(A, b, c, cut, detected_mask)
    idx = (Ellipsis,) + tuple(int(n) for n in pattern)
    return out[idx]


def level_points(cutoffs, total):
    """The lattice points n (0 <= n_j < C_j) with |n| <= total, level by
    level (S = |n| = 0, 1, ...), each level in lexicographic order with the
    first mode slowest; returns (points, level offsets)."""
    cut = [int(C) for C in cutoffs]
    smax = min(int(total), sum(C - 1 for C in cut))

    def compositions(S, d):
        if d == len(cut) - 1:
            if S < cut[d]:
                yield (S,)
            return
        for v in range(min(cut[d] - 1, S) + 1):
            for rest in compositions(S - v, d + 1):
                yield (v,) + rest

    pts, offs = [], [0]
    for S in range(smax + 1):
        pts.extend(compositions(S, 0))
        offs.append(len(pts))
    return pts, offs


def probs_total(A, b, c, cutoffs, total):
    """p(n) for 0 <= n_j < C_j with a total photon cutoff |n| <= total
    (Sec. 3.1 with the sweep ending at level total), in the order of
    ``level_points``.  No entry depends on the cutoffs (each level only reads
    lower ones): read off the box with per-mode cutoffs min(C_j, total + 1)
    when that is small, else pattern by pattern (Tier B)."""
    mask = (1 << len(cutoffs)) - 1
    pts, offs = level_points(cutoffs, total)
    dims = [min(int(C), int(total) + 1) for C in cutoffs]
    if math.prod(d * d for d in dims) <= 4_000_000:   # the whole box is cheap: read it off
        box = detection_probs(A, b, c, dims)
        return np.array([box[n] for n in pts], dtype=np.complex128), offs
    vals = [complex(fock_diag_pattern(A, b, c, cutoffs, mask, n)) for n in pts]
    return np.array(vals, dtype=np.complex128), offs


def stop_level(level_mass, eps):
    """Probability-sum stopping: the first level S* with sum_{S <= S*} mass(S)
    >= 1 - eps (None if the sum stays below)."""
    acc = 0.0
    for S, m in enumerate(level_mass):
        acc += float(np.real(m))
        if acc >= 1.0 - eps:
            return S
    return None


# --------------------------------------------------------------------------
# Tier E: brute-force loop hafnian expansion of the generating function
# --------------------------------------------------------------------------
def loop_hafnian(X) -> complex:
    """Sum over all partitions of the vertex set into pairs {u, v} (weight X_uv)
    and singletons {u} (weight X_uu)."""
    X = np.asarray(X, dtype=np.complex128)
    n = X.shape[0]
    Xl = X.tolist()

    @lru_cache(maxsize=None)
    def rec(mask: int) -> complex:
        if mask == 0:
            return 1.0 + 0.0j
        i = (mask & -mask).bit_length() - 1
        rest = mask & ~(1 << i)
        total = Xl[i][i] * rec(rest)
        m = rest
        while m:
            j = (m & -m).bit_length() - 1
            m &= m - 1
            total += Xl[i][j] * rec(rest & ~(1 << j))
        return total

    return rec((1 << n) - 1)


def amplitude_bruteforce(A, b, c, k) -> complex:
    """rho_k = c * lhaf(X) / sqrt(prod k_i!), where X repeats row/column i of A
    k_i times and carries b on its diagonal (loops).  Derivation: expanding
    exp(1/2 z^T A z + b^T z) and differentiating k_i times along each z_i picks
    one factor z_i per derivative, paired through A or taken alone through b."""
    A = np.asarray(A, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    L = [i for i, ki in enumerate(k) for _ in range(int(ki))]
    X = A[np.ix_(L, L)].copy()
    X[np.diag_indices(len(L))] = b[L]
    norm = math.sqrt(math.prod(math.factorial(int(ki)) for ki in k))
    return complex(c) * loop_hafnian(X) / norm


# --------------------------------------------------------------------------
# gradients
# --------------------------------------------------------------------------
def adjoint_closed_form(Ai, bi, c, rho_box, gbar_box):
    """VJP of the amplitudes in a box, from the generating function directly.

    With A entering F through 1/2 z^T A z (A symmetric):
      d rho_k / d A_il = 1/2 sqrt(k_i k_l) rho_{k-1_i-1_l}       (i != l)
      d rho_k / d A_ii = 1/2 sqrt(k_i (k_i-1)) rho_{k-2*1_i}
      d rho_k / d b_i  = sqrt(k_i) rho_{k-1_i}
      d rho_k / d c    = rho_k / c
    and the cotangent convention of Sec. 2.5 (Eqs. dL_dB, dL_dA): the
    returned Abar = sum_k gbar_k * conj(d rho_k / d A), likewise bbar, cbar.
    Interleaved order in and out.  ``gbar_box`` has the box's shape.
    """
    R = np.asarray(rho_box, dtype=np.complex128)
    Gb = np.asarray(gbar_box, dtype=np.complex128)
    D = R.ndim
    dims = R.shape
    Abar = np.zeros((D, D), dtype=np.complex128)
    bbar = np.zeros(D, dtype=np.complex128)
    for i in range(D):
        if dims[i] < 2:
            continue
        hi = [slice(None)] * D
        lo = [slice(None)] * D
        hi[i] = slice(1, None)
        lo[i] = slice(0, dims[i] - 1)
        w = np.sqrt(np.arange(1, dims[i], dtype=np.float64)).reshape(
            [dims[i] - 1 if a == i else 1 for a in range(D)])
        bbar[i] = np.sum(Gb[tuple(hi)] * np.conj(w * R[tuple(lo)]))
    for i in range(D):
        for l in range(D):
            if i == l:
                if dims[i] < 3:
                    continue
                hi = [slice(None)] * D
                lo = [slice(None)] * D
                hi[i] = slice(2, None)
                lo[i] = slice(0, dims[i] - 2)
                kk = np.arange(2, dims[i], dtype=np.float64)
                w = (0.5 * np.sqrt(kk * (kk - 1))).reshape([dims[i] - 2 if a == i else 1 for a in range(D)])
            else:
                if dims[i] < 2 or dims[l] < 2:
                    continue
                hi = [slice(None)] * D
                lo = [slice(None)] * D
                hi[i] = slice(1, None)
                hi[l] = slice(1, None)
                lo[i] = slice(0, dims[i] - 1)
                lo[l] = slice(0, dims[l] - 1)
                wi = np.sqrt(np.arange(1, dims[i], dtype=np.float64)).reshape(
                    [dims[i] - 1 if a == i else 1 for a in range(D)])
                wl = np.sqrt(np.arange(1, dims[l], dtype=np.float64)).reshape(
                    [dims[l] - 1 if a == l else 1 for a in range(D)])
                w = 0.5 * wi * wl
            Abar[i, l] = np.sum(Gb[tuple(hi)] * np.conj(w * R[tuple(lo)]))
    cbar = np.sum(Gb * np.conj(R / c))
    return Abar, bbar, complex(cbar)


def _scatter_outputs(shape_box, detected_mask: int, M: int, gbar_out):
    """Place a cotangent of rho[k_U, l_U, n_D] into a zero box of interleaved shape."""
    det = [j for j in range(M) if (detected_mask >> j) & 1]
    und = [j for j in range(M) if not (detected_mask >> j) & 1]
    G = np.zeros(shape_box, dtype=np.complex128)
    g = np.asarray(gbar_out, dtype=np.complex128)
    nU = len(und)
    for idx in np.ndindex(*g.shape):
        ks, ls, ns = idx[:nU], idx[nU:2 * nU], idx[2 * nU:]
        full = [0] * (2 * M)
        for t, j in enumerate(und):
            full[2 * j], full[2 * j + 1] = ks[t], ls[t]
        for t, j in enumerate(det):
            full[2 * j] = full[2 * j + 1] = ns[t]
        G[tuple(full)] = g[idx]
    return G


def fock_diag_vjp(A, b, c, cutoffs, detected_mask: int, gbar_out):
    """(dA, db, dc) in block order for the cotangent ``gbar_out`` of
    rho[k_U, l_U, n_D] (closed-form adjoint evaluated on the full box).  The
    gradient is taken w.r.t. the symmetric use of A, so dA is symmetric."""
    M = len(cutoffs)
    Ai, bi = to_interleaved(A, b)
    R = full_density_matrix(A, b, c, cutoffs)
    Gb = _scatter_outputs(R.shape, detected_mask, M, gbar_out)
    Abar, bbar, cbar = adjoint_closed_form(Ai, bi, c, R, Gb)
    dA, db = from_interleaved(Abar, bbar)
    return dA, db, cbar


def tangent_recurrences(Ai, bi, c, dims):
    """Forward-mode derivatives by the paper's tangent recurrences (Sec. 2.5,
    Eqs. recrel_dB and recrel_dA), walked together with Eq. recrel over the
    box in the same order as ``taylor_box``.

    Returns (G, dG_db, dG_dA) with dG_db[m] = dG/db_m and dG_dA[m, n] =
    dG/dA_mn, where A_mn is the coefficient that multiplies the read of
    direction n when writing along direction m.
    """
    A = np.asarray(Ai, dtype=np.complex128)
    b = np.asarray(bi, dtype=np.complex128)
    dims = tuple(dims)
    D = len(dims)
    G = np.zeros(dims, dtype=np.complex128)
    dB = np.zeros((D,) + dims, dtype=np.complex128)
    dA = np.zeros((D, D) + dims, dtype=np.complex128)
    G[(0,) * D] = c
    for d in range(D - 1, -1, -1):
        sG = G[(0,) * d]
        sB = dB[(slice(None),) + (0,) * d]
        sA = dA[(slice(None), slice(None)) + (0,) * d]
        nrest = D - d - 1
        roots = {l: _sqrt_index(dims[l], l - d - 1, nrest) for l in range(d + 1, D)}
        for k in range(dims[d] - 1):
            # reads G_{p - 1_l} for the pivot p = (0.., k, rest), times sqrt(p_l)
            reads_G = {}
            if k >= 1:
                reads_G[d] = math.sqrt(k) * sG[k - 1]
            for l in range(d + 1, D):
                reads_G[l] = roots[l] * _shift_down(sG[k], l - d - 1)
            newG = b[d] * sG[k] + sum(A[d, l] * v for l, v in reads_G.items())
            # tangent w.r.t. b_m: same recurrence on dG, plus G_p when m == d
            newB = b[d] * sB[:, k]
            if k >= 1:
                newB = newB + math.sqrt(k) * A[d, d] * sB[:, k - 1]
            for l in range(d + 1, D):
                newB = newB + A[d, l] * (roots[l][None] * _shift_down(sB[:, k], l - d))
            newB[d] = newB[d] + sG[k]
            # tangent w.r.t. A_mn: same recurrence, plus sqrt(p_n) G_{p-1_n} when m == d
            newA = b[d] * sA[:, :, k]
            if k >= 1:
                newA = newA + math.sqrt(k) * A[d, d] * sA[:, :, k - 1]
            for l in range(d + 1, D):
                newA = newA + A[d, l] * (roots[l][None, None] * _shift_down(sA[:, :, k], l - d + 1))
            for n, v in reads_G.items():
                newA[d, n] = newA[d, n] + v
            s = math.sqrt(k + 1)
            sG[k + 1] = newG / s
            sB[:, k + 1] = newB / s
            sA[:, :, k + 1] = newA / s
    return G, dB, dA


def fock_diag_jvp(A, b, c, cutoffs, detected_mask: int, dA, db, dc):
    """(rho, drho): rho[k_U, l_U, n_D] and its derivative along the direction
    (dA, db, dc), from the paper's tangent recurrences (Sec. 2.5) over the full
    interleaved box.  A enters through (A + A^T) / 2 and so does dA; G is
    proportional to c, so its c-tangent is G dc / c.  Small boxes only: the
    recurrences carry D + D^2 tangents of every entry."""
    A, dA = np.asarray(A, dtype=np.complex128), np.asarray(dA, dtype=np.complex128)
    Ai, bi = to_interleaved(0.5 * (A + A.T), b)
    dAi, dbi = to_interleaved(0.5 * (dA + dA.T), db)
    dims = [C for C in cutoffs for _ in range(2)]
    G, dGb, dGA = tangent_recurrences(Ai, bi, c, dims)
    dG = (np.tensordot(dbi, dGb, axes=(0, 0)) + np.tensordot(dAi, dGA, axes=([0, 1], [0, 1]))
          + G * (complex(dc) / complex(c)))
    return select_outputs(G, detected_mask), select_outputs(dG, detected_mask)


def _shift(X: np.ndarray, shifts) -> np.ndarray:
    """Y[n] = X[n - shifts] (zero where some n_j < shifts_j)."""
    Y = np.zeros_like(X)
    src = tuple(slice(0, X.shape[j] - s) for j, s in enumerate(shifts))
    dst = tuple(slice(s, None) for s in shifts)
    Y[dst] = X[src]
    return Y


def probs_vjp_pure(psi, c, gbar):
    """Closed-form adjoint of every detection probability of a PURE state, at
    full size.  For rho = psi psi^dag (Sec. 2.2: the density triple of a pure
    state is the ket triple and its conjugate), the amplitude at interleaved
    index (kappa kets, beta bras) is psi_kappa conj(psi_beta), so the
    off-diagonal amplitudes the closed form needs next to the diagonal are
    products of two state-vector entries.  With p(n) = rho_{d(n)} and the
    derivatives of ``adjoint_closed_form`` (d rho_k/d A_il = 1/2 sqrt(k_i k_l)
    rho_{k-1_i-1_l}, i != l; 1/2 sqrt(k_i (k_i-1)) rho_{k-2*1_i}, i = l;
    d rho_k/d b_i = sqrt(k_i) rho_{k-1_i}; d rho_k/d c = rho_k / c):
        k = d(n), i = ket p:  k - 1_i has kets n - 1_p and bras n,
        i = bra p:            kets n and bras n - 1_p.
    ``psi`` is the state vector over the whole box (cutoffs C_j), ``c`` the
    density triple's c (= |c_psi|^2, used by dc only), ``gbar`` the cotangent
    of p over the same box.  Returns (dA, db, dc) in block order, as
    ``fock_diag_vjp`` does for the all-detected output of the density triple."""
    psi = np.asarray(psi, dtype=np.complex128)
    G = np.asarray(gbar, dtype=np.complex128)
    M = psi.ndim
    dims = psi.shape
    D = 2 * M
    cpsi = np.conj(psi)
    e = lambda *ps: tuple(sum(1 for q in ps if q == j) for j in range(M))
    root = [np.sqrt(np.arange(dims[j], dtype=np.float64)).reshape([dims[j] if a == j else 1 for a in range(M)])
            for j in range(M)]
    n_of = [np.arange(dims[j], dtype=np.float64).reshape([dims[j] if a == j else 1 for a in range(M)])
            for j in range(M)]

    def amp(kets, bras):
        # rho at kets n - e(kets), bras n - e(bras), as an array over n
        return _shift(psi, e(*kets)) * _shift(cpsi, e(*bras))

    def side(pos):
        return ("ket" if pos % 2 == 0 else "bra"), pos // 2

    Abar = np.zeros((D, D), dtype=np.complex128)
    bbar = np.zeros(D, dtype=np.complex128)
    for i in range(D):
        si, p = side(i)
        R = amp([p], []) if si == "ket" else amp([], [p])
        bbar[i] = np.sum(G * np.conj(root[p] * R))
        for l in range(D):
            sl, q = side(l)
            kets = [x for s_, x in ((si, p), (sl, q)) if s_ == "ket"]
            bras = [x for s_, x in ((si, p), (sl, q)) if s_ == "bra"]
            if i == l:
                w = 0.5 * np.sqrt(n_of[p] * np.maximum(n_of[p] - 1.0, 0.0))
            else:
                w = 0.5 * root[p] * root[q]
            Abar[i, l] = np.sum(G * np.conj(w * amp(kets, bras)))
    cbar = np.sum(G * np.conj(psi * cpsi / complex(c)))
    dA, db = from_interleaved(Abar, bbar)
    return dA, db, complex(cbar)


# --------------------------------------------------------------------------
# error metric
# --------------------------------------------------------------------------
def rel_err(x, ref) -> float:
    """Normwise relative error ||x - ref||_2 / ||ref||_2 (0 if both vanish)."""
    x = np.asarray(x, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    nr = np.linalg.norm(ref)
    nd = np.linalg.norm(x - ref)
    if nr == 0.0:
        return float(nd)
    return float(nd / nr)
