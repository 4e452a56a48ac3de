"""Slow pure-Python model of the GPU library's schedule (test-side only).

It mirrors, entry by entry, the order of work of the HIP kernels: the
canonical-parent ("pull") form of Algorithms 1 and 2 (Sec. 3.1.3 and 3.2),
with amplitudes stored as families diag + offset (Sec. 3.1.4 and App. B.2),
and the reverse sweep in which every off-diagonal cotangent slot is written by
its single reader.  The tests run it against the oracle on small cases so that
a mistake in the family / parent / reader bookkeeping shows up on the CPU.

Layout conventions (same as the library):
* modes with cutoff 1 are dropped; undetected modes first, then detected;
* U block coordinates kappa = (k_u..., l_u...) in C order;
* internal positions: U kets 0..MU-1, U bras MU..2MU-1, then for detected
  mode j: ket 2MU+2j, bra 2MU+2j+1.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


class Model:
    def __init__(self, M, cutoffs, detected_mask, b_zero):
        self.M = M
        self.cut = list(cutoffs)
        self.mask = detected_mask
        act = [j for j in range(M) if cutoffs[j] >= 2]
        self.U = [j for j in act if not (detected_mask >> j) & 1]
        self.D = [j for j in act if (detected_mask >> j) & 1]
        self.MU, self.MD = len(self.U), len(self.D)
        self.CU = [cutoffs[j] for j in self.U]
        self.CD = [cutoffs[j] for j in self.D]
        self.udims = self.CU + self.CU
        self.B = int(np.prod(self.udims)) if self.udims else 1
        self.ustride = [int(np.prod(self.udims[q + 1:])) for q in range(len(self.udims))]
        self.odd = (not b_zero) or self.MU > 0
        # internal position -> block-order index of the caller's A
        self.pos2blk = [j for j in self.U] + [M + j for j in self.U]
        for j in self.D:
            self.pos2blk += [j, M + j]
        self.smax = sum(c - 1 for c in self.CD)

    # ------------------------------------------------------------ positions
    def ket(self, j):
        return 2 * self.MU + 2 * j

    def bra(self, j):
        return 2 * self.MU + 2 * j + 1

    def kcoords(self, e):
        out = []
        for q in range(len(self.udims)):
            out.append((e // self.ustride[q]) % self.udims[q])
        return out

    # ------------------------------------------------------------- families
    def valid(self, fam, n):
        C = self.CD
        t = fam[0]
        if t == "F0":
            return True
        if t in ("F1k", "F1b"):
            j = fam[1]
            lim0 = C[0] - 2 if (t == "F1k" or j > 0) else C[0] - 3
            if n[0] > lim0:
                return False
            if j > 0 and n[j] > C[j] - 2:
                return False
            return True
        K = fam[1]
        if any(n[i] != 0 for i in range(K)):
            return False
        if t == "F2":
            return n[K] <= C[K] - 3
        j = fam[2]
        return n[K] <= C[K] - 2 and n[j] <= C[j] - 2

    def families(self):
        f = [("F0",)]
        if self.odd:
            f += [("F1k", j) for j in range(self.MD)] + [("F1b", j) for j in range(self.MD)]
        f += [("F2", K) for K in range(self.MD)]
        for K in range(self.MD):
            for j in range(K + 1, self.MD):
                f += [("F1010", K, j), ("F1001", K, j)]
        return f

    def lattice(self, S):
        for n in itertools.product(*[range(c) for c in self.CD]):
            if sum(n) == S:
                yield n

    # ------------------------------------------------------------- triple prep
    def prep(self, A, b, c):
        A = np.asarray(A, dtype=np.complex128)
        b = np.asarray(b, dtype=np.complex128)
        P = self.pos2blk
        As = 0.5 * (A + A.T)
        return As[np.ix_(P, P)], b[P], complex(c)

    # ------------------------------------------------------------- forward
    def ufill(self, A, b, c):
        """Step 1 of Algorithm 2: the whole U block at zero detections."""
        G = np.zeros(self.B, dtype=np.complex128)
        G[0] = c
        nq = len(self.udims)
        for e in range(1, self.B):
            kap = self.kcoords(e)
            q = next(i for i in range(nq) if kap[i] > 0)
            p = list(kap)
            p[q] -= 1
            pe = e - self.ustride[q]
            acc = b[q] * G[pe]
            for q2 in range(nq):
                if p[q2] > 0:
                    acc += math.sqrt(p[q2]) * A[q, q2] * G[pe - self.ustride[q2]]
            G[e] = acc / math.sqrt(p[q] + 1)
        return G

    def _apply(self, A, b, i, piv, reads, scale):
        """One target block: (b_i piv + sum_q sqrt(kappa_q) A_iq piv[e - s_q]
        + sum_l coef_l A_il x_l) * scale, reads = [(l, coef, block)]."""
        out = np.zeros(self.B, dtype=np.complex128)
        for e in range(self.B):
            acc = 0j
            if piv is not None:
                acc += b[i] * piv[e]
                kap = self.kcoords(e)
                for q in range(len(self.udims)):
                    if kap[q] > 0:
                        acc += math.sqrt(kap[q]) * A[i, q] * piv[e - self.ustride[q]]
            for (l, coef, x) in reads:
                acc += coef * A[i, l] * x[e]
            out[e] = acc * scale
        return out

    def forward(self, A, b, c, keep_all=True):
        A, b, c = self.prep(A, b, c)
        C = self.CD
        MD = self.MD
        st = {}                      # (family, n) -> block
        self.writes = {}
        st[(("F0",), (0,) * MD)] = self.ufill(A, b, c)

        def put(fam, n, val):
            key = (fam, tuple(n))
            assert self.valid(fam, n), key
            assert key not in st, ("written twice", key)
            st[key] = val

        for S in range(self.smax + 1):
            for m in self.lattice(S):
                m = list(m)
                # diagonal pivot d(m): writes type-1 offsets (Alg. 1 diag pivots)
                if self.odd and MD > 0 and m[0] <= C[0] - 2:
                    piv = st[(("F0",), tuple(m))]
                    reads = []
                    for j in range(MD):
                        if m[j] > 0:
                            mm = list(m)
                            mm[j] -= 1
                            reads.append((self.ket(j), math.sqrt(m[j]), st[(("F1b", j), tuple(mm))]))
                            reads.append((self.bra(j), math.sqrt(m[j]), st[(("F1k", j), tuple(mm))]))
                    for j in range(MD):
                        for (fam, i) in ((("F1k", j), self.ket(j)), (("F1b", j), self.bra(j))):
                            if self.valid(fam, m):
                                put(fam, m, self._apply(A, b, i, piv, reads, 1 / math.sqrt(m[j] + 1)))
                # off-diagonal / bridge pivots d(m) + 1_ketK
                K0 = next((j for j in range(MD) if m[j] > 0), MD)
                for K in range(min(K0 + 1, MD)):
                    if m[K] > C[K] - 2:
                        continue
                    piv = st[(("F1k", K), tuple(m))] if self.odd else None
                    reads = [(self.ket(K), math.sqrt(m[K] + 1), st[(("F0",), tuple(m))])]
                    if m[K] > 0:
                        mm = list(m)
                        mm[K] -= 1
                        reads.append((self.bra(K), math.sqrt(m[K]), st[(("F2", K), tuple(mm))]))
                    for j in range(K + 1, MD):
                        if m[j] > 0:
                            mm = list(m)
                            mm[j] -= 1
                            reads.append((self.ket(j), math.sqrt(m[j]), st[(("F1001", K, j), tuple(mm))]))
                            reads.append((self.bra(j), math.sqrt(m[j]), st[(("F1010", K, j), tuple(mm))]))
                    mp = list(m)
                    mp[K] += 1
                    put(("F0",), mp, self._apply(A, b, self.bra(K), piv, reads, 1 / math.sqrt(m[K] + 1)))
                    if self.valid(("F2", K), m):
                        put(("F2", K), m, self._apply(A, b, self.ket(K), piv, reads, 1 / math.sqrt(m[K] + 2)))
                    for j in range(K + 1, MD):
                        for (fam, i) in ((("F1010", K, j), self.ket(j)), (("F1001", K, j), self.bra(j))):
                            if self.valid(fam, m):
                                put(fam, m, self._apply(A, b, i, piv, reads, 1 / math.sqrt(m[j] + 1)))
        self.st = st
        self.Aint, self.bint, self.c = A, b, c
        return self.output(st)

    def output(self, st):
        shape = [self.cut[j] for j in range(self.M) if not (self.mask >> j) & 1] * 2 + \
                [self.cut[j] for j in range(self.M) if (self.mask >> j) & 1]
        out = np.zeros(shape, dtype=np.complex128)
        act_shape = self.udims + self.CD
        view = np.zeros(act_shape, dtype=np.complex128)
        for n in itertools.product(*[range(c) for c in self.CD]):
            blk = st[(("F0",), n)]
            view[(Ellipsis,) + n] = blk.reshape(self.udims) if self.udims else blk[0]
        # size-1 (dropped) modes are index 0 of their axis
        U_all = [j for j in range(self.M) if not (self.mask >> j) & 1]
        D_all = [j for j in range(self.M) if (self.mask >> j) & 1]
        sl = []
        for j in U_all:
            sl.append(slice(None) if j in self.U else 0)
        for j in U_all:
            sl.append(slice(None) if j in self.U else 0)
        for j in D_all:
            sl.append(slice(None) if j in self.D else 0)
        out[tuple(sl)] = view
        return out

    def stored_counts(self):
        cnt = {}
        for (fam, n) in self.st:
            cnt[fam[0]] = cnt.get(fam[0], 0) + 1
        return cnt

    # ------------------------------------------------------------- reverse
    def vjp(self, gout):
        """Reverse sweep; every off-diagonal cotangent slot is *set* by its single
        reader, F1k(K)(m) additionally receives the K-pivot's pivot-value
        contribution from the lattice point m itself."""
        A, b, st = self.Aint, self.bint, self.st
        C, MD = self.CD, self.MD
        npos = 2 * self.MU + 2 * MD
        Abar = np.zeros((npos, npos), dtype=np.complex128)
        bbar = np.zeros(npos, dtype=np.complex128)
        slot = {}                      # off-diagonal cotangent slots
        gF0 = {}                       # final F0 cotangents
        # drho in active-node form
        U_all = [j for j in range(self.M) if not (self.mask >> j) & 1]
        D_all = [j for j in range(self.M) if (self.mask >> j) & 1]
        sl = []
        for j in U_all + U_all:
            sl.append(slice(None) if j in self.U else 0)
        for j in D_all:
            sl.append(slice(None) if j in self.D else 0)
        gview = np.asarray(gout)[tuple(sl)]

        def drho(n):
            return np.array(gview[(Ellipsis,) + tuple(n)], dtype=np.complex128).reshape(self.B)

        def setslot(fam, n, val):
            key = (fam, tuple(n))
            assert key not in slot, ("slot set twice", key)
            slot[key] = val

        def take(fam, n):
            return slot[(fam, tuple(n))]

        nq = len(self.udims)

        def accumulate(i, h, reads, piv):
            # Abar_il += conj(coef_l x_l) h ; bbar_i += conj(piv) h ; U neighbours
            for (l, coef, x) in reads:
                Abar[i, l] += np.sum(np.conj(coef * x) * h)
            if piv is not None:
                bbar[i] += np.sum(np.conj(piv) * h)
                for e in range(self.B):
                    kap = self.kcoords(e)
                    for q in range(nq):
                        if kap[q] > 0:
                            Abar[i, q] += np.conj(math.sqrt(kap[q]) * piv[e - self.ustride[q]]) * h[e]

        def pivot_adjoint(targets):
            """sum_i conj(b_i) h_i and the U-neighbour pull, for the pivot block."""
            g = np.zeros(self.B, dtype=np.complex128)
            for (i, h) in targets:
                g += np.conj(b[i]) * h
                for e in range(self.B):
                    kap = self.kcoords(e)
                    for q in range(nq):
                        if kap[q] + 1 < self.udims[q]:
                            g[e] += math.sqrt(kap[q] + 1) * np.conj(A[i, q]) * h[e + self.ustride[q]]
            return g

        def read_adjoint(l, coef, targets):
            g = np.zeros(self.B, dtype=np.complex128)
            for (i, h) in targets:
                g += coef * np.conj(A[i, l]) * h
            return g

        for S in range(self.smax, -1, -1):
            for m in reversed(list(self.lattice(S))):
                m = list(m)
                g0 = drho(m)
                K0 = next((j for j in range(MD) if m[j] > 0), MD)
                for K in range(min(K0 + 1, MD)):
                    if m[K] > C[K] - 2:
                        continue
                    piv = st[(("F1k", K), tuple(m))] if self.odd else None
                    reads = [(self.ket(K), math.sqrt(m[K] + 1), st[(("F0",), tuple(m))], None)]
                    if m[K] > 0:
                        mm = list(m); mm[K] -= 1
                        reads.append((self.bra(K), math.sqrt(m[K]), st[(("F2", K), tuple(mm))], (("F2", K), mm)))
                    for j in range(K + 1, MD):
                        if m[j] > 0:
                            mm = list(m); mm[j] -= 1
                            reads.append((self.ket(j), math.sqrt(m[j]), st[(("F1001", K, j), tuple(mm))], (("F1001", K, j), mm)))
                            reads.append((self.bra(j), math.sqrt(m[j]), st[(("F1010", K, j), tuple(mm))], (("F1010", K, j), mm)))
                    targets = []
                    mp = list(m); mp[K] += 1
                    targets.append((self.bra(K), gF0[tuple(mp)] / math.sqrt(m[K] + 1)))
                    if self.valid(("F2", K), m):
                        targets.append((self.ket(K), take(("F2", K), m) / math.sqrt(m[K] + 2)))
                    for j in range(K + 1, MD):
                        for (fam, i) in ((("F1010", K, j), self.ket(j)), (("F1001", K, j), self.bra(j))):
                            if self.valid(fam, m):
                                targets.append((i, take(fam, m) / math.sqrt(m[j] + 1)))
                    for (i, h) in targets:
                        accumulate(i, h, [(l, cf, x) for (l, cf, x, _) in reads], piv)
                    for (l, cf, x, dest) in reads:
                        g = read_adjoint(l, cf, targets)
                        if dest is None:
                            g0 = g0 + g
                        else:
                            setslot(dest[0], dest[1], g)
                    if self.odd:
                        gp = pivot_adjoint(targets)
                        has_diag_reader = (K > 0 or m[0] + 1 <= C[0] - 2)
                        base = take(("F1k", K), m) if has_diag_reader else 0
                        slot[(("F1k", K), tuple(m))] = base + gp
                if self.odd and MD > 0 and m[0] <= C[0] - 2:
                    piv = st[(("F0",), tuple(m))]
                    reads = []
                    for j in range(MD):
                        if m[j] > 0:
                            mm = list(m); mm[j] -= 1
                            reads.append((self.ket(j), math.sqrt(m[j]), st[(("F1b", j), tuple(mm))], (("F1b", j), mm)))
                            reads.append((self.bra(j), math.sqrt(m[j]), st[(("F1k", j), tuple(mm))], (("F1k", j), mm)))
                    targets = []
                    for j in range(MD):
                        for (fam, i) in ((("F1k", j), self.ket(j)), (("F1b", j), self.bra(j))):
                            if self.valid(fam, m):
                                targets.append((i, take(fam, m) / math.sqrt(m[j] + 1)))
                    for (i, h) in targets:
                        accumulate(i, h, [(l, cf, x) for (l, cf, x, _) in reads], piv)
                    for (l, cf, x, dest) in reads:
                        setslot(dest[0], dest[1], read_adjoint(l, cf, targets))
                    g0 = g0 + pivot_adjoint(targets)
                gF0[tuple(m)] = g0
        # reverse of the U-block fill, gather form by U weight
        G = st[(("F0",), (0,) * MD)]
        g = gF0[(0,) * MD].copy()
        wt = [sum(self.kcoords(e)) for e in range(self.B)]
        gfin = np.zeros(self.B, dtype=np.complex128)
        for w in range(max(wt), -1, -1):
            for e in range(self.B):
                if wt[e] != w:
                    continue
                x = self.kcoords(e)
                acc = g[e]
                first0 = 0
                while first0 < nq and x[first0] == 0:
                    first0 += 1
                for q in range(nq):
                    if q > first0:
                        break   # x + 1_q has first non-zero q only if x_{<q} = 0
                    if x[q] + 1 >= self.udims[q]:
                        continue
                    t = e + self.ustride[q]
                    ht = gfin[t] / math.sqrt(x[q] + 1)
                    acc += np.conj(b[q]) * ht
                for q in range(nq):
                    if q > first0:
                        break
                    for q2 in range(q, nq):
                        # t = x + 1_q2 + 1_q, parent p = x + 1_q2, direction q
                        xp = list(x); xp[q2] += 1
                        if xp[q2] >= self.udims[q2] or xp[q] + 1 >= self.udims[q]:
                            continue
                        t = e + self.ustride[q2] + self.ustride[q]
                        ht = gfin[t] / math.sqrt(xp[q] + 1)
                        acc += math.sqrt(xp[q2]) * np.conj(A[q, q2]) * ht
                gfin[e] = acc
        for e in range(1, self.B):
            kap = self.kcoords(e)
            q = next(i for i in range(nq) if kap[i] > 0)
            p = list(kap); p[q] -= 1
            pe = e - self.ustride[q]
            h = gfin[e] / math.sqrt(p[q] + 1)
            bbar[q] += np.conj(G[pe]) * h
            for q2 in range(nq):
                if p[q2] > 0:
                    Abar[q, q2] += np.conj(math.sqrt(p[q2]) * G[pe - self.ustride[q2]]) * h
        cbar = gfin[0]
        # back to the caller's block order; symmetrise
        Asym = 0.5 * (Abar + Abar.T)
        dA = np.zeros((2 * self.M, 2 * self.M), dtype=np.complex128)
        db = np.zeros(2 * self.M, dtype=np.complex128)
        P = self.pos2blk
        for p_ in range(npos):
            db[P[p_]] = bbar[p_]
            for q_ in range(npos):
                dA[P[p_], P[q_]] = Asym[p_, q_]
        return dA, db, complex(cbar), slot
