"""CPU model of the tiled state-vector derivative kernels (test-side only).

The forward- and reverse-mode kernels split psi (C order) into tiles of the
trailing modes and serve each term of the closed-form derivatives from one of
three places: the staged tile t (shift in trailing modes only), the staged
tile t - 1_i (leading part 1_i) or one amplitude of tile t - 1_i - 1_l read
straight from memory (two leading modes).  This model walks the same phases
and the same per-XCD tile order, asserts that every read stays inside its
tile or the box, and compares the results with the oracle's tangent
recurrences (forward mode) and closed-form adjoint (reverse mode), with small
tile sizes so that several modes are leading."""
import math

import numpy as np
import pytest

import oracle as O


def tiles(C, tmax):
    MD = len(C)
    stride = [0] * MD
    s = 1
    for d in range(MD - 1, -1, -1):
        stride[d] = s
        s *= C[d]
    sp, T = MD, 1
    while sp > 0 and T * C[sp - 1] <= tmax:
        sp -= 1
        T *= C[sp]
    return sp, T, s // T, stride, s


def tile_of(nt, v):
    return v if nt % 8 else (v % 8) * (nt // 8) + v // 8


def digits(x, C, stride):
    return [(x // stride[d]) % C[d] for d in range(len(C))]


def terms_of_tile(C, tmax, t):
    """(shift, weight function of the entry digits, source) of every term the
    kernels serve for tile t, source 'tile' / 'lead' / 'mem'; also checks
    that each read index lies in the tile (or the box for 'mem')."""
    MD = len(C)
    sp, T, nt, stride, tot = tiles(C, tmax)
    x0 = t * T
    ks = digits(x0, C, stride)
    out = []   # (term key, per-entry list of (weight, read index))
    for f in range(T):
        k = digits(f, C, stride)
        x = x0 + f
        reads = [("c", 1.0, x)]
        for i in range(sp, MD):
            if k[i] >= 1:
                assert 0 <= f - stride[i] < T
                reads.append((("b", i), math.sqrt(k[i]), x - stride[i]))
            for l in range(i, MD):
                kl = k[l] - (l == i)
                if k[i] >= 1 and kl >= 1:
                    assert 0 <= f - stride[i] - stride[l] < T
                    reads.append((("A", i, l), 0.5 * math.sqrt(k[i] * kl), x - stride[i] - stride[l]))
        for i in range(sp):
            if ks[i] < 1:
                continue
            xs = x0 - stride[i]
            assert xs >= 0
            wi = math.sqrt(ks[i])
            reads.append((("b", i), wi, xs + f))
            for l in range(sp, MD):
                if k[l] >= 1:
                    assert 0 <= f - stride[l] < T
                    reads.append((("A", i, l), 0.5 * wi * math.sqrt(k[l]), xs + f - stride[l]))
            for l in range(i, sp):
                kl = ks[l] - (l == i)
                if kl >= 1:
                    y = xs + f - stride[l]
                    assert 0 <= y < tot
                    reads.append((("A", i, l), 0.5 * wi * math.sqrt(kl), y))
        out.append((x, reads))
    return out


def model_jvp(C, tmax, psi, r, tb, S):
    sp, T, nt, stride, tot = tiles(C, tmax)
    out = np.zeros(tot, complex)
    seen = set()
    for v in range(nt):
        t = tile_of(nt, v)
        seen.add(t)
        for x, reads in terms_of_tile(C, tmax, t):
            acc = 0j
            for key, w, y in reads:
                coef = r if key == "c" else (tb[key[1]] if key[0] == "b" else S[key[1], key[2]])
                acc += coef * w * psi[y]
            out[x] = acc
    assert seen == set(range(nt))   # the per-XCD order visits every tile once
    return out


def model_vjp(C, tmax, psi, g):
    sp, T, nt, stride, tot = tiles(C, tmax)
    MD = len(C)
    bbar, Abar, csum = np.zeros(MD, complex), np.zeros((MD, MD), complex), 0j
    for v in range(nt):
        for x, reads in terms_of_tile(C, tmax, tile_of(nt, v)):
            for key, w, y in reads:
                val = g[x] * np.conj(w * psi[y])
                if key == "c":
                    csum += val
                elif key[0] == "b":
                    bbar[key[1]] += val
                else:
                    Abar[key[1], key[2]] += val
    return bbar, Abar, csum


SHAPES = [([3, 4, 2, 3], 8), ([3, 4, 2, 3], 4096), ([2, 3, 3, 2, 2], 6), ([5], 2), ([4, 3], 1), ([3, 3, 3], 9),
          ([2, 2, 2, 2, 2, 2], 4)]


@pytest.mark.parametrize("C,tmax", SHAPES)
def test_tile_phases_forward_mode(C, tmax):
    rng = np.random.default_rng(sum(C) + tmax)
    M = len(C)
    X = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    A, b, c = 0.2 * (X + X.T), 0.3 * (rng.standard_normal(M) + 1j * rng.standard_normal(M)), 0.8 - 0.1j
    tA = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    tb = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    tc = 0.3 + 0.2j
    G, dB, dAr = O.tangent_recurrences(A, b, c, C)
    Ts = 0.5 * (tA + tA.T)
    ref = (tc / c * G + np.tensordot(tb, dB, axes=(0, 0)) + np.tensordot(Ts, dAr, axes=([0, 1], [0, 1]))).ravel()
    # the kernels' coefficients: S_il = dA_il + dA_li (i < l), dA_ii
    S = tA + tA.T - np.diag(np.diag(tA))
    got = model_jvp(C, tmax, O.state_vector(A, b, c, C).ravel(), tc / c, tb, S)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("C,tmax", SHAPES)
def test_tile_phases_reverse_mode(C, tmax):
    rng = np.random.default_rng(2 * sum(C) + tmax)
    M = len(C)
    X = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    A, b, c = 0.2 * (X + X.T), 0.3 * (rng.standard_normal(M) + 1j * rng.standard_normal(M)), 0.8 - 0.1j
    psi = O.state_vector(A, b, c, C)
    g = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    rA, rb, rc = O.adjoint_closed_form(A, b, c, psi, g)
    bbar, Abar, csum = model_vjp(C, tmax, psi.ravel(), g.ravel())
    # the final kernel's assembly: Abar mirrored, cbar = sum g conj(psi) / conj(c)
    Afull = Abar + Abar.T - np.diag(np.diag(Abar))
    got = np.concatenate([Afull.ravel(), bbar, [csum / np.conj(c)]])
    ref = np.concatenate([np.asarray(rA).ravel(), np.asarray(rb).ravel(), [rc]])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_full_size_geometry():
    # the 8-mode cutoff-8 state: the forward mode's 4096-entry tiles leave
    # four leading modes and 4096 tiles in eight per-XCD ranges, the reverse
    # mode's 512-entry tiles five leading modes
    sp, T, nt, _, _ = tiles([8] * 8, 4096)
    assert (sp, T, nt) == (4, 4096, 4096)
    assert sorted(tile_of(nt, v) for v in range(nt)) == list(range(nt))
    sp, T, nt, _, _ = tiles([8] * 8, 512)
    assert (sp, T, nt) == (5, 512, 32768)
