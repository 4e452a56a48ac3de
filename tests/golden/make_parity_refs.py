"""Writes tests/golden/parity_*.npz: oracle references for the full-size GPU
parity tests.  Calls only the oracle and the seeded input generators.

A detection pattern's conditional block rho[:, :, n] (and the adjoint of a
cotangent supported on it) needs only the box whose detected cutoffs are
n_j + 1 (Tier B: Taylor coefficients do not depend on the cutoffs), so every
reference below is exact at the workloads' full sizes:

* parity_patterns.npz -- for the 4-mode conditional state (undetected cutoff
  30, detected 12, b != 0), the 5-mode one (undetected 40, detected 10), the
  8-mode all-detected state (cutoff 8) and the first circuit of the 6-mode
  gradient batch (undetected 30, detected 8): blocks at high patterns, a
  seeded cotangent per pattern and the adjoint of each;
* parity_pure8.npz -- the 8-mode state of cutoff 8 without loss: the adjoint
  of a dense seeded cotangent over all 8^8 detection probabilities
  (``probs_vjp_pure``, the state-vector route);
* parity_batch.npz -- sampled patterns of every circuit of the 256-circuit
  uneven batch.

Run from the repository root:  python tests/golden/make_parity_refs.py
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2303_08879_amd import workloads as W  # noqa: E402

# (workload, patterns): boxes of at most ~5M entries
PATTERNS = {
    "config2": [(11, 3, 0), (0, 4, 11), (5, 5, 1), (3, 0, 7), (2, 7, 2)],
    "config4": [(9, 0, 0, 1), (0, 3, 3, 2), (1, 1, 1, 5), (2, 0, 6, 0), (4, 0, 4, 0)],
    "config5": [(7, 7, 7, 0, 0, 0, 0, 0), (0, 0, 0, 0, 0, 7, 7, 7), (7, 0, 0, 7, 0, 0, 0, 6),
                (3, 3, 3, 3, 0, 0, 0, 0), (1, 1, 1, 1, 1, 1, 1, 1), (2, 2, 2, 2, 2, 2, 0, 0),
                (4, 0, 3, 0, 2, 0, 1, 5), (0, 6, 0, 0, 5, 0, 4, 0)],
    "config5b": [(7, 0, 0, 0, 0), (1, 1, 1, 1, 1), (0, 3, 0, 3, 1), (7, 7, 0, 0, 0), (0, 0, 2, 2, 6)],
}
PURE8 = dict(seed=505, M=8, cut=8, r_lo=0.5, r_hi=1.0, cot_seed=21)


def circuit(name):
    if name == "config2":
        return W.config2()
    if name == "config4":
        return W.config4()
    if name == "config5":
        return W.config5()
    if name == "config5b":
        return W.config5b(n=1)[0]
    raise KeyError(name)


def pattern_task(args):
    name, k, n = args
    ci = circuit(name)
    blk = O.fock_diag_pattern(ci.A, ci.b, ci.c, ci.cutoffs, ci.detected_mask, n)
    rng = np.random.default_rng(1000 + 17 * k + 1)
    g = rng.standard_normal(blk.shape) + 1j * rng.standard_normal(blk.shape)
    det = [j for j in range(ci.M) if (ci.detected_mask >> j) & 1]
    cut = list(ci.cutoffs)
    for j, x in zip(det, n):
        cut[j] = x + 1
    G = np.zeros(O.fock_diag(ci.A, ci.b, ci.c, cut, ci.detected_mask).shape, complex)
    G[(Ellipsis,) + tuple(n)] = g
    dA, db, dc = O.fock_diag_vjp(ci.A, ci.b, ci.c, cut, ci.detected_mask, G)
    return name, k, np.asarray(blk, complex), g, dA, db, dc


def batch_patterns(ci):
    det = [j for j in range(ci.M) if (ci.detected_mask >> j) & 1]
    nd = len(det)
    C = [ci.cutoffs[j] for j in det]
    pats = [tuple([C[0] - 1] + [0] * (nd - 1))]
    if nd == ci.M:   # all detected: scalar outputs, cheap boxes
        pats.append(tuple([0] * (nd - 1) + [C[-1] - 1]))
        pats.append(tuple([1] * nd))
        pats.append(tuple([C[0] - 1, C[1] - 1] + [0] * (nd - 2)))
    else:
        pats.append(tuple([1] * min(3, nd) + [0] * (nd - min(3, nd))))
    return pats


def batch_task(i):
    ci = W.config3()[i]
    out = []
    for n in batch_patterns(ci):
        out.append((n, np.asarray(O.fock_diag_pattern(ci.A, ci.b, ci.c, ci.cutoffs, ci.detected_mask, n), complex)))
    return i, out


def main():
    t0 = time.time()
    tasks = [(name, k, n) for name, pats in PATTERNS.items() for k, n in enumerate(pats)]
    with Pool(6) as pool:
        res = pool.map(pattern_task, tasks, chunksize=1)
        print(f"patterns done {time.time() - t0:.0f} s", flush=True)
        bres = pool.map(batch_task, range(256), chunksize=4)
        print(f"batch done {time.time() - t0:.0f} s", flush=True)
    arrs = {}
    for name, k, blk, g, dA, db, dc in res:
        arrs[f"{name}_pattern_{k}"] = np.array(PATTERNS[name][k])
        arrs[f"{name}_rho_{k}"] = blk
        arrs[f"{name}_g_{k}"] = g
        arrs[f"{name}_dA_{k}"] = dA
        arrs[f"{name}_db_{k}"] = db
        arrs[f"{name}_dc_{k}"] = np.array([dc])
    np.savez_compressed(os.path.join(HERE, "parity_patterns.npz"), **arrs)
    circ_idx, pats, offs, vals = [], [], [0], []
    for i, lst in sorted(bres):
        for n, v in lst:
            circ_idx.append(i)
            pats.append(list(n) + [-1] * (8 - len(n)))
            vals.append(v.reshape(-1))
            offs.append(offs[-1] + v.size)
    np.savez_compressed(os.path.join(HERE, "parity_batch.npz"), circ=np.array(circ_idx), pattern=np.array(pats),
                        offsets=np.array(offs), values=np.concatenate(vals))
    # pure 8-mode state: dense cotangent over every detection probability
    ci = W.pure_state(PURE8["seed"], PURE8["M"], [PURE8["cut"]] * PURE8["M"], PURE8["r_lo"], PURE8["r_hi"])
    A, b, c = ci.params["rho_triple"]
    psi = O.state_vector(ci.A, ci.b, ci.c, ci.cutoffs)
    print(f"psi done {time.time() - t0:.0f} s", flush=True)
    g = W.random_cotangent(tuple(ci.cutoffs), seed=PURE8["cot_seed"])
    dA, db, dc = O.probs_vjp_pure(psi, c, g)
    np.savez_compressed(os.path.join(HERE, "parity_pure8.npz"), dA=dA, db=db, dc=np.array([dc]),
                        **{k: np.array(v) for k, v in PURE8.items()})
    print(f"all done {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
