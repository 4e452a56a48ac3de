"""Parity criteria of the GPU results against the oracle.

The bar in complex128 is a relative error of 1e-10.  Every comparison checks
  * normwise:      ||x - r||_2 / ||r||_2 <= tol;
  * entry by entry, on the entries with |r| >= floor * max|r|:
                   |x - r| <= tol * |r|;
  * the remaining (tiny) entries in absolute terms:
                   |x - r| <= SMALL_ABS * max|r|,
so an error confined to small entries cannot hide behind the large ones.
SMALL_ABS = 1e-14 is about 45 units in the last place of the largest entry:
tiny entries come out of sums of terms as large as that entry, so their
rounding is measured on its scale (the full 8-mode pure-state forward, 16.8M
entries, shows 3.9e-16).
The measured figures are printed (pytest -s / -v logs keep them).
"""
from __future__ import annotations

import numpy as np

TOL = 1e-10
FLOOR = 1e-6
SMALL_ABS = 1e-14


def compare(got, ref, floor=FLOOR):
    x = np.asarray(got, dtype=np.complex128).ravel()
    r = np.asarray(ref, dtype=np.complex128).ravel()
    assert x.shape == r.shape, (x.shape, r.shape)
    d = np.abs(x - r)
    a = np.abs(r)
    amax = float(a.max()) if a.size else 0.0
    nr = float(np.linalg.norm(r))
    out = {"n": int(r.size), "max_ref": amax,
           "normwise": float(np.linalg.norm(d)) / nr if nr > 0 else float(np.linalg.norm(d))}
    if amax == 0.0:
        out.update(elementwise_large=0.0, small_abs_over_max=float(d.max()) if d.size else 0.0, n_large=0)
        return out
    big = a >= floor * amax
    out["n_large"] = int(big.sum())
    out["elementwise_large"] = float((d[big] / a[big]).max())
    out["small_abs_over_max"] = float(d[~big].max()) / amax if (~big).any() else 0.0
    return out


def assert_close(got, ref, tol=TOL, floor=FLOOR, label=""):
    s = compare(got, ref, floor)
    print(f"[parity] {label} n={s['n']} large={s['n_large']} normwise={s['normwise']:.2e} "
          f"elementwise={s['elementwise_large']:.2e} small_abs/max={s['small_abs_over_max']:.2e}", flush=True)
    assert s["normwise"] <= tol, (label, s)
    assert s["elementwise_large"] <= tol, (label, s)
    assert s["small_abs_over_max"] <= max(tol * floor, SMALL_ABS), (label, s)
    return s


def grad_vector(dA, db, dc):
    return np.concatenate([np.ravel(dA), np.ravel(db), np.ravel([dc])]).astype(np.complex128)


def assert_grad_close(got, ref, tol=TOL, floor=FLOOR, label="", zero=()):
    """(dA, db, dc) against the reference, element-wise over the concatenated
    gradient.  ``zero`` names components that vanish by construction (e.g.
    'db' when b = 0 and every output has even weight): their reference must
    be below 1e-12 of the gradient's largest entry, and the element-wise
    check then holds them to the absolute floor."""
    names = ("dA", "db", "dc")
    scale = float(np.max(np.abs(grad_vector(*ref))))
    for name, r in zip(names, ref):
        if name in zero:
            assert np.max(np.abs(np.ravel([r]))) <= 1e-12 * scale, (label, name)
    return assert_close(grad_vector(*got), grad_vector(*ref), tol, floor, label)
