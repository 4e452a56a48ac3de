"""Selective CPU oracle (Tier D) -- TEST INFRASTRUCTURE ONLY.

``fock_diag_selective`` runs the paper's pivot schedules as printed
(Algorithm 1, Sec. 3.1; Algorithm 2 with its step 1 and coarse-grained step 2,
Sec. 3.2) on the CPU: plain C in ``fock_selective.c``, every amplitude kept
in a hash map keyed by its 2M-index, every pivot writing its increments by
Eq. recrel.  It returns the same selected outputs as ``fock_diag`` without
the full box, so it reaches sizes the Taylor box cannot (eight detected modes
at cutoff 4, for one), and it checks the schedule while it runs: a read of
an amplitude that no earlier pivot wrote, or two writes of one amplitude that
disagree, is an error.

The C library is compiled on first use (gcc, in ``oracle/_build/``) or by
``__graft_entry__.build()``; it shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .fock_oracle import to_interleaved

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fock_selective.c")
LIB = os.path.join(HERE, "_build", "libfock_selective.so")

_lib = None

ERRORS = {1: "a pivot read an amplitude that no earlier pivot wrote",
          2: "two writes of one amplitude disagree",
          3: "out of memory", 4: "bad arguments"}


def build(force: bool = False) -> str:
    """Compiles the C oracle (gcc -O2, OpenMP) unless an up-to-date build exists."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"],
                       check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        L.fd_oracle_selective.argtypes = [ctypes.c_int, ip, ip, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_int]
        L.fd_oracle_selective.restype = ctypes.c_int
        _lib = L
    return _lib


def fock_diag_selective(A, b, c, cutoffs, detected_mask: int, nthreads: int = 1):
    """(rho, pivots): rho[k_U, l_U, n_D] as ``fock_diag`` returns it, and the
    number of pivots the schedule applied.  A and b in block order
    [ket_1..ket_M, bra_1..bra_M] (A enters through its symmetric part)."""
    M0 = len(cutoffs)
    A = np.asarray(A, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    det0 = [(detected_mask >> j) & 1 for j in range(M0)]
    shape0 = tuple([cutoffs[j] for j in range(M0) if not det0[j]] * 2 + [cutoffs[j] for j in range(M0) if det0[j]])
    # a mode with cutoff 1 never carries a photon: no pivot increments its
    # indices, so the amplitudes are those of the triple without its rows and
    # columns (the schedules as printed need C >= 2 in the modes they sweep)
    keep = [j for j in range(M0) if cutoffs[j] >= 2]
    if not keep:
        return np.full(shape0, complex(c), dtype=np.complex128), 0
    sel = keep + [M0 + j for j in keep]
    A, b = A[np.ix_(sel, sel)], b[sel]
    cutoffs = [cutoffs[j] for j in keep]
    detected_mask = sum(1 << k for k, j in enumerate(keep) if det0[j])
    M = len(cutoffs)
    Ai, bi = to_interleaved(A, b)
    Ai = np.ascontiguousarray(Ai, dtype=np.complex128)
    bi = np.ascontiguousarray(bi, dtype=np.complex128)
    cc = np.array([complex(c)], dtype=np.complex128)
    det = [(detected_mask >> j) & 1 for j in range(M)]
    U = [j for j in range(M) if not det[j]]
    D = [j for j in range(M) if det[j]]
    shape = tuple([cutoffs[j] for j in U] * 2 + [cutoffs[j] for j in D])
    out = np.zeros(int(np.prod(shape)) if shape else 1, dtype=np.complex128)
    cut = (ctypes.c_int * M)(*cutoffs)
    dm = (ctypes.c_int * M)(*det)
    piv = ctypes.c_int64(0)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib().fd_oracle_selective(M, cut, dm, Ai.ctypes.data_as(dp), bi.ctypes.data_as(dp), cc.ctypes.data_as(dp),
                                   out.ctypes.data_as(dp), ctypes.byref(piv), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"selective oracle: {ERRORS.get(rc, rc)}")
    return out.reshape(shape0), int(piv.value)
