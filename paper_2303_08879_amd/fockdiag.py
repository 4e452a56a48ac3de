"""Thin ctypes binding of libfockdiag.so (include/fockdiag.h), same names.

Only argument marshalling happens here: tensors become device pointers and
sizes, the current torch stream becomes the hipStream_t.  Every step of the
computation runs in the library's HIP kernels; if the library is missing the
calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfockdiag.so")

FD_OK, FD_ERR_INVALID_ARG, FD_ERR_UNSUPPORTED, FD_ERR_WORKSPACE, FD_ERR_OOM, FD_ERR_HIP, FD_ERR_NONFINITE = range(7)
FD_C128, FD_C64 = 0, 1
FD_B_AUTO, FD_B_ZERO, FD_B_GENERAL = 0, 1, 2
(FD_Q_OUT_ELEMS, FD_Q_LEVELS, FD_Q_PIVOTS, FD_Q_STORED_NODES, FD_Q_TARGETS, FD_Q_READ_TERMS, FD_Q_BLOCK,
 FD_Q_NODES_F0, FD_Q_NODES_F1, FD_Q_NODES_F2, FD_Q_NODES_F1010, FD_Q_NODES_F1001, FD_Q_B_SCHEDULE) = range(13)

EXPORTS = [
    "fd_plan_create", "fd_plan_destroy", "fd_plan_workspace", "fd_plan_query", "fock_diag_fwd",
    "fock_diag_vjp", "detection_probs", "fock_diag_fwd_batch", "fd_last_error", "fd_device_status",
    "fd_plan_timing", "fd_plan_kernel_times", "fd_plan_use_graphs", "fd_batch_set_tuning", "fd_batch_get_tuning",
    "fock_diag_vjp_batch", "fd_state_plan_create", "fd_state_plan_destroy", "fd_state_plan_workspace",
    "fock_state_fwd", "fd_state_device_status", "fd_state_plan_timing", "fd_state_plan_kernel_times",
    "fd_plan_create_total", "fd_plan_level_offsets", "detection_probs_until", "fd_state_plan_vjp_workspace",
    "fock_state_vjp", "fock_state_jvp", "fd_plan_jvp_workspace", "fock_diag_jvp", "fock_diag_fwd_static",
    "fd_plan_set_checkpoint", "fd_plan_set_write_counters",
]
(FD_K_PREP, FD_K_UFILL, FD_K_FWD_LEVEL, FD_K_OUT_PERM, FD_K_PERM_IN, FD_K_VJP_LEVEL, FD_K_UFILL_VJP,
 FD_K_VJP_FINAL, FD_K_ZERO, FD_K_BATCH_PREP, FD_K_BATCH_SWEEP, FD_K_BATCH_OUT) = range(12)

_lib = None
# Every plan object not yet destroyed: released in order at interpreter exit
# (see _release_all).
_live = weakref.WeakSet()


class BatchTuning(ctypes.Structure):
    """fd_batch_tuning: scheduling knobs of fock_diag_fwd_batch."""
    _fields_ = [("min_block_units", ctypes.c_int32), ("min_point_units", ctypes.c_int32),
                ("items_per_wave", ctypes.c_int32), ("fill_waves", ctypes.c_int32), ("use_graph", ctypes.c_int32)]

    def as_tuple(self):
        return (self.min_block_units, self.min_point_units, self.items_per_wave, self.fill_waves, self.use_graph)


class FockDiagError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fockdiag status {status}: {msg}")
        self.status = status


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_2303_08879_amd/build.py (or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, u32, i64p = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int64)
    L.fd_plan_create.argtypes = [i32, ctypes.POINTER(ctypes.c_int), u32, i32, u32, ctypes.POINTER(vp)]
    L.fd_plan_destroy.argtypes = [vp]
    L.fd_plan_workspace.argtypes = [vp, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.fd_plan_query.argtypes = [vp, i32, i64p]
    L.fock_diag_fwd.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp, sz, vp]
    L.fock_diag_fwd_static.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fock_diag_vjp.argtypes = [vp, vp, vp, vp, vp, sz, vp, vp, vp, vp, vp, sz, vp]
    L.detection_probs.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.fock_diag_fwd_batch.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(sz), vp]
    L.fock_diag_vjp_batch.argtypes = [i32] + [ctypes.POINTER(vp)] * 5 + [ctypes.POINTER(sz)] + \
        [ctypes.POINTER(vp)] * 5 + [ctypes.POINTER(sz), vp]
    L.fd_last_error.argtypes = []
    L.fd_last_error.restype = ctypes.c_char_p
    L.fd_device_status.argtypes = [vp, vp]
    L.fd_plan_timing.argtypes = [vp, u32]
    L.fd_plan_use_graphs.argtypes = [vp, i32]
    L.fd_plan_set_checkpoint.argtypes = [vp, i32]
    L.fd_plan_set_write_counters.argtypes = [vp, vp, sz]
    L.fd_plan_kernel_times.argtypes = [vp, i32, i64p, ctypes.POINTER(ctypes.c_double)]
    L.fd_batch_set_tuning.argtypes = [ctypes.POINTER(BatchTuning)]
    L.fd_batch_get_tuning.argtypes = [ctypes.POINTER(BatchTuning)]
    L.fd_plan_create_total.argtypes = [i32, ctypes.POINTER(ctypes.c_int), i32, i32, u32, ctypes.POINTER(vp)]
    L.fd_plan_level_offsets.argtypes = [vp, i64p, i32]
    L.detection_probs_until.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    L.fd_plan_jvp_workspace.argtypes = [vp, ctypes.POINTER(sz)]
    L.fock_diag_jvp.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.fd_state_plan_create.argtypes = [i32, ctypes.POINTER(ctypes.c_int), i32, u32, ctypes.POINTER(vp)]
    L.fd_state_plan_destroy.argtypes = [vp]
    L.fd_state_plan_vjp_workspace.argtypes = [vp, ctypes.POINTER(sz)]
    L.fock_state_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.fock_state_jvp.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.fd_state_plan_workspace.argtypes = [vp, ctypes.POINTER(sz)]
    L.fock_state_fwd.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.fd_state_device_status.argtypes = [vp, vp]
    L.fd_state_plan_timing.argtypes = [vp, u32]
    L.fd_state_plan_kernel_times.argtypes = [vp, i32, i64p, ctypes.POINTER(ctypes.c_double)]
    for name in EXPORTS:
        if name != "fd_last_error":
            getattr(L, name).restype = i32
    _lib = L
    atexit.register(_release_all)
    return L


def _release_all():
    """Destroys every live plan at interpreter exit, while the HIP runtime (and
    any profiler attached to it) is still fully up: plans own device tables,
    captured graphs, a capture stream and the batched sweep's cached
    schedules, and leaving them to the garbage collection of module globals
    would release them at an unspecified point of the shutdown.  Pending work
    is waited for first."""
    if _lib is None:
        return
    try:
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except RuntimeError:
        pass
    for p in list(_live):
        p.close()


def _check(status):
    if status != FD_OK:
        raise FockDiagError(status, lib().fd_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


class Plan:
    """fd_plan_create / fd_plan_destroy.  ``dtype`` is torch.complex128 or
    torch.complex64; ``b_mode`` one of 'auto', 'zero', 'general'."""

    def __init__(self, cutoffs, detected_mask, dtype=torch.complex128, b_mode="auto", total_cutoff=None):
        """total_cutoff: a total photon cutoff (fd_plan_create_total; every mode
        detected, output p(n) in level order)."""
        self.cutoffs = [int(c) for c in cutoffs]
        self.M = len(self.cutoffs)
        self.detected_mask = int(detected_mask)
        self.dtype = dtype
        self.total_cutoff = total_cutoff
        dt = FD_C128 if dtype == torch.complex128 else FD_C64
        flags = {"auto": FD_B_AUTO, "zero": FD_B_ZERO, "general": FD_B_GENERAL}[b_mode]
        arr = (ctypes.c_int * self.M)(*self.cutoffs)
        h = ctypes.c_void_p()
        if total_cutoff is None:
            _check(lib().fd_plan_create(self.M, arr, self.detected_mask, dt, flags, ctypes.byref(h)))
        else:
            _check(lib().fd_plan_create_total(self.M, arr, int(total_cutoff), dt, flags, ctypes.byref(h)))
            self.detected_mask = (1 << self.M) - 1
        self.handle = h
        _live.add(self)

    def close(self):
        """fd_plan_destroy (idempotent; the plan is unusable afterwards)."""
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.fd_plan_destroy(h)
        self.handle = None

    def __del__(self):
        self.close()

    def level_offsets(self):
        """fd_plan_level_offsets (plans with every mode detected)."""
        n = self.query(FD_Q_LEVELS) + 1
        arr = (ctypes.c_int64 * n)()
        _check(lib().fd_plan_level_offsets(self.handle, arr, n))
        return list(arr)

    @property
    def out_shape(self):
        if self.total_cutoff is not None:
            return (self.query(FD_Q_OUT_ELEMS),)
        U = [j for j in range(self.M) if not (self.detected_mask >> j) & 1]
        D = [j for j in range(self.M) if (self.detected_mask >> j) & 1]
        return tuple([self.cutoffs[j] for j in U] * 2 + [self.cutoffs[j] for j in D])

    def workspace(self, with_vjp=False):
        """(workspace bytes, saved bytes) -- fd_plan_workspace."""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().fd_plan_workspace(self.handle, int(bool(with_vjp)), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def jvp_workspace(self):
        """Workspace bytes of fock_diag_jvp -- fd_plan_jvp_workspace."""
        n = ctypes.c_size_t()
        _check(lib().fd_plan_jvp_workspace(self.handle, ctypes.byref(n)))
        return n.value

    def query(self, what):
        v = ctypes.c_int64()
        _check(lib().fd_plan_query(self.handle, int(what), ctypes.byref(v)))
        return v.value


class StatePlan:
    """fd_state_plan_create / fd_state_plan_destroy: the state vector psi of a
    pure state over ``cutoffs`` (shape = cutoffs, C order)."""

    def __init__(self, cutoffs, dtype=torch.complex128, b_mode="auto"):
        self.cutoffs = [int(c) for c in cutoffs]
        self.M = len(self.cutoffs)
        self.dtype = dtype
        dt = FD_C128 if dtype == torch.complex128 else FD_C64
        flags = {"auto": FD_B_AUTO, "zero": FD_B_ZERO, "general": FD_B_GENERAL}[b_mode]
        arr = (ctypes.c_int * self.M)(*self.cutoffs)
        h = ctypes.c_void_p()
        _check(lib().fd_state_plan_create(self.M, arr, dt, flags, ctypes.byref(h)))
        self.handle = h
        _live.add(self)

    def close(self):
        """fd_state_plan_destroy (idempotent)."""
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.fd_state_plan_destroy(h)
        self.handle = None

    def __del__(self):
        self.close()

    @property
    def out_shape(self):
        return tuple(self.cutoffs)

    def workspace(self):
        n = ctypes.c_size_t()
        _check(lib().fd_state_plan_workspace(self.handle, ctypes.byref(n)))
        return n.value

    def vjp_workspace(self):
        n = ctypes.c_size_t()
        _check(lib().fd_state_plan_vjp_workspace(self.handle, ctypes.byref(n)))
        return n.value


def fock_state_fwd(plan, A, b, c, psi, workspace, stream=None):
    _check(lib().fock_state_fwd(plan.handle, _ptr(A), _ptr(b), _ptr(c), _ptr(psi), _ptr(workspace),
                                _nbytes(workspace), _stream(stream)))


def fock_state_vjp(plan, c, psi, dpsi, dA, db, dc, workspace, stream=None):
    _check(lib().fock_state_vjp(plan.handle, _ptr(c), _ptr(psi), _ptr(dpsi), _ptr(dA), _ptr(db), _ptr(dc),
                                _ptr(workspace), _nbytes(workspace), _stream(stream)))


def fock_state_jvp(plan, c, psi, dA, db, dc, dpsi, stream=None):
    _check(lib().fock_state_jvp(plan.handle, _ptr(c), _ptr(psi), _ptr(dA), _ptr(db), _ptr(dc), _ptr(dpsi),
                                _stream(stream)))


def fd_state_device_status(plan, stream=None):
    _check(lib().fd_state_device_status(plan.handle, _stream(stream)))


def fd_state_plan_timing(plan, kind_mask):
    _check(lib().fd_state_plan_timing(plan.handle, int(kind_mask)))


def fd_state_plan_kernel_times(plan, kind):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().fd_state_plan_kernel_times(plan.handle, int(kind), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def fock_diag_fwd(plan, A, b, c, rho, workspace, saved=None, stream=None):
    _check(lib().fock_diag_fwd(plan.handle, _ptr(A), _ptr(b), _ptr(c), _ptr(rho), _ptr(workspace),
                               _nbytes(workspace), _ptr(saved), _nbytes(saved), _stream(stream)))


def fock_diag_fwd_static(plan, A, b, c, rho, stream=None):
    """fock_diag_fwd with the library's static scratch (no allocation)."""
    _check(lib().fock_diag_fwd_static(plan.handle, _ptr(A), _ptr(b), _ptr(c), _ptr(rho), _stream(stream)))


def fock_diag_jvp(plan, A, b, c, dA, db, dc, rho, drho, workspace, stream=None):
    _check(lib().fock_diag_jvp(plan.handle, _ptr(A), _ptr(b), _ptr(c), _ptr(dA), _ptr(db), _ptr(dc), _ptr(rho),
                               _ptr(drho), _ptr(workspace), _nbytes(workspace), _stream(stream)))


def detection_probs(plan, A, b, c, probs, workspace, stream=None):
    _check(lib().detection_probs(plan.handle, _ptr(A), _ptr(b), _ptr(c), _ptr(probs), _ptr(workspace),
                                 _nbytes(workspace), _stream(stream)))


def detection_probs_until(plan, A, b, c, probs, eps, workspace, stream=None):
    """Returns (levels_done, mass)."""
    n, m = ctypes.c_int(), ctypes.c_double()
    _check(lib().detection_probs_until(plan.handle, _ptr(A), _ptr(b), _ptr(c), _ptr(probs), float(eps),
                                       ctypes.byref(n), ctypes.byref(m), _ptr(workspace), _nbytes(workspace),
                                       _stream(stream)))
    return n.value, m.value


def fock_diag_vjp(plan, A, b, c, saved, drho, dA, db, dc, workspace, stream=None):
    _check(lib().fock_diag_vjp(plan.handle, _ptr(A), _ptr(b), _ptr(c), _ptr(saved), _nbytes(saved), _ptr(drho),
                               _ptr(dA), _ptr(db), _ptr(dc), _ptr(workspace), _nbytes(workspace),
                               _stream(stream)))


def fock_diag_fwd_batch(plans, As, bs, cs, rhos, workspaces, stream=None):
    n = len(plans)
    P = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    mk = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])
    sizes = (ctypes.c_size_t * n)(*[_nbytes(w) for w in workspaces])
    _check(lib().fock_diag_fwd_batch(n, P, mk(As), mk(bs), mk(cs), mk(rhos), mk(workspaces), sizes,
                                     _stream(stream)))


def fd_batch_set_tuning(min_block_units, min_point_units, items_per_wave, fill_waves=2048, use_graph=0):
    t = BatchTuning(int(min_block_units), int(min_point_units), int(items_per_wave), int(fill_waves),
                    int(use_graph))
    _check(lib().fd_batch_set_tuning(ctypes.byref(t)))


def fd_batch_get_tuning():
    t = BatchTuning()
    _check(lib().fd_batch_get_tuning(ctypes.byref(t)))
    return t.as_tuple()


def fock_diag_vjp_batch(plans, As, bs, cs, saveds, drhos, dAs, dbs, dcs, workspaces, stream=None):
    """saveds: list of tensors or None entries (recompute), or None for all."""
    n = len(plans)
    arr = lambda ts: (ctypes.c_void_p * n)(*[None if t is None else t.data_ptr() for t in ts])
    szs = lambda ts: (ctypes.c_size_t * n)(*[_nbytes(t) for t in ts])
    P = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    saveds = saveds if saveds is not None else [None] * n
    _check(lib().fock_diag_vjp_batch(n, P, arr(As), arr(bs), arr(cs), arr(saveds), szs(saveds), arr(drhos),
                                     arr(dAs), arr(dbs), arr(dcs), arr(workspaces), szs(workspaces),
                                     _stream(stream)))


def fd_device_status(plan, stream=None):
    _check(lib().fd_device_status(plan.handle, _stream(stream)))


def fd_plan_set_checkpoint(plan, every):
    """Reverse-sweep checkpoint interval in levels (0: keep every level)."""
    _check(lib().fd_plan_set_checkpoint(plan.handle, int(every)))


def fd_plan_set_write_counters(plan, counters=None):
    """Debug write counters of fock_diag_fwd with a saved buffer: `counters`
    is a zeroed device tensor of 32-bit ints with at least one entry per
    element of the saved buffer, or None to switch the mode off."""
    if counters is None:
        _check(lib().fd_plan_set_write_counters(plan.handle, None, 0))
    else:
        _check(lib().fd_plan_set_write_counters(plan.handle, _ptr(counters), counters.numel()))


def fd_plan_use_graphs(plan, enable=True):
    _check(lib().fd_plan_use_graphs(plan.handle, int(bool(enable))))


def fd_plan_timing(plan, kind_mask):
    _check(lib().fd_plan_timing(plan.handle, int(kind_mask)))


def fd_plan_kernel_times(plan, kind):
    """(launches, total milliseconds) of kernel kind `kind` since timing was enabled."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().fd_plan_kernel_times(plan.handle, int(kind), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def fd_last_error():
    return lib().fd_last_error().decode()
