"""Host-side runner of fock_diag_fwd_batch for batches larger than device
memory, and the autotuner of the batched sweep's scheduling knobs.

A batch whose outputs and workspaces exceed the memory budget is packed into
groups (first-fit decreasing by bytes) that each fit one arena; every group is
one fock_diag_fwd_batch call, i.e. one persistent sweep launch.  Groups run one
after the other on the current stream and reuse the arena, so the outputs of a
group are valid until the next group runs (``run(callback)`` hands each
group's outputs to the caller in between).
"""
from __future__ import annotations

import time

import torch

from . import fockdiag as F


def _al(x, a=256):
    return (int(x) + a - 1) // a * a


class BatchRunner:
    def __init__(self, shapes, triples, dtype=torch.complex128, b_mode="zero", budget_bytes=None,
                 device="cuda"):
        """shapes: list of (cutoffs, detected_mask); triples: list of (A, b, c)."""
        self.dtype = dtype
        self.eb = 16 if dtype == torch.complex128 else 8
        self.plans = [F.Plan(cut, mask, dtype, b_mode) for cut, mask in shapes]
        self.ws_bytes = [p.workspace(False)[0] for p in self.plans]
        self.out_elems = [p.query(F.FD_Q_OUT_ELEMS) for p in self.plans]
        need = [_al(w) + _al(o * self.eb) for w, o in zip(self.ws_bytes, self.out_elems)]
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.6 * free)
        budget_bytes = max(int(budget_bytes), max(need))
        order = sorted(range(len(need)), key=lambda i: -need[i])
        self.groups, load = [], []
        for i in order:
            for g in range(len(self.groups)):
                if load[g] + need[i] <= budget_bytes:
                    self.groups[g].append(i)
                    load[g] += need[i]
                    break
            else:
                self.groups.append([i])
                load.append(need[i])
        self.arena = torch.empty(max(load), dtype=torch.uint8, device=device)
        self.inputs = [(torch.as_tensor(A, dtype=dtype, device=device).contiguous(),
                        torch.as_tensor(b, dtype=dtype, device=device).contiguous(),
                        torch.as_tensor(c, dtype=dtype, device=device).reshape(1).contiguous())
                       for A, b, c in triples]
        self.views = [self._carve(g) for g in self.groups]

    def _carve(self, g):
        off, rho, ws = 0, {}, {}
        for i in g:
            ws[i] = self.arena[off:off + self.ws_bytes[i]]
            off += _al(self.ws_bytes[i])
            n = self.out_elems[i] * self.eb
            rho[i] = self.arena[off:off + n].view(self.dtype).view(self.plans[i].out_shape)
            off += _al(n)
        return rho, ws

    def run_group(self, k, batched=True):
        g, (rho, ws) = self.groups[k], self.views[k]
        if batched:
            F.fock_diag_fwd_batch([self.plans[i] for i in g], [self.inputs[i][0] for i in g],
                                  [self.inputs[i][1] for i in g], [self.inputs[i][2] for i in g],
                                  [rho[i] for i in g], [ws[i] for i in g])
        else:
            for i in g:
                F.fock_diag_fwd(self.plans[i], *self.inputs[i], rho[i], ws[i])
        return rho

    def run(self, batched=True, callback=None):
        """Every group; callback(group_index, {circuit: rho}) after each."""
        for k in range(len(self.groups)):
            rho = self.run_group(k, batched)
            if callback is not None:
                callback(k, rho)

    def check_status(self):
        for p in self.plans:
            F.fd_device_status(p)


# Winners of earlier autotune calls, per batch signature (dtype and every
# circuit's cutoffs and detection mask).
_tuned = {}

DEFAULT_TUNING = (2, 64, 4, 2048, 0)


def _signature(runner):
    return (str(runner.dtype),) + tuple((tuple(p.cutoffs), p.detected_mask) for p in runner.plans)


def _time(runner, cand, reps):
    F.fd_batch_set_tuning(*cand)
    runner.run(True)           # builds the schedules (and graphs) under this tuning
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        runner.run(True)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def autotune(runner, candidates=None, reps=1, use_cache=True):
    """Times the runner's batched calls under candidate knob sets
    (min_block_units, min_point_units, items_per_wave, fill_waves, use_graph),
    keeps the fastest (set process-wide through fd_batch_set_tuning) and
    returns (best, {candidate: seconds}).

    Without explicit candidates the search goes one knob group at a time from
    the defaults: the item sizes, then the routing threshold fill_waves
    (circuits whose levels average that many wavefront units run their own
    level launches), then graph replay of the whole call.  The winner is
    remembered per batch signature; a later call with the same signature sets
    it without timing (``use_cache=False`` times again)."""
    sig = _signature(runner)
    if candidates is None and use_cache and sig in _tuned:
        F.fd_batch_set_tuning(*_tuned[sig])
        return _tuned[sig], {}
    times = {}
    if candidates is not None:
        for cand in candidates:
            cand = tuple(cand) + DEFAULT_TUNING[len(cand):]
            times[cand] = _time(runner, cand, reps)
    else:
        best = DEFAULT_TUNING
        for items in [(2, 64, 4), (4, 128, 2), (1, 64, 8), (8, 256, 2)]:
            cand = items + best[3:]
            times[cand] = _time(runner, cand, reps)
        best = min(times, key=times.get)
        for fill in (1024, 4096):
            cand = best[:3] + (fill, best[4])
            times[cand] = _time(runner, cand, reps)
        best = min(times, key=times.get)
        cand = best[:4] + (1,)
        t = _time(runner, cand, reps)
        if F.fd_batch_get_tuning()[4] == 1:   # -1: the runtime refused the capture
            times[cand] = t
    best = min(times, key=times.get)
    F.fd_batch_set_tuning(*best)
    _tuned[sig] = best
    return best, times
