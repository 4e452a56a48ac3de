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


def autotune(runner, candidates=None, reps=1):
    """Times the batched sweep of the runner's batch under each candidate
    (min_block_units, min_point_units, items_per_wave), keeps the fastest
    (set process-wide through fd_batch_set_tuning) and returns
    (best, {candidate: seconds})."""
    if candidates is None:
        candidates = [(2, 64, 4), (4, 128, 2), (1, 64, 8), (8, 256, 2)]
    times = {}
    for cand in candidates:
        F.fd_batch_set_tuning(*cand)
        runner.run(True)           # builds the schedules under this tuning
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            runner.run(True)
        torch.cuda.synchronize()
        times[cand] = (time.perf_counter() - t0) / reps
    best = min(times, key=times.get)
    F.fd_batch_set_tuning(*best)
    return best, times
