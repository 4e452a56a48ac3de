#!/usr/bin/env python3
"""Benchmark of the selective Fock-amplitude path on one MI355X.

Headline workload (default): 8 modes, all detected, cutoff 8 (the 8^8 =
16.8M detection probabilities of a lossy squeezed state through a Haar
interferometer, b = 0), seeded synthetic triple; one step = forward (every
intermediate kept for the reverse sweep) + reverse sweep with a dense seeded
cotangent, complex128.  `value` = output Fock amplitudes (entries of rho) per
second of whole-step wall time, inputs already resident in HBM.

Roofline: the dominant level kernel's algorithmic bytes (32 B per computed
amplitude forward, 48 B reverse, complex128) over its HIP-event time, against
8 TB/s.  Extra legs in the same line: the other single-circuit workloads
(2 modes; 4 modes with an undetected mode; 5 modes with an undetected mode),
the complex64 variant of every single-circuit workload with its measured
error against the complex128 result, the 64-circuit gradient batch, the
256-circuit uneven batch (persistent batched launch against a graph-replayed
per-circuit loop), the pure-state, total-cutoff and forward-mode legs, and
the CPU oracle on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "Fock amplitudes/s (c128, fwd+VJP) and batched circuits/s at ≤1e-10 rel err"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def workload(name):
    from paper_2303_08879_amd import workloads as W
    if name == "config1":
        return W.config1(), "M=2 both detected C=10, eta=0.9, b=0"
    if name == "config2":
        return W.config2(), "M=4 conditional state: mode 0 undetected C_U=30, modes 1-3 detected C_D=12, b!=0"
    if name == "config4":
        return W.config4(), "M=5 conditional state: mode 0 undetected C_U=40, modes 1-4 detected C_D=10, b=0"
    if name == "config5":
        return W.config5(), "M=8 all detected C=8 (16.8M detection probabilities), b=0"
    raise SystemExit(f"unknown workload {name}")


# Sources each level kernel is compiled from: a counter summary applies to a
# kernel only while these hash to the value recorded with it.
KERNEL_SOURCES = {
    "k_vjp_point": ["kernels_vjp.hip", "vjp_common.h", "fd_device.h"],
    "k_vjp_block": ["kernels_vjp_block.hip", "vjp_common.h", "fd_device.h"],
    "k_fwd_point": ["kernels_fwd.hip", "fwd_units.h", "fd_device.h"],
    "k_fwd_block": ["kernels_fwd.hip", "fwd_units.h", "fd_device.h"],
    "k_state_level": ["kernels_state.hip", "fd_device.h"],
    "k_state_jvp": ["kernels_state.hip", "fd_device.h"],
    "k_state_vjp": ["kernels_state.hip", "fd_device.h"],
}


def kernel_source_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, "paper_2303_08879_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, kernel):
    """HBM bytes per launch of `kernel` on `workload_name` from the committed
    rocprofv3 counter summary profiles/hbm_traffic_<workload>.md (FETCH_SIZE
    and WRITE_SIZE per dispatch, each scaled by what the counter reads for a
    plain copy of known size), or None when no summary covers it or the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(HERE, "profiles", f"hbm_traffic_{workload_name}.md")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    vals = {}
    for line in open(path):
        parts = line.split()
        if len(parts) >= 2 and parts[0] in ("fetch_scale", "write_scale"):
            vals[parts[0]] = float(parts[1])
        elif len(parts) == 5 and parts[0] == "kib":
            vals[parts[1]] = (float(parts[2]), float(parts[3]), parts[4])
    if kernel not in vals or vals[kernel][2] != kernel_source_hash(kernel):
        return None
    fetch, write, _ = vals[kernel]
    return 1024.0 * (fetch * vals["fetch_scale"] + write * vals["write_scale"])


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": model}


class CircuitStep:
    """One circuit in one complex dtype: plan, device buffers and the step
    forward (intermediates kept) + reverse sweep; whole sweeps replay one
    captured graph each (the buffers stay fixed)."""

    def __init__(self, circ, dtype, cot_seed=7):
        import numpy as np
        import torch
        from paper_2303_08879_amd import fockdiag as F
        from paper_2303_08879_amd import workloads as W
        self.F = F
        dev = "cuda"
        self.b_zero = not np.any(circ.b)
        self.plan = F.Plan(circ.cutoffs, circ.detected_mask, dtype, "zero" if self.b_zero else "general")
        self.A = torch.tensor(circ.A, dtype=dtype, device=dev)
        self.b = torch.tensor(circ.b, dtype=dtype, device=dev)
        self.c = torch.tensor([circ.c], dtype=dtype, device=dev)
        self.g = torch.tensor(W.random_cotangent(self.plan.out_shape, seed=cot_seed), dtype=dtype, device=dev)
        wsb, svb = self.plan.workspace(True)
        self.ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        self.saved = torch.empty(svb, dtype=torch.uint8, device=dev)
        self.rho = torch.empty(self.plan.out_shape, dtype=dtype, device=dev)
        self.dA, self.db, self.dc = torch.empty_like(self.A), torch.empty_like(self.b), torch.empty_like(self.c)
        F.fd_plan_use_graphs(self.plan, True)

    def step(self):
        F = self.F
        F.fock_diag_fwd(self.plan, self.A, self.b, self.c, self.rho, self.ws, self.saved)
        F.fock_diag_vjp(self.plan, self.A, self.b, self.c, self.saved, self.g, self.dA, self.db, self.dc, self.ws)

    def timed(self, steps, warmup):
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        self.F.fd_device_status(self.plan)
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def level_events(self, steps):
        """The same steps launched kernel by kernel with HIP events around every
        level-sweep launch (graph replay is off while timing is on):
        (forward launches, forward ms, reverse launches, reverse ms)."""
        import torch
        F = self.F
        F.fd_plan_timing(self.plan, (1 << F.FD_K_FWD_LEVEL) | (1 << F.FD_K_VJP_LEVEL))
        torch.cuda.synchronize()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        n_f, ms_f = F.fd_plan_kernel_times(self.plan, F.FD_K_FWD_LEVEL)
        n_v, ms_v = F.fd_plan_kernel_times(self.plan, F.FD_K_VJP_LEVEL)
        F.fd_plan_timing(self.plan, 0)
        F.fd_device_status(self.plan)
        return n_f, ms_f, n_v, ms_v

    def release(self):
        self.plan.close()
        for k in ("A", "b", "c", "g", "ws", "saved", "rho", "dA", "db", "dc"):
            setattr(self, k, None)


def errors_vs(x, ref):
    """Normwise relative error, max |x - ref| / max |ref|, and the largest
    element-wise relative error over the entries with |ref| >= 1e-6 max |ref|
    (computed on the device in float64)."""
    import torch
    x = x.to(torch.complex128).reshape(-1)
    ref = ref.to(torch.complex128).reshape(-1)
    d = (x - ref).abs()
    a = ref.abs()
    amax = float(a.max())
    big = a >= 1e-6 * amax
    return {"normwise": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(a)),
            "max_abs_over_max": float(d.max()) / amax,
            "elementwise_max_on_large": float((d[big] / a[big]).max())}


def grad_errors(s64, s128):
    import torch
    x = torch.cat([s64.dA.reshape(-1), s64.db.reshape(-1), s64.dc.reshape(-1)]).to(torch.complex128)
    r = torch.cat([s128.dA.reshape(-1), s128.db.reshape(-1), s128.dc.reshape(-1)])
    return float(torch.linalg.vector_norm(x - r) / torch.linalg.vector_norm(r))


def single_leg(name, steps, warmup, events=True, keep=False):
    """One single-circuit workload: complex128 step timing (+ level events),
    then the complex64 variant and its error against the complex128 result."""
    import torch
    circ, desc = workload(name)
    s = CircuitStep(circ, torch.complex128)
    sec = s.timed(steps, warmup)
    out_elems = s.plan.query(s.F.FD_Q_OUT_ELEMS)
    targets = s.plan.query(s.F.FD_Q_TARGETS)
    terms = s.plan.query(s.F.FD_Q_READ_TERMS)
    leg = {"workload": f"{name}: {desc}; one step = forward + VJP",
           "out_amplitudes": out_elems, "computed_amplitudes": targets, "read_terms": terms,
           "ms_per_step": 1e3 * sec / steps, "value": out_elems * steps / sec, "unit": "Fock amplitudes/s",
           "computed_amplitudes_per_s": targets * steps / sec, "steps": steps}
    if events:
        n_f, ms_f, n_v, ms_v = s.level_events(steps)
        leg.update({"fwd_level_launches_per_step": n_f // steps, "vjp_level_launches_per_step": n_v // steps,
                    "fwd_level_ms_per_step": ms_f / steps, "vjp_level_ms_per_step": ms_v / steps,
                    "fwd_level_GBs": 32.0 * targets * steps / (ms_f * 1e-3) / 1e9,
                    "vjp_level_GBs": 48.0 * targets * steps / (ms_v * 1e-3) / 1e9,
                    "fwd_level_GFLOPs": 8.0 * terms * steps / (ms_f * 1e-3) / 1e9,
                    "_ev": (n_f, ms_f, n_v, ms_v)})
    s.step()
    torch.cuda.synchronize()
    s64 = CircuitStep(circ, torch.complex64)
    sec64 = s64.timed(steps, warmup)
    s64.step()
    torch.cuda.synchronize()
    leg["c64"] = {"ms_per_step": 1e3 * sec64 / steps, "value": out_elems * steps / sec64,
                  "rho_error_vs_c128": errors_vs(s64.rho, s.rho),
                  "grad_rel_error_vs_c128": grad_errors(s64, s),
                  "note": "the complex128 result it is compared with matches the float64 oracle to <= 1e-10 "
                          "(tests); errors are relative to the complex128 values"}
    s64.release()
    if keep:
        return leg, s, circ
    s.release()
    torch.cuda.empty_cache()
    return leg


def cpu_baseline(circ, s128, s64, corner):
    """The oracle, unchanged, on a bounded sample of the same workload: every
    detection pattern with n_j < corner[j] (a Tier B box: the oracle's full
    Taylor box over the small cutoffs is exact for those patterns), forward
    plus the closed-form adjoint for the cotangent restricted to that sample;
    also the GPU's complex128 and complex64 errors on the sample."""
    import numpy as np
    import oracle as O
    import torch
    M = circ.M
    cut = [circ.cutoffs[j] if not (circ.detected_mask >> j) & 1 else corner[j] for j in range(M)]
    nU = sum(1 for j in range(M) if not (circ.detected_mask >> j) & 1)
    sl = (slice(None),) * (2 * nU) + tuple(slice(0, corner[j]) for j in range(M) if (circ.detected_mask >> j) & 1)
    from threadpoolctl import threadpool_limits
    g_full = s128.g.cpu().numpy()
    with threadpool_limits(1):   # one thread, library routines included
        t0 = time.perf_counter()
        out = O.fock_diag(circ.A, circ.b, circ.c, cut, circ.detected_mask)
        O.fock_diag_vjp(circ.A, circ.b, circ.c, cut, circ.detected_mask, g_full[sl])
        dt = time.perf_counter() - t0
    rho128 = s128.rho.cpu().numpy()[sl]
    rho64 = s64.rho.cpu().numpy()[sl].astype(np.complex128) if s64 is not None else None
    res = dict(value=out.size / dt, unit="Fock amplitudes/s", cores=1, kind="oracle",
               sample=(f"every detection pattern with n < {list(corner)} ({out.size} of {s128.rho.numel()} "
                       f"output amplitudes): the oracle's Taylor box over those cutoffs (exact for them), forward "
                       f"+ closed-form adjoint, numpy float64, one thread"),
               seconds=dt, host=host_info(),
               sample_rel_err_gpu_c128_vs_oracle=O.rel_err(rho128, out))
    if rho64 is not None:
        res["sample_rel_err_gpu_c64_vs_oracle"] = O.rel_err(rho64, out)
    del torch
    return res


def cpu_selective(circ, s128, s64):
    """The selective CPU oracle (the paper's pivot schedules run as printed,
    plain C, every host thread) on the largest corner of the workload whose
    patterns it reaches in a few seconds: forward only (it has no reverse
    mode), with the GPU's complex128 and complex64 results compared on every
    output of the corner, entry by entry."""
    import os
    from oracle import selective as S
    M = circ.M
    det = [(circ.detected_mask >> j) & 1 for j in range(M)]
    corner = [min(circ.cutoffs[j], 5 if M >= 8 else 6) if det[j] else circ.cutoffs[j] for j in range(M)]
    nU = M - sum(det)
    sl = (slice(None),) * (2 * nU) + tuple(slice(0, corner[j]) for j in range(M) if det[j])
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ref, piv = S.fock_diag_selective(circ.A, circ.b, circ.c, corner, circ.detected_mask, nthreads=threads)
    dt = time.perf_counter() - t0
    import torch
    ref_t = torch.from_numpy(ref).to(s128.rho.device)
    e128 = errors_vs(s128.rho[sl], ref_t)
    res = dict(value=ref.size / dt, unit="Fock amplitudes/s (forward only)", cores=threads, kind="oracle",
               sample=f"every detection pattern with n < {corner} ({ref.size} outputs, {piv} pivots)",
               seconds=dt, gpu_c128_vs_oracle=e128)
    if s64 is not None:
        res["gpu_c64_vs_oracle"] = errors_vs(s64.rho[sl], ref_t)
    return res


def batched_leg(reps=1):
    """The uneven batch (256 circuits, M 3..6, cutoffs 8..16, 0 or 1 undetected
    mode with cutoff 20..40, b = 0, complex128): batched persistent launches
    (one per memory group) against a loop of per-circuit fock_diag_fwd calls on
    the same stream and buffers, each replaying its captured graph; then the
    complex64 variant of every circuit (per-circuit calls, equal to the batched
    result bit for bit) against its complex128 result."""
    import torch
    from paper_2303_08879_amd import batching as Bt
    from paper_2303_08879_amd import fockdiag as F
    from paper_2303_08879_amd import workloads as W
    circs = W.config3()
    runner = Bt.BatchRunner([(c.cutoffs, c.detected_mask) for c in circs], [(c.A, c.b, c.c) for c in circs],
                            budget_bytes=int(150e9))
    best, tune = Bt.autotune(runner, reps=1, use_cache=False)
    runner.check_status()

    def timed(batched):
        runner.run(batched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            runner.run(batched)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    tb = timed(True)
    tl_eager = timed(False)
    for p in runner.plans:
        F.fd_plan_use_graphs(p, True)
    tl = timed(False)
    runner.check_status()
    n = len(circs)
    targets = sum(p.query(F.FD_Q_TARGETS) for p in runner.plans)
    outs = sum(p.query(F.FD_Q_OUT_ELEMS) for p in runner.plans)
    out = dict(workload="config3: 256 circuits, M~U{3..6}, C_D~U{8..16}, 0/1 undetected mode C_U~U{20..40}, b=0, "
                        "complex128", circuits=n, memory_groups=len(runner.groups),
               computed_amplitudes=targets, out_amplitudes=outs,
               batched_circuits_per_s=n / tb, loop_circuits_per_s=n / tl, speedup_vs_loop=tl / tb,
               loop_eager_circuits_per_s=n / tl_eager,
               batched_s=tb, loop_s=tl, loop_eager_s=tl_eager, tuning=list(best),
               tuning_trials_s={str(list(k)): v for k, v in tune.items()},
               batched_algorithmic_GBs=32.0 * targets / tb / 1e9,
               batched_roofline={"bound": "hbm", "achieved": 32.0 * targets / tb / 1e9, "peak": 8000.0,
                                 "unit": "GB/s", "frac": 32.0 * targets / tb / 1e9 / 8000.0},
               note="loop = per-circuit fock_diag_fwd calls replaying one captured graph each (loop_eager: "
                    "the same calls launched kernel by kernel); algorithmic bytes 32 B per computed amplitude "
                    "over the whole batched call (its launches of the largest circuits included)")
    for p in runner.plans:
        F.fd_plan_use_graphs(p, False)
    del runner
    torch.cuda.empty_cache()
    # complex64 per circuit against complex128, same calls one after another
    worst, worst_el, errs = 0.0, 0.0, []
    for ci in circs:
        r = {}
        for dt in (torch.complex128, torch.complex64):
            p = F.Plan(ci.cutoffs, ci.detected_mask, dt, "zero")
            ws = torch.empty(max(p.workspace(False)[0], 256), dtype=torch.uint8, device="cuda")
            rho = torch.empty(p.out_shape, dtype=dt, device="cuda")
            F.fock_diag_fwd(p, torch.tensor(ci.A, dtype=dt, device="cuda"), torch.tensor(ci.b, dtype=dt, device="cuda"),
                            torch.tensor([ci.c], dtype=dt, device="cuda"), rho, ws)
            r[dt] = rho
            del ws
            p.close()
        e = errors_vs(r[torch.complex64], r[torch.complex128])
        errs.append(e["normwise"])
        worst = max(worst, e["normwise"])
        worst_el = max(worst_el, e["elementwise_max_on_large"])
        del r
    torch.cuda.empty_cache()
    errs.sort()
    out["c64"] = {"worst_circuit_rel_err_vs_c128": worst, "median_circuit_rel_err_vs_c128": errs[len(errs) // 2],
                  "worst_circuit_elementwise_max_on_large": worst_el}
    return out


def gradient_leg(n=64):
    """The batched gradient workload: n circuits with M = 6, mode 0 undetected
    (cutoff 30), five detected modes (cutoff 8), b = 0, complex128; per circuit
    one forward keeping every intermediate and one reverse sweep with a seeded
    dense cotangent, circuits one after another (each sweep fills the device;
    a circuit's intermediates take 9.9 GB, so the saved buffer and the
    workspace are reused)."""
    import torch
    from paper_2303_08879_amd import fockdiag as F
    from paper_2303_08879_amd import workloads as W
    circs = W.config5b(n=n)
    dt, dev = torch.complex128, "cuda"
    plan = F.Plan(circs[0].cutoffs, circs[0].detected_mask, dt, "zero")
    wb, sb = plan.workspace(True)
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    saved = torch.empty(sb, dtype=torch.uint8, device=dev)
    rho = torch.empty(plan.out_shape, dtype=dt, device=dev)
    g = torch.tensor(W.random_cotangent(plan.out_shape, seed=11), dtype=dt, device=dev)
    ins = [(torch.tensor(c.A, dtype=dt, device=dev), torch.tensor(c.b, dtype=dt, device=dev),
            torch.tensor([c.c], dtype=dt, device=dev)) for c in circs]
    grads = [(torch.empty_like(A), torch.empty_like(b), torch.empty_like(c)) for A, b, c in ins]

    def step():
        for (A, b, c), (dA, db, dc) in zip(ins, grads):
            F.fock_diag_fwd(plan, A, b, c, rho, ws, saved)
            F.fock_diag_vjp(plan, A, b, c, saved, g, dA, db, dc, ws)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    F.fd_device_status(plan)
    targets = plan.query(F.FD_Q_TARGETS)
    res = dict(workload="config5b: 64 circuits, M=6, mode 0 undetected C_U=30, 5 detected C_D=8, b=0, complex128; "
                        "forward (intermediates kept) + VJP per circuit",
               circuits=n, seconds=sec, circuits_per_s=n / sec, computed_amplitudes_per_circuit=targets,
               output_amplitudes_per_s=n * plan.query(F.FD_Q_OUT_ELEMS) / sec,
               saved_bytes_per_circuit=sb, workspace_bytes=wb)
    # the same step with checkpointed reverse sweeps (every ceil(sqrt(L)) levels)
    levels = plan.query(F.FD_Q_LEVELS)
    every = math.ceil(math.sqrt(levels))
    ref = [(dA.clone(), db.clone(), dc.clone()) for dA, db, dc in grads]
    del ws, saved
    torch.cuda.empty_cache()
    F.fd_plan_set_checkpoint(plan, every)
    wb, sb = plan.workspace(True)
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    saved = torch.empty(sb, dtype=torch.uint8, device=dev)
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    sec_c = time.perf_counter() - t0
    F.fd_device_status(plan)
    same = all(torch.equal(a, r) for x, y in zip(grads, ref) for a, r in zip(x, y))
    res["checkpointed"] = dict(every_levels=every, levels=levels, saved_bytes_per_circuit=sb, workspace_bytes=wb,
                               seconds=sec_c, circuits_per_s=n / sec_c, gradients_bitwise_equal=bool(same))
    plan.close()
    del ws, saved, rho, g, ins, grads, ref
    torch.cuda.empty_cache()
    return res


def level_counts(cutoffs):
    """Points n of the box 0 <= n_j < C_j with |n| = S, for every S."""
    import numpy as np
    cnt = np.ones(1, dtype=np.int64)
    for C in cutoffs:
        cnt = np.convolve(cnt, np.ones(int(C), dtype=np.int64))
    return cnt


def state_leg(steps=20):
    """The pure-state workload (8 squeezed modes through a Haar interferometer,
    no loss, b = 0, cutoff 8: the 8^8 amplitudes of psi), complex128.  Under
    b = 0 one launch per even level S computes level S from level S - 2 and
    clears level S - 1; algorithmic bytes of that launch: 16 per amplitude
    written (levels S and S - 1) plus 16 per amplitude of level S - 2 read
    once.  The output permutation to C order is timed apart."""
    import numpy as np
    import torch
    from paper_2303_08879_amd import fockdiag as F
    from paper_2303_08879_amd import workloads as W
    ci = W.state8()
    dt, dev = torch.complex128, "cuda"
    plan = F.StatePlan(ci.cutoffs, dt, "zero")
    A = torch.tensor(ci.A, dtype=dt, device=dev)
    b = torch.tensor(ci.b, dtype=dt, device=dev)
    c = torch.tensor([ci.c], dtype=dt, device=dev)
    ws = torch.empty(plan.workspace(), dtype=torch.uint8, device=dev)
    psi = torch.empty(plan.out_shape, dtype=dt, device=dev)

    def call():
        F.fock_state_fwd(plan, A, b, c, psi, ws)

    for _ in range(3):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    F.fd_state_plan_timing(plan, (1 << F.FD_K_FWD_LEVEL) | (1 << F.FD_K_OUT_PERM))
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    nl, ms_l = F.fd_state_plan_kernel_times(plan, F.FD_K_FWD_LEVEL)
    _, ms_p = F.fd_state_plan_kernel_times(plan, F.FD_K_OUT_PERM)
    F.fd_state_plan_timing(plan, 0)
    F.fd_state_device_status(plan)
    # reverse mode with a seeded cotangent: dA, db, dc (45 dot products over the box)
    g = torch.tensor(W.random_cotangent(plan.out_shape, seed=5), dtype=dt, device=dev)
    vws = torch.empty(plan.vjp_workspace(), dtype=torch.uint8, device=dev)
    dA = torch.empty((8, 8), dtype=dt, device=dev)
    db = torch.empty(8, dtype=dt, device=dev)
    dc = torch.empty(1, dtype=dt, device=dev)
    F.fock_state_vjp(plan, c, psi, g, dA, db, dc, vws)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        F.fock_state_vjp(plan, c, psi, g, dA, db, dc, vws)
    torch.cuda.synchronize()
    sec_v = time.perf_counter() - t2
    # forward mode along a seeded direction of the triple: one pass over the box
    rng = np.random.default_rng(6)
    tA = torch.tensor(rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)), dtype=dt, device=dev)
    tb = torch.tensor(rng.standard_normal(8) + 1j * rng.standard_normal(8), dtype=dt, device=dev)
    tc = torch.tensor([0.3 - 0.1j], dtype=dt, device=dev)
    dpsi = torch.empty_like(psi)
    F.fock_state_jvp(plan, c, psi, tA, tb, tc, dpsi)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(steps):
        F.fock_state_jvp(plan, c, psi, tA, tb, tc, dpsi)
    torch.cuda.synchronize()
    sec_j = time.perf_counter() - t3
    # the derivative kernels alone, HIP events around each launch
    F.fd_state_plan_timing(plan, (1 << F.FD_K_FWD_LEVEL) | (1 << F.FD_K_VJP_LEVEL))
    for _ in range(steps):
        F.fock_state_vjp(plan, c, psi, g, dA, db, dc, vws)
        F.fock_state_jvp(plan, c, psi, tA, tb, tc, dpsi)
    torch.cuda.synchronize()
    nv, ms_v = F.fd_state_plan_kernel_times(plan, F.FD_K_VJP_LEVEL)
    nj, ms_j = F.fd_state_plan_kernel_times(plan, F.FD_K_FWD_LEVEL)
    F.fd_state_plan_timing(plan, 0)

    def deriv_roofline(kernel, n, ms, amps):
        # 32 B per amplitude: two complex128 streams (psi and the cotangent
        # read, or psi read and the tangent written), each entry once
        us = 1e3 * ms / max(n, 1)
        gbs = 32.0 * amps / (us * 1e-6) / 1e9
        return {"bound": "hbm", "kernel": kernel, "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 5), "avg_launch_us": round(us, 3),
                "algorithmic_bytes_per_launch": 32 * amps, "traffic": measured_traffic("state8", kernel)}
    N = level_counts(ci.cutoffs)
    smax = len(N) - 1
    alg = sum(16 * (N[S] + N[S - 1] + N[S - 2]) for S in range(2, smax + 1, 2))
    if smax % 2:
        alg += 16 * N[smax]   # the last odd level, cleared alone
    launches = nl // steps
    amps = int(N.sum())
    gbs = alg * steps / (ms_l * 1e-3) / 1e9
    plan.close()
    return dict(workload="state8: pure state, M=8 squeezed modes r~U(0.3,0.7), Haar interferometer, no loss, b=0, "
                         "cutoff 8 (8^8 amplitudes of psi), complex128",
                amplitudes=amps, calls=steps, ms_per_call=1e3 * sec / steps,
                value=amps * steps / sec, unit="state-vector amplitudes/s",
                level_ms_per_call=ms_l / steps, out_perm_ms_per_call=ms_p / steps,
                roofline={"bound": "hbm", "kernel": "k_state_level (even levels)", "achieved": round(gbs, 2),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
                          "launches": launches, "avg_launch_us": round(1e3 * ms_l / nl, 3),
                          "algorithmic_bytes_per_launch": int(alg // max(launches, 1)),
                          "traffic": measured_traffic("state8", "k_state_level")},
                norm2=float((psi.abs() ** 2).sum()),
                vjp={"ms_per_call": 1e3 * sec_v / steps,
                     "note": "the 45 cotangent dot products (8 of b, 36 of the symmetric A, 1 of c) over the box, "
                             "one tiled pass plus the final slot sums",
                     "algorithmic_GBs": round(32 * amps * steps / sec_v / 1e9, 1),
                     "algorithmic_bytes": "32 B per amplitude: the cotangent and psi read once",
                     "roofline": deriv_roofline("k_state_vjp", nv, ms_v, amps)},
                jvp={"ms_per_call": 1e3 * sec_j / steps, "launches": 1,
                     "note": "one tiled pass: reads psi (and its shifted neighbours), writes the tangent: "
                             "32 B per amplitude",
                     "algorithmic_GBs": round(32 * amps * steps / sec_j / 1e9, 1),
                     "roofline": deriv_roofline("k_state_jvp", nj, ms_j, amps)})


def total_leg(steps=20, N=16, eps=0.05):
    """Total photon cutoff: the 8-mode lossy state of the headline workload
    (r~U(0.5,1.0), eta~U(0.8,0.95), b = 0) with per-mode cutoff 40 and
    |n| <= N, p(n) of the C(N+8, 8) points in level order (complex128); then
    the same sweep with probability-sum stopping at 1 - eps (the stream is
    synchronised once per 4 levels)."""
    import torch
    from paper_2303_08879_amd import fockdiag as F
    from paper_2303_08879_amd import workloads as W
    ci = W.config5()
    dt, dev = torch.complex128, "cuda"
    plan = F.Plan([40] * 8, 0, dt, "zero", total_cutoff=N)
    A = torch.tensor(ci.A, dtype=dt, device=dev)
    b = torch.tensor(ci.b, dtype=dt, device=dev)
    c = torch.tensor([ci.c], dtype=dt, device=dev)
    ws = torch.empty(plan.workspace(False)[0], dtype=torch.uint8, device=dev)
    out = torch.empty(plan.out_shape, dtype=dt, device=dev)
    for _ in range(3):
        F.detection_probs(plan, A, b, c, out, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        F.detection_probs(plan, A, b, c, out, ws)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    full_mass = float(out.real.sum())
    levels, mass = F.detection_probs_until(plan, A, b, c, out, eps, ws)
    t1 = time.perf_counter()
    for _ in range(steps):
        levels, mass = F.detection_probs_until(plan, A, b, c, out, eps, ws)
    sec_stop = time.perf_counter() - t1
    F.fd_device_status(plan)
    pts = plan.query(F.FD_Q_OUT_ELEMS)
    plan.close()
    return dict(workload=f"config5 state (8 modes, b=0), per-mode cutoff 40, total photon cutoff {N}: "
                         f"p(n) for the {pts} points with |n| <= {N}, complex128",
                points=pts, ms_per_call=1e3 * sec / steps, value=pts * steps / sec, unit="probabilities/s",
                mass_below_cutoff=full_mass,
                stopping={"eps": eps, "levels_done": levels, "mass": mass, "ms_per_call": 1e3 * sec_stop / steps})


def jvp_leg(steps=10):
    """Forward mode of rho on the headline workload (8 modes, all detected,
    cutoff 8: 16.8M outputs; b = 0 at the base point, so the general schedule
    that a non-zero db needs): rho and its tangent along a seeded direction in
    one sweep, against the forward alone on the same schedule."""
    import numpy as np
    import torch
    from paper_2303_08879_amd import fockdiag as F
    from paper_2303_08879_amd import workloads as W
    ci = W.config5()
    dt, dev = torch.complex128, "cuda"
    plan = F.Plan(ci.cutoffs, ci.detected_mask, dt, "general")
    T = lambda x: torch.tensor(np.asarray(x), dtype=dt, device=dev)
    A, b, c = T(ci.A), T(ci.b), T([ci.c])
    rng = np.random.default_rng(3)
    D = 2 * ci.M
    dA = T(rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)))
    db = T(rng.standard_normal(D) + 1j * rng.standard_normal(D))
    dc = T([0.3 + 0.1j])
    wj = torch.empty(plan.jvp_workspace(), dtype=torch.uint8, device=dev)
    wf = torch.empty(plan.workspace(False)[0], dtype=torch.uint8, device=dev)
    rho = torch.empty(plan.out_shape, dtype=dt, device=dev)
    drho = torch.empty_like(rho)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        F.fd_plan_timing(plan, 1 << F.FD_K_FWD_LEVEL)
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        n, ms = F.fd_plan_kernel_times(plan, F.FD_K_FWD_LEVEL)
        F.fd_plan_timing(plan, 0)
        return 1e3 * sec / steps, ms / steps, n // steps

    ms_j, lvl_j, launches = timed(lambda: F.fock_diag_jvp(plan, A, b, c, dA, db, dc, rho, drho, wj))
    ms_f, lvl_f, _ = timed(lambda: F.fock_diag_fwd(plan, A, b, c, rho, wf))
    F.fd_device_status(plan)
    n = plan.query(F.FD_Q_OUT_ELEMS)
    # algorithmic bytes per computed amplitude: value and tangent each written
    # once and read once by their reader (64 B; the forward alone 32 B)
    t = plan.query(F.FD_Q_TARGETS)
    gbs = lambda nbytes, ms: nbytes / (ms * 1e-3) / 1e9
    plan.close()
    return dict(workload="config5: M=8 all detected C=8 (16.8M outputs), b=0 at the base point, general schedule, "
                         "one seeded direction (dA, db, dc), complex128",
                outputs=n, ms_per_call=ms_j, value=n * 1e3 / ms_j, unit="outputs (rho and drho)/s",
                level_ms_per_call=lvl_j, level_launches=launches, forward_only_ms_per_call=ms_f,
                forward_only_level_ms_per_call=lvl_f, cost_vs_forward=ms_j / ms_f,
                level_GBs_algorithmic=gbs(64.0 * t, lvl_j), forward_level_GBs_algorithmic=gbs(32.0 * t, lvl_f))


def progress(what, t0):
    print(f"[bench] {what} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the other single-circuit workloads")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-circuits leg")
    ap.add_argument("--no-gradient", action="store_true", help="skip the 64-circuit gradient batch")
    ap.add_argument("--no-state", action="store_true", help="skip the pure-state (state vector) leg")
    ap.add_argument("--no-total", action="store_true", help="skip the total-photon-cutoff leg")
    ap.add_argument("--no-jvp", action="store_true", help="skip the forward-mode (JVP) leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 1 GiB device-to-device copies (the reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library runs each circuit on a single device; sharding "
              f"across GPUs is a design, not an implementation (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        # a plain copy kernel of known size: each copy reads and writes 1 GiB
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "copies": 5}), flush=True)
        return

    # headline: forward + VJP of the named workload, complex128, graph replay
    t_start = time.perf_counter()
    head, s128, circ = single_leg(args.workload, args.steps, args.warmup, events=True, keep=True)
    progress(f"headline {args.workload}", t_start)
    n_f, ms_f, n_v, ms_v = head.pop("_ev")
    targets = head["computed_amplitudes"]
    kind = "block" if s128.plan.query(s128.F.FD_Q_BLOCK) > 1 else "point"
    if ms_v >= ms_f:
        dom = dict(kernel=f"k_vjp_{kind} (reverse level sweep)", short=f"k_vjp_{kind}", ms=ms_v, launches=n_v,
                   bytes_per_unit=48)
    else:
        dom = dict(kernel=f"k_fwd_{kind} (forward level sweep)", short=f"k_fwd_{kind}", ms=ms_f, launches=n_f,
                   bytes_per_unit=32)
    # algorithmic bytes of one launch: bytes per computed amplitude x computed
    # amplitudes per level launch (the step's amplitudes over its launches)
    per_step = max(dom["launches"] // args.steps, 1)
    alg_per_launch = dom["bytes_per_unit"] * targets / per_step
    avg_s = dom["ms"] * 1e-3 / max(dom["launches"], 1)
    achieved = alg_per_launch / avg_s / 1e9
    traffic = measured_traffic(args.workload, dom["short"])
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": None if traffic is None else round(traffic), "kernel": dom["kernel"],
            "avg_launch_us": round(avg_s * 1e6, 3), "launches": dom["launches"],
            "algorithmic_bytes_per_amplitude": dom["bytes_per_unit"],
            "algorithmic_bytes_per_launch": round(alg_per_launch),
            "traffic_over_algorithmic": None if traffic is None else round(traffic / alg_per_launch, 3)}
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "Fock amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": head["workload"] + ", complex128",
                   "out_amplitudes": head["out_amplitudes"], "computed_amplitudes": targets},
        "roofline": roof,
        "detail": {k: head[k] for k in ("computed_amplitudes_per_s", "fwd_level_ms_per_step",
                                        "vjp_level_ms_per_step", "fwd_level_GBs", "vjp_level_GBs",
                                        "fwd_level_GFLOPs", "read_terms")},
        "c64": head["c64"],
    }
    line["detail"]["fp64_peak_TFLOPs"] = FP64_PEAK_TFLOPS
    if not args.no_cpu_baseline:
        import numpy as np
        s64 = CircuitStep(circ, torch.complex64)
        s64.step()
        torch.cuda.synchronize()
        # the oracle's cost grows with the box (prod of the sample's cutoffs, squared):
        # time the smallest sample, then report the largest one predicted to take
        # at most ~25 s on this host
        if circ.M == 8:
            corners = [[3] * k + [2] * (8 - k) for k in (5, 6, 7)]
        else:
            corners = [[c] * circ.M for c in (3, 4, 5)]
        size = lambda cn: math.prod(c * c for c in cn)
        first = cpu_baseline(circ, s128, s64, corners[0])
        per = first["seconds"] / size(corners[0])
        pick = max((cn for cn in corners if per * size(cn) <= 25.0), key=size, default=corners[0])
        line["cpu_baseline"] = first if pick is corners[0] else cpu_baseline(circ, s128, s64, pick)
        line["cpu_selective_oracle"] = cpu_selective(circ, s128, s64)
        s64.release()
        progress("cpu_baseline", t_start)
        del np
    s128.release()
    torch.cuda.empty_cache()
    if not args.no_legs:
        line["legs"] = {}
        for name in ("config1", "config2", "config4", "config5"):
            if name == args.workload:
                continue
            steps = 200 if name == "config1" else 20
            leg = single_leg(name, steps, 3, events=True)
            leg.pop("_ev", None)
            line["legs"][name] = leg
            progress(name, t_start)
    if not args.no_gradient:
        line["gradient_batch"] = gradient_leg()
        progress("gradient_batch", t_start)
    if not args.no_batched:
        line["batched"] = batched_leg()
        progress("batched", t_start)
    if not args.no_state:
        line["state_vector"] = state_leg()
        progress("state_vector", t_start)
    if not args.no_total:
        line["total_cutoff"] = total_leg()
        progress("total_cutoff", t_start)
    if not args.no_jvp:
        line["density_jvp"] = jvp_leg()
        progress("density_jvp", t_start)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
