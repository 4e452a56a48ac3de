"""fock_diag_fwd_static (the entry point that allocates nothing: library-owned
scratch in a static device array) against fock_diag_fwd on the same plans and
inputs, called through the C ABI.  Two calls in a row on the shared scratch,
the second with a smaller problem; complex128 and complex64; the host-side
rejections (oversized sweep, plan without device tables)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_2303_08879_amd import fockdiag as F
from paper_2303_08879_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10
SCRATCH = 64 << 20


def static_fn():
    L = F.lib()
    fn = L.fock_diag_fwd_static
    fn.argtypes = [ctypes.c_void_p] * 6
    fn.restype = ctypes.c_int
    return fn


def inputs(circ, dtype):
    T = lambda x: torch.tensor(np.asarray(x), dtype=dtype, device="cuda")
    return T(circ.A), T(circ.b), T([circ.c])


def run_both(circ, dtype, b_mode):
    print(f"[static fwd] cut={circ.cutoffs} mask={bin(circ.detected_mask)} dtype={dtype} b_mode={b_mode}", flush=True)
    plan = F.Plan(circ.cutoffs, circ.detected_mask, dtype, b_mode)
    A, b, c = inputs(circ, dtype)
    ws = torch.empty(plan.workspace(False)[0], dtype=torch.uint8, device="cuda")
    ref = torch.empty(plan.out_shape, dtype=dtype, device="cuda")
    F.fock_diag_fwd(plan, A, b, c, ref, ws)          # also puts the plan's tables on the device
    out = torch.full(plan.out_shape, float("nan"), dtype=dtype, device="cuda")
    st = static_fn()(plan.handle, A.data_ptr(), b.data_ptr(), c.data_ptr(), out.data_ptr(),
                     torch.cuda.current_stream().cuda_stream)
    assert st == F.FD_OK, F.fd_last_error()
    torch.cuda.synchronize()
    F.fd_device_status(plan)
    return plan, out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_static_matches_workspace_entry_two_calls(dtype):
    big = W.config2()                       # undetected mode, b != 0: block units and odd levels
    small = W.config2(c_u=6, c_d=4)
    assert F.Plan(big.cutoffs, big.detected_mask, dtype, "general").workspace(False)[0] <= SCRATCH
    tol = TOL if dtype == torch.complex128 else 1e-5
    for circ in (big, small):
        _, out, ref = run_both(circ, dtype, "general")
        # same kernels and schedule as the workspace entry point: identical bits
        assert np.array_equal(out, ref)
        assert O.rel_err(out, ref) <= tol
    # the small case against the oracle too (the scratch kept the big call's contents)
    orc = O.fock_diag(small.A, small.b, small.c, small.cutoffs, small.detected_mask)
    assert O.rel_err(out, orc) <= tol


def test_static_b_zero_plans():
    # an all-detected plan with b = 0: under FD_B_ZERO both entry points take the
    # b = 0 schedule; under FD_B_AUTO the static one takes the general schedule
    # (it never reads b on the host), which gives the same amplitudes
    circ = W.config1()
    _, out, ref = run_both(circ, torch.complex128, "zero")
    assert np.array_equal(out, ref)
    _, out, ref = run_both(circ, torch.complex128, "auto")
    assert O.rel_err(out, ref) <= TOL
    assert O.rel_err(out, O.fock_diag(circ.A, circ.b, circ.c, circ.cutoffs, circ.detected_mask)) <= TOL


def test_static_rejections_on_the_host():
    fn = static_fn()
    stream = torch.cuda.current_stream().cuda_stream
    circ = W.config2(c_u=6, c_d=4)
    A, b, c = inputs(circ, torch.complex128)
    out = torch.empty(circ.out_shape, dtype=torch.complex128, device="cuda")
    # a plan that has not run on this device: no tables, nothing launched
    fresh = F.Plan(circ.cutoffs, circ.detected_mask, torch.complex128, "general")
    assert fn(fresh.handle, A.data_ptr(), b.data_ptr(), c.data_ptr(), out.data_ptr(), stream) == F.FD_ERR_INVALID_ARG
    # a sweep larger than the static array (8 modes, cutoff 8: F0 alone is 268 MB)
    big = F.Plan([8] * 8, 0xFF, torch.complex128, "zero")
    assert big.workspace(False)[0] > SCRATCH
    A8 = torch.zeros((16, 16), dtype=torch.complex128, device="cuda")
    b8 = torch.zeros(16, dtype=torch.complex128, device="cuda")
    assert fn(big.handle, A8.data_ptr(), b8.data_ptr(), c.data_ptr(), out.data_ptr(), stream) == F.FD_ERR_WORKSPACE
    assert "static array" in F.fd_last_error()
    assert fn(None, A.data_ptr(), b.data_ptr(), c.data_ptr(), out.data_ptr(), stream) == F.FD_ERR_INVALID_ARG
