"""fdlb_step_static (the entry point for callers that cannot allocate device memory) against
fdlb_step: from the same state, on the same tile, both give bit-identical populations.

Two calls in a row share the static scratch: the second, on a smaller problem, must not see the
first call's moments, control block or tables.  Through the C ABI (ctypes), no Python wrapper.
"""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_0692_amd as F
    return F


def _bytes(t, ptr, n):
    """n bytes of the aligned region that starts at device address ptr inside tensor t, on the host."""
    off = ptr - t.data_ptr()
    return t[off:off + n].cpu().numpy()


def _state_copy(F, p):
    """A fresh aligned device buffer holding a copy of p's whole state buffer."""
    import torch
    t, ptr = F._alloc(p.state_bytes, p.device)
    src_off = p._state - p._state_t.data_ptr()
    dst_off = ptr - t.data_ptr()
    torch.cuda.synchronize()
    t[dst_off:dst_off + p.state_bytes].copy_(p._state_t[src_off:src_off + p.state_bytes])
    torch.cuda.synchronize()
    return t, ptr


def _check(F, case, prec, n, seed):
    import torch
    p = F.Problem(case, precision=prec)
    rho, ux, uy = W.random_fields(case.nx, case.ny, seed, amp=0.01)
    p.init_equilibrium(rho, ux, uy)
    t, ptr = _state_copy(F, p)
    stream = torch.cuda.Stream(device=p.device)
    code = F._lib.lib.fdlb_step_static(p._h, C.c_void_p(ptr), int(n), C.c_void_p(stream.cuda_stream))
    assert code == 0, F._lib.lib.fdlb_last_error()
    stream.synchronize()
    p.step(n)
    p.stream.synchronize()
    half = p.state_bytes // 2
    par = n % 2
    got = _bytes(t, ptr + par * half, half)
    ref = _bytes(p._state_t, p._state + par * half, half)
    assert np.array_equal(got, ref), (case.name, prec, n)
    # the bound problem's own state and step counter were not touched by the static call
    assert p.last_residual()[1] == n
    return p


def test_static_step_matches_bound_step_two_calls(F):
    big = W.cavity(96, ny=80, kn=0.1, order=3, name="cavity96x80_q36")
    small = W.cavity(24, ny=20, kn=0.3, order=2, name="cavity24x20_q16")
    _check(F, big, "fp64", 37, seed=11)
    _check(F, small, "fp32", 20, seed=12)
    _check(F, W.couette(50, kn=0.2, qy=("half", 3), qx=("full", 3)), "fp64", 9, seed=13)


def test_static_step_rejects_what_does_not_fit(F):
    import torch
    big = F.Problem(W.cavity(1024, kn=1.0, order=2), precision="fp32", bind=False)
    t, ptr = F._alloc(256, "cuda:0")
    s = torch.cuda.current_stream()
    assert F._lib.lib.fdlb_step_static(big._h, C.c_void_p(ptr), 1, C.c_void_p(s.cuda_stream)) == F._lib.EINVAL
    assert "static scratch" in F._lib.lib.fdlb_last_error().decode()
    mixed = F.Problem(W.cavity(24, kn=0.2, order=2), precision="mixed", bind=False)
    assert F._lib.lib.fdlb_step_static(mixed._h, C.c_void_p(ptr), 1, C.c_void_p(s.cuda_stream)) == F._lib.EINVAL
    small = F.Problem(W.cavity(24, kn=0.2, order=2), precision="fp64", bind=False)
    assert F._lib.lib.fdlb_step_static(small._h, C.c_void_p(ptr + 8), 1, C.c_void_p(s.cuda_stream)) == F._lib.EINVAL
    assert F._lib.lib.fdlb_step_static(small._h, C.c_void_p(ptr), -1, C.c_void_p(s.cuda_stream)) == F._lib.EINVAL
