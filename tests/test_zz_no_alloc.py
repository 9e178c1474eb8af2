"""The allocation-free FD entry point (afieti_apply_fd_noalloc), called
through the C ABI: its output equals afieti_apply_fd's bit for bit (same
kernels, the intermediate tensor in the fixed device array instead of
handle memory) on two calls in a row, the second on a smaller problem; a
problem whose intermediate does not fit the array is refused."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _call(L, fn, h, r, z, torch):
    code = getattr(L, fn)(h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()),
                          C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_fd_equals_apply_fd(prec):
    torch = _torch()
    from paper_2001_09626_amd import Solver, _native as N
    L = N.lib()
    # larger problem first, then a smaller one on the same GPU
    probs = [W.make_c2(n_el=12, p=3, seed=2), W.make_c3(n_el=3, p=2, grid=(2, 3, 2), seed=4)]
    for j, prob in enumerate(probs):
        print(f"\n[noalloc {prec} call {j}: {len(prob['patches'])} patches]", flush=True)
        s = Solver(prob, fd_precision=prec)
        r = torch.from_numpy(W.random_vector(s.n_dof, 40 + j)).cuda()
        z_ref = torch.full_like(r, float("nan"))
        z = torch.full_like(r, float("nan"))
        assert _call(L, "afieti_apply_fd", s._h, r, z_ref, torch) == N.OK
        assert _call(L, "afieti_apply_fd_noalloc", s._h, r, z, torch) == N.OK
        torch.cuda.synchronize()
        assert torch.isfinite(z).all()
        assert torch.equal(z, z_ref), float((z - z_ref).abs().max())
        s.close()


def test_noalloc_fd_refuses_oversized_intermediate():
    torch = _torch()
    from paper_2001_09626_amd import Solver, _native as N
    L = N.lib()
    # 8 patches x 3 components x 43^3 FP64 intermediate entries = 15.3 MB > 8 MiB
    s = Solver(W.make_c2(n_el=40, p=3, seed=0), fd_precision="fp64")
    r = torch.zeros(s.n_dof, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    assert _call(L, "afieti_apply_fd_noalloc", s._h, r, z, torch) == -7
    assert b"exceeds" in L.afieti_last_error(s._h)
    s.close()
