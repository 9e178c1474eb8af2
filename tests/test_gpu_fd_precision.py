"""FD precision variants against the FP64 oracle: FP32 and BF16 mode
products on the matrix cores (FP32 accumulation) and FP32 on the vector
ALU.  Bounds from the unit round-off u of the operand type and the
O(n) terms of each of the six contractions: FP32 (u = 6e-8) to 2e-5 of
the largest entry, BF16 (u = 3.9e-3) to 0.1.  Solves with each variant
converge and land as close to the converged solution as the FP64-FD
iterate does (within a factor 3); BF16 is reported, with a looser bound."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI

pytestmark = pytest.mark.gpu

CASES = {"c2_small": lambda: W.make_c2(n_el=5, p=3, seed=2),
         "c3_ragged": lambda: W.make_c3(n_el=3, p=2, grid=(2, 3, 2), seed=4),
         "c1_2d": lambda: W.make_c1(n_el=6, p=2, seed=1)}
BOUND = {"fp32": 2e-5, "fp32_valu": 2e-5, "bf16": 0.1, "fp64": 1e-12, "fp64_valu": 1e-12}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp64_valu", "fp32", "fp32_valu", "bf16"])
def test_fd_precision(case, prec):
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = CASES[case]()
    o = AFIETI(prob)
    s = Solver(prob, fd_precision=prec, tol=1e-8)
    r = W.random_vector(o.n_dof, 60)
    z = s.apply_fd(torch.from_numpy(r).cuda()).cpu().numpy()
    ref = o.apply_PA_inv(r)
    e = np.abs(z - ref).max() / np.abs(ref).max()
    # the interior solve of S-hat uses the same kernels
    x = W.random_vector(o.n_dof, 61)
    zi = s.apply("fd_interior", torch.from_numpy(x).cuda()).cpu().numpy()
    refi = []
    for k, xk in enumerate(o.split(x)):
        inner = tuple(slice(1, -1) for _ in range(o.dim))
        blk = np.zeros_like(xk)
        for l in range(o.dim):
            blk[l][inner] = o.fd_solve_interior(k, l, xk[l][inner])
        refi.append(blk)
    refi = o.join(refi)
    ei = np.abs(zi - refi).max() / np.abs(refi).max()
    u, _, st = s.solve(want_lambda=False, allow_not_converged=True)
    tight = o.solve(tol=1e-13)
    ref8 = o.solve(tol=1e-8)
    nu = np.linalg.norm(tight["u"])
    eu = np.linalg.norm(u.cpu().numpy() - tight["u"]) / nu
    e64 = np.linalg.norm(ref8["u"] - tight["u"]) / nu
    print(f"  {case} {prec}: FD {e:.2e}, interior FD {ei:.2e}; solve {st['iterations']} it "
          f"(FP64 {ref8['iters']}), error vs converged {eu:.2e} (FP64-FD iterate {e64:.2e})")
    assert e <= BOUND[prec] and ei <= BOUND[prec]
    assert st["converged"]
    if prec != "bf16":
        assert eu <= 3 * e64 + 1e-12
    else:
        assert eu <= 1e-5
