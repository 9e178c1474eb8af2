"""No kernel reads device memory that the library has not written.  Device
memory is filled with NaN through torch and handed back to the driver before
the handles are created, so the library's own allocations are likely to
reuse it; every operator output and every solve must stay finite and
converge in the oracle's iteration count.  (An earlier version left the
coarse coefficients of the three modes a 2D patch does not have unset, and
P_chi turned them into NaN on reused memory.)"""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from minres_band import same_iterations

pytestmark = pytest.mark.gpu

OPS_DOF = ("fd_interior", "stiffness", "B", "P_u", "Shat", "Ahat", "mass", "load")
OPS_C = ("Bt", "P_chi", "P_S")
OPS_ALL = ("prec", "saddle")


def _poison(torch, gib=2):
    t = torch.full((gib * (1 << 27),), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    del t
    torch.cuda.empty_cache()


@pytest.mark.parametrize("case", ["c1_2d", "c2_small", "batch"])
def test_no_uninitialised_reads(case):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_09626_amd import Solver
    probs = {"c1_2d": [W.make_c1(n_el=6, p=2, seed=1)],
             "c2_small": [W.make_c2(n_el=5, p=3, seed=2)],
             "batch": [W.make_c1(n_el=4, p=3, seed=2), W.make_c3(n_el=2, p=3, grid=(2, 2, 1), seed=3)]}[case]
    _poison(torch)
    s = Solver(probs, tol=1e-8)
    nd, nc = s.n_dof, s.n_c

    def finite(t):
        return bool(torch.isfinite(t).all())

    xd = torch.from_numpy(W.random_vector(nd, 1)).cuda()
    xc = torch.from_numpy(W.random_vector(nc, 2)).cuda()
    xa = torch.from_numpy(W.random_vector(nd + nc, 3)).cuda()
    bad = [op for op in OPS_DOF if not finite(s.apply(op, xd))]
    bad += [op for op in OPS_C if not finite(s.apply(op, xc))]
    bad += [op for op in OPS_ALL if not finite(s.apply(op, xa))]
    bad += [] if finite(s.apply_fd(xd)) else ["fd"]
    assert not bad, f"non-finite output of {bad}"
    u, lam, st = s.solve()
    assert finite(u) and finite(lam)
    its = s.problem_stats()[0]
    for j, pr in enumerate(probs):
        ref = AFIETI(pr).solve(tol=1e-8)
        alt = AFIETI(pr, eig_driver="gv").solve(tol=1e-8)
        assert same_iterations(int(its[j]), ref, 1e-8, alt=alt), (j, its[j], ref["iters"])
    s.close()
