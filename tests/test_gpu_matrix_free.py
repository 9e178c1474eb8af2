"""The matrix-free stiffness operator (sum-factorised quadrature per brick
of elements, deterministic per-node gather) against the oracle and against
the assembled stencil, for p = 1..6 on perturbed multi-patch cubes with
partial bricks (element counts that are not multiples of the brick's 2
elements per direction for p <= 4), one brick or several per direction."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("p,n_el", [(1, 3), (2, 3), (2, 6), (3, 3), (3, 4), (3, 6), (4, 2), (4, 5), (5, 2), (6, 1)])
def test_matrix_free_matches_oracle_and_assembled(p, n_el):
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = W.make_c3(seed=p, p=p, n_el=n_el, grid=(2, 1, 2))
    o = AFIETI(prob)
    smf = Solver(prob, stiffness="matrix_free", tol=1e-12)
    sas = Solver(prob, stiffness="assembled", tol=1e-12)
    x = torch.from_numpy(W.random_vector(o.n_dof, 40 + p)).cuda()
    ymf = smf.apply("stiffness", x).cpu().numpy()
    yas = sas.apply("stiffness", x).cpu().numpy()
    ref = o.apply_A(x.cpu().numpy())
    e1 = np.abs(ymf - ref).max() / np.abs(ref).max()
    e2 = np.abs(ymf - yas).max() / np.abs(yas).max()
    print(f"  p={p} n_el={n_el}: matrix-free vs oracle {e1:.2e}, vs assembled {e2:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12
    u1, _, st1 = smf.solve(want_lambda=False)
    u2, _, st2 = sas.solve(want_lambda=False)
    assert abs(st1["iterations"] - st2["iterations"]) <= max(1, st2["iterations"] // 50)
    d = float(torch.linalg.norm(u1 - u2) / torch.linalg.norm(u2))
    print(f"  solves at tol 1e-12: {st1['iterations']} / {st2['iterations']} it, rel diff {d:.2e}")
    assert d <= 1e-9


def test_matrix_free_saddle_with_fused_bt():
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = W.make_c2(n_el=5, p=3, seed=4)
    o = AFIETI(prob)
    s = Solver(prob, stiffness="matrix_free")
    r = W.random_vector(o.n_dof + o.n_c, 50)
    y = s.apply("saddle", torch.from_numpy(r).cuda()).cpu().numpy()
    ref = o.apply_op(r)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
