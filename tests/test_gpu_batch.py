"""Ragged batches: independent problems of different dimension, patch
counts, sizes and degrees in one handle.  Each problem's solution and
iteration count match the oracle; a problem solved inside a batch is
bitwise identical to the same problem solved alone (identical chunking,
and converged problems are masked out of the kernels); replaying the
captured iteration graph is bitwise identical to launching the kernels one
by one."""
import numpy as np
import pytest

import workloads as W
from oracle.afieti import AFIETI
from minres_band import same_iterations

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _batch():
    return [W.make_c2(n_el=3, p=2, seed=1),
            W.make_c1(n_el=4, p=3, seed=2),
            W.make_c3(n_el=2, p=3, grid=(2, 2, 1), seed=3),
            W.make_c4(seed=5, n_problems=1, el_range=(4, 7))[0],
            W.make_c3(n_el=3, p=2, grid=(1, 3, 2), seed=6)]


def test_batch_matches_oracle_per_problem():
    torch = _torch()
    from paper_2001_09626_amd import Solver
    probs = _batch()
    for tol in (1e-8, 1e-12):
        s = Solver(probs, tol=tol)
        u, lam, st = s.solve()
        u, lam = _host(u), _host(lam)
        its, rel, sta = s.problem_stats()
        for j, pr in enumerate(probs):
            o = AFIETI(pr)
            ref = o.solve(tol=tol)
            a, b = s.dof_offsets[sum(len(p["patches"]) for p in probs[:j])], None
            uj = u[a:a + o.n_dof]
            lj = lam[s.c_offsets[j]:s.c_offsets[j + 1]]
            e = np.linalg.norm(uj - ref["u"]) / np.linalg.norm(ref["u"])
            el = np.linalg.norm(lj - ref["lam"]) / np.linalg.norm(ref["lam"])
            print(f"  tol {tol:.0e} problem {j}: {its[j]} it (oracle {ref['iters']}), u {e:.2e}, lam {el:.2e}")
            assert sta[j] == 1
            alt = AFIETI(pr, eig_driver="gv").solve(tol=tol)
            assert same_iterations(int(its[j]), ref, tol, alt=alt)
            if tol == 1e-12:
                assert e <= 1e-10 and el <= 1e-9
            else:
                assert e <= 1e-8
        s.close()


def test_batch_bitwise_equals_single_and_graph_equals_eager():
    torch = _torch()
    from paper_2001_09626_amd import Solver
    probs = _batch()
    sb = Solver(probs, tol=1e-8)
    ub, _, _ = sb.solve(want_lambda=False)
    its_b = sb.problem_stats()[0]
    se = Solver(probs, tol=1e-8, use_graph=False)
    ue, _, _ = se.solve(want_lambda=False)
    assert torch.equal(ub, ue), "graph replay differs from eager launches"
    assert np.array_equal(its_b, se.problem_stats()[0])
    off = 0
    for j, pr in enumerate(probs):
        s1 = Solver(pr, tol=1e-8)
        u1, _, st = s1.solve(want_lambda=False)
        n = s1.n_dof
        assert torch.equal(ub[off:off + n], u1), f"problem {j} differs between batch and single"
        assert st["iterations"] == its_b[j]
        off += n
        s1.close()


def test_c4_ragged_batch_full():
    """The full ragged batch: 32 problems, 1..27 patches, 8..40 elements
    per direction, p in {2,3,4}; FP32 FD; every problem converges, its
    solution satisfies B u = O(tol), and three problems are bitwise equal
    to their single-problem solves."""
    torch = _torch()
    from paper_2001_09626_amd import Solver
    probs = W.make_c4(seed=0)
    print("\n[c4: setup]", flush=True)
    s = Solver(probs, tol=1e-8, fd_precision="fp32")
    u, lam, st = s.solve()
    its, rel, sta = s.problem_stats()
    print(f"  32 problems, {s.n_dof} DOF, {s.n_c} multipliers: {st['ms']:.0f} ms, iterations "
          f"min {its.min()} max {its.max()}", flush=True)
    assert np.all(sta == 1) and np.all(rel <= 1e-8)
    pstart = np.cumsum([0] + [len(p["patches"]) for p in probs])
    for j in (0, 13, 22):
        s1 = Solver(probs[j], tol=1e-8, fd_precision="fp32")
        u1, _, st1 = s1.solve(want_lambda=False)
        a = s.dof_offsets[pstart[j]]
        assert torch.equal(u[a:a + s1.n_dof], u1), j
        assert st1["iterations"] == its[j]
        s1.close()
