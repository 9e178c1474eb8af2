"""Exit paths of the GPU solve, forced from the host through options the
C ABI exposes (no kernel is made to fail):
  * maxit below the iterations needed: AFIETI_NOT_CONVERGED, per-problem
    status 3, and the returned iterate is the oracle's MINRES iterate after
    the same number of steps, recovered the same way;
  * a negative weight of the preconditioner's multiplier block makes the
    preconditioner indefinite: AFIETI_EBREAKDOWN, per-problem status 2;
  * a weight of 1 (the default) gives bitwise the default solve.
Both graph replay (six iterations per launch, maxit not a multiple of six)
and one-by-one launches, one problem and a batch."""
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


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("maxit", [5, 14])
def test_maxit_not_converged(use_graph, maxit):
    _torch()
    from paper_2001_09626_amd import Solver, AfietiError, _native as N
    prob = W.make_c2(n_el=3, p=2, seed=1)
    print(f"\n[maxit {maxit} graph {use_graph}]", flush=True)
    s = Solver(prob, tol=1e-12, maxit=maxit, use_graph=use_graph)
    with pytest.raises(AfietiError) as ei:
        s.solve()
    assert ei.value.code == N.NOT_CONVERGED
    u, lam, st = s.solve(allow_not_converged=True)
    assert st["code"] == N.NOT_CONVERGED and not st["converged"]
    assert st["iterations"] == maxit
    its, rel, status = s.problem_stats()
    assert list(its) == [maxit] and list(status) == [3] and rel[0] > 1e-12
    ref = AFIETI(prob).solve(tol=1e-12, maxit=maxit)
    assert ref["iters"] == maxit
    u = _host(u)
    err = np.abs(u - ref["u"]).max() / np.abs(ref["u"]).max()
    print(f"  iterate after {maxit} steps: rel diff {err:.2e}", flush=True)
    assert err <= 1e-12
    s.close()


def test_maxit_batch_stops_each_problem():
    """A batch where some problems converge within maxit and others do not:
    converged ones report status 1, the rest 3, and the call returns
    NOT_CONVERGED with the converged solutions intact."""
    _torch()
    from paper_2001_09626_amd import Solver, _native as N
    probs = [W.make_c1(n_el=3, p=2, seed=0), W.make_c2(n_el=4, p=3, seed=2)]
    full = Solver(probs, tol=1e-8)
    uf, _, _ = full.solve()
    its_full, _, _ = full.problem_stats()
    lim = int((its_full[0] + its_full[1]) // 2)
    assert its_full[0] < lim < its_full[1]
    s = Solver(probs, tol=1e-8, maxit=lim)
    u, _, st = s.solve(allow_not_converged=True)
    its, rel, status = s.problem_stats()
    print(f"\n  full its {list(its_full)}, maxit {lim}: its {list(its)} status {list(status)}", flush=True)
    assert st["code"] == N.NOT_CONVERGED
    assert list(status) == [1, 3] and its[0] == its_full[0] and its[1] == lim
    n0 = int(s.dof_offsets[len(probs[0]["patches"])])
    assert np.array_equal(_host(u)[:n0], _host(uf)[:n0])
    s.close()
    full.close()


@pytest.mark.parametrize("use_graph", [True, False])
def test_indefinite_preconditioner_breaks_down(use_graph):
    _torch()
    from paper_2001_09626_amd import Solver, AfietiError, _native as N
    probs = [W.make_c1(n_el=3, p=2, seed=0), W.make_c2(n_el=3, p=2, seed=1)]
    s = Solver(probs, tol=1e-8, ps_weight=-1e6, use_graph=use_graph)
    with pytest.raises(AfietiError) as ei:
        s.solve()
    assert ei.value.code == N.EBREAKDOWN
    its, rel, status = s.problem_stats()
    print(f"\n  breakdown: its {list(its)} status {list(status)}", flush=True)
    assert list(status) == [2, 2]
    s.close()


def test_unit_weight_is_the_default():
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = W.make_c2(n_el=3, p=2, seed=1)
    a, b = Solver(prob), Solver(prob, ps_weight=1.0)
    ua, _, sa = a.solve()
    ub, _, sb = b.solve()
    assert sa["iterations"] == sb["iterations"] and torch.equal(ua, ub)
    a.close()
    b.close()


def test_caller_allocator():
    """With the caller's allocator (torch's caching allocator through the
    dev_alloc / dev_free options) the handle's memory is torch's while the
    handle lives and goes back at close; results equal the default
    allocator's bitwise."""
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = W.make_c2(n_el=3, p=2, seed=1)
    ref = Solver(prob)
    u0, _, st0 = ref.solve()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    s = Solver(prob, allocator="torch")
    held = torch.cuda.memory_allocated() - base
    print(f"\n  handle memory {s.device_bytes} B, torch allocator holds {held} B more", flush=True)
    assert held >= s.device_bytes
    u1, _, st1 = s.solve()
    assert st1["iterations"] == st0["iterations"] and torch.equal(u0, u1)
    del u1
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base <= 0
    ref.close()
