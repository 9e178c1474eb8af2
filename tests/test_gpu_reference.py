"""GPU solves of the full-size workloads against stored oracle solutions
(tests/golden/ref_*.json, written by tests/golden/make_reference.py, which
calls only the oracle): C2 (1,029,000 DOF), the problems of the C4 ragged
batch solved in one batched handle as a whole batch, and C3's 4x4x4 patch
grid at p = 2..5 on 4^3 elements per patch (the full 24^3 is beyond the
oracle's reach on a CPU).

Each reference stores the oracle's MINRES iteration count and |eta|/gamma_1
history, u and lambda at 4096 seeded indices, and three projections of u.
Rules (the parity rules of the small cases, at full size); u* is the tol
1e-12 oracle solution, distances are the largest sampled entry difference
over the largest sampled entry:
  * FP64 FD at tol 1e-8: the oracle's iteration count under the band rule
    and the GPU-oracle difference under the iterate rule of
    tests/minres_band.py, both measured against the oracle's own rounding
    sensitivity where a second reference with LAPACK's 'gv' eigensolver
    driver exists (ref_*_gv.json); without a tol 1e-12 reference: below
    1e-8.
  * FP64 FD at tol 1e-12: band rule, u within 1e-10 of u*.
  * FP32 / BF16 FD at tol 1e-8: they reach the same discrete solution
    along other iterates, so they are compared with u*.  MINRES stops on
    the residual in the norm of the preconditioner, so a solve with another
    preconditioner at the same tolerance ends at another distance from u*.
    FP32 FD perturbs the preconditioner by about 1e-6: at most 1.5 times
    the FP64 oracle's own distance (measured 0.86 to 1.16 over C2, C3 and
    C4).  BF16 FD perturbs it by about 1e-2: at most 3 times (measured 0.64
    to 1.72, the largest at C3 p = 5).  A "1e-8 relative" bound in this
    norm would fail the FP64 oracle itself, whose own distance is 1.1e-8
    (C2) to 9.4e-8 (C3 p = 5).
"""
import glob
import json
import os

import numpy as np
import pytest

import workloads as W
from minres_band import iterate_bound, same_iterations

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ref(name, tol, driver=None):
    path = os.path.join(GOLDEN, f"ref_{name}_{tol:.0e}" + (f"_{driver}" if driver else "") + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return dict(d["solves"][0], n_dof=d["n_dof"], n_c=d["n_c"])


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _sample_diff(u, ref):
    idx = np.asarray(ref["u_idx"])
    val = np.asarray(ref["u_val"])
    return np.abs(u[idx] - val).max() / np.abs(val).max()


def _proj_diff(u, ref):
    """Largest relative difference of the stored projections r_s . u."""
    out = 0.0
    for s, v in ref["u_proj"].items():
        r = W.random_vector(len(u), int(s))
        out = max(out, abs(r @ u - v) / (np.linalg.norm(r) * ref["u_norm"]))
    return out


def _own(ref8, ref12):
    """The oracle's own distance at tol 1e-8 from its tol 1e-12 solution,
    at the sampled entries (both files sample the same indices)."""
    assert ref8["u_idx"] == ref12["u_idx"]
    a, b = np.asarray(ref8["u_val"]), np.asarray(ref12["u_val"])
    return np.abs(a - b).max() / np.abs(b).max()


def _check(tag, u, lam, its, ref8, ref12, prec, tol, alt8=None, alt12=None):
    """The rules of the module docstring for one solve."""
    if prec == "fp64" and tol == 1e-8:
        d8 = _sample_diff(u, ref8)
        lidx = np.asarray(ref8["lam_idx"])
        dl = np.abs(lam[lidx] - np.asarray(ref8["lam_val"])).max() / np.abs(ref8["lam_val"]).max()
        msg = (f"  {tag}: its {its} (oracle {ref8['iters']}), |u-u_or| {d8:.2e}, |lam-lam_or| {dl:.2e}, "
               f"proj {_proj_diff(u, ref8):.2e}")
        bound = 1e-8
        if ref12 is not None:
            own = _own(ref8, ref12)
            pair = _own(ref8, alt8) if alt8 is not None else 0.0
            msg += f", oracle own error {own:.2e}, ratio {d8 / own:.3f}, oracle pair {pair:.2e}"
            bound = iterate_bound(own, pair)
        print(msg, flush=True)
        assert same_iterations(its, ref8, 1e-8, alt=alt8), msg
        assert d8 <= bound, msg
    elif prec == "fp64":
        d = _sample_diff(u, ref12)
        print(f"  {tag}: its {its} (oracle {ref12['iters']}), |u-u_or| {d:.2e}, "
              f"proj {_proj_diff(u, ref12):.2e}", flush=True)
        assert same_iterations(its, ref12, 1e-12, alt=alt12)
        assert d <= 1e-10
    elif ref12 is None:
        print(f"  {tag}: its {its} (oracle fp64 {ref8['iters']}), |u-u_or(tol 1e-8)| {_sample_diff(u, ref8):.2e}"
              " (no tol 1e-12 reference: not checked)", flush=True)
    else:
        d, own = _sample_diff(u, ref12), _own(ref8, ref12)
        print(f"  {tag}: its {its} (oracle fp64 {ref8['iters']}), |u-u*| {d:.2e}, "
              f"fp64 oracle at tol 1e-8: {own:.2e}, ratio {d / own:.2f}", flush=True)
        assert d <= (1.5 if prec == "fp32" else 3.0) * own


# ------------------------------------------------------------------- C2
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp64", 1e-12), ("fp32", 1e-8), ("bf16", 1e-8)])
def test_c2_against_oracle(prec, tol):
    ref8, ref12 = _ref("c2", 1e-8), _ref("c2", 1e-12)
    alt8, alt12 = _ref("c2", 1e-8, "gv"), _ref("c2", 1e-12, "gv")
    need = ref8 if tol == 1e-8 and prec == "fp64" else (ref12 if tol == 1e-12 else (ref12 or ref8))
    if need is None or ref8 is None:
        pytest.skip("C2 oracle reference not generated")
    _torch()
    from paper_2001_09626_amd import Solver
    print(f"\n[c2 {prec} tol {tol:.0e}]", flush=True)
    s = Solver(W.make_c2(seed=0), tol=tol, fd_precision=prec, maxit=5000)
    u, lam, st = s.solve()
    assert st["converged"]
    _check(f"c2 {prec}", _host(u), _host(lam), st["iterations"], ref8, ref12, prec, tol, alt8, alt12)
    s.close()


# ------------------------------------------------------------------- C3
C3_REFS = sorted({os.path.basename(p)[4:].rsplit("_", 1)[0]
                  for p in glob.glob(os.path.join(GOLDEN, "ref_c3_*.json")) if not p.endswith("_gv.json")})


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("name", C3_REFS or ["c3_missing"])
def test_c3_against_oracle(name, prec):
    if name == "c3_missing":
        pytest.skip("no C3 oracle reference generated")
    ref8, ref12 = _ref(name, 1e-8), _ref(name, 1e-12)
    alt8, alt12 = _ref(name, 1e-8, "gv"), _ref(name, 1e-12, "gv")
    _torch()
    from paper_2001_09626_amd import Solver
    p, n_el = (int(t[1:]) for t in name.split("_")[1:3])
    prob = W.make_c3(seed=0, p=p, n_el=n_el)
    print(f"\n[{name} {prec}]", flush=True)
    s = Solver(prob, tol=1e-8, fd_precision=prec, maxit=5000)
    u, lam, st = s.solve()
    assert st["converged"]
    _check(f"{name} {prec}", _host(u), _host(lam), st["iterations"], ref8, ref12, prec, 1e-8, alt8, alt12)
    s.close()
    if prec == "fp64" and ref12 is not None:
        s = Solver(prob, tol=1e-12, fd_precision="fp64", maxit=5000)
        u, lam, st = s.solve()
        _check(f"{name} fp64 tol 1e-12", _host(u), _host(lam), st["iterations"], ref8, ref12, "fp64", 1e-12,
               alt8, alt12)
        s.close()


# ------------------------------------------------------------------- C4
def _c4_refs():
    out = {}
    for p in glob.glob(os.path.join(GOLDEN, "ref_c4_*_1e-08.json")):
        j = int(os.path.basename(p).split("_")[2])
        out[j] = (_ref(f"c4_{j}", 1e-8), _ref(f"c4_{j}", 1e-12), _ref(f"c4_{j}", 1e-8, "gv"))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_c4_batch_against_oracle(prec):
    refs = _c4_refs()
    if not refs:
        pytest.skip("no C4 oracle reference generated")
    _torch()
    from paper_2001_09626_amd import Solver
    probs = W.make_c4(seed=0)
    print(f"\n[c4 batch of {len(probs)} problems, {prec}; references for {sorted(refs)}]", flush=True)
    s = Solver(probs, tol=1e-8, fd_precision=prec, maxit=5000)
    u, lam, st = s.solve()
    u, lam = _host(u), _host(lam)
    its, rel, status = s.problem_stats()
    assert (status == 1).all()
    first = np.concatenate([[0], np.cumsum([len(p["patches"]) for p in probs])])
    for j, (ref8, ref12, alt8) in sorted(refs.items()):
        d0, d1 = s.dof_offsets[first[j]], s.dof_offsets[first[j + 1]]
        c0, c1 = s.c_offsets[j], s.c_offsets[j + 1]
        assert (d1 - d0, c1 - c0) == (ref8["n_dof"], ref8["n_c"])
        _check(f"c4[{j}] {prec}", u[d0:d1], lam[c0:c1], int(its[j]), ref8, ref12, prec, 1e-8, alt8)
    s.close()


# ---------------------------------------------- non-conforming three-cube box
NC_REFS = sorted({os.path.basename(p)[4:].rsplit("_", 1)[0]
                  for p in glob.glob(os.path.join(GOLDEN, "ref_nc_p*.json")) if not p.endswith("_gv.json")})


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp64", 1e-12), ("fp32", 1e-8)])
@pytest.mark.parametrize("name", NC_REFS or ["nc_missing"])
def test_nonconforming_box_against_oracle(name, prec, tol):
    """The paper's non-conforming test (Section 6): the box (0,1)x(0,3)x(0,1)
    in three cubes of 4, 8 and 16 elements per direction, nested knot
    vectors on both interfaces, Dirichlet data of the exact solution on the
    whole boundary."""
    ref8, ref12 = _ref(name, 1e-8), _ref(name, 1e-12)
    alt8, alt12 = _ref(name, 1e-8, "gv"), _ref(name, 1e-12, "gv")
    if ref8 is None or (tol == 1e-12 and ref12 is None):
        pytest.skip("oracle reference not generated")
    _torch()
    from paper_2001_09626_amd import Solver
    p = int(name.split("_p")[1])
    print(f"\n[{name} {prec} tol {tol:.0e}]", flush=True)
    s = Solver(W.make_nonconforming(p=p), tol=tol, fd_precision=prec, maxit=5000)
    assert (s.n_dof, s.n_c) == (ref8["n_dof"], ref8["n_c"])
    u, lam, st = s.solve()
    assert st["converged"]
    _check(f"{name} {prec}", _host(u), _host(lam), st["iterations"], ref8, ref12, prec, tol, alt8, alt12)
    s.close()
