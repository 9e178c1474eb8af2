"""Write oracle reference solutions of full-size workloads for the GPU
parity tests (tests/test_gpu_reference.py).

    python tests/golden/make_reference.py c2 1e-8       # C2 at one tolerance
    python tests/golden/make_reference.py c4 1e-8 0 3 5 ...  # problems of the C4 batch
    python tests/golden/make_reference.py c3 p n_el     # C3's 4x4x4 patches, degree p,
                                                        # n_el^3 elements (tol 1e-8, 1e-12)
    python tests/golden/make_reference.py nc 1 2 3 4    # the non-conforming three-cube box,
                                                        # degrees p (tol 1e-8, 1e-12)
    AFIETI_REF_DRIVER=gv python tests/golden/make_reference.py ...
        # the same with LAPACK's 'gv' eigensolver driver: ref_<name>_<tol>_gv.json,
        # the oracle's own rounding sensitivity for the parity rules

Only the oracle (``oracle/``) and the seeded workload generators are called.
Each output file holds, per tolerance: the MINRES iteration count and the
history of |eta| / gamma_1, the norms of u and lambda, u and lambda at a
seeded sample of indices, and the projections of u onto seeded N(0, 1)
vectors (``workloads.random_vector(n_dof, seed)``), so that a test can
compare the whole solution without storing it.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.afieti import AFIETI  # noqa: E402

N_SAMPLES = 4096
PROJ_SEEDS = (101, 102, 103)


def summarise(o, res, tol):
    rng = np.random.default_rng(1234)
    iu = np.sort(rng.choice(o.n_dof, size=min(N_SAMPLES, o.n_dof), replace=False))
    il = np.sort(rng.choice(o.n_c, size=min(N_SAMPLES, o.n_c), replace=False))
    u, lam = res["u"], res["lam"]
    return dict(tol=tol, iters=int(res["iters"]), history=[float(h) for h in res["history"]],
                u_norm=float(np.linalg.norm(u)), lam_norm=float(np.linalg.norm(lam)),
                u_idx=iu.tolist(), u_val=u[iu].tolist(), lam_idx=il.tolist(), lam_val=lam[il].tolist(),
                u_proj={str(s): float(W.random_vector(o.n_dof, s) @ u) for s in PROJ_SEEDS})


def write(name, prob, *tols):
    """Oracle solves of ``prob`` at each tolerance, each summarised into
    ref_<name>_<tol>[_<driver>].json beside this script."""
    driver = os.environ.get("AFIETI_REF_DRIVER") or None
    o = AFIETI(prob, eig_driver=driver)
    for tol in tols:
        t0 = time.time()
        res = o.solve(tol=tol, maxit=5000)
        out = dict(workload=name, n_dof=int(o.n_dof), n_c=int(o.n_c), solves=[summarise(o, res, tol)])
        path = os.path.join(HERE, f"ref_{name}_{tol:.0e}" + (f"_{driver}" if driver else "") + ".json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"{name} tol {tol:.0e}: {res['iters']} iterations; wrote {path} ({time.time() - t0:.0f} s)",
              flush=True)


def main(argv):
    what = argv[1]
    if what == "c2":
        write("c2", W.make_c2(seed=0), float(argv[2]))
    elif what == "c3":
        p, n_el = int(argv[2]), int(argv[3])
        write(f"c3_p{p}_e{n_el}", W.make_c3(seed=0, p=p, n_el=n_el), 1e-8, 1e-12)
    elif what == "nc":
        # the non-conforming three-cube box (4, 8, 16 elements per direction)
        for p in argv[2:]:
            write(f"nc_p{int(p)}", W.make_nonconforming(p=int(p)), 1e-8, 1e-12)
    elif what == "c4":
        probs = W.make_c4(seed=0)
        for j in argv[3:]:
            write(f"c4_{int(j)}", probs[int(j)], float(argv[2]))
    else:
        raise SystemExit(f"unknown workload {what}")


if __name__ == "__main__":
    main(sys.argv)
