"""The launch shapes of the matrix-core FD kernels (components of a patch
together or one per workgroup, 64 or 128 columns per mode-3 block) sum
every output element over the same depth order, so every shape gives
bitwise the same P_A^{-1} and interior solve, and the autotuned handle
equals them; ragged batches included (with tensors that need the largest
depth extent)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CASES = {"c2_small": lambda: W.make_c2(n_el=5, p=3, seed=2),
         "c1_2d": lambda: W.make_c1(n_el=6, p=2, seed=1),
         "ragged": lambda: [W.make_c3(n_el=3, p=2, grid=(2, 3, 2), seed=4),
                            W.make_c4(seed=5, n_problems=1, el_range=(4, 9))[0],
                            W.make_c1(n_el=5, p=3, seed=2),
                            W.make_c2(n_el=38, p=3, grid=(1, 1, 2), seed=3)]}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp64"])
def test_fd_launch_shapes_bitwise_equal(case, prec):
    torch = _torch()
    from paper_2001_09626_amd import Solver
    prob = CASES[case]()
    print(f"\n[fd shapes {case} {prec}]", flush=True)
    outs = []
    for tune in [-1] + list(range(4)):
        s = Solver(prob, fd_precision=prec, fd_tune=tune)
        r = torch.from_numpy(W.random_vector(s.n_dof, 70)).cuda()
        z = s.apply_fd(r)
        zi = s.apply("fd_interior", r)
        torch.cuda.synchronize()
        assert torch.isfinite(z).all() and torch.isfinite(zi).all()
        outs.append((tune, z, zi))
        s.close()
    for tune, z, zi in outs[1:]:
        assert torch.equal(z, outs[0][1]), f"shape {tune}: {float((z - outs[0][1]).abs().max())}"
        assert torch.equal(zi, outs[0][2]), f"shape {tune} interior"
