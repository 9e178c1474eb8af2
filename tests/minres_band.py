"""Iteration-count agreement of two MINRES runs on the same system.

The stopping test |eta_j| <= tol gamma_1 is applied to a residual estimate
that rounding perturbs more and more as the Lanczos vectors lose
orthogonality.  Measured on the oracle alone:
  * two runs that differ only in the summation order of the stiffness
    product (assembled matrix vs quadrature apply) give |eta|/gamma_1 =
    1.0522e-8 and 1.0699e-8 after 258 iterations of a ragged-batch problem
    (1.7 %);
  * two runs that differ only in LAPACK's generalised eigensolver driver
    (their fast-diagonalization inverses 4e-14 apart) give estimates up to
    6.8 % apart at iterations 320-323 of the flattest C4 problem (323
    iterations to 1e-8 in both runs).
  * on a C1 problem whose estimates stall (2.03, 2.00, then 1.20 times tol
    at iterations 58-60) the same driver change moves the estimate at
    iteration 57 by 14 %.
Counts therefore agree exactly, or the GPU stops earlier where the oracle's
own estimate at the GPU's stopping iteration lies within a factor `band`
of tol (|eta| never increases, so every estimate in between lies in that
band too: on flat tails such as C2 at 1e-12, 1.031, 1.020 and 0.813 times
tol at iterations 244-246, this can be two iterations), or later where the
oracle's estimate at the GPU's last continuing iteration lies within the
band (one iteration late: the estimate at the oracle's own stop; more: the
same oracle run continued to a smaller tolerance, whose estimates up to its
stop are the same arithmetic, gives the estimates past it; on C2-small at
1e-12 they read 1.0015 and 1.0002 times tol at iterations 150 and 151, and
runs on two hosts' LAPACK builds stop at 150 and 152).
Where a second oracle run with another eigensolver driver (``alt``) is at
hand, the band widens by twice the largest relative spread between the two
oracle runs' estimates over the last ten iterations (up to the later of the
two stops, with both runs continued past their stops where ``ext`` and
``alt_ext`` are given): the GPU is held to the oracle's own rounding
sensitivity, not tighter.  At a stagnation step the estimates of two
runs can differ by tens of per cent (C2-small at 1e-12: 1.0002 and about
0.7 times tol at iteration 151 on two hosts).
"""

import math


def same_iterations(gpu_its, ref, tol, band=1.1, alt=None, ext=None, alt_ext=None):
    o = int(ref["iters"])
    h = ref["history"]
    hx = ext["history"] if ext is not None else h
    if alt is not None:
        ha = (alt_ext if alt_ext is not None else alt)["history"]
        # the ten iterations before the later of the two stops, as far as
        # both (continued) histories reach
        hi = min(len(hx), len(ha), max(gpu_its, o) + 1)
        spread = max((abs(math.log(hx[j] / ha[j])) for j in range(max(1, hi - 10), hi)), default=0.0)
        band = band * math.exp(2.0 * spread)
    if gpu_its == o:
        return True
    if gpu_its < o:           # stopped early: the oracle was still just above tol
        return h[gpu_its] <= band * tol
    # late: the oracle's estimate at the GPU's last continuing iteration
    # (gpu_its - 1) lies within the band; past the oracle's own stop that
    # estimate comes from the same run continued to a smaller tolerance
    # (``ext``: its iterations up to the stop are the same arithmetic)
    if gpu_its - 1 < len(hx):
        return hx[gpu_its - 1] >= tol / band
    return False


def iterate_bound(own, pair):
    """Bound on the distance between the GPU's and the oracle's iterates at
    tolerance 1e-8 (relative 2-norms).  ``own`` is the oracle iterate's
    distance to the converged solution, ``pair`` its distance to the
    oracle's own iterate with LAPACK's 'gv' eigensolver driver instead of
    the default (U, D perturbed at rounding level; fast-diagonalization
    inverses about 4e-14 apart).  The GPU's perturbation is a few times
    larger (its host eigensolver is another rounding of the same pencils,
    1e-13 from the oracle's FD, plus other summation orders); measured GPU
    distance / pair: 2.0 (C1, 0.19 / 0.094 of own), 1.8 (C2), 1.6 (C2 with
    geometry inclusion).  Bound: the larger of a tenth of own and four
    times pair."""
    return max(0.1 * own, 4.0 * pair)
