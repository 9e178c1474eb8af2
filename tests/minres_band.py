"""Iteration-count agreement of two MINRES runs on the same system.

The stopping test |eta_j| <= tol gamma_1 is applied to a residual estimate
that rounding perturbs more and more as the Lanczos vectors lose
orthogonality: two oracle runs that differ only in the summation order of
the stiffness product (assembled matrix vs quadrature apply) give
|eta|/gamma_1 = 1.0522e-8 and 1.0699e-8 after 258 iterations of the ragged
batch problem (1.7 %).  Counts therefore agree exactly, or differ by one
where the oracle's own estimate at the earlier stopping iteration lies
within a factor `band` of tol.
"""


def same_iterations(gpu_its, ref, tol, band=1.1):
    o = int(ref["iters"])
    h = ref["history"]
    if gpu_its == o:
        return True
    if gpu_its == o - 1:      # stopped one step early: the oracle was just above tol
        return h[gpu_its] <= band * tol
    if gpu_its == o + 1:      # one step late: the oracle was just below tol
        return h[o] >= tol / band
    return False
