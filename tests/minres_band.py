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
Counts therefore agree exactly, or the GPU stops earlier where the oracle's
own estimate at the GPU's stopping iteration lies within a factor `band`
of tol (|eta| never increases, so every estimate in between lies in that
band too: on flat tails such as C2 at 1e-12, 1.031, 1.020 and 0.813 times
tol at iterations 244-246, this can be two iterations), or one iteration
later where the oracle's estimate at its own stop lies within the band.
"""


def same_iterations(gpu_its, ref, tol, band=1.1):
    o = int(ref["iters"])
    h = ref["history"]
    if gpu_its == o:
        return True
    if gpu_its < o:           # stopped early: the oracle was still just above tol
        return h[gpu_its] <= band * tol
    if gpu_its == o + 1:      # one step late: the oracle was just below tol
        return h[o] >= tol / band
    return False
