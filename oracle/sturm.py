"""Sturm-sequence eigenvalue counts of a symmetric tridiagonal matrix (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Textbook fact (Sylvester's law of inertia): the number of eigenvalues of T
smaller than x equals the number of negative pivots q_i of the LDL^T
factorisation of T - xI, q_1 = a_1 - x, q_i = (a_i - x) - b_{i-1}^2/q_{i-1}.
This gives any single eigenvalue lambda_k by bisection in O(N) per step, at
any N, independently of divide-and-conquer.
"""
import numpy as np


def count_below(diag, off, x):
    """Number of eigenvalues < x, for every x in the array x (vectorised)."""
    a = np.asarray(diag, np.float64)
    b2 = np.asarray(off, np.float64) ** 2
    x = np.atleast_1d(np.asarray(x, np.float64))
    tiny = np.finfo(np.float64).tiny
    cnt = np.zeros(x.shape, np.int64)
    q = a[0] - x
    for i in range(len(a)):
        if i > 0:
            q = (a[i] - x) - b2[i - 1] / q
        q = np.where(q == 0.0, -tiny, q)
        cnt += q < 0
    return cnt


def eigenvalues_by_index(diag, off, ks):
    """lambda_k (0-based k, ascending) for every k in ks, by bisection on counts.

    Bisects over the ordered set of representable doubles, so the result is
    the smallest double x with count_below(x) > k, up to the rounding of the
    pivot recurrence.
    """
    a = np.asarray(diag, np.float64)
    b = np.abs(np.asarray(off, np.float64))
    r = np.zeros_like(a)
    r[:-1] += b
    r[1:] += b
    lo = float(np.min(a - r)) - 1.0
    hi = float(np.max(a + r)) + 1.0
    ks = np.atleast_1d(np.asarray(ks, np.int64))
    L = np.full(ks.shape, lo)
    H = np.full(ks.shape, hi)
    for _ in range(2200):
        M = 0.5 * (L + H)
        done = (M <= L) | (M >= H)
        if np.all(done):
            break
        c = count_below(a, b, M)
        up = c > ks  # lambda_k < M
        H = np.where(~done & up, M, H)
        L = np.where(~done & ~up, M, L)
    return H
