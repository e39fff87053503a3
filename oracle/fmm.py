"""Fast sampling of the Cauchy-like eigenvector matrix (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The random sampling of Algorithm 2 multiplies the off-diagonal blocks of the
Cauchy-like matrix A_ij = uh_i v_j / (d_i - lam_j) by Omega, which costs
O(K^2 s).  The paper names fast multipole (FMM) summation of these Cauchy
sums as the way to lower that cost (Sections 1, 3 and 5) without giving an
algorithm.  This module is the formulation used here: a one-dimensional FMM
with Chebyshev interpolation on both sides of the kernel 1/(x - y) (the
"black-box" form of Fong and Darve, 2009), over the same binary tree as the
HSS matrix.

Quantities (0-based, leaf t(i) holds index i):
  Y_ic = uh_i  sum_{j not in t(i)} v_j  Omega_jc / (d_i - lam_j)    (Phi)
  Z_jc = v_j   sum_{i not in t(j)} uh_i Omega_ic / (d_i - lam_j)    (Theta)
Y has targets d_i and sources lam_j; Z has targets lam_j and sources d_i and
the kernel 1/(source - target).

Geometry.  A node with index range [lo, hi) covers the points d_lo .. d_{hi-1}
and lam_lo .. lam_{hi-1}; the smallest is d_lo, the largest
lam_{hi-1} = d_{hi-1} + gam_{hi-1}.  Coordinates are local to the node's
anchor pole d_lo: a pole maps to d_i - d_lo and a root to (d_j - d_lo) + gam_j,
so no large coordinate is ever subtracted from another.  The node's interval
is [0, w], w = (d_{hi-1} - d_lo) + gam_{hi-1}, with centre and half-width w/2
and p Chebyshev points tau_k = w/2 (1 + cos((2k+1) pi / (2p))).  Between a
node T and a node S to its right the gap is
(d_{lo_S} - d_{hi_T}) + mu_{hi_T - 1} (eq. d-lambda).  T and S are
well separated (admissible) when the gap is at least eta times the larger of
their widths (eta = 1): a point of one node then lies at least three
half-widths from the other's centre, where Chebyshev interpolation of
1/(x - y) converges like (3 + sqrt 8)^-p.

Interaction lists.  A dual traversal from (root, root): an admissible pair
is a far pair; a non-admissible pair of leaves is a near pair unless both are
the same leaf (the diagonal block, left out of Phi and Theta); otherwise the
four pairs of children are visited.  Every (i, j) off the diagonal blocks is
then covered exactly once.

Operators (l, k index Chebyshev points; ell^N(x) is the vector of Lagrange
basis values of node N's points at x, by the barycentric formula):
  P2M  M_S = sum_{j in S} ell^S(y_j) q_j^T                 (leaf S)
  M2M  M_P = sum_{children C} E_PC M_C,  E_PC[k, l] = ell_k^P(tau_l^C + d_lo(C) - d_lo(P))
  M2L  L_T += G_TS M_S,  G_TS[l, k] = sigma / ((d_lo(T) - d_lo(S)) + (tau_l^T - tau_k^S))
  L2L  L_C += E_PC^T L_P
  L2P  out_i = ell^T(x_i) . L_T + near sums
with q_jc = v_j Omega_jc, sigma = +1 for Y and q_ic = uh_i Omega_ic,
sigma = -1 for Z; near sums use the differences of eq. (d-lambda)
(Remark 1) entry by entry, and the result is scaled by uh_i (Y) or v_j (Z).
"""
import math

import numpy as np

from . import secular as _sec
from .hss import build_tree

ETA = 1.0


def cheb_points(p):
    """Chebyshev points of the first kind on [-1, 1] and their barycentric
    weights (Berrut and Trefethen, 2004)."""
    k = np.arange(p)
    th = (2 * k + 1) * math.pi / (2 * p)
    return np.cos(th), ((-1.0) ** k) * np.sin(th)


def lagrange(x, centre, half, p):
    """ell (p x len(x)): Lagrange basis of the p Chebyshev points of
    [centre - half, centre + half] at the points x (barycentric formula)."""
    t, beta = cheb_points(p)
    nodes = centre + half * t
    x = np.atleast_1d(np.asarray(x, np.float64))
    diff = x[None, :] - nodes[:, None]
    out = np.zeros((p, x.size))
    exact = diff == 0.0
    hit = exact.any(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = beta[:, None] / diff
    q[:, hit] = 0.0
    out[:, ~hit] = q[:, ~hit] / q[:, ~hit].sum(axis=0)
    for col in np.nonzero(hit)[0]:
        out[np.argmax(exact[:, col]), col] = 1.0
    return out


def node_width(d, gam, lo, hi):
    """w = lam_{hi-1} - d_lo in the node's local coordinates."""
    return (d[hi - 1] - d[lo]) + gam[hi - 1]


def gap(d, mu, T, S):
    """Distance between node T and node S (disjoint index ranges)."""
    if S.lo >= T.hi:
        return (d[S.lo] - d[T.hi]) + mu[T.hi - 1]
    return (d[T.lo] - d[S.hi]) + mu[S.hi - 1]


def interaction_lists(d, gam, mu, root):
    """(far, near): lists of (T, S) node pairs by the dual traversal."""
    far, near = [], []

    def visit(T, S):
        if T is not S and (T.hi <= S.lo or S.hi <= T.lo):
            wt = node_width(d, gam, T.lo, T.hi)
            ws = node_width(d, gam, S.lo, S.hi)
            if gap(d, mu, T, S) >= ETA * max(wt, ws):
                far.append((T, S))
                return
        if T.leaf and S.leaf:
            if T is not S:
                near.append((T, S))
            return
        for a in (T.left, T.right):
            for b in (S.left, S.right):
                visit(a, b)

    visit(root, root)
    return far, near


def _local(d, gam, side_is_root, lo, idx):
    """Local coordinates (anchor d_lo) of the poles (side_is_root False) or
    roots (True) with indices idx."""
    base = d[idx] - d[lo]
    return base + gam[idx] if side_is_root else base


def sample_fmm(gen, Omega, bounds, p=24):
    """(Y, Z) = (Phi, Theta) of Algorithm 2 by the FMM described above.
    gen = (d, uh, gam, mu, v); Omega is K x s; bounds are the leaf starts
    (a power of two of leaves) followed by K."""
    d, uh, gam, mu, v = (np.asarray(x, np.float64) for x in gen)
    Omega = np.asarray(Omega, np.float64)
    K, s = Omega.shape
    root, post = build_tree(list(bounds))
    far, near = interaction_lists(d, gam, mu, root)
    t, _ = cheb_points(p)
    geo = {}
    for nd in post:
        w = node_width(d, gam, nd.lo, nd.hi)
        geo[nd] = (w / 2.0, w / 2.0, (w / 2.0) * (1.0 + t))  # centre, half-width, points
    out = []
    for side in (0, 1):
        # side 0: targets d (poles), sources lam (roots), q = v Omega, sigma = +1
        # side 1: targets lam, sources d, q = uh Omega, sigma = -1
        src_root = side == 0
        q = (v if side == 0 else uh)[:, None] * Omega
        sigma = 1.0 if side == 0 else -1.0
        M = {}
        for nd in post:  # children before parents
            c, h, _ = geo[nd]
            if nd.leaf:
                idx = np.arange(nd.lo, nd.hi)
                M[nd] = lagrange(_local(d, gam, src_root, nd.lo, idx), c, h, p) @ q[idx]
            else:
                acc = np.zeros((p, s))
                for ch in (nd.left, nd.right):
                    pts = geo[ch][2] + (d[ch.lo] - d[nd.lo])
                    acc += lagrange(pts, c, h, p) @ M[ch]
                M[nd] = acc
        Lc = {nd: np.zeros((p, s)) for nd in post}
        for T, S in far:
            G = sigma / ((d[T.lo] - d[S.lo]) + (geo[T][2][:, None] - geo[S][2][None, :]))
            Lc[T] += G @ M[S]
        for nd in reversed(post):  # parents before children
            if nd.leaf:
                continue
            c, h, _ = geo[nd]
            for ch in (nd.left, nd.right):
                pts = geo[ch][2] + (d[ch.lo] - d[nd.lo])
                Lc[ch] += lagrange(pts, c, h, p).T @ Lc[nd]
        res = np.zeros((K, s))
        for nd in post:
            if not nd.leaf:
                continue
            idx = np.arange(nd.lo, nd.hi)
            c, h, _ = geo[nd]
            res[idx] = lagrange(_local(d, gam, not src_root, nd.lo, idx), c, h, p).T @ Lc[nd]
        for T, S in near:
            ti = np.arange(T.lo, T.hi)
            sj = np.arange(S.lo, S.hi)
            if side == 0:
                dl = _sec.d_minus_lambda(d, gam, mu, ti, sj)      # d_i - lam_j, i in T
                res[ti] += (1.0 / dl) @ q[sj]
            else:
                dl = _sec.d_minus_lambda(d, gam, mu, sj, ti)      # d_i - lam_j, i in S, j in T
                res[ti] += (1.0 / dl).T @ q[sj]
        out.append((uh if side == 0 else v)[:, None] * res)
    return out[0], out[1]


def sample_direct(gen, Omega, bounds):
    """(Y, Z) by their definition: the Cauchy-like matrix with its diagonal
    leaf blocks set to zero, times Omega and its transpose times Omega."""
    d, uh, gam, mu, v = (np.asarray(x, np.float64) for x in gen)
    K = len(d)
    A = uh[:, None] * v[None, :] / _sec.d_minus_lambda(d, gam, mu)
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        A[lo:hi, lo:hi] = 0.0
    return A @ Omega, A.T @ Omega
