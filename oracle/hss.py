"""Randomized HSS approximation of the Cauchy-like eigenvector matrix (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper in its own order:
  * random sampling (Section 3): Y = A Omega, Z = A^T Omega with one Gaussian
    Omega for both (Omega1 = Omega2, as the paper does in practice);
  * interpolative decomposition (Section 3): B ~ B(:, J) X with X holding an
    identity block, computed here by column-pivoted Householder QR truncated
    at |R_kk| <= tol |R_11|, X = R11^{-1} R12;
  * Algorithm 2 (random HSS construction for Cauchy-like matrices), bottom-up
    over a postordered binary tree;
  * Algorithm 3 (HSS matrix times a general matrix from the right), with the
    sibling term added at the leaves and the downsweep split by columns
    (the printed listing omits the first and stacks the second);
  * eq. (new-hss): the dense expansion of an HSS matrix, used to check it;
  * eq. (bounds) with the neighbouring-segment rules of Section 4.1 for the
    rank estimate: r_b = ceil(log(16/eps) log(8R)/pi^2), R = (b^ - a^)/dist,
    boundaries moved by up to 5 rows when dist < 1e-10, r capped at 100.
"""
import math

import numpy as np

from . import secular as _sec
from .rng import philox_normal


# ----------------------------------------------------------------------------
# tree
# ----------------------------------------------------------------------------
class Node:
    __slots__ = ("lo", "hi", "level", "left", "right", "parent", "idx",
                 "U", "V", "B", "skel_r", "skel_c", "k_r", "k_c")

    def __init__(self, lo, hi, level):
        self.lo, self.hi, self.level = lo, hi, level
        self.left = self.right = self.parent = None
        self.idx = -1
        self.U = self.V = self.B = None
        self.skel_r = self.skel_c = None
        self.k_r = self.k_c = 0

    @property
    def leaf(self):
        return self.left is None


def hss_levels(K, m):
    """Number of levels below the root: L = ceil(log2(K/m)), at least 1 when K > m."""
    if K <= m:
        return 0
    return int(math.ceil(math.log2(K / m)))


def leaf_boundaries(K, L):
    """Leaf start indices of the balanced tree (split at floor(n/2))."""
    ranges = [(0, K)]
    for _ in range(L):
        nxt = []
        for lo, hi in ranges:
            h = (hi - lo) // 2
            nxt.append((lo, lo + h))
            nxt.append((lo + h, hi))
        ranges = nxt
    return [lo for lo, _ in ranges] + [K]


def build_tree(bounds):
    """Postordered binary tree over the leaf ranges [bounds[i], bounds[i+1])."""
    nleaf = len(bounds) - 1
    L = int(round(math.log2(nleaf))) if nleaf > 0 else 0
    assert (1 << L) == nleaf, "leaf count must be a power of two"
    level_nodes = [Node(bounds[i], bounds[i + 1], L) for i in range(nleaf)]
    levels = [level_nodes]
    for lev in range(L - 1, -1, -1):
        prev = levels[-1]
        cur = []
        for a in range(0, len(prev), 2):
            p = Node(prev[a].lo, prev[a + 1].hi, lev)
            p.left, p.right = prev[a], prev[a + 1]
            prev[a].parent = prev[a + 1].parent = p
            cur.append(p)
        levels.append(cur)
    root = levels[-1][0]
    post = []

    def visit(n):
        if not n.leaf:
            visit(n.left)
            visit(n.right)
        n.idx = len(post)
        post.append(n)
    visit(root)
    return root, post


# ----------------------------------------------------------------------------
# interpolative decomposition
# ----------------------------------------------------------------------------
def cpqr_id(A, tol, kmax=None):
    """Column interpolative decomposition A ~ A[:, J] @ X.

    Businger-Golub column-pivoted Householder QR: at every step the column of
    largest remaining norm (recomputed, not downdated) is pivoted to the front;
    stop when that norm is <= tol * |R_11| or kmax columns are taken.  Returns
    (J, X, rdiag) with X (k x n), X[:, J] = I, X = P [I, R11^-1 R12].
    """
    A = np.array(A, np.float64, copy=True)
    s, n = A.shape
    kmax = min(s, n) if kmax is None else min(kmax, s, n)
    perm = np.arange(n)
    rdiag = []
    k = 0
    r11 = None
    while k < kmax:
        norms = np.sqrt(np.sum(A[k:, k:] ** 2, axis=0))
        p = k + int(np.argmax(norms))
        nrm = norms[p - k]
        if r11 is None:
            r11 = nrm
        if nrm <= tol * r11 or nrm == 0.0:
            break
        if p != k:
            A[:, [k, p]] = A[:, [p, k]]
            perm[[k, p]] = perm[[p, k]]
        x = A[k:, k].copy()
        alpha = -math.copysign(nrm, x[0]) if x[0] != 0 else -nrm
        vvec = x.copy()
        vvec[0] -= alpha
        vn = np.sqrt(np.sum(vvec * vvec))
        if vn > 0:
            vvec /= vn
            A[k:, k:] -= 2.0 * np.outer(vvec, vvec @ A[k:, k:])
        A[k, k] = alpha
        A[k + 1:, k] = 0.0
        rdiag.append(abs(alpha))
        k += 1
    R11 = np.triu(A[:k, :k])
    R12 = A[:k, k:]
    T = np.linalg.solve(R11, R12) if k > 0 else np.zeros((0, n))
    X = np.zeros((k, n))
    X[:, perm[:k]] = np.eye(k)
    X[:, perm[k:]] = T
    return perm[:k].copy(), X, np.array(rdiag)


# ----------------------------------------------------------------------------
# rank estimate (eq. bounds + Section 4.1 rules)
# ----------------------------------------------------------------------------
def rank_bound(R, eps):
    """Smallest integer r with r >= log(16/eps) log(8R) / pi^2 (eq. bounds)."""
    return int(math.ceil(math.log(16.0 / eps) * math.log(8.0 * R) / math.pi ** 2))


def boundary_dist(d, gam, mu, b):
    """Distance of neighbouring segments split before index b:
    min(lam_b - d_{b-1}, d_b - lam_{b-1}) with the accurate differences."""
    K = len(d)
    # lam_b - d_{b-1} = (d_b - d_{b-1}) + gam_b ; d_b - lam_{b-1} = mu_{b-1}
    x = (d[b] - d[b - 1]) + gam[b] if b < K else np.inf
    y = mu[b - 1]
    return min(abs(x), abs(y))


def estimate_rank(d, gam, mu, bounds, eps=1e-16, shift_thresh=1e-10, max_shift=5, r_cap=100):
    """HSS rank estimate over the leaf boundaries; may move boundaries.

    Returns (r, new_bounds, per_boundary_ranks)."""
    d = np.asarray(d)
    K = len(d)
    span = (d[K - 1] + gam[K - 1]) - d[0]   # b^ - a^ = lam_K - d_1
    nb = list(bounds)
    ranks = []
    for t in range(1, len(nb) - 1):
        b = nb[t]
        dist = boundary_dist(d, gam, mu, b)
        if dist < shift_thresh:
            best, bestd = b, dist
            lo = max(nb[t - 1] + 1, b - max_shift)
            hi = min(nb[t + 1] - 1, b + max_shift)
            for bb in range(lo, hi + 1):
                dd = boundary_dist(d, gam, mu, bb)
                if dd > bestd:
                    best, bestd = bb, dd
            nb[t] = best
            dist = bestd
        R = span / dist if dist > 0 else np.inf
        ranks.append(r_cap if not np.isfinite(R) else min(r_cap, rank_bound(max(R, 1.0), eps)))
    r = max(ranks) if ranks else 0
    return min(r, r_cap), nb, ranks


# ----------------------------------------------------------------------------
# Algorithm 2
# ----------------------------------------------------------------------------
def cauchy_block(gen, rows, cols):
    """A(rows, cols) of the Cauchy-like matrix A_ij = uh_i v_j / (d_i - lam_j)."""
    d, uh, gam, mu, v = gen
    dl = _sec.d_minus_lambda(d, gam, mu, rows, cols)
    return np.asarray(uh)[np.asarray(rows)][:, None] * np.asarray(v)[np.asarray(cols)][None, :] / dl


def rshss(gen, Omega, bounds, tol, sample="paper"):
    """Algorithm 2 with a given Omega (K x s).  Returns (root, postorder, info).

    sample="paper": Phi_i = Y_i - D_i Omega_i and Theta_i = Z_i - D_i^T Omega_i
    as printed.  sample="offdiag": the same quantities by their definition,
    the HSS block row A(t_i, I \\ t_i) times Omega(I \\ t_i) (and the column
    likewise), which avoids the cancellation of the subtraction."""
    d = gen[0]
    K = len(d)
    A = cauchy_block(gen, np.arange(K), np.arange(K))
    if sample == "offdiag":
        Aoff = A.copy()
        for lo, hi in zip(bounds[:-1], bounds[1:]):
            Aoff[lo:hi, lo:hi] = 0.0
        Y = Aoff @ Omega
        Z = Aoff.T @ Omega
        A_for_D = np.zeros_like(A)
    else:
        Y = A @ Omega
        Z = A.T @ Omega
        A_for_D = A
    root, post = build_tree(bounds)
    L = max(n.level for n in post)
    Phi, Theta, Yh, Zh = {}, {}, {}, {}
    s = Omega.shape[1]
    for lev in range(L, 0, -1):
        for nd in [n for n in post if n.level == lev]:
            if nd.leaf:
                t = np.arange(nd.lo, nd.hi)
                D = A_for_D[np.ix_(t, t)]
                phi = Y[t] - D @ Omega[t]
                theta = Z[t] - D.T @ Omega[t]
                rows_r, rows_c = t, t
                Om_r, Om_c = Omega[t], Omega[t]
            else:
                a, b = nd.left, nd.right
                a.B = A[np.ix_(a.skel_r, b.skel_c)]
                b.B = A[np.ix_(b.skel_r, a.skel_c)]
                phi = np.vstack([Phi[a.idx] - a.B @ Yh[b.idx], Phi[b.idx] - b.B @ Yh[a.idx]])
                theta = np.vstack([Theta[a.idx] - b.B.T @ Zh[b.idx], Theta[b.idx] - a.B.T @ Zh[a.idx]])
                rows_r = np.concatenate([a.skel_r, b.skel_r])
                rows_c = np.concatenate([a.skel_c, b.skel_c])
                Om_r = np.vstack([Yh[a.idx], Yh[b.idx]])   # stacked Yhat of children
                Om_c = np.vstack([Zh[a.idx], Zh[b.idx]])   # stacked Zhat of children
            Jr, Xr, _ = cpqr_id(phi.T, tol)
            Jc, Xc, _ = cpqr_id(theta.T, tol)
            nd.U = Xr.T
            nd.V = Xc.T
            nd.skel_r = rows_r[Jr]
            nd.skel_c = rows_c[Jc]
            nd.k_r, nd.k_c = len(Jr), len(Jc)
            Phi[nd.idx] = phi[Jr]
            Theta[nd.idx] = theta[Jc]
            # Yhat_i = V_i^T Omega_i (leaf) or V_i^T [Yhat_i1; Yhat_i2] (parent),
            # Zhat_i likewise with U_i
            Yh[nd.idx] = nd.V.T @ Om_r
            Zh[nd.idx] = nd.U.T @ Om_c
    if not root.leaf:
        a, b = root.left, root.right
        a.B = A[np.ix_(a.skel_r, b.skel_c)]
        b.B = A[np.ix_(b.skel_r, a.skel_c)]
    ranks = [max(n.k_r, n.k_c) for n in post if n is not root]
    info = dict(s=s, max_rank=max(ranks) if ranks else 0, levels=L)
    return root, post, info


class HSS:
    """An HSS matrix: postordered nodes with generators, plus the Cauchy
    generators from which the leaf diagonal blocks D_i are regenerated."""

    def __init__(self, root, post, gen, info):
        self.root, self.post, self.gen, self.info = root, post, gen, info
        self.K = len(gen[0])

    def D(self, nd):
        t = np.arange(nd.lo, nd.hi)
        return cauchy_block(self.gen, t, t)


def hss_dense(H):
    """Dense expansion of an HSS matrix by eq. (new-hss)."""
    def expand(nd):
        if nd.leaf:
            return H.D(nd), nd.U, nd.V
        Da, Ua, Va = expand(nd.left)
        Db, Ub, Vb = expand(nd.right)
        a, b = nd.left, nd.right
        Dh = np.block([[Da, Ua @ a.B @ Vb.T], [Ub @ b.B @ Va.T, Db]])
        if nd is H.root:
            return Dh, None, None
        from scipy.linalg import block_diag
        Uh = block_diag(Ua, Ub) @ nd.U
        Vh = block_diag(Va, Vb) @ nd.V
        return Dh, Uh, Vh
    return expand(H.root)[0]


# ----------------------------------------------------------------------------
# Algorithm 3: X * H
# ----------------------------------------------------------------------------
def hss_matmul_right(X, H):
    """X (P x K) times the HSS matrix H (Algorithm 3)."""
    X = np.asarray(X, np.float64)
    root = H.root
    if root.leaf:
        return X @ H.D(root)
    post = H.post
    L = max(n.level for n in post)
    G, F = {}, {}
    # upsweep
    for lev in range(L, 0, -1):
        for nd in [n for n in post if n.level == lev]:
            if nd.leaf:
                G[nd.idx] = X[:, nd.lo:nd.hi] @ nd.U
            else:
                G[nd.idx] = np.hstack([G[nd.left.idx], G[nd.right.idx]]) @ nd.U

    def sib(nd):
        p = nd.parent
        return p.right if p.left is nd else p.left
    # downsweep
    out = np.empty_like(X)
    for lev in range(1, L + 1):
        for nd in [n for n in post if n.level == lev]:
            j = sib(nd)
            Fi = G[j.idx] @ j.B
            if lev > 1:
                Fi = Fi + F[nd.idx]
            if nd.leaf:
                out[:, nd.lo:nd.hi] = X[:, nd.lo:nd.hi] @ H.D(nd) + Fi @ nd.V.T
            else:
                W = Fi @ nd.V.T
                ka = nd.left.k_c
                F[nd.left.idx] = W[:, :ka]
                F[nd.right.idx] = W[:, ka:]
    return out


# ----------------------------------------------------------------------------
# the HSS update of one merge (rank estimate, sampling, check, retries)
# ----------------------------------------------------------------------------
def adc_hss_update(d, uh, gam, mu, opts, Omega=None):
    """Build H ~ Q' for one merge.  opts keys: leaf (m), p, id_tol, eps,
    seed, stream, max_retries, check_tol, nprobe, fixed_rank (optional)."""
    d = np.asarray(d)
    K = len(d)
    m = opts.get("leaf", 128)
    p = opts.get("p", 10)
    L = max(1, hss_levels(K, m))
    bounds = leaf_boundaries(K, L)
    # v_j from the Cauchy columns
    _, v = _sec.cauchy_vectors(d, uh, gam, mu)
    gen = (d, np.asarray(uh), np.asarray(gam), np.asarray(mu), v)
    r, bounds, _ = estimate_rank(d, gam, mu, bounds, eps=opts.get("eps", 1e-16))
    if opts.get("fixed_rank") is not None:
        r = int(opts["fixed_rank"])
    s = min(K, r + p)
    seed = opts.get("seed", 0)
    stream = opts.get("stream", 0)
    retries = 0
    Qp = cauchy_block(gen, np.arange(K), np.arange(K))
    nprobe = opts.get("nprobe", 4)
    W = philox_normal(K, nprobe, seed, stream * 2 + 1)
    WQ = W.T @ Qp
    while True:
        Om = Omega if (Omega is not None and retries == 0) else philox_normal(K, s, seed, stream * 2)
        root, post, info = rshss(gen, Om, bounds, opts.get("id_tol", 1e-14))
        H = HSS(root, post, gen, info)
        err = np.linalg.norm(WQ - hss_matmul_right(W.T, H)) / np.linalg.norm(WQ)
        # the probe error alone decides; a node whose ID kept every sample
        # column is only reported
        info.update(check_err=float(err), retries=retries, r_est=r,
                    saturated=bool(info["max_rank"] >= s and s < K))
        if err <= opts.get("check_tol", 1e-12):
            return H, info
        if retries >= opts.get("max_retries", 2):
            info["fallback"] = True
            return _DenseAsHSS(Qp, gen), info
        retries += 1
        s = min(K, 2 * s)


class _DenseAsHSS(HSS):
    """Dense fallback wearing the HSS interface: a single leaf."""

    def __init__(self, Qp, gen):
        nd = Node(0, Qp.shape[0], 0)
        nd.idx = 0
        super().__init__(nd, [nd], gen, dict(fallback=True))
        self._Q = Qp

    def D(self, nd):
        return self._Q
