"""Plain fp64 Cuppen / Gu-Eisenstat divide-and-conquer (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1 (ADC) of the paper, step by step:
  * leaf (size <= leaf): dense eigendecomposition.  The paper uses QR; the
    oracle uses cyclic Jacobi (an exact-arithmetic-equivalent textbook method).
  * tear (eq. T2): T = diag(T1, T2) + |b_k| v v^T with v = e_k +- e_{k+1};
    T1 loses |b_k| at its last diagonal entry, T2 at its first.  k = floor(n/2).
  * merge (eq. T3): d = [Lambda1; Lambda2], u = [last row of Q1; first row
    of Q2] (second half negated when b_k < 0); rho = |b_k| ||u||^2, z = u/||u||.
  * deflation: the two-type rule of the DC literature (a component of z too
    small to matter, or two nearly equal poles combined by a Givens rotation).
  * secular roots, Loewner recompute, Cauchy-like eigenvectors (Theorem 1,
    eq. ev_z, Remark 1) and the eigenvector update diag(Q1, Q2) * Q'.
  * the update is either the dense product or, when the secular size is large,
    an HSS approximation of Q' (Algorithm 2) applied with Algorithm 3.
"""
import numpy as np

from . import secular as _sec

EPS = np.finfo(np.float64).eps


# ----------------------------------------------------------------------------
# leaves: cyclic Jacobi (textbook; batched over leaves of equal size)
# ----------------------------------------------------------------------------
def jacobi_eigh(A, max_sweeps=60):
    """Eigendecomposition of a batch of small symmetric matrices by cyclic Jacobi.

    A: (B, m, m).  Returns (w, V) with w ascending per matrix, A = V diag(w) V^T.
    """
    A = np.array(A, np.float64, copy=True)
    if A.ndim == 2:
        w, V = jacobi_eigh(A[None], max_sweeps)
        return w[0], V[0]
    B, m, _ = A.shape
    V = np.broadcast_to(np.eye(m), (B, m, m)).copy()
    fro = np.sqrt(np.sum(A * A, axis=(1, 2)))
    offmask = ~np.eye(m, dtype=bool)
    for _ in range(max_sweeps):
        off = np.sqrt(np.sum((A * A)[:, offmask], axis=1))
        if np.all(off <= EPS * fro):
            break
        for p in range(m - 1):
            for q in range(p + 1, m):
                apq = A[:, p, q]
                nz = apq != 0.0
                if not np.any(nz):
                    continue
                app = A[:, p, p]
                aqq = A[:, q, q]
                with np.errstate(over="ignore", divide="ignore"):
                    theta = np.where(nz, (aqq - app) / (2.0 * np.where(nz, apq, 1.0)), 0.0)
                    t = np.where(theta >= 0, 1.0, -1.0) / (np.abs(theta) + np.sqrt(1.0 + theta * theta))
                t = np.where(nz, t, 0.0)
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = t * c
                # A <- J^T A J with J the rotation in the (p, q) plane
                Ap = A[:, :, p].copy()
                Aq = A[:, :, q].copy()
                A[:, :, p] = c[:, None] * Ap - s[:, None] * Aq
                A[:, :, q] = s[:, None] * Ap + c[:, None] * Aq
                Ap = A[:, p, :].copy()
                Aq = A[:, q, :].copy()
                A[:, p, :] = c[:, None] * Ap - s[:, None] * Aq
                A[:, q, :] = s[:, None] * Ap + c[:, None] * Aq
                Vp = V[:, :, p].copy()
                Vq = V[:, :, q].copy()
                V[:, :, p] = c[:, None] * Vp - s[:, None] * Vq
                V[:, :, q] = s[:, None] * Vp + c[:, None] * Vq
    w = np.diagonal(A, axis1=1, axis2=2).copy()
    order = np.argsort(w, axis=1, kind="stable")
    w = np.take_along_axis(w, order, axis=1)
    V = np.take_along_axis(V, order[:, None, :], axis=2)
    return w, V


def tridiag_dense(diag, off):
    n = len(diag)
    T = np.diag(np.asarray(diag, np.float64))
    if n > 1:
        T += np.diag(off, 1) + np.diag(off, -1)
    return T


# ----------------------------------------------------------------------------
# tree
# ----------------------------------------------------------------------------
def split_tree(n, leaf):
    """Balanced binary DC tree over [0, n): nodes (s0, n, n1); leaves have n1=0.

    Returned as a list of levels, top (root) first; level l holds 2^l nodes or
    fewer.  The split is k = floor(n/2).
    """
    levels = [[(0, n)]]
    while True:
        nxt = []
        for s0, m in levels[-1]:
            if m > leaf:
                h = m // 2
                nxt.append((s0, h))
                nxt.append((s0 + h, m - h))
        if not nxt:
            break
        levels.append(nxt)
    return levels


def torn_diagonal(diag, off, leaf):
    """Diagonal with every tear correction of the tree applied (eq. T2)."""
    a = np.array(diag, np.float64, copy=True)
    for lev in split_tree(len(a), leaf):
        for s0, m in lev:
            if m > leaf:
                k = s0 + m // 2 - 1
                beta = abs(off[k])
                a[k] -= beta
                a[k + 1] -= beta
    return a


# ----------------------------------------------------------------------------
# deflation
# ----------------------------------------------------------------------------
def deflate(d, z, rho):
    """Deflation of D + rho z z^T with d ascending (may contain ties).

    tol = 8 eps max(max|d|, rho max|z|).  Scanning in ascending order:
      type 1: |rho z_j| <= tol  -> j deflates with eigenvalue d_j;
      type 2: with i the previous surviving index, r = hypot(z_i, z_j),
              c = z_j/r, s = -z_i/r; if |(d_j - d_i) c s| <= tol the pair is
              rotated: i deflates with c^2 d_i + s^2 d_j, j keeps z_j = r and
              d_j = s^2 d_i + c^2 d_j.  The rotation acts on columns (i, j)
              of the eigenvector basis as [U_i, U_j] <- [c U_i + s U_j, -s U_i + c U_j].
    Returns dict(surv, defl, dval, zval, rot) where surv/defl are index lists
    (in scan order), dval/zval the updated d/z, and rot the ordered list of
    rotations (i, j, c, s).
    """
    d = np.array(d, np.float64, copy=True)
    z = np.array(z, np.float64, copy=True)
    n = d.shape[0]
    tol = 8.0 * EPS * max(np.max(np.abs(d)) if n else 0.0, rho * (np.max(np.abs(z)) if n else 0.0))
    surv, defl, rot = [], [], []
    prev = -1
    for j in range(n):
        if rho * abs(z[j]) <= tol:
            defl.append(j)
            continue
        if prev < 0:
            prev = j
            continue
        i = prev
        r = np.hypot(z[i], z[j])
        c = z[j] / r
        s = -z[i] / r
        if abs((d[j] - d[i]) * c * s) <= tol:
            di, dj = d[i], d[j]
            d[i] = c * c * di + s * s * dj
            d[j] = s * s * di + c * c * dj
            z[j] = r
            z[i] = 0.0
            rot.append((i, j, c, s))
            defl.append(i)
            prev = j
        else:
            surv.append(i)
            prev = j
    if prev >= 0:
        surv.append(prev)
    return dict(surv=np.array(surv, np.int64), defl=np.array(defl, np.int64),
                dval=d, zval=z, rot=rot, tol=tol)


# ----------------------------------------------------------------------------
# one merge
# ----------------------------------------------------------------------------
def merge_vectors(d1, Q1, d2, Q2, beta):
    """The rank-one problem of eq. (T3) from the two children.

    Returns (d, z, rho, U, order): d ascending (stable merge of the two
    sorted spectra), z normalised, rho >= 0, U = diag(Q1, Q2) with columns in
    the same order as d.
    """
    n1, n2 = len(d1), len(d2)
    u = np.concatenate([Q1[n1 - 1, :], Q2[0, :] * (1.0 if beta >= 0 else -1.0)])
    nu = np.sqrt(np.sum(u * u))
    rho = abs(beta) * nu * nu
    z = u / nu if nu > 0 else u
    dd = np.concatenate([d1, d2])
    order = np.argsort(dd, kind="stable")
    U = np.zeros((n1 + n2, n1 + n2))
    U[:n1, :n1] = Q1
    U[n1:, n1:] = Q2
    return dd[order], z[order], rho, U[:, order], order


def merge(d1, Q1, d2, Q2, beta, update="dense", hss_opts=None, report=None):
    """Eigendecomposition of diag(T1', T2') + |beta| v v^T from the children's."""
    d, z, rho, U, _ = merge_vectors(d1, Q1, d2, Q2, beta)
    n = len(d)
    df = deflate(d, z, rho)
    U = U.copy()
    for (i, j, c, s) in df["rot"]:
        ui = U[:, i].copy()
        uj = U[:, j].copy()
        U[:, i] = c * ui + s * uj
        U[:, j] = -s * ui + c * uj
    surv, defl = df["surv"], df["defl"]
    ds, zs = df["dval"][surv], df["zval"][surv]
    K = len(surv)
    lam_all = np.empty(n)
    Qn = np.empty((n, n))
    used_hss = False
    if K > 0:
        lam, gam, mu, _ = _sec.secular_roots(ds, zs, rho)
        uh = _sec.lowner_z(ds, rho, gam, mu, np.sign(zs))
        if update == "hss" and hss_opts is not None and K >= hss_opts.get("min_k", 2048):
            from . import hss as _hss
            H, info = _hss.adc_hss_update(ds, uh, gam, mu, hss_opts)
            newcols = _hss.hss_matmul_right(U[:, surv], H)
            used_hss = True
            if report is not None:
                report.setdefault("hss", []).append(info)
        else:
            Qp, _ = _sec.cauchy_vectors(ds, uh, gam, mu)
            newcols = U[:, surv] @ Qp
        vals = np.concatenate([lam, df["dval"][defl]])
        cols = np.concatenate([newcols, U[:, defl]], axis=1)
    else:
        vals = df["dval"][defl]
        cols = U[:, defl]
    order = np.argsort(vals, kind="stable")
    lam_all[:] = vals[order]
    Qn[:] = cols[:, order]
    if report is not None:
        report.setdefault("merges", []).append(dict(n=n, K=K, hss=used_hss))
    return lam_all, Qn


def stedc(diag, off, leaf=32, update="dense", hss_opts=None, report=None):
    """Full eigendecomposition of the symmetric tridiagonal T (Algorithm 1).

    diag: (N,), off: (N-1,).  Returns (w ascending, Z) with T Z = Z diag(w).
    update: "dense" (plain DC) or "hss" (merges with K >= hss_opts['min_k'] in
    the top hss_opts['levels'] levels use the randomized HSS update).
    """
    diag = np.asarray(diag, np.float64)
    off = np.asarray(off, np.float64)
    N = diag.shape[0]
    if N == 0:
        return np.zeros(0), np.zeros((0, 0))
    a = torn_diagonal(diag, off, leaf)
    levels = split_tree(N, leaf)
    # leaves: all nodes with size <= leaf, batched by size for the Jacobi sweeps
    blocks = {}
    leaves = [(s0, m) for lev in levels for (s0, m) in lev if m <= leaf]
    by_size = {}
    for s0, m in leaves:
        by_size.setdefault(m, []).append(s0)
    for m, starts in by_size.items():
        T = np.zeros((len(starts), m, m))
        for b, s0 in enumerate(starts):
            T[b] = tridiag_dense(a[s0:s0 + m], off[s0:s0 + m - 1])
        w, V = jacobi_eigh(T)
        for b, s0 in enumerate(starts):
            blocks[(s0, m)] = (w[b], V[b])
    depth_of = {}
    for lvl, lev in enumerate(levels):
        for node in lev:
            depth_of[node] = lvl
    for lvl in range(len(levels) - 1, -1, -1):
        for (s0, m) in levels[lvl]:
            if m <= leaf:
                continue
            h = m // 2
            d1, Q1 = blocks.pop((s0, h))
            d2, Q2 = blocks.pop((s0 + h, m - h))
            beta = off[s0 + h - 1]
            upd = update
            if update == "hss" and hss_opts is not None and lvl >= hss_opts.get("levels", 10 ** 9):
                upd = "dense"
            blocks[(s0, m)] = merge(d1, Q1, d2, Q2, beta, upd, hss_opts, report)
    return blocks[(0, N)]


# ----------------------------------------------------------------------------
# accuracy metrics (Section 5, Example 3 text; norms as stated in the docstring)
# ----------------------------------------------------------------------------
def tnorm1(diag, off):
    """||T||_1 = max_i (|b_{i-1}| + |a_i| + |b_i|)."""
    a = np.abs(np.asarray(diag, np.float64))
    b = np.abs(np.asarray(off, np.float64))
    s = a.copy()
    s[:-1] += b
    s[1:] += b
    return float(np.max(s)) if len(s) else 0.0


def residual(diag, off, w, Z):
    """||T Z - Z diag(w)||_F / (N ||T||_1)."""
    N = len(diag)
    TZ = np.asarray(diag)[:, None] * Z
    if N > 1:
        TZ[:-1] += np.asarray(off)[:, None] * Z[1:]
        TZ[1:] += np.asarray(off)[:, None] * Z[:-1]
    R = TZ - Z * np.asarray(w)[None, :]
    return float(np.sqrt(np.sum(R * R)) / (N * tnorm1(diag, off)))


def orthogonality(Z):
    """||Z^T Z - I||_max."""
    G = Z.T @ Z
    G[np.diag_indices_from(G)] -= 1.0
    return float(np.max(np.abs(G)))
