"""Secular equation, Loewner recompute and Cauchy-like eigenvectors (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The rank-one problem is M = D + rho z z^T with D = diag(d), d strictly
increasing, ||z|| = 1 and rho > 0 (Theorem 1, Bunch-Nielsen-Sorensen).  Its
eigenvalues are the roots of the secular function

    f(lam) = 1 + rho * sum_j z_j^2 / (d_j - lam),

one in each interval (d_i, d_{i+1}) and the last in (d_K, d_K + rho]
(interlacing, Theorem 1).  The paper leaves the root finder to LAPACK; the
oracle uses plain bisection in the shifted variable tau = lam - d_o, where the
origin d_o is the nearer pole, and bisects over the ordered set of
representable doubles so that it ends on two adjacent floating-point numbers.
The outputs are gamma_i = lam_i - d_i and mu_i = d_{i+1} - lam_i, the
distances the paper carries to keep the eigenvectors orthogonal (Remark 1 and
the description of the merge routine in Section 4.3).  mu_K is +inf: there is
no d_{K+1}.
"""
import numpy as np

_CHUNK_ELEMS = 1 << 22  # entries of the (roots x K) work matrix per chunk


def _tau_from_bits(bits, sgn):
    return sgn * bits.view(np.float64)


def secular_function(d, z, rho, lam):
    """f(lam) = 1 + rho * sum_j z_j^2/(d_j - lam) evaluated directly (Theorem 1)."""
    d = np.asarray(d, np.float64)
    z = np.asarray(z, np.float64)
    lam = np.atleast_1d(np.asarray(lam, np.float64))
    return 1.0 + rho * np.sum((z * z)[None, :] / (d[None, :] - lam[:, None]), axis=1)


def _g_shifted(delta_rows, z2, rho, tau):
    # g(tau) = 1/rho + sum_j z_j^2 / (delta_j - tau), delta_j = d_j - d_origin
    return 1.0 / rho + np.sum(z2[None, :] / (delta_rows - tau[:, None]), axis=1)


def secular_roots(d, z, rho):
    """All K roots of the secular equation.

    Returns (lam, gam, mu, origin): lam_i; gam_i = lam_i - d_i; mu_i = d_{i+1}
    - lam_i (inf for the last root); origin_i in {i, i+1} is the pole the
    shifted variable was measured from.
    """
    d = np.ascontiguousarray(d, np.float64)
    z = np.ascontiguousarray(z, np.float64)
    K = d.shape[0]
    if K == 0:
        e = np.zeros(0)
        return e, e, e, np.zeros(0, np.int64)
    if not (rho > 0):
        raise ValueError("rho must be positive")
    if K > 1 and not np.all(np.diff(d) > 0):
        raise ValueError("d must be strictly increasing")
    z2 = z * z
    gap = np.empty(K)
    gap[:-1] = d[1:] - d[:-1]
    gap[-1] = np.inf

    # Choose the origin: the root lies left of the midpoint iff f(mid) >= 0.
    origin = np.arange(K, dtype=np.int64)
    sgn = np.ones(K)
    hi = np.empty(K)
    rows = max(1, _CHUNK_ELEMS // K)
    for r0 in range(0, K - 1, rows):
        r1 = min(K - 1, r0 + rows)
        idx = np.arange(r0, r1)
        delta = d[None, :] - d[idx][:, None]
        g_mid = _g_shifted(delta, z2, rho, 0.5 * gap[idx])
        right = g_mid < 0.0
        origin[idx[right]] += 1
        sgn[idx[right]] = -1.0
        hi[idx] = 0.5 * gap[idx]
    hi[K - 1] = rho  # last root: (d_K, d_K + rho], g(rho) >= 0

    # Bisection on |tau| over representable doubles.  For sgn=+1, g rises with
    # |tau| (g(0+) = -inf); for sgn=-1, g falls with |tau| (g(0-) = +inf).
    lo_bits = np.zeros(K, np.uint64)
    hi_bits = hi.view(np.uint64).copy()
    tau = np.empty(K)
    for r0 in range(0, K, rows):
        r1 = min(K, r0 + rows)
        idx = np.arange(r0, r1)
        delta = d[None, :] - d[origin[idx]][:, None]
        lo = lo_bits[idx].copy()
        hb = hi_bits[idx].copy()
        s = sgn[idx]
        for _ in range(70):
            active = (hb - lo) > 1
            if not np.any(active):
                break
            mid = lo + (hb - lo) // np.uint64(2)
            g = _g_shifted(delta, z2, rho, _tau_from_bits(mid, s))
            # "root beyond mid" means: for s=+1, g(mid) < 0; for s=-1, g(mid) >= 0
            beyond = np.where(s > 0, g < 0.0, g >= 0.0)
            lo = np.where(active & beyond, mid, lo)
            hb = np.where(active & ~beyond, mid, hb)
        # lo is never 0 for the answer unless the bracket collapsed onto 0;
        # pick the endpoint with the smaller |g| among the valid ones.
        t_hi = _tau_from_bits(hb, s)
        g_hi = np.abs(_g_shifted(delta, z2, rho, t_hi))
        t_lo = _tau_from_bits(lo, s)
        lo_valid = lo > 0
        g_lo = np.full(len(idx), np.inf)
        if np.any(lo_valid):
            g_lo[lo_valid] = np.abs(_g_shifted(delta[lo_valid], z2, rho, t_lo[lo_valid]))
        tau[idx] = np.where(g_lo < g_hi, t_lo, t_hi)

    lam = d[origin] + tau
    gam = np.where(sgn > 0, tau, gap + tau)
    mu = np.where(sgn > 0, gap - tau, -tau)
    mu[K - 1] = np.inf
    return lam, gam, mu, origin


def d_minus_lambda(d, gam, mu, rows=None, cols=None):
    """Matrix (d_i - lam_j) for i in rows, j in cols, computed as in Remark 1:

        d_i - lam_j = (d_i - d_j) - gam_j       if i <= j
                    = (d_i - d_{j+1}) + mu_j    if i >  j
    """
    d = np.asarray(d, np.float64)
    K = d.shape[0]
    rows = np.arange(K) if rows is None else np.asarray(rows)
    cols = np.arange(K) if cols is None else np.asarray(cols)
    I = rows[:, None]
    J = cols[None, :]
    jp1 = np.minimum(J + 1, K - 1)
    upper = (d[I] - d[J]) - gam[J]
    lower = (d[I] - d[jp1]) + mu[J]
    return np.where(I <= J, upper, lower)


def lowner_z(d, rho, gam, mu, zsign):
    """Loewner recompute of the rank-one vector (eq. ev_z, with 1/rho and sign).

    uhat_i^2 = (lam_i - d_i)/rho * prod_{j != i} (lam_j - d_i)/(d_j - d_i),
    taken in the paper's pairing, as a running product whose binary exponent
    is split off after every factor so that no partial product over- or
    underflows.  sign(uhat_i) = sign(z_i).
    """
    d = np.asarray(d, np.float64)
    K = d.shape[0]
    if K == 0:
        return np.zeros(0)
    mant = np.ones(K)
    expo = np.zeros(K, np.int64)
    i = np.arange(K)
    for j in range(K):
        # lam_j - d_i over all i, from the differences of Remark 1
        if j + 1 < K:
            lam_minus_d = np.where(i <= j, gam[j] - (d - d[j]), -((d - d[j + 1]) + mu[j]))
        else:
            lam_minus_d = gam[j] - (d - d[j])
        fac = np.where(i == j, lam_minus_d, lam_minus_d / np.where(i == j, 1.0, d[j] - d))
        mant = mant * fac
        m, e = np.frexp(mant)
        mant = m
        expo += e
    u2 = np.ldexp(mant / rho, expo)
    return np.where(np.asarray(zsign) < 0, -1.0, 1.0) * np.sqrt(u2)


def cauchy_vectors(d, uh, gam, mu):
    """Eigenvector matrix of D + rho*uh*uh^T (eq. EVec / eq. Ev-Q).

    Q'_{ij} = uh_i v_j / (d_i - lam_j), v_j = 1/||uh/(d - lam_j)||, with the
    differences d_i - lam_j of Remark 1.  Returns (Q', v).
    """
    dl = d_minus_lambda(d, gam, mu)
    C = np.asarray(uh)[:, None] / dl
    v = 1.0 / np.sqrt(np.sum(C * C, axis=0))
    return C * v[None, :], v
