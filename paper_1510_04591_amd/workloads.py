"""Seeded synthetic inputs (no method arithmetic here).

Matrices are returned as numpy fp64 (diag, offdiag) pairs; merge problems as
(d, z, rho).  Every generator is deterministic in its arguments.
"""
import numpy as np


def toeplitz(N, a=2.0, b=1.0):
    """Tridiagonal Toeplitz: diagonal a, off-diagonal b (Example 3)."""
    return np.full(N, float(a)), np.full(max(N - 1, 0), float(b))


def random_uniform(N, seed=2):
    """Diagonal iid U(-1, 1), then off-diagonal iid U(0, 1), one generator."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, N)
    b = rng.uniform(0.0, 1.0, N - 1)
    return a, b


def batched(count=256, seed=4, nmin=200, nmax=4000):
    """count matrices with N ~ U{nmin..nmax}; the first half Toeplitz (2, 1),
    the second half random as in random_uniform, drawn from the same
    generator in index order."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(nmin, nmax + 1, count)
    mats = []
    for i, N in enumerate(Ns):
        N = int(N)
        if i < count // 2:
            mats.append(toeplitz(N))
        else:
            a = rng.uniform(-1.0, 1.0, N)
            b = rng.uniform(0.0, 1.0, N - 1)
            mats.append((a, b))
    return mats


def clement(n):
    """Clement-type matrix of order n+1: zero diagonal, b_i = sqrt(i (n+1-i))."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.zeros(n + 1), np.sqrt(i * (n + 1 - i))


def hermite(n):
    """Hermite-type matrix of order n: zero diagonal, b_i = sqrt(i)."""
    return np.zeros(n), np.sqrt(np.arange(1, n, dtype=np.float64))


def legendre(n):
    """Legendre-type matrix of order n: zero diagonal, b_i = i/sqrt((2i-1)(2i+1)), i = 2..n."""
    i = np.arange(2, n + 1, dtype=np.float64)
    return np.zeros(n), i / np.sqrt((2 * i - 1) * (2 * i + 1))


def laguerre(n):
    """Laguerre-type matrix of order n: diagonal 3, 5, ..., 2n+1; off-diagonal 2, 3, ..., n."""
    return 2.0 * np.arange(1, n + 1, dtype=np.float64) + 1.0, np.arange(2, n + 1, dtype=np.float64)


def example1_merge(N, seed=1, a=1.0, b=9.0):
    """Rank-one problem of Example 1: d_i = i (b-a)/N, u a random unit vector, rho = 1."""
    d = np.arange(1, N + 1, dtype=np.float64) * (b - a) / N
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(N)
    return d, u / np.linalg.norm(u), 1.0


def random_merge(K, seed=0, spread="uniform"):
    """Random rank-one problem: strictly increasing d, unit z, rho in [0.5, 2]."""
    rng = np.random.default_rng(seed)
    if spread == "uniform":
        d = np.sort(rng.uniform(-1.0, 1.0, K))
    elif spread == "clustered":
        c = rng.uniform(-1.0, 1.0, max(1, K // 16))
        d = np.sort(c[rng.integers(0, len(c), K)] + rng.uniform(-1e-6, 1e-6, K))
    else:
        d = np.sort(rng.standard_normal(K))
    d = np.unique(d)
    while len(d) < K:
        d = np.unique(np.concatenate([d, rng.uniform(-1, 1, K - len(d))]))
    z = rng.standard_normal(len(d))
    return d, z / np.linalg.norm(z), float(rng.uniform(0.5, 2.0))


def planted_merge(K, pairs, seed=0):
    """Random rank-one problem with planted close poles: d sorted U(0, 1)
    with d[j] = d[j-1] + gap for every (j, gap) in `pairs` (pairs applied in
    index order, the rest of d shifted to stay increasing), z a random unit
    vector, rho = 1."""
    rng = np.random.default_rng(seed)
    g = rng.uniform(0.5, 1.5, K)
    for j, gap in pairs:
        g[j] = 0.0
    d = np.cumsum(g)
    d = d / d[-1]
    for j, gap in sorted(pairs):
        d[j:] += (d[j - 1] + gap) - d[j]
    z = rng.standard_normal(K)
    return d, z / np.linalg.norm(z), 1.0


def spectrum(kind, N, seed=5):
    """Prescribed spectra: 'uniform' sorted U(0,1); 'geometric' 10^(-6(i-1)/(N-1));
    'clusters' 10 clusters centred at (k+0.5)/10 of width 1e-8."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        lam = np.sort(rng.uniform(0.0, 1.0, N))
    elif kind == "geometric":
        lam = 10.0 ** (-6.0 * np.arange(N) / (N - 1))[::-1]
    elif kind == "clusters":
        counts = [N // 10 + (1 if k < N % 10 else 0) for k in range(10)]
        lam = np.sort(np.concatenate([(k + 0.5) / 10 + rng.uniform(-5e-9, 5e-9, c) for k, c in enumerate(counts)]))
    else:
        raise ValueError(kind)
    w = rng.standard_normal(N)
    return lam, w / np.linalg.norm(w)


def jacobi_from_spectrum(lam, w):
    """Tridiagonal (diag, |offdiag|) with eigenvalues lam whose eigenvector
    matrix has first row w (unit vector): Lanczos on diag(lam) from w, by
    the O(n^2) Givens reconstruction in jacobi_gen.c (built next to this
    file by build.build_gen)."""
    import ctypes
    import os
    lib_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libadcgen.so")
    if not os.path.exists(lib_path):
        from . import build as _build
        _build.build_gen(verbose=False)
    L = ctypes.CDLL(lib_path)
    P = ctypes.POINTER(ctypes.c_double)
    L.adc_gen_jacobi.argtypes = [ctypes.c_int, P, P, P, P]
    L.adc_gen_jacobi.restype = ctypes.c_int
    lam = np.ascontiguousarray(lam, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    n = len(lam)
    a = np.zeros(n)
    b = np.zeros(max(n - 1, 0))
    st = L.adc_gen_jacobi(n, lam.ctypes.data_as(P), w.ctypes.data_as(P), a.ctypes.data_as(P),
                          b.ctypes.data_as(P) if n > 1 else None)
    if st != 0:
        raise MemoryError("adc_gen_jacobi")
    return a, b


def prescribed_tridiagonal(kind, N, seed=5, method="givens"):
    """Tridiagonal matrix with the spectrum `spectrum(kind, N, seed)`: the
    Jacobi matrix of the weights w_i^2 at the nodes lam_i, i.e. Lanczos on
    diag(lam) started from w.  method "givens": the O(N^2) reconstruction of
    jacobi_from_spectrum; "householder": the Householder tridiagonalization
    (scipy, O(N^3)) of H diag(lam) H with H the reflector taking e_1 to w (the
    first column of the reduction's basis stays e_1).  Off-diagonals are
    returned as absolute values (a diagonal sign similarity)."""
    lam, w = spectrum(kind, N, seed)
    if method == "givens":
        return jacobi_from_spectrum(lam, w)
    from scipy.linalg import hessenberg
    u = w.copy()
    u[0] -= 1.0 if w[0] < 0 else -1.0  # u = w + sign(w_0) e_1: H e_1 = -sign(w_0) w
    u /= np.linalg.norm(u)
    Lu = lam * u
    A = np.diag(lam) - 2.0 * (np.outer(u, Lu) + np.outer(Lu, u)) + 4.0 * float(u @ Lu) * np.outer(u, u)
    Hs = hessenberg(A, overwrite_a=True, check_finite=False)
    return np.diag(Hs).copy(), np.abs(np.diag(Hs, -1)).copy()
