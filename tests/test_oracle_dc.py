"""Pins of the oracle's divide-and-conquer (Algorithm 1) and its pieces.

Fixed by: closed-form spectra (Toeplitz, Clement), library nodes (Gauss-
Hermite), LAPACK via numpy/scipy, Sturm counts (textbook), the exact tear
identity (eq. T2), the persymmetry of Toeplitz merges, and invariants.
"""
import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

from oracle import dc, secular as sec, sturm
from paper_1510_04591_amd import workloads

EPS = np.finfo(np.float64).eps


def test_jacobi_vs_lapack():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((6, 32, 32))
    A = A + A.transpose(0, 2, 1)
    w, V = dc.jacobi_eigh(A)
    for b in range(6):
        ref = np.linalg.eigvalsh(A[b])
        assert np.max(np.abs(w[b] - ref)) <= 64 * EPS * np.max(np.abs(ref))
        assert np.max(np.abs(V[b].T @ V[b] - np.eye(32))) <= 1e-14
        assert np.max(np.abs(A[b] @ V[b] - V[b] * w[b])) <= 1e-13 * np.max(np.abs(ref))


def test_tear_identity_exact():
    a, b = workloads.random_uniform(200, 7)
    b = b.copy()
    b[50] = -b[50]
    at = dc.torn_diagonal(a, b, leaf=32)
    T = dc.tridiag_dense(a, b)
    # rebuild T from diag(T1', T2', ...) and the rank-one terms |b_k| v v^T,
    # v = e_k + sign(b_k) e_{k+1} (eq. T2)
    bb = b.copy()
    splits = [s0 + m // 2 - 1 for lev in dc.split_tree(200, 32) for s0, m in lev if m > 32]
    bb[splits] = 0.0
    R = dc.tridiag_dense(at, bb)
    for k in splits:
        v = np.zeros(200)
        v[k] = 1.0
        v[k + 1] = 1.0 if b[k] >= 0 else -1.0
        R += abs(b[k]) * np.outer(v, v)
    assert np.max(np.abs(R - T)) <= 2 * EPS * np.max(np.abs(a))
    assert np.array_equal(R == 0, T == 0)


@pytest.mark.parametrize("N", [1, 2, 31, 32, 33, 100, 1024])
def test_toeplitz_closed_form(N):
    a, b = workloads.toeplitz(N)
    w, Z = dc.stedc(a, b, leaf=32)
    k = np.arange(1, N + 1)
    exact = np.sort(2 + 2 * np.cos(k * np.pi / (N + 1)))
    assert np.max(np.abs(w - exact)) <= 1e-13 * 4
    # eigenvectors: q_k(i) = sqrt(2/(N+1)) sin(i k pi/(N+1)) up to sign
    kk = np.arange(N, 0, -1)  # ascending eigenvalues <-> descending k
    i = np.arange(1, N + 1)
    Q = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(i, kk) * np.pi / (N + 1))
    assert np.min(np.abs(np.sum(Q * Z, axis=0))) >= 1 - 1e-10


def test_clement_closed_form():
    n = 300
    a, b = workloads.clement(n)
    w, Z = dc.stedc(a, b, leaf=32)
    assert np.max(np.abs(w - np.arange(-n, n + 1, 2))) <= 1e-13 * dc.tnorm1(a, b)
    assert dc.residual(a, b, w, Z) <= 1e-14 and dc.orthogonality(Z) <= 1e-13


def test_hermite_gauss_nodes():
    n = 400
    a, b = workloads.hermite(n)
    w, Z = dc.stedc(a, b, leaf=32)
    nodes = np.polynomial.hermite_e.hermegauss(n)[0]
    assert np.max(np.abs(w - np.sort(nodes))) <= 1e-12 * dc.tnorm1(a, b)


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_small(seed):
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(2, 65))
    a = rng.standard_normal(N)
    b = rng.standard_normal(N - 1) * (rng.random(N - 1) > 0.1)  # some zeros, mixed signs
    w, Z = dc.stedc(a, b, leaf=int(rng.integers(2, 9)))
    wj, _ = dc.jacobi_eigh(dc.tridiag_dense(a, b))
    ref = np.linalg.eigvalsh(dc.tridiag_dense(a, b))
    scale = dc.tnorm1(a, b)
    assert np.max(np.abs(w - ref)) <= 1e-13 * scale
    assert np.max(np.abs(wj - ref)) <= 1e-13 * scale
    assert dc.residual(a, b, w, Z) <= 1e-14 and dc.orthogonality(Z) <= 1e-13


def test_random_vs_lapack_and_sturm():
    N = 1500
    a, b = workloads.random_uniform(N, 2)
    w, Z = dc.stedc(a, b, leaf=32)
    ref = eigh_tridiagonal(a, b, eigvals_only=True, lapack_driver="stebz")
    assert np.max(np.abs(w - ref)) <= 1e-13 * dc.tnorm1(a, b)
    ks = np.array([0, 7, 700, N - 1])
    assert np.max(np.abs(w[ks] - sturm.eigenvalues_by_index(a, b, ks))) <= 1e-13 * dc.tnorm1(a, b)
    assert dc.residual(a, b, w, Z) <= 1e-14 and dc.orthogonality(Z) <= 1e-13


def test_sturm_toeplitz():
    N = 5000
    a, b = workloads.toeplitz(N)
    ks = np.array([0, 1, 2500, N - 1])
    k = N - ks  # ascending order index -> k of the closed form
    exact = 2 + 2 * np.cos(k * np.pi / (N + 1))
    assert np.max(np.abs(sturm.eigenvalues_by_index(a, b, ks) - exact)) <= 8 * EPS * 4


def test_deflation_toeplitz_mirror_and_eigs():
    # top merge of a Toeplitz matrix: T2' is the flip of T1', so exactly half
    # of the poles coincide and deflate by rotation (K = n/2)
    N = 256
    a, b = workloads.toeplitz(N)
    at = dc.torn_diagonal(a, b, leaf=N // 2)
    h = N // 2
    w1, Q1 = np.linalg.eigh(dc.tridiag_dense(at[:h], b[:h - 1]))
    w2, Q2 = np.linalg.eigh(dc.tridiag_dense(at[h:], b[h:]))
    d, z, rho, U, _ = dc.merge_vectors(w1, Q1, w2, Q2, b[h - 1])
    df = dc.deflate(d, z, rho)
    assert len(df["surv"]) == h and len(df["rot"]) == h
    # eigenvalues after deflation: deflated values plus secular roots equal the
    # spectrum of D + rho z z^T
    surv, defl = df["surv"], df["defl"]
    lam, _, _, _ = sec.secular_roots(df["dval"][surv], df["zval"][surv], rho)
    allv = np.sort(np.concatenate([lam, df["dval"][defl]]))
    ref = np.linalg.eigvalsh(np.diag(d) + rho * np.outer(z, z))
    assert np.max(np.abs(allv - ref)) <= 1e-13 * 4


def test_negative_and_zero_offdiagonals():
    rng = np.random.default_rng(3)
    N = 300
    a = rng.uniform(-1, 1, N)
    b = rng.uniform(-1, 1, N - 1)
    b[[40, 149, 151]] = 0.0
    w, Z = dc.stedc(a, b, leaf=16)
    ref = eigh_tridiagonal(a, b, eigvals_only=True, lapack_driver="stebz")
    assert np.max(np.abs(w - ref)) <= 1e-13 * dc.tnorm1(a, b)
    assert dc.residual(a, b, w, Z) <= 1e-14 and dc.orthogonality(Z) <= 1e-13


@pytest.mark.parametrize("kind", ["uniform", "geometric", "clusters"])
def test_prescribed_spectrum_generator(kind):
    """The generated Jacobi matrix has the prescribed eigenvalues (LAPACK)
    and a positive off-diagonal."""
    from scipy.linalg import eigh_tridiagonal
    a, b = workloads.prescribed_tridiagonal(kind, 512)
    lam, _ = workloads.spectrum(kind, 512)
    ev = eigh_tridiagonal(a, b, eigvals_only=True)
    assert np.max(np.abs(ev - np.sort(lam))) <= 1e-13
    assert np.all(b > 0)


@pytest.mark.parametrize("kind", ["uniform", "geometric"])
def test_givens_generator_matches_householder(kind):
    """The O(n^2) reconstruction and the Householder tridiagonalization
    produce the same Jacobi matrix (it is unique for given nodes and weights
    with positive off-diagonals) where it is well conditioned."""
    a1, b1 = workloads.prescribed_tridiagonal(kind, 512, method="givens")
    a2, b2 = workloads.prescribed_tridiagonal(kind, 512, method="householder")
    assert np.max(np.abs(a1 - a2)) <= 1e-10 and np.max(np.abs(b1 - b2)) <= 1e-10
