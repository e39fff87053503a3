"""Pins of the oracle's fast sampling (one-dimensional Chebyshev FMM).

Fixed by: exactness of barycentric interpolation on polynomials below the
point count; a brute-force count showing that the far pairs, near pairs and
diagonal leaf blocks cover every (i, j) exactly once; the separation of every
far pair recomputed from lam = d + gam; and agreement with the samples taken
by their definition (dense Cauchy-like matrix with zeroed diagonal blocks)
within the interpolation error, which falls as the point count grows.
"""
import math

import numpy as np
import pytest

from oracle import fmm, hss, secular as sec
from paper_1510_04591_amd import workloads


def _gen(d, z, rho):
    lam, gam, mu, _ = sec.secular_roots(d, z, rho)
    uh = sec.lowner_z(d, rho, gam, mu, np.sign(z))
    _, v = sec.cauchy_vectors(d, uh, gam, mu)
    return (d, uh, gam, mu, v), lam


def _bounds(K, m):
    return hss.leaf_boundaries(K, hss.hss_levels(K, m))


@pytest.mark.parametrize("p", [4, 9, 24])
def test_lagrange_reproduces_polynomials(p):
    g = np.random.default_rng(p)
    c, h = 0.3, 1.7
    coef = g.standard_normal(p)                  # degree p - 1
    nodes = c + h * fmm.cheb_points(p)[0]
    f = np.polynomial.polynomial.polyval(nodes, coef)
    x = np.concatenate([g.uniform(c - h, c + h, 50), nodes[:3]])
    got = fmm.lagrange(x, c, h, p).T @ f
    want = np.polynomial.polynomial.polyval(x, coef)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    L = fmm.lagrange(nodes, c, h, p)
    assert np.array_equal(L, np.eye(p))


@pytest.mark.parametrize("K,m,spread", [(600, 16, "uniform"), (1000, 32, "clustered"), (777, 8, "normal")])
def test_interaction_lists_partition_the_off_diagonal_blocks(K, m, spread):
    d, z, rho = workloads.random_merge(K, seed=3, spread=spread)
    (d, uh, gam, mu, v), lam = _gen(d, z, rho)
    bounds = _bounds(len(d), m)
    root, post = hss.build_tree(bounds)
    far, near = fmm.interaction_lists(d, gam, mu, root)
    cover = np.zeros((len(d), len(d)), dtype=np.int32)
    for T, S in far + near:
        cover[T.lo:T.hi, S.lo:S.hi] += 1
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        cover[lo:hi, lo:hi] += 1
    assert np.all(cover == 1)
    assert all(T.leaf and S.leaf for T, S in near)
    # separation from the roots themselves
    for T, S in far:
        pts_t = np.concatenate([d[T.lo:T.hi], lam[T.lo:T.hi]])
        pts_s = np.concatenate([d[S.lo:S.hi], lam[S.lo:S.hi]])
        g = max(pts_s.min() - pts_t.max(), pts_t.min() - pts_s.max())
        w = max(np.ptp(pts_t), np.ptp(pts_s))
        assert g >= fmm.ETA * w * (1 - 1e-12)
    assert len(far) > 0


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("case", ["example1", "paired", "clustered", "normal"])
def test_fmm_samples_match_definition(case):
    if case == "example1":
        d, z, rho = workloads.example1_merge(1500, seed=2)
    elif case == "paired":
        # poles in close pairs around a Toeplitz spectrum (two nearly equal halves)
        n1 = 512
        k = np.arange(1, n1 + 1)
        lam1 = 2 + 2 * np.cos(k * math.pi / (n1 + 1))
        d = np.sort(np.concatenate([lam1 - 1e-3 * k / n1, lam1 + 1e-3 * k / n1]))
        z = np.random.default_rng(5).standard_normal(len(d))
        z /= np.linalg.norm(z)
        rho = 1.0
    else:
        d, z, rho = workloads.random_merge(1200, seed=7, spread=case)
    gen, _ = _gen(d, z, rho)
    K = len(gen[0])
    Omega = np.random.default_rng(11).standard_normal((K, 24))
    bounds = _bounds(K, 32)
    Yd, Zd = fmm.sample_direct(gen, Omega, bounds)
    Yf, Zf = fmm.sample_fmm(gen, Omega, bounds, p=24)
    assert _rel(Yf, Yd) <= 1e-13
    assert _rel(Zf, Zd) <= 1e-13


def test_fmm_error_falls_with_point_count():
    d, z, rho = workloads.random_merge(800, seed=1, spread="uniform")
    gen, _ = _gen(d, z, rho)
    K = len(gen[0])
    Omega = np.random.default_rng(2).standard_normal((K, 8))
    bounds = _bounds(K, 16)
    Yd, Zd = fmm.sample_direct(gen, Omega, bounds)
    errs = []
    for p in (4, 8, 16):
        Yf, Zf = fmm.sample_fmm(gen, Omega, bounds, p=p)
        errs.append(max(_rel(Yf, Yd), _rel(Zf, Zd)))
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    # geometric rate: at least (3 + sqrt 8)^-p up to a modest constant
    assert errs[1] <= 1e3 * (3 + math.sqrt(8)) ** -8


def test_diagonal_block_left_out():
    d, z, rho = workloads.random_merge(300, seed=4)
    gen, _ = _gen(d, z, rho)
    K = len(gen[0])
    bounds = _bounds(K, 16)
    # Omega supported on one leaf: Y on that leaf's rows must be zero
    lo, hi = bounds[3], bounds[4]
    Omega = np.zeros((K, 3))
    Omega[lo:hi] = np.random.default_rng(0).standard_normal((hi - lo, 3))
    Yf, Zf = fmm.sample_fmm(gen, Omega, bounds, p=16)
    assert np.all(Yf[lo:hi] == 0.0) and np.all(Zf[lo:hi] == 0.0)
    assert np.linalg.norm(Yf) > 0
