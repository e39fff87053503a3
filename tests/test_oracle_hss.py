"""Pins of the oracle's interpolative decomposition, Algorithm 2, Algorithm 3,
the rank estimate of eq. (bounds) and the Philox generator.

Fixed by: exact reconstruction of exactly-low-rank matrices; exactness of
Algorithm 2 at full rank and zero tolerance; the dense expansion of an HSS
matrix (eq. new-hss, which is an identity of the representation, computed
here recursively and independently of Algorithm 3); the worked example after
eq. (bounds); the Philox known-answer vectors.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import hss, rng, secular as sec
from paper_1510_04591_amd import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _example(N, seed=1):
    d, u, rho = workloads.example1_merge(N, seed)
    lam, gam, mu, _ = sec.secular_roots(d, u, rho)
    uh = sec.lowner_z(d, rho, gam, mu, np.sign(u))
    Q, v = sec.cauchy_vectors(d, uh, gam, mu)
    return (d, uh, gam, mu, v), Q


@pytest.mark.parametrize("shape,r", [((40, 90), 7), ((60, 60), 1), ((25, 200), 25)])
def test_cpqr_id_exact_low_rank(shape, r):
    g = np.random.default_rng(r)
    A = g.standard_normal((shape[0], r)) @ g.standard_normal((r, shape[1]))
    J, X, _ = hss.cpqr_id(A, 1e-12)
    assert len(J) == r
    assert np.allclose(X[:, J], np.eye(r))
    assert np.max(np.abs(A[:, J] @ X - A)) <= 1e-12 * np.max(np.abs(A))


def test_cpqr_id_tolerance_on_cauchy_block():
    gen, Q = _example(1000)
    B = Q[:200, 200:]
    J, X, rd = hss.cpqr_id(B, 1e-14)
    err = np.max(np.abs(B[:, J] @ X - B))
    assert err <= 1e-12 and len(J) < 60


def test_rshss_exact_at_full_rank():
    gen, Q = _example(256, seed=3)
    K = 256
    bounds = hss.leaf_boundaries(K, 2)  # leaves of 64
    Om = rng.philox_normal(K, 200, 11, 0)  # s >= 3 * leaf: every ID is exact
    root, post, info = hss.rshss(gen, Om, bounds, 0.0)
    H = hss.HSS(root, post, gen, info)
    assert np.max(np.abs(hss.hss_dense(H) - Q)) <= 1e-13


def test_rshss_accuracy_and_alg3():
    gen, Q = _example(1200)
    K = 1200
    L = hss.hss_levels(K, 128)
    r, bounds, _ = hss.estimate_rank(gen[0], gen[2], gen[3], hss.leaf_boundaries(K, L))
    Om = rng.philox_normal(K, r + 10, 5, 0)
    root, post, info = hss.rshss(gen, Om, bounds, 1e-14)
    H = hss.HSS(root, post, gen, info)
    Hd = hss.hss_dense(H)
    assert np.max(np.abs(Hd - Q)) <= 1e-12
    assert info["max_rank"] < r + 10
    X = np.random.default_rng(0).standard_normal((77, K))
    assert np.max(np.abs(hss.hss_matmul_right(X, H) - X @ Hd)) <= 1e-12


def test_alg3_sibling_term_needed():
    """Planted mistake: the leaf step without the sibling term G_j B_j (as
    printed) misses the coupling between sibling leaves."""
    gen, Q = _example(512)
    K = 512
    bounds = hss.leaf_boundaries(K, 2)
    Om = rng.philox_normal(K, 60, 5, 0)
    root, post, info = hss.rshss(gen, Om, bounds, 1e-14)
    H = hss.HSS(root, post, gen, info)
    X = np.random.default_rng(1).standard_normal((10, K))
    good = hss.hss_matmul_right(X, H)
    # recompute leaves with F_i only
    leaves = [n for n in post if n.leaf]
    G = {n.idx: X[:, n.lo:n.hi] @ n.U for n in leaves}
    bad = good.copy()
    for n in leaves:
        p = n.parent
        j = p.right if p.left is n else p.left
        bad[:, n.lo:n.hi] -= (G[j.idx] @ j.B) @ n.V.T
    ref = X @ hss.hss_dense(H)
    assert np.max(np.abs(good - ref)) <= 1e-12 < np.max(np.abs(bad - ref))


def test_rank_bound_worked_example():
    g = json.load(open(os.path.join(GOLD, "rank_bound_example.json")))
    r = hss.rank_bound(g["R"], g["eps"])
    raw = math.log(16 / g["eps"]) * math.log(8 * g["R"]) / math.pi ** 2
    assert abs(raw - g["printed_rank"]) < 0.5
    assert r in (g["printed_rank"], g["printed_rank"] + 1)


def test_estimate_rank_rules():
    gen, Q = _example(2000)
    d, uh, gam, mu, v = gen
    b0 = hss.leaf_boundaries(2000, 4)
    r, b1, ranks = hss.estimate_rank(d, gam, mu, b0)
    assert 1 <= r <= 100 and len(ranks) == len(b0) - 2
    assert all(abs(x - y) <= 5 for x, y in zip(b0, b1))
    # a tiny cap and a huge epsilon are respected
    assert hss.estimate_rank(d, gam, mu, b0, r_cap=7)[0] == 7


def test_adaptive_check_retries_on_underestimate():
    gen, Q = _example(1500)
    d, uh, gam, mu, v = gen
    H, info = hss.adc_hss_update(d, uh, gam, mu, dict(leaf=128, p=10, seed=3, fixed_rank=4))
    assert info["retries"] >= 1
    X = np.random.default_rng(2).standard_normal((5, 1500))
    assert np.max(np.abs(hss.hss_matmul_right(X, H) - X @ Q)) <= 1e-11


def test_philox_known_answers():
    g = json.load(open(os.path.join(GOLD, "philox_kat.json")))
    h = lambda x: int(x, 16) if isinstance(x, str) else int(x)
    for v in g["vectors"]:
        c = [h(x) for x in v["ctr"]]
        k = [h(x) for x in v["key"]]
        out = rng.philox4x32(c[0], c[1], c[2], c[3], k[0], k[1])
        assert [int(o) for o in out] == [h(x) for x in v["out"]]


def test_philox_normal_moments():
    x = rng.philox_normal(4000, 16, 123, 7).ravel()
    assert abs(np.mean(x)) < 0.02 and abs(np.std(x) - 1) < 0.02
    assert not np.array_equal(rng.philox_normal(10, 3, 1, 0), rng.philox_normal(10, 3, 1, 1))
