"""GPU parity of the rank estimate (eq. bounds with the boundary moves of
Section 4.1): the library's integer rank and moved leaf boundaries must equal
the oracle's exactly on the same FP64 generators.

The generators (d, gam, mu) come from the oracle's secular solver, so both
sides read identical bytes; the oracle's estimate is pinned against the
pair-minimum definition of the segment distance in test_oracle_rank.py.
Both entry points that produce the estimate are covered: adc_rank_estimate
(the solver's kernel on one merge) and adc_hss_build (its leaf nodes and its
sample count s = r + p when the first check passes)."""
import numpy as np
import pytest
from scipy.linalg import eigh_tridiagonal

from oracle import dc as odc, hss as ohss, secular as osec
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu


def _gens(d, z, rho):
    _, gam, mu, _ = osec.secular_roots(d, z, rho)
    _gens.last = (np.asarray(z), rho)
    return np.asarray(d), np.asarray(gam), np.asarray(mu)


def _toeplitz_top(N=2048):
    """The top merge of Toeplitz(2, 1) after deflation: children torn at
    N/2 (eq. T2), their eigenpairs by LAPACK, merged and deflated by the oracle."""
    a, b = workloads.toeplitz(N)
    k = N // 2
    beta = b[k - 1]
    a1 = a[:k].copy()
    a1[-1] -= beta
    a2 = a[k:].copy()
    a2[0] -= beta
    w1, Q1 = eigh_tridiagonal(a1, b[:k - 1])
    w2, Q2 = eigh_tridiagonal(a2, b[k:])
    d, z, rho, _, _ = odc.merge_vectors(w1, Q1, w2, Q2, beta)
    df = odc.deflate(d, z, rho)
    s = df["surv"]
    return df["dval"][s], df["zval"][s], rho


def _case(name):
    if name == "example1":
        return _gens(*workloads.example1_merge(3000, 1)), 128
    if name == "planted":
        pairs = [(80, 1e-12), (160, 1e-12), (162, 1e-12), (243, 1e-12), (370, 1e-12), (480, 1e-9)]
        return _gens(*workloads.planted_merge(640, pairs, 3)), 80
    if name == "toeplitz_top":
        return _gens(*_toeplitz_top()), 128
    if name == "clustered":
        return _gens(*workloads.random_merge(2500, 7, "clustered")), 64
    if name == "wide_cluster":
        pairs = [(j, 1e-13) for j in range(120, 140)]
        return _gens(*workloads.planted_merge(256, pairs, 5)), 128
    raise ValueError(name)


CASES = ["example1", "planted", "toeplitz_top", "clustered", "wide_cluster"]


@pytest.mark.parametrize("name", CASES)
def test_rank_estimate_matches_oracle(ctx, name):
    (d, gam, mu), leaf = _case(name)
    K = len(d)
    L = max(1, ohss.hss_levels(K, leaf))
    bounds = ohss.leaf_boundaries(K, L)
    r_o, nb_o, _ = ohss.estimate_rank(d, gam, mu, bounds)
    st, r, nb = adc.adc_rank_estimate(ctx.h, K, cuda(d), cuda(gam), cuda(mu), adc.opts(hss_leaf=leaf))
    assert st == adc.ADC_OK, adc.status_string(st)
    print(f"{name}: K={K} leaf={leaf} r={r} (oracle {r_o}), moved={sum(x != y for x, y in zip(nb, bounds))}")
    assert r == r_o
    assert nb == nb_o
    if name in ("planted", "wide_cluster"):
        assert nb != bounds  # the moves are exercised


@pytest.mark.parametrize("name", ["example1", "planted", "toeplitz_top"])
def test_hss_build_uses_the_estimate(ctx, name):
    """adc_hss_build draws s = r + p samples and builds on the moved leaves."""
    (d, gam, mu), leaf = _case(name)
    z, rho = _gens.last
    K = len(d)
    uh = osec.lowner_z(d, rho, gam, mu, np.sign(z))
    _, v = osec.cauchy_vectors(d, uh, gam, mu)
    L = max(1, ohss.hss_levels(K, leaf))
    r_o, nb_o, _ = ohss.estimate_rank(d, gam, mu, ohss.leaf_boundaries(K, L))
    p = 16
    o = adc.opts(hss_leaf=leaf, oversample=p)
    st, h = adc.adc_hss_build(ctx.h, K, cuda(d), cuda(gam), cuda(mu), cuda(uh), cuda(v), None, 0, o)
    assert st == adc.ADC_OK, adc.status_string(st)
    try:
        info = adc.adc_hss_info(h)
        nodes = adc.adc_hss_nodes(h)
    finally:
        adc.adc_hss_free(h)
    assert info["retries"] == 0
    assert info["samples"] == r_o + p
    # heap order: the last 2^L nodes are the leaves, left to right
    leaf_nodes = nodes[len(nodes) - (1 << L):]
    assert [n["lo"] for n in leaf_nodes] + [leaf_nodes[-1]["hi"]] == nb_o


def test_rank_estimate_errors(ctx):
    (d, gam, mu), leaf = _case("planted")
    K = len(d)
    st, _, _ = adc.adc_rank_estimate(ctx.h, K, cuda(d), cuda(gam), cuda(mu), adc.opts(hss_leaf=leaf), cap=4)
    assert st == adc.ADC_ERR_ARG  # 9 boundaries do not fit in 4
    st, _, _ = adc.adc_rank_estimate(ctx.h, 1, cuda(d), cuda(gam), cuda(mu), adc.opts(hss_leaf=leaf))
    assert st == adc.ADC_ERR_ARG
    st, _, _ = adc.adc_rank_estimate(ctx.h, K, cuda(d), cuda(gam), cuda(mu), adc.opts(hss_leaf=8))
    assert st == adc.ADC_ERR_ARG  # invalid options
