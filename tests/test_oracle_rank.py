"""Pins of the oracle's rank estimate (eq. bounds with the neighbouring-segment
rules of Section 4.1) against the definitions, computed by brute force.

dist(I1, I2) is defined after eq. (dist_xy) as the smallest |d_i - lam_j| with
d_i in one segment and lam_j in the other.  Here it is evaluated over every
such pair of the two neighbouring segments, with lam_j = d_j + gam_j formed
in extended precision, independently of the oracle's two-term formula.

A note on what this can and cannot detect.  For interlacing poles and roots
(d_j < lam_j < d_{j+1}) the pair minimum across a boundary b is always
mu_{b-1} = d_b - lam_{b-1}: every pair (d left, lam right) is at least
lam_b - d_{b-1} = (d_b - d_{b-1}) + gam_b, which exceeds d_b - d_{b-1} >=
mu_{b-1}.  The oracle's min(|(d_b - d_{b-1}) + gam_b|, |mu_{b-1}|) therefore
returns mu_{b-1}, and so would the same expression with gam_{b-1} in place
of gam_b: that variant is output-equivalent and no test can tell them apart.
A variant that changes the result (mu_b instead of mu_{b-1}, the pole gap
alone, a one-sided distance) fails the pair-minimum test below.

The boundary moves (rule (1) after eq. bounds, threshold 1e-10, at most 5
rows) and the rank (eq. bounds with eps = 1e-16, rule (2) cap 100) are then
recomputed from those brute-force distances and compared with the oracle
exactly.  The inputs are chosen so that no decision sits at a rounding edge
(checked in the tests).
"""
import math

import numpy as np
import pytest

from oracle import hss, mlp, secular as sec
from paper_1510_04591_amd import workloads

EPS_RANK = 1e-16
THRESH = 1e-10
SHIFT = 5
CAP = 100


def _roots(d, z, rho):
    _, gam, mu, _ = sec.secular_roots(d, z, rho)
    return np.asarray(gam), np.asarray(mu)


def _pair_min(d, gam, seg_a, seg_b):
    """min |d_i - lam_j| over d_i in seg_a and lam_j in seg_b and the other way
    round, lam = d + gam in extended precision."""
    dl = np.asarray(d, np.longdouble)
    lam = dl + np.asarray(gam, np.longdouble)
    a0, a1 = seg_a
    b0, b1 = seg_b
    x = np.min(np.abs(dl[a0:a1][:, None] - lam[b0:b1][None, :]))
    y = np.min(np.abs(dl[b0:b1][:, None] - lam[a0:a1][None, :]))
    return float(min(x, y))


def _expected(d, gam, bounds):
    """Boundary moves and ranks recomputed from pair minima (the rules of
    Section 4.1 applied to each interior boundary in order)."""
    K = len(d)
    span = float(np.longdouble(d[K - 1]) + np.longdouble(gam[K - 1]) - np.longdouble(d[0]))
    nb = list(bounds)
    raw = []
    for t in range(1, len(nb) - 1):
        b = nb[t]
        dist = _pair_min(d, gam, (nb[t - 1], b), (b, nb[t + 1]))
        if dist < THRESH:
            lo = max(nb[t - 1] + 1, b - SHIFT)
            hi = min(nb[t + 1] - 1, b + SHIFT)
            cand = {bb: _pair_min(d, gam, (nb[t - 1], bb), (bb, nb[t + 1])) for bb in range(lo, hi + 1)}
            best = max(cand.values())
            winners = [bb for bb, v in cand.items() if v == best]
            assert len(winners) == 1
            # the winner stands clear of the runner-up: no rounding decides it
            rest = sorted(cand.values())[-2]
            assert rest < best * (1 - 1e-6)
            nb[t] = winners[0]
            dist = best
        else:
            assert dist > THRESH * 1.01
        R = span / dist
        raw.append(math.log(16.0 / EPS_RANK) * math.log(8.0 * max(R, 1.0)) / math.pi ** 2)
    for x in raw:  # no rank sits at a rounding edge of the ceiling
        assert abs(x - round(x)) > 1e-6
    ranks = [min(CAP, int(math.ceil(x))) for x in raw]
    return min(max(ranks), CAP), nb, ranks


def _planted(K=640, seed=3):
    # leaf boundaries at multiples of 80 (8 leaves): a close pair exactly at
    # 80; two close pairs at 160 and 162 (the window around 160 contains
    # another close boundary); one at 243 (inside a leaf, 3 rows after a
    # boundary: no boundary moves onto it); one at 370 (far from any
    # boundary); and a pole gap of 1e-9 at 480 (above the threshold)
    pairs = [(80, 1e-12), (160, 1e-12), (162, 1e-12), (243, 1e-12), (370, 1e-12), (480, 1e-9)]
    d, z, rho = workloads.planted_merge(K, pairs, seed)
    gam, mu = _roots(d, z, rho)
    return d, gam, mu


def _example1(K=600, seed=1):
    d, z, rho = workloads.example1_merge(K, seed)
    gam, mu = _roots(d, z, rho)
    return d, gam, mu


@pytest.mark.parametrize("case", ["example1", "planted"])
def test_boundary_dist_is_the_pair_minimum(case):
    d, gam, mu = _example1() if case == "example1" else _planted()
    K = len(d)
    bounds = hss.leaf_boundaries(K, 3)
    for t in range(1, len(bounds) - 1):
        lo, hi = bounds[t - 1], bounds[t + 1]
        # every split position inside the two leaves, not only the boundary
        for b in range(lo + 1, hi):
            ref = _pair_min(d, gam, (lo, b), (b, hi))
            got = hss.boundary_dist(d, gam, mu, b)
            assert abs(got - ref) <= 1e-5 * ref, (b, got, ref)
            assert abs(mlp._dist(d, gam, mu, b) - ref) <= 1e-5 * ref


@pytest.mark.parametrize("case", ["example1", "planted"])
def test_estimate_rank_by_brute_force(case):
    d, gam, mu = _example1() if case == "example1" else _planted()
    K = len(d)
    bounds = hss.leaf_boundaries(K, 3)
    r, nb, ranks = hss.estimate_rank(d, gam, mu, bounds)
    r_ref, nb_ref, ranks_ref = _expected(d, gam, bounds)
    assert nb == nb_ref
    assert ranks == ranks_ref
    assert r == r_ref


def test_planted_pairs_move_the_boundaries():
    d, gam, mu = _planted()
    bounds = hss.leaf_boundaries(len(d), 3)
    assert bounds[1:8] == [80, 160, 240, 320, 400, 480, 560]
    _, nb, ranks = hss.estimate_rank(d, gam, mu, bounds)
    moved = [t for t in range(1, 8) if nb[t] != bounds[t]]
    # 80 and 160 sit on close pairs and move (160 not onto 162); 240 is
    # clear although its window holds the pair at 243; 480's gap of 1e-9
    # keeps its distance above the threshold
    assert moved == [1, 2]
    assert nb[2] not in (160, 162)
    assert all(abs(nb[t] - bounds[t]) <= SHIFT for t in range(len(nb)))
    # after the moves no boundary is closer than the threshold
    for t in range(1, 8):
        assert hss.boundary_dist(d, gam, mu, nb[t]) >= THRESH


def test_rank_cap_and_unmoved_close_boundary():
    # a cluster wider than the window: every candidate stays below the
    # threshold, so the boundary keeps its best candidate and the rank is capped
    K = 256
    pairs = [(j, 1e-13) for j in range(120, 140)]
    d, z, rho = workloads.planted_merge(K, pairs, 5)
    gam, mu = _roots(d, z, rho)
    bounds = hss.leaf_boundaries(K, 1)
    r, nb, ranks = hss.estimate_rank(d, gam, mu, bounds)
    lo, hi = 128 - SHIFT, 128 + SHIFT
    cand = {bb: _pair_min(d, gam, (0, bb), (bb, K)) for bb in range(lo, hi + 1)}
    assert all(v < THRESH for v in cand.values())
    assert nb[1] == max(cand, key=cand.get)
    R = ((d[-1] + gam[-1]) - d[0]) / cand[nb[1]]
    raw = math.log(16.0 / EPS_RANK) * math.log(8.0 * R) / math.pi ** 2
    assert r == min(CAP, math.ceil(raw))
    assert hss.estimate_rank(d, gam, mu, bounds, r_cap=30)[0] == 30
