"""Full eigendecomposition on the GPU vs the oracle and closed forms."""
import numpy as np
import pytest
import torch

from oracle import dc as odc, sturm
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu


def solve(ctx, a, b, **kw):
    w, Z, rep = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b) if len(a) > 1 else None, **kw)
    torch.cuda.synchronize()
    return w.cpu().numpy(), Z.cpu().numpy(), rep


def check_result(a, b, w, Z, w_ref, res_tol=1e-13, orth_tol=1e-12):
    tn = odc.tnorm1(a, b) if len(a) > 1 else abs(a[0])
    assert np.max(np.abs(w - w_ref)) <= 1e-13 * max(tn, 1e-300)
    assert np.all(np.diff(w) >= 0)
    assert odc.residual(a, b, w, Z) <= res_tol
    assert odc.orthogonality(Z) <= orth_tol


@pytest.mark.parametrize("N", [1, 2, 3, 32, 33, 64, 65, 100, 1024])
def test_toeplitz_dense(ctx, N):
    print(f"toeplitz N={N}", flush=True)
    a, b = workloads.toeplitz(N)
    w, Z, rep = solve(ctx, a, b, force_dense=1)
    k = np.arange(1, N + 1)
    exact = np.sort(2 + 2 * np.cos(k * np.pi / (N + 1)))
    check_result(a, b, w, Z, exact)


@pytest.mark.parametrize("N,seed", [(64, 1), (200, 2), (1000, 3), (2048, 2)])
def test_random_dense_vs_oracle(ctx, N, seed):
    print(f"random N={N} seed={seed}", flush=True)
    a, b = workloads.random_uniform(N, seed)
    w, Z, rep = solve(ctx, a, b, force_dense=1)
    w_o, Z_o = odc.stedc(a, b, leaf=32)
    check_result(a, b, w, Z, w_o)
    ks = np.array([0, N // 3, N - 1])
    assert np.max(np.abs(w[ks] - sturm.eigenvalues_by_index(a, b, ks))) <= 1e-13 * odc.tnorm1(a, b)


def glued(copies, m=20, glue=1e-10, seed=7):
    """copies of one random m x m tridiagonal block joined by tiny off-diagonals:
    every eigenvalue of the block appears `copies` times to within ~glue, so
    deflation meets chains of nearly equal poles."""
    rng = np.random.default_rng(seed)
    a0 = rng.uniform(-1, 1, m)
    b0 = rng.uniform(0.1, 1, m - 1)
    a = np.tile(a0, copies)
    b = np.concatenate([np.concatenate([b0, [glue]]) for _ in range(copies)])[:-1]
    return a, b


@pytest.mark.parametrize("leaf", [2, 3, 17, 63, 64])
def test_leaf_sizes_vs_oracle(ctx, leaf):
    """The DC leaf sizes the options allow, at both ends and between: the leaf
    eigensolves (their LDS sized to the leaf; above 63 rows more than the
    default dynamic LDS) and the tree above them against the oracle with the
    same leaf size, with equal deflation counts per level; a matrix that is a
    single leaf against its closed form."""
    print(f"leaf size {leaf}", flush=True)
    a, b = workloads.random_uniform(700, 9)
    w, Z, rep = solve(ctx, a, b, force_dense=1, dc_leaf=leaf)
    rep_o = {}
    w_o, _ = odc.stedc(a, b, leaf=leaf, report=rep_o)
    check_result(a, b, w, Z, w_o)
    lev = odc.split_tree(len(a), leaf)
    idx = 0
    for t in range(len(lev) - 1, -1, -1):
        cnt = sum(1 for (s0, m) in lev[t] if m > leaf)
        if cnt:
            k = sum(rep_o["merges"][idx + u]["K"] for u in range(cnt))
            assert rep["K_per_level"][t] == k, (t, rep["K_per_level"][t], k)
            idx += cnt
    a, b = workloads.toeplitz(leaf)
    w, Z, rep = solve(ctx, a, b, force_dense=1, dc_leaf=leaf)
    assert rep["merges"] == 0
    k = np.arange(1, leaf + 1)
    check_result(a, b, w, Z, np.sort(2 + 2 * np.cos(k * np.pi / (leaf + 1))))


@pytest.mark.parametrize("kind", ["toeplitz", "random", "glued"])
def test_deflation_counts_match_oracle(ctx, kind):
    """Integer parity: the number of survivors of deflation, summed per tree
    level, equals the oracle's (same tolerance, same scan order)."""
    print(f"deflation counts {kind}", flush=True)
    if kind == "toeplitz":
        a, b = workloads.toeplitz(3000)
    elif kind == "random":
        a, b = workloads.random_uniform(3000, 5)
    else:
        a, b = glued(120)
    w, Z, rep = solve(ctx, a, b, force_dense=1)
    rep_o = {}
    w_o, _ = odc.stedc(a, b, leaf=32, report=rep_o)
    # oracle merges in processing order: deepest level first, left to right
    lev = odc.split_tree(len(a), 32)
    per = []
    idx = 0
    for t in range(len(lev) - 1, -1, -1):
        cnt = sum(1 for (s0, m) in lev[t] if m > 32)
        if cnt:
            per.append((t, sum(rep_o["merges"][idx + u]["K"] for u in range(cnt))))
            idx += cnt
    for t, k in per:
        assert rep["K_per_level"][t] == k, (t, rep["K_per_level"][t], k)
    check_result(a, b, w, Z, w_o)


def test_glued_clusters(ctx):
    print("glued clusters", flush=True)
    a, b = glued(200, glue=1e-12)
    w, Z, rep = solve(ctx, a, b, force_dense=1)
    ks = np.array([0, 1, 2, 1000, len(a) - 1])
    ref = sturm.eigenvalues_by_index(a, b, ks)
    assert np.max(np.abs(w[ks] - ref)) <= 1e-13 * odc.tnorm1(a, b)
    assert odc.residual(a, b, w, Z) <= 1e-13 and odc.orthogonality(Z) <= 1e-12
