"""GPU randomized HSS (Algorithms 2 and 3) against the oracle, and the HSS-ADC
solver against closed forms and the oracle."""
import numpy as np
import pytest
import torch

from oracle import dc as odc, hss as ohss, rng as orng, secular as osec, sturm
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu


def generators(d, z, rho):
    lam, gam, mu, _ = osec.secular_roots(d, z, rho)
    uh = osec.lowner_z(d, rho, gam, mu, np.sign(z))
    Q, v = osec.cauchy_vectors(d, uh, gam, mu)
    return (d, uh, gam, mu, v), Q


def gpu_build(ctx, gen, omega=None, s=0, **kw):
    d, uh, gam, mu, v = gen
    o = adc.opts(**kw)
    st, h = adc.adc_hss_build(ctx.h, len(d), cuda(d), cuda(gam), cuda(mu), cuda(uh), cuda(v),
                              cuda(omega) if omega is not None else None, s, o)
    assert st == adc.ADC_OK, adc.status_string(st)
    return h


def gpu_apply(ctx, h, X):
    P, K = X.shape
    Xg = cuda(np.asfortranarray(X).ravel(order="F"))
    Yg = torch.empty(P * K, dtype=torch.float64, device="cuda")
    st = adc.adc_hss_apply(ctx.h, h, P, Xg, P, Yg, P)
    assert st == adc.ADC_OK
    torch.cuda.synchronize()
    return Yg.cpu().numpy().reshape((K, P)).T


@pytest.mark.parametrize("K,leaf", [(2000, 128), (1000, 64), (3001, 200)])
def test_hss_same_omega_vs_oracle(ctx, K, leaf):
    print(f"hss K={K} leaf={leaf}", flush=True)
    d, u, rho = workloads.example1_merge(K, seed=1)
    gen, Q = generators(d, u, rho)
    L = ohss.hss_levels(K, leaf)
    r, bounds, _ = ohss.estimate_rank(gen[0], gen[2], gen[3], ohss.leaf_boundaries(K, L))
    s = r + 10
    Om = orng.philox_normal(K, s, 77, 0)
    # the GPU forms Phi_i / Theta_i from the off-diagonal block rows; the
    # oracle's "offdiag" reading computes the same quantities
    root, post, info = ohss.rshss(gen, Om, bounds, 1e-14, sample="offdiag")
    Ho = ohss.HSS(root, post, gen, info)
    h = gpu_build(ctx, gen, Om, s, hss_leaf=leaf)
    inf = adc.adc_hss_info(h)
    assert inf["levels"] == L and inf["samples"] == s
    # node by node: same tree; ranks within two (the truncation |R_kk| <=
    # tol |R_11| sits at the rounding level of the samples)
    gn = adc.adc_hss_nodes(h)
    om = {(n.level, n.lo): n for n in post}
    for i, g in enumerate(gn[1:], start=1):
        lvl = int(np.floor(np.log2(i + 1)))
        n = om[(lvl, g["lo"])]
        assert n.hi == g["hi"]
        assert abs(n.k_r - g["kr"]) <= 2 and abs(n.k_c - g["kc"]) <= 2, (i, g, n.k_r, n.k_c)
    X = np.random.default_rng(K).standard_normal((300, K))
    Yg = gpu_apply(ctx, h, X)
    Yo = ohss.hss_matmul_right(X, Ho)
    ref = X @ Q
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(Yg - ref)) <= 1e-12 * scale
    assert np.max(np.abs(Yg - Yo)) <= 1e-12 * scale
    # the paper's literal Y - D Omega gives another valid H of the same accuracy
    root2, post2, info2 = ohss.rshss(gen, Om, bounds, 1e-14, sample="paper")
    Yp = ohss.hss_matmul_right(X, ohss.HSS(root2, post2, gen, info2))
    assert np.max(np.abs(Yp - ref)) <= 1e-12 * scale
    # the dense expansion (X = I) matches the oracle's eq. (new-hss) expansion
    Hg = gpu_apply(ctx, h, np.eye(K))
    assert np.max(np.abs(Hg - ohss.hss_dense(Ho))) <= 1e-12
    adc.adc_hss_free(h)


def test_hss_adaptive_retry(ctx):
    print("hss adaptive", flush=True)
    d, u, rho = workloads.example1_merge(1500, seed=2)
    gen, Q = generators(d, u, rho)
    h = gpu_build(ctx, gen, None, 0, rank_mode=adc.ADC_RANK_FIXED, fixed_rank=4, hss_leaf=128)
    inf = adc.adc_hss_info(h)
    assert inf["retries"] >= 1 and inf["check_err"] <= 1e-12
    X = np.random.default_rng(0).standard_normal((64, 1500))
    assert np.max(np.abs(gpu_apply(ctx, h, X) - X @ Q)) <= 1e-11
    adc.adc_hss_free(h)


@pytest.mark.parametrize("nprobe", [1, 4, 8, 13])
def test_check_error_by_its_definition(ctx, nprobe):
    """The reported check error equals ||W^T (Q' - H)||_F / ||W^T Q'||_F with
    the probes W drawn by the oracle's Philox stream (element (i, c) is normal
    number i*nprobe + c of stream 1 for a single build), Q' from the oracle and
    W^T H by applying the handle.  A deliberately low fixed rank without
    retries makes the error large, so that rounding does not blur it."""
    print(f"check error by definition, {nprobe} probes", flush=True)
    d, u, rho = workloads.example1_merge(1500, seed=2)
    gen, Q = generators(d, u, rho)
    K = len(d)
    seed = adc.opts().seed
    h = gpu_build(ctx, gen, None, 0, rank_mode=adc.ADC_RANK_FIXED, fixed_rank=6, max_retries=0, hss_leaf=128,
                  nprobe=nprobe)
    inf = adc.adc_hss_info(h)
    W = orng.philox_normal(K, nprobe, seed, 1)
    WQ = W.T @ Q
    WH = gpu_apply(ctx, h, np.ascontiguousarray(W.T))
    want = np.linalg.norm(WQ - WH) / np.linalg.norm(WQ)
    print(f"  reported {inf['check_err']:.6e} definition {want:.6e}", flush=True)
    assert want > 1e-10
    assert abs(inf["check_err"] - want) <= 1e-8 * want
    adc.adc_hss_free(h)


def solve(ctx, a, b, **kw):
    w, Z, rep = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), **kw)
    torch.cuda.synchronize()
    return w.cpu().numpy(), Z.cpu().numpy(), rep


@pytest.mark.parametrize("N,leaf,minK", [(2048, 64, 256), (4096, 128, 512), (5000, 128, 1000)])
def test_stedc_hss_toeplitz(ctx, N, leaf, minK):
    print(f"stedc hss toeplitz N={N}", flush=True)
    a, b = workloads.toeplitz(N)
    w, Z, rep = solve(ctx, a, b, hss_leaf=leaf, hss_min_k=minK, hss_levels=-1, hss_min_flops=0)
    assert rep["hss_merges"] >= 1 and rep["hss_fallbacks"] == 0
    k = np.arange(1, N + 1)
    exact = np.sort(2 + 2 * np.cos(k * np.pi / (N + 1)))
    assert np.max(np.abs(w - exact)) <= 1e-13 * 4
    assert odc.residual(a, b, w, Z) <= 1e-13
    assert odc.orthogonality(Z) <= 1e-12


def test_stedc_hss_random_matches_oracle(ctx):
    print("stedc hss random", flush=True)
    a, b = workloads.random_uniform(3000, 9)
    w, Z, rep = solve(ctx, a, b, hss_leaf=32, hss_min_k=16, hss_levels=-1, hss_min_flops=0)
    w_o, _ = odc.stedc(a, b, leaf=32)
    assert np.max(np.abs(w - w_o)) <= 1e-13 * odc.tnorm1(a, b)
    assert odc.residual(a, b, w, Z) <= 1e-13 and odc.orthogonality(Z) <= 1e-12


@pytest.mark.parametrize("rank", [4, 48, 64])
def test_stedc_hss_retries_rebuild_failing_merges(ctx, rank):
    """Too few samples on purpose (fixed rank, no oversampling): merges that
    fail the check are rebuilt with doubled samples while the ones that
    passed keep their first HSS form; the result must still be exact."""
    print(f"stedc hss retries rank={rank}", flush=True)
    N = 8192
    a, b = workloads.toeplitz(N)
    w, Z, rep = solve(ctx, a, b, hss_leaf=128, hss_min_k=1024, hss_levels=-1, hss_min_flops=0,
                      rank_mode=adc.ADC_RANK_FIXED, fixed_rank=rank, oversample=0, max_retries=6)
    print(f"  hss merges {rep['hss_merges']} retries {rep['retries']} samples {rep['samples']}", flush=True)
    assert rep["hss_merges"] >= 3 and rep["hss_fallbacks"] == 0
    if rank == 4:
        assert rep["retries"] >= rep["hss_merges"]
    k = np.arange(1, N + 1)
    exact = np.sort(2 + 2 * np.cos(k * np.pi / (N + 1)))
    assert np.max(np.abs(w - exact)) <= 1e-13 * 4
    assert odc.residual(a, b, w, Z) <= 1e-13
    assert odc.orthogonality(Z) <= 1e-12


@pytest.mark.parametrize("case", ["toeplitz", "legendre"])
def test_stedc_dense_fallback_after_failed_check(ctx, case):
    """Two samples and no retries: every HSS merge fails the check and falls
    back to the dense update of its packed (leaf-grouped) columns, whose
    unsupported halves are zero-filled first; the result stays exact.  With
    strict, the failed check is an error."""
    print(f"stedc dense fallback {case}", flush=True)
    N = 6000
    a, b = workloads.toeplitz(N) if case == "toeplitz" else workloads.legendre(N)
    kw = dict(hss_leaf=128, hss_min_k=1024, hss_levels=-1, hss_min_flops=0, rank_mode=adc.ADC_RANK_FIXED,
              fixed_rank=2, oversample=0, max_retries=0)
    w, Z, rep = solve(ctx, a, b, **kw)
    assert rep["hss_merges"] >= 1 and rep["hss_fallbacks"] == rep["hss_merges"]
    ks = np.array([0, 1, N // 3, N // 2, N - 1])
    assert np.max(np.abs(w[ks] - sturm.eigenvalues_by_index(a, b, ks))) <= 1e-13 * odc.tnorm1(a, b)
    assert odc.residual(a, b, w, Z) <= 1e-13
    assert odc.orthogonality(Z) <= 1e-12
    with pytest.raises(adc.AdcError) as ei:
        adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), strict=1, **kw)
    assert ei.value.status == adc.ADC_ERR_ACCURACY


def test_saturation_guard_forces_retry(ctx):
    """Four samples and no oversampling saturate the interpolative
    decompositions (node ranks equal to s with more candidates than s).  With
    a check tolerance so loose that every probe error passes, the merges are
    accepted and reported as saturated; with sat_guard a saturated merge
    fails its check like a large probe error and is rebuilt with doubled
    samples, so no accepted merge saturates and the result is exact."""
    print("saturation guard", flush=True)
    N = 8192
    a, b = workloads.toeplitz(N)
    kw = dict(hss_leaf=128, hss_min_k=1024, hss_levels=-1, hss_min_flops=0, rank_mode=adc.ADC_RANK_FIXED,
              fixed_rank=4, oversample=0, max_retries=6, check_tol=1.0)
    _, _, rep = solve(ctx, a, b, **kw)
    print(f"  unguarded: merges {rep['hss_merges']} saturated {rep['hss_saturated']} nodes {rep['hss_sat_nodes']}",
          flush=True)
    assert rep["hss_merges"] >= 3 and rep["retries"] == 0
    assert rep["hss_saturated"] == rep["hss_merges"] and rep["hss_sat_nodes"] >= rep["hss_merges"]
    w, Z, rep = solve(ctx, a, b, sat_guard=1, **kw)
    print(f"  guarded: retries {rep['retries']} samples {rep['samples']} saturated {rep['hss_saturated']} "
          f"fallbacks {rep['hss_fallbacks']}", flush=True)
    assert rep["retries"] >= rep["hss_merges"] - rep["hss_fallbacks"]
    assert rep["hss_saturated"] == 0
    k = np.arange(1, N + 1)
    exact = np.sort(2 + 2 * np.cos(k * np.pi / (N + 1)))
    assert np.max(np.abs(w - exact)) <= 1e-13 * 4
    assert odc.residual(a, b, w, Z) <= 1e-13
    assert odc.orthogonality(Z) <= 1e-12
