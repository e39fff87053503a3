"""Full-size solves in the configurations the benchmark times, checked on
quantities the oracle can compute one by one: eigenvalues against the
Toeplitz closed form, Sturm counts at sampled indices or the prescribed
spectrum; residual and orthogonality on the device (chunked)."""
import numpy as np
import pytest
import torch

from oracle import dc as odc, sturm
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu

HEADLINE = dict(dc_leaf=32, hss_leaf=128, hss_levels=-1, hss_min_k=2048, hss_min_flops=2.5e10, oversample=16)


def device_checks(a, b, w, Z, cb=4096):
    """||T Z - Z diag(w)||_F / (N ||T||_1) and ||Z^T Z - I||_max, in column blocks."""
    N = a.shape[0]
    ad, bd = cuda(a), cuda(b)
    res2, orth = 0.0, 0.0
    for c0 in range(0, N, cb):
        Zc = Z[:, c0:c0 + cb]
        TZ = ad[:, None] * Zc
        TZ[:-1] += bd[:, None] * Zc[1:]
        TZ[1:] += bd[:, None] * Zc[:-1]
        R = TZ - Zc * w[None, c0:c0 + cb]
        res2 += float(torch.sum(R * R))
        G = Z.t() @ Zc
        G[c0:c0 + cb].diagonal().sub_(1.0)
        orth = max(orth, float(torch.max(torch.abs(G))))
        del TZ, R, G
    return float(np.sqrt(res2)) / (N * odc.tnorm1(a, b)), orth


def test_toeplitz_32768_headline_configuration(ctx):
    print("toeplitz 32768 headline configuration", flush=True)
    N = 32768
    a, b = workloads.toeplitz(N)
    w, Z, rep = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), **HEADLINE)
    torch.cuda.synchronize()
    # HSS at the top four merge levels, as the configuration states
    assert rep["hss_per_level"][:5] == [1, 2, 4, 8, 0]
    assert rep["hss_fallbacks"] == 0
    exact = np.sort(2 + 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)))
    assert np.max(np.abs(w.cpu().numpy() - exact)) <= 1e-13 * 4
    res, orth = device_checks(a, b, w, Z)
    print(f"  resid {res:.2e} orth {orth:.2e}", flush=True)
    assert res <= 1e-13 and orth <= 1e-12


def test_random_8192_leaf64_against_dense_and_sturm(ctx):
    print("random 8192, HSS leaf 64 at K >= 2048", flush=True)
    N = 8192
    a, b = workloads.random_uniform(N, 2)
    tn = odc.tnorm1(a, b)
    w, Z, rep = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), hss_leaf=64, hss_min_k=2048, hss_min_flops=0,
                                     hss_levels=-1)
    wd, Zd, _ = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), force_dense=1)
    torch.cuda.synchronize()
    wh, wdh = w.cpu().numpy(), wd.cpu().numpy()
    assert np.max(np.abs(wh - wdh)) <= 1e-13 * tn
    ks = np.array([0, 1, 7, N // 5, N // 2, 3 * N // 4, N - 2, N - 1])
    assert np.max(np.abs(wh[ks] - sturm.eigenvalues_by_index(a, b, ks))) <= 1e-13 * tn
    res, orth = device_checks(a, b, w, Z)
    print(f"  hss merges {rep['hss_merges']} K top {rep['K_per_level'][0]} resid {res:.2e} orth {orth:.2e}",
          flush=True)
    assert res <= 1e-13 and orth <= 1e-12


def test_prescribed_uniform_spectrum_32768(ctx):
    print("prescribed uniform spectrum 32768", flush=True)
    N = 32768
    a, b = workloads.prescribed_tridiagonal("uniform", N)
    lam, _ = workloads.spectrum("uniform", N)
    w, Z, rep = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), hss_min_k=2048, hss_min_flops=0, hss_levels=-1)
    torch.cuda.synchronize()
    tn = odc.tnorm1(a, b)
    err = np.max(np.abs(w.cpu().numpy() - np.sort(lam))) / tn
    res, orth = device_checks(a, b, w, Z)
    print(f"  hss merges {rep['hss_merges']} retries {rep['retries']} eig err {err:.1e} resid {res:.2e} "
          f"orth {orth:.2e}", flush=True)
    assert rep["hss_merges"] >= 7 and rep["hss_fallbacks"] == 0
    assert err <= 1e-13
    assert res <= 1e-13 and orth <= 1e-12
