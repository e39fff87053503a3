"""GPU parity of the merge-step kernels against the oracle (same inputs)."""
import numpy as np
import pytest
import torch

from oracle import secular as osec
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def gpu_secular(ctx, d, z, rho):
    K = len(d)
    dd, zz = cuda(d), cuda(z)
    lam = torch.empty(K, dtype=torch.float64, device="cuda")
    gam = torch.empty_like(lam)
    mu = torch.empty_like(lam)
    st = adc.adc_secular(ctx.h, K, dd, zz, rho, lam, gam, mu)
    assert st == adc.ADC_OK, adc.status_string(st)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), gam.cpu().numpy(), mu.cpu().numpy()


CASES = [(1, 0, "uniform"), (2, 1, "uniform"), (3, 2, "normal"), (64, 3, "uniform"), (100, 4, "clustered"),
         (1000, 5, "normal"), (1111, 6, "clustered"), (4097, 7, "uniform")]


@pytest.mark.parametrize("K,seed,spread", CASES)
def test_secular_parity(ctx, K, seed, spread):
    d, z, rho = workloads.random_merge(K, seed, spread)
    K = len(d)
    print(f"secular K={K} seed={seed} spread={spread}", flush=True)
    lam_g, gam_g, mu_g = gpu_secular(ctx, d, z, rho)
    lam_o, gam_o, mu_o, _ = osec.secular_roots(d, z, rho)
    scale = max(np.max(np.abs(d)), rho)
    assert np.max(np.abs(lam_g - lam_o)) <= 1e-13 * scale
    # the small distance to the nearer pole agrees to a few ulps of itself
    small_g = np.minimum(gam_g, mu_g)
    small_o = np.minimum(gam_o, mu_o)
    rel = np.abs(small_g - small_o) / small_o
    assert np.max(rel) <= 1e-12, (np.max(rel), np.argmax(rel))
    # interlacing (Theorem 1)
    assert np.all(gam_g > 0) and np.all(mu_g[:-1] > 0)


@pytest.mark.parametrize("K,seed,spread", CASES)
def test_lowner_parity(ctx, K, seed, spread):
    d, z, rho = workloads.random_merge(K, seed, spread)
    K = len(d)
    print(f"lowner K={K} seed={seed}", flush=True)
    lam_o, gam_o, mu_o, _ = osec.secular_roots(d, z, rho)
    uh_o = osec.lowner_z(d, rho, gam_o, mu_o, np.sign(z))
    _, v_o = osec.cauchy_vectors(d, uh_o, gam_o, mu_o)
    uh = torch.empty(K, dtype=torch.float64, device="cuda")
    v = torch.empty_like(uh)
    st = adc.adc_lowner(ctx.h, K, cuda(d), cuda(z), rho, cuda(gam_o), cuda(mu_o), uh, v)
    assert st == adc.ADC_OK
    torch.cuda.synchronize()
    uh_g, v_g = uh.cpu().numpy(), v.cpu().numpy()
    # products of K factors: relative rounding ~ K eps
    assert np.max(np.abs(uh_g - uh_o) / np.abs(uh_o)) <= 4 * K * EPS + 1e-14
    assert np.max(np.abs(v_g - v_o) / np.abs(v_o)) <= 4 * K * EPS + 1e-14


@pytest.mark.parametrize("P,K", [(1, 1), (37, 5), (128, 128), (300, 257), (1000, 700)])
def test_cauchy_gemm_parity(ctx, P, K):
    print(f"cauchy_gemm P={P} K={K}", flush=True)
    d, z, rho = workloads.random_merge(K, 11 + K, "uniform")
    K = len(d)
    lam, gam, mu, _ = osec.secular_roots(d, z, rho)
    uh = osec.lowner_z(d, rho, gam, mu, np.sign(z))
    Qp, v = osec.cauchy_vectors(d, uh, gam, mu)
    X = np.random.default_rng(P).standard_normal((P, K))
    Xg = cuda(np.asfortranarray(X).ravel(order="F"))
    Yg = torch.empty(P * K, dtype=torch.float64, device="cuda")
    st = adc.adc_cauchy_gemm(ctx.h, P, K, cuda(d), cuda(gam), cuda(mu), cuda(uh), cuda(v), Xg, P, Yg, P)
    assert st == adc.ADC_OK
    torch.cuda.synchronize()
    Y = Yg.cpu().numpy().reshape((K, P)).T
    ref = X @ Qp
    err = np.max(np.abs(Y - ref)) / max(1.0, np.max(np.abs(ref)))
    assert err <= 1e-13 * np.sqrt(K), err
