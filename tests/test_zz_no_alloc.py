"""The allocation-free Cauchy update against the allocating one (same kernels)
and the oracle: two calls in a row on one stream, the second smaller, then a
size beyond the static scratch."""
import numpy as np
import pytest
import torch

from oracle import secular as osec
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu


def _problem(P, K, seed):
    d, z, rho = workloads.random_merge(K, seed, "uniform")
    K = len(d)
    _, gam, mu, _ = osec.secular_roots(d, z, rho)
    uh = osec.lowner_z(d, rho, gam, mu, np.sign(z))
    Qp, v = osec.cauchy_vectors(d, uh, gam, mu)
    X = np.random.default_rng(seed).standard_normal((P, K))
    return (d, gam, mu, uh, v), Qp, X


def test_noalloc_matches_allocating_entry(ctx):
    outs = []
    for P, K, seed in ((3000, 2048, 5), (1000, 700, 6)):
        print(f"noalloc cauchy_gemm P={P} K={K}", flush=True)
        gen, Qp, X = _problem(P, K, seed)
        g = [cuda(x) for x in gen]
        Xg = cuda(np.asfortranarray(X).ravel(order="F"))
        Y1 = torch.full((P * K,), np.nan, dtype=torch.float64, device="cuda")
        Y2 = torch.full((P * K,), np.nan, dtype=torch.float64, device="cuda")
        assert adc.adc_cauchy_gemm(ctx.h, P, K, *g, Xg, P, Y1, P) == adc.ADC_OK
        torch.cuda.synchronize()
        assert adc.adc_cauchy_gemm_noalloc(ctx.h, P, K, *g, Xg, P, Y2, P) == adc.ADC_OK
        torch.cuda.synchronize()
        a, b = Y1.cpu().numpy(), Y2.cpu().numpy()
        assert np.all(np.isfinite(b))
        ref = (X @ Qp).T.ravel()
        scale = max(1.0, float(np.max(np.abs(ref))))
        assert np.max(np.abs(b - a)) / scale <= 1e-13 * np.sqrt(K)
        assert np.max(np.abs(b - ref)) / scale <= 1e-13 * np.sqrt(K)
        outs.append(bool(np.array_equal(a, b)))
    print(f"  bit-identical to the allocating entry: {outs}", flush=True)


def test_noalloc_rejects_large_k(ctx):
    K = 2049
    z = torch.zeros(K, dtype=torch.float64, device="cuda")
    X = torch.zeros(4 * K, dtype=torch.float64, device="cuda")
    st = adc.adc_cauchy_gemm_noalloc(ctx.h, 4, K, z, z, z, z, z, X, 4, X.clone(), 4)
    assert st == adc.ADC_ERR_UNSUPPORTED
