"""Fast sampling on the GPU (adc_hss_sample, sample_mode FMM) against the
samples by their definition (oracle: dense Cauchy-like matrix with zeroed
diagonal leaf blocks), against the oracle's FMM, and the whole solver with
fast sampling against closed forms."""
import math

import numpy as np
import pytest
import torch

from oracle import dc as odc, fmm as ofmm, hss as ohss, secular as osec
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu


def generators(d, z, rho):
    lam, gam, mu, _ = osec.secular_roots(d, z, rho)
    uh = osec.lowner_z(d, rho, gam, mu, np.sign(z))
    _, v = osec.cauchy_vectors(d, uh, gam, mu)
    return (d, uh, gam, mu, v)


def merge_case(case):
    if case == "example1":
        return workloads.example1_merge(1500, seed=2)
    if case == "paired":
        n1 = 700
        k = np.arange(1, n1 + 1)
        lam1 = 2 + 2 * np.cos(k * math.pi / (n1 + 1))
        d = np.sort(np.concatenate([lam1 - 1e-3 * k / n1, lam1 + 1e-3 * k / n1]))
        z = np.random.default_rng(5).standard_normal(len(d))
        return d, z / np.linalg.norm(z), 1.0
    if case == "geometric":
        K = 1800
        d = 10.0 ** (-6.0 * np.arange(K)[::-1] / (K - 1))
        z = np.random.default_rng(6).standard_normal(K)
        return d, z / np.linalg.norm(z), 0.7
    return workloads.random_merge(2100, seed=7, spread=case)


def gpu_sample(ctx, gen, Omega, mode, leaf, order=20):
    d, uh, gam, mu, v = gen
    K, s = Omega.shape
    phi = torch.empty(K * s, dtype=torch.float64, device="cuda")
    theta = torch.empty(K * s, dtype=torch.float64, device="cuda")
    o = adc.opts(hss_leaf=leaf, sample_mode=mode, fmm_order=order)
    st = adc.adc_hss_sample(ctx.h, K, cuda(d), cuda(gam), cuda(mu), cuda(uh), cuda(v),
                            cuda(np.ascontiguousarray(Omega)), s, o, phi, theta)
    assert st == adc.ADC_OK, adc.status_string(st)
    torch.cuda.synchronize()
    return phi.cpu().numpy().reshape(K, s), theta.cpu().numpy().reshape(K, s)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("case,leaf,s", [("example1", 64, 24), ("paired", 32, 70), ("clustered", 128, 33),
                                         ("normal", 64, 96), ("uniform", 16, 9), ("geometric", 64, 40)])
def test_fmm_sampling_matches_definition(ctx, case, leaf, s):
    print(f"fmm sampling {case} leaf={leaf} s={s}", flush=True)
    gen = generators(*merge_case(case))
    K = len(gen[0])
    Omega = np.random.default_rng(3).standard_normal((K, s))
    bounds = ohss.leaf_boundaries(K, max(1, ohss.hss_levels(K, leaf)))
    Yd, Zd = ofmm.sample_direct(gen, Omega, bounds)
    Yf, Zf = gpu_sample(ctx, gen, Omega, adc.ADC_SAMPLE_FMM, leaf)
    Yg, Zg = gpu_sample(ctx, gen, Omega, adc.ADC_SAMPLE_DIRECT, leaf)
    print(f"  fmm {rel(Yf, Yd):.1e} {rel(Zf, Zd):.1e}  direct {rel(Yg, Yd):.1e} {rel(Zg, Zd):.1e}", flush=True)
    assert rel(Yg, Yd) <= 1e-14 and rel(Zg, Zd) <= 1e-14
    assert rel(Yf, Yd) <= 1e-13 and rel(Zf, Zd) <= 1e-13
    # the same algorithm on the CPU: agreement to rounding
    Yo, Zo = ofmm.sample_fmm(gen, Omega, bounds, p=20)
    assert rel(Yf, Yo) <= 1e-14 and rel(Zf, Zo) <= 1e-14


def test_fmm_order_controls_error(ctx):
    gen = generators(*merge_case("uniform"))
    K = len(gen[0])
    Omega = np.random.default_rng(4).standard_normal((K, 16))
    Yg, Zg = gpu_sample(ctx, gen, Omega, adc.ADC_SAMPLE_DIRECT, 64)
    errs = []
    for p in (6, 12, 24):
        Yf, Zf = gpu_sample(ctx, gen, Omega, adc.ADC_SAMPLE_FMM, 64, order=p)
        errs.append(max(rel(Yf, Yg), rel(Zf, Zg)))
    print("  errors by order", errs, flush=True)
    assert errs[0] > 100 * errs[1] and errs[2] <= 1e-14


def test_fmm_sampling_rejects_bad_order(ctx):
    gen = generators(*merge_case("example1"))
    d, uh, gam, mu, v = gen
    K = len(d)
    phi = torch.empty(K * 4, dtype=torch.float64, device="cuda")
    o = adc.opts(sample_mode=adc.ADC_SAMPLE_FMM, fmm_order=40)
    st = adc.adc_hss_sample(ctx.h, K, cuda(d), cuda(gam), cuda(mu), cuda(uh), cuda(v), cuda(np.ones((K, 4))), 4, o,
                            phi, phi)
    assert st == adc.ADC_ERR_ARG


@pytest.mark.parametrize("N", [8192, 20000])
def test_solver_with_fast_sampling(ctx, N):
    """Toeplitz: the same eigenvalues (closed form), residual and
    orthogonality with fast and with direct sampling."""
    print(f"solver fast sampling toeplitz N={N}", flush=True)
    a, b = workloads.toeplitz(N)
    k = np.arange(1, N + 1)
    exact = np.sort(2 + 2 * np.cos(k * np.pi / (N + 1)))
    res = {}
    for mode in (adc.ADC_SAMPLE_FMM, adc.ADC_SAMPLE_DIRECT):
        w, Z, rep = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), hss_min_k=2048, hss_min_flops=0, hss_levels=-1,
                                         sample_mode=mode)
        torch.cuda.synchronize()
        wh = w.cpu().numpy()
        assert rep["hss_merges"] >= 3 and rep["hss_fallbacks"] == 0
        assert np.max(np.abs(wh - exact)) <= 1e-13 * 4
        ad, bd = cuda(a), cuda(b)
        TZ = ad[:, None] * Z
        TZ[:-1] += bd[:, None] * Z[1:]
        TZ[1:] += bd[:, None] * Z[:-1]
        resid = float(torch.linalg.norm(TZ - Z * w[None, :])) / (N * 4)
        G = Z.t() @ Z
        G.diagonal().sub_(1.0)
        orth = float(G.abs().max())
        res[mode] = (resid, orth, rep["retries"], rep["samples"])
        del Z, TZ, G
    print("  ", res, flush=True)
    for resid, orth, _, _ in res.values():
        assert resid <= 1e-13 and orth <= 1e-12


def test_hss_from_fast_samples_as_accurate_as_from_direct(ctx):
    """adc_hss_build with fast and with direct sampling: the adaptive check
    measures the same approximation error."""
    gen = generators(*merge_case("example1"))
    d, uh, gam, mu, v = gen
    K = len(d)
    errs = {}
    for mode in (adc.ADC_SAMPLE_FMM, adc.ADC_SAMPLE_DIRECT):
        o = adc.opts(hss_leaf=64, sample_mode=mode)
        st, h = adc.adc_hss_build(ctx.h, K, cuda(d), cuda(gam), cuda(mu), cuda(uh), cuda(v), None, 0, o)
        assert st == adc.ADC_OK
        errs[mode] = adc.adc_hss_info(h)["check_err"]
        adc.adc_hss_free(h)
    print("  check errors", errs, flush=True)
    e1, e2 = errs[adc.ADC_SAMPLE_FMM], errs[adc.ADC_SAMPLE_DIRECT]
    assert 0 < e1 <= 1e-13 and 0 < e2 <= 1e-13
    assert abs(e1 - e2) <= 0.5 * max(e1, e2)
