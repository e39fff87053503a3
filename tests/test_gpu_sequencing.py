"""Levels sequenced on the device against levels sequenced by the host.

A level on which no merge can take the HSS route runs with worst-case
launches and device-built GEMM problems; a level where HSS is possible but
no merge qualifies runs the host-sequenced route with the dense update.
Both use the same kernels in the same configuration, so the results must
be identical bit for bit, and so must the report's integer counts and the
dense update's counted work.  Also: a solve without a report, a solve whose
top level is host-sequenced above device-sequenced levels with HSS at the
top, and the oracle's eigenvalues for all of them."""
import numpy as np
import pytest
import torch

from oracle import dc as odc
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu


def run(ctx, a, b, rep=True, **kw):
    n = len(a)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    Zt = torch.empty((n, n), dtype=torch.float64, device="cuda")
    r = adc.adc_report() if rep else None
    st = adc.adc_stedc(ctx.h, n, cuda(a), cuda(b), w, Zt, n, None, 0, adc.opts(**kw), r)
    assert st == adc.ADC_OK, adc.status_string(st)
    torch.cuda.synchronize()
    return w.cpu().numpy(), Zt.t().cpu().numpy(), (r.as_dict() if rep else None)


@pytest.mark.parametrize("kind", ["toeplitz", "random"])
def test_host_and_device_levels_agree_bitwise(ctx, kind):
    N = 4096
    print(f"sequencing {kind} N={N}", flush=True)
    a, b = workloads.toeplitz(N) if kind == "toeplitz" else workloads.random_uniform(N, 9)
    # every level on the device
    w_d, Z_d, r_d = run(ctx, a, b, force_dense=1)
    # the top level host-sequenced (2 n^3 reaches the threshold) but no merge
    # takes HSS (its dense update stays below it); the levels below on the device
    w_h, Z_h, r_h = run(ctx, a, b, hss_min_k=2048, hss_min_flops=1.2e11, hss_levels=-1)
    assert r_h["hss_merges"] == 0
    assert np.array_equal(w_d, w_h)
    assert np.array_equal(Z_d, Z_h)
    for key in ("K_per_level", "n_per_level", "hss_per_level"):
        assert r_d[key] == r_h[key], key
    assert r_d["merges"] == r_h["merges"] and r_d["levels"] == r_h["levels"]
    assert r_d["phase_flops"][4] == r_h["phase_flops"][4]
    assert r_d["phase_bytes"][4] == r_h["phase_bytes"][4]
    # the oracle: eigenvalues, residual, orthogonality
    w_o, _ = odc.stedc(a, b, leaf=32)
    tn = odc.tnorm1(a, b)
    assert np.max(np.abs(w_d - w_o)) <= 1e-13 * tn
    assert odc.residual(a, b, w_d, Z_d) <= 1e-13
    assert odc.orthogonality(Z_d) <= 1e-12


def test_without_report(ctx):
    """The counts of device-sequenced levels are read back only for a
    report; without one the solve is the same bit for bit."""
    N = 3000
    print(f"no report N={N}", flush=True)
    a, b = workloads.random_uniform(N, 4)
    w_r, Z_r, _ = run(ctx, a, b, force_dense=1)
    w_n, Z_n, _ = run(ctx, a, b, rep=False, force_dense=1)
    assert np.array_equal(w_r, w_n) and np.array_equal(Z_r, Z_n)


def test_hss_top_over_device_levels(ctx):
    """HSS at the top level only (hss_levels=1): the levels below are
    sequenced on the device, the top one by the host with HSS."""
    N = 6000
    print(f"hss top N={N}", flush=True)
    a, b = workloads.toeplitz(N)
    w, Z, r = run(ctx, a, b, hss_min_k=512, hss_leaf=64, hss_levels=1, hss_min_flops=0)
    assert r["hss_per_level"][0] == 1 and sum(r["hss_per_level"][1:r["levels"]]) == 0
    exact = np.sort(2 + 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)))
    tn = odc.tnorm1(a, b)
    assert np.max(np.abs(w - exact)) <= 1e-13 * tn
    assert odc.residual(a, b, w, Z) <= 1e-13
    assert odc.orthogonality(Z) <= 1e-12
    # the same levels below the top as a solve that is dense everywhere
    w_d, _, r_d = run(ctx, a, b, force_dense=1)
    assert r["K_per_level"][1:r["levels"]] == r_d["K_per_level"][1:r_d["levels"]]
