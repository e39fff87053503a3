"""Level-batched solver (many matrices, one launch per phase and level, HIP
graph replay) vs the oracle, closed forms and Sturm counts."""
import numpy as np
import pytest
import torch

from oracle import dc as odc, sturm
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu


def run_batch(ctx, mats, reps=1, **kw):
    ns = [len(a) for a, _ in mats]
    ds = [cuda(a) for a, _ in mats]
    os_ = [cuda(b) if len(a) > 1 else None for a, b in mats]
    ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in ns]
    Zs = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n in ns]
    o = adc.opts(**kw)
    outs = []
    for _ in range(reps):
        rep = adc.adc_report()
        st = adc.adc_stedc_batched(ctx.h, ns, ds, os_, ws, Zs, ns, o, rep)
        assert st == adc.ADC_OK, adc.status_string(st)
        torch.cuda.synchronize()
        outs.append(([w.clone() for w in ws], [Z.clone() for Z in Zs], rep.as_dict()))
    return outs


def test_mixed_small_batch_vs_oracle(ctx):
    """Sizes around the leaf size and the tile sizes, Toeplitz and random."""
    print("mixed small batch", flush=True)
    sizes = [1, 2, 31, 32, 33, 64, 65, 100, 257, 1000]
    mats = []
    for i, n in enumerate(sizes):
        mats.append(workloads.toeplitz(n) if i % 2 == 0 else workloads.random_uniform(n, 30 + i))
    (ws, Zs, rep), = run_batch(ctx, mats, force_dense=1)
    for (a, b), w, Zt in zip(mats, ws, Zs):
        w = w.cpu().numpy()
        Z = Zt.t().cpu().numpy()
        n = len(a)
        if n == 1:
            assert w[0] == a[0] and abs(abs(Z[0, 0]) - 1.0) == 0.0
            continue
        w_o, _ = odc.stedc(a, b, leaf=32)
        tn = odc.tnorm1(a, b)
        assert np.max(np.abs(w - w_o)) <= 1e-13 * tn, n
        assert np.all(np.diff(w) >= 0)
        assert odc.residual(a, b, w, Z) <= 1e-13 and odc.orthogonality(Z) <= 1e-12, n


def test_leaf_64_batch_and_replay(ctx):
    """The largest leaf size through the batched solver: the leaves' LDS
    above the default dynamic limit, eager call and graph replay, against the
    oracle with the same leaf size."""
    print("batched leaf 64", flush=True)
    mats = [workloads.random_uniform(500, 61), workloads.toeplitz(64), workloads.random_uniform(129, 62)]
    outs = run_batch(ctx, mats, reps=2, force_dense=1, dc_leaf=64)
    for i, (a, b) in enumerate(mats):
        w = outs[0][0][i].cpu().numpy()
        Z = outs[0][1][i].t().cpu().numpy()
        w_o, _ = odc.stedc(a, b, leaf=64)
        assert np.max(np.abs(w - w_o)) <= 1e-13 * odc.tnorm1(a, b)
        assert odc.residual(a, b, w, Z) <= 1e-13 and odc.orthogonality(Z) <= 1e-12
        assert np.array_equal(w, outs[1][0][i].cpu().numpy())
        assert np.array_equal(outs[0][1][i].cpu().numpy(), outs[1][1][i].cpu().numpy())


def test_deflation_counts_match_oracle(ctx):
    """Integer parity: survivors of deflation summed per tree depth over the
    batch equal the oracle's."""
    mats = [workloads.toeplitz(700), workloads.random_uniform(900, 41), workloads.toeplitz(1500),
            workloads.random_uniform(300, 42)]
    (ws, Zs, rep), = run_batch(ctx, mats, force_dense=1)
    expect = {}
    for a, b in mats:
        rep_o = {}
        odc.stedc(a, b, leaf=32, report=rep_o)
        lev = odc.split_tree(len(a), 32)
        idx = 0
        for t in range(len(lev) - 1, -1, -1):
            cnt = sum(1 for (s0, m) in lev[t] if m > 32)
            if cnt:
                expect[t] = expect.get(t, 0) + sum(rep_o["merges"][idx + u]["K"] for u in range(cnt))
                idx += cnt
    for t, k in expect.items():
        assert rep["K_per_level"][t] == k, (t, rep["K_per_level"][t], k)


def test_graph_replays_match_the_eager_call(ctx):
    """The first call runs eagerly and captures; later calls replay the graph.
    Every replay, with unrelated eager work and synchronisations between
    them, gives the eager call's results bit for bit."""
    print("graph replays", flush=True)
    mats = [workloads.toeplitz(513), workloads.random_uniform(777, 43), workloads.toeplitz(64)]
    outs = []
    ns = [len(a) for a, _ in mats]
    ds = [cuda(a) for a, _ in mats]
    os_ = [cuda(b) for _, b in mats]
    ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in ns]
    Zs = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n in ns]
    o = adc.opts(force_dense=1)
    for r in range(4):
        for Z in Zs:
            Z.fill_(float("nan"))
        st = adc.adc_stedc_batched(ctx.h, ns, ds, os_, ws, Zs, ns, o, None)
        assert st == adc.ADC_OK
        torch.cuda.synchronize()
        outs.append(([w.cpu().numpy() for w in ws], [Z.cpu().numpy() for Z in Zs]))
        x = torch.randn(512, 512, device="cuda", dtype=torch.float64)
        (x @ x).sum().item()  # eager work between replays
    for r in range(1, 4):
        for a_, b_ in zip(outs[0][0], outs[r][0]):
            assert np.array_equal(a_, b_)
        for a_, b_ in zip(outs[0][1], outs[r][1]):
            assert np.array_equal(a_, b_)
    # new output buffers (pointer refresh before the replay)
    ws2 = [torch.empty(n, dtype=torch.float64, device="cuda") for n in ns]
    Zs2 = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n in ns]
    assert adc.adc_stedc_batched(ctx.h, ns, ds, os_, ws2, Zs2, ns, o, None) == adc.ADC_OK
    torch.cuda.synchronize()
    for w, w0 in zip(ws2, outs[0][0]):
        assert np.array_equal(w.cpu().numpy(), w0)
    for Z, Z0 in zip(Zs2, outs[0][1]):
        assert np.array_equal(Z.cpu().numpy(), Z0)


def gpu_checks(a, b, w, Zt):
    """Residual ||TZ - Z diag(w)||_F / (n ||T||_1) and ||Z^T Z - I||_max on
    the device (Zt is the row-major buffer, Z = Zt^T)."""
    ad = cuda(a)
    bd = cuda(b)
    Z = Zt.t()
    TZ = ad[:, None] * Z
    TZ[:-1] += bd[:, None] * Z[1:]
    TZ[1:] += bd[:, None] * Z[:-1]
    R = TZ - Z * w[None, :]
    n = len(a)
    tn = odc.tnorm1(a, b)
    res = float(torch.linalg.norm(R)) / (n * tn)
    G = Zt @ Zt.t()
    G.diagonal().sub_(1.0)
    return res, float(G.abs().max())


def test_full_batch_256_matrices(ctx):
    """The benchmark's batch at full size (256 matrices, N in [200, 4000],
    half Toeplitz, half random): every matrix by residual and orthogonality,
    closed-form spectra for the Toeplitz half, Sturm-count eigenvalues at
    sampled indices for the random half."""
    print("full batch", flush=True)
    mats = workloads.batched(256, 4)
    outs = run_batch(ctx, mats, reps=2, force_dense=1)
    ws, Zs, rep = outs[1]
    for i, ((a, b), w, Zt) in enumerate(zip(mats, ws, Zs)):
        n = len(a)
        res, orth = gpu_checks(a, b, w, Zt)
        assert res <= 1e-13 and orth <= 1e-12, (i, n, res, orth)
        wh = w.cpu().numpy()
        tn = odc.tnorm1(a, b)
        if i < 128:
            k = np.arange(1, n + 1)
            assert np.max(np.abs(wh - np.sort(2 + 2 * np.cos(k * np.pi / (n + 1))))) <= 1e-13 * tn
        else:
            ks = np.array([0, n // 2, n - 1])
            assert np.max(np.abs(wh[ks] - sturm.eigenvalues_by_index(a, b, ks))) <= 1e-13 * tn
        assert np.array_equal(wh, outs[0][0][i].cpu().numpy())


@pytest.mark.parametrize("variant", ["default", "direct_sampling", "retries", "fallback", "split"])
def test_batch_with_hss_matrices_vs_oracle(ctx, variant):
    """A batch mixing matrices that take the HSS route (solved together, one
    level loop over all of them) with small dense ones (graph path): every
    result against the oracle / closed form, the HSS merges counted once per
    merge, and the HSS-eligible matrices' level counts equal to solo solves
    with the same options (the forest changes the launches, not the
    deflation)."""
    print(f"batch with HSS matrices ({variant})", flush=True)
    kw = dict(hss_min_k=512, hss_leaf=64, hss_levels=-1, hss_min_flops=0)
    if variant == "direct_sampling":
        kw["sample_mode"] = adc.ADC_SAMPLE_DIRECT
    elif variant == "retries":
        # too few samples: merges of the forest fail the check and are rebuilt
        kw.update(rank_mode=adc.ADC_RANK_FIXED, fixed_rank=4, oversample=0, max_retries=6)
    elif variant == "fallback":
        # two samples, no retry: every HSS merge falls back to the dense update
        kw.update(rank_mode=adc.ADC_RANK_FIXED, fixed_rank=2, oversample=0, max_retries=0)
    elif variant == "split":
        # a group bound of 400 MB: the HSS-eligible matrices form three
        # groups (3000 + 2500, then 4097 alone although it exceeds the bound,
        # then 2000)
        kw["batch_bytes"] = 400e6
    mats = [workloads.toeplitz(3000), workloads.random_uniform(300, 51), workloads.clement(2500),
            workloads.toeplitz(4097), workloads.random_uniform(40, 52), workloads.legendre(2000)]
    (ws, Zs, rep), = run_batch(ctx, mats, **kw)
    assert rep["hss_merges"] > 0
    if variant == "retries":
        assert rep["retries"] > 0
    if variant == "fallback":
        assert rep["hss_fallbacks"] == rep["hss_merges"]
    hss_solo = 0
    for (a, b), w, Zt in zip(mats, ws, Zs):
        w = w.cpu().numpy()
        Z = Zt.t().cpu().numpy()
        n = len(a)
        tn = odc.tnorm1(a, b)
        w_o, _ = odc.stedc(a, b, leaf=32)
        assert np.max(np.abs(w - w_o)) <= 1e-13 * tn, n
        assert np.all(np.diff(w) >= 0)
        assert odc.residual(a, b, w, Z) <= 1e-13 and odc.orthogonality(Z) <= 1e-12, n
        if n >= 512:
            ws1, Z1, r1 = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), **kw)
            hss_solo += r1["hss_merges"]
    assert rep["hss_merges"] == hss_solo
