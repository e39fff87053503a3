"""Benchmark: full symmetric tridiagonal eigendecomposition on one MI355X.

Workload (the headline configuration): N = 32768 tridiagonal Toeplitz
(diagonal 2, off-diagonal 1), DC leaf 32, randomized HSS update at the
merges whose dense update would cost at least 2.5e10 flops (the top four
levels here; HSS leaf 128, p = 16, adaptive oversampling), compared
with the plain dense FP64 MFMA update on the same GPU.

A step is one complete eigendecomposition (all eigenvalues and eigenvectors)
through adc_stedc with the inputs resident in HBM.  Each step is bracketed by
device synchronisation and timed on the host clock; after each step (outside
the timed spans) its result is validated: eigenvalues against the closed
form, the residual on the device and, for the first step, the orthogonality;
every later step must reproduce the first step's eigenvectors bit for bit,
or it is validated in full as well.  The JSON line reports the HSS-ADC
seconds per step as `value`, the dense-DC time beside it (warmed up like the
headline), the roofline of the dominant kernel (HIP-event durations recorded
by the library on its stream inside the timed steps), Algorithm 3 against its
least-traffic model, the other configurations (random N = 8192, the headline
with HSS at exactly the top three levels, the learned rank predictor on a
prescribed spectrum, the 256-matrix batch, a batch of 16 matrices that take
the HSS route) and the CPU oracle timed on a
bounded sample, with the GPU time at the same size.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM traffic per launch from rocprofv3 counter passes (FETCH_SIZE, then
# WRITE_SIZE, each in its own run over `--mode hss --steps 1 --warmup 0
# --no-cpu --no-validate --no-batched --no-extra`, and the same with
# `--mode dense --dense-steps 1 --dense-warmup 0`), scaled by what the same counters
# read for a 1 GiB device copy (`--calibrate-copy`: FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0).  A record holds only while the sources that define the
# kernel and its launches are unchanged (first 16 hex digits of their
# SHA-256); otherwise the traffic is reported as null.
TRAFFIC = {
    "k_gemm_f64": {"bytes_per_launch": 1657.8e6,
                   "sources": {"gemm.hip": "1de54d48df37fd0d", "hss.hip": "8a7821e8e03d41b3"}},
    "k_gemm_f64_n64": {"bytes_per_launch": 841.0e6,
                       "sources": {"gemm.hip": "1de54d48df37fd0d", "hss.hip": "8a7821e8e03d41b3"}},
    "k_gemm_f64_n96": {"bytes_per_launch": 356.2e6,
                       "sources": {"gemm.hip": "1de54d48df37fd0d", "hss.hip": "8a7821e8e03d41b3"}},
    "k_pack_rot": {"bytes_per_launch": 2302.1e6,
                   "sources": {"merge.hip": "039045ecc7c2eae4", "dc.hip": "6b29df377f3fd2e0"}},
}
# the dense-update GEMM of the dense-DC run (bench.py --mode dense)
TRAFFIC_DENSE = {
    "k_gemm_f64_big": {"bytes_per_launch": 29047.6e6,
                       "sources": {"gemm.hip": "1de54d48df37fd0d", "dc.hip": "6b29df377f3fd2e0"}},
}


HEADLINE = dict(dc_leaf=32, hss_leaf=128, hss_levels=-1, hss_min_k=2048, hss_min_flops=2.5e10, oversample=16)
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
METRIC = "N=32768 tridiag eig wall time: HSS-ADC vs dense DC, 1 GPU, resid≤1e-13"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=32768)
    p.add_argument("--hss-leaf", type=int, default=128, help="HSS leaf size of the headline options")
    p.add_argument("--id-tol", type=float, default=1e-14, help="ID truncation tolerance of the headline options")
    p.add_argument("--dense-steps", type=int, default=3)
    p.add_argument("--dense-warmup", type=int, default=1)
    p.add_argument("--no-extra", action="store_true",
                   help="skip the other configurations (random 8192, top three levels, predictor, "
                        "the five families at 25000)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-validate", action="store_true")
    p.add_argument("--mode", choices=["both", "hss", "dense"], default="both")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only copy 1 GiB between two device buffers three times (HBM counter calibration)")
    p.add_argument("--batched-only", action="store_true")
    p.add_argument("--c5", action="store_true",
                   help="only the learned rank predictor at N = 32768 on prescribed spectra (trains first)")
    p.add_argument("--families", action="store_true",
                   help="only the five matrix families of Example 3 at 5k..25k: HSS-ADC against dense DC")
    p.add_argument("--family-sizes", default="5000,10000,15000,20000,25000")
    return p.parse_args()


def validate(torch, a, b, w, Z, exact):
    """Residual ||TZ - Z diag(w)||_F/(N||T||_1), orthogonality ||Z^T Z - I||_max,
    max |w - exact| / ||T||_1, computed with plain torch ops on the device."""
    N = a.shape[0]
    ad = torch.from_numpy(a).cuda()
    bd = torch.from_numpy(b).cuda()
    tn = float(np.max(np.abs(a) + np.concatenate([[0], np.abs(b)]) + np.concatenate([np.abs(b), [0]])))
    res2 = 0.0
    orth = 0.0
    cb = 4096
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
    werr = float(np.max(np.abs(w.cpu().numpy() - exact))) / tn
    return dict(resid=float(np.sqrt(res2)) / (N * tn), orth=orth, eig_err_rel=werr)


def host_info():
    """Host cores visible to this process and the CPU model name."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return nproc, model


def cpu_baseline(n=7168):
    """The oracle (plain fp64 numpy DC) timed on a bounded sample: the full
    dense DC of the same Toeplitz family at order n on the host cores.  The
    value in the metric's unit is that measurement times (32768/n)^3 (the
    dense update's O(N^3) term dominates), an estimate; the measured seconds
    and the sample are reported beside it."""
    from oracle import dc as odc
    from paper_1510_04591_amd import workloads
    a, b = workloads.toeplitz(n)
    t = time.perf_counter()
    odc.stedc(a, b, leaf=32)
    dt = time.perf_counter() - t
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((x.get("num_threads", 1) for x in threadpool_info()), default=1)
    except Exception:
        threads = os.cpu_count()
    nproc, model = host_info()
    scale = (32768 / n) ** 3
    return {"value": dt * scale, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle dense DC of Toeplitz N={n}, measured {dt:.2f} s on the host; value = that x{scale:.0f} "
                      f"(N^3) to N=32768, an estimate",
            "measured_s": dt, "measured_n": n, "nproc": nproc, "cpu_model": model}


def run_batched(torch, adc, ctx, steps, warmup, sequential=True):
    """256 matrices, N ~ U{200..4000}, half Toeplitz half random (seed 4),
    dense update, through adc_stedc_batched: the first call tunes and
    captures the HIP graph (warm-up), the timed calls replay it.  Also the
    same batch through adc_stedc one matrix at a time, for context."""
    from paper_1510_04591_amd import workloads
    mats = workloads.batched(256, 4)
    ns = [len(a) for a, _ in mats]
    ds = [torch.from_numpy(a).cuda() for a, _ in mats]
    os_ = [torch.from_numpy(b).cuda() for _, b in mats]
    ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in ns]
    Zs = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n in ns]
    o = adc.opts(dc_leaf=32, force_dense=1)

    def call():
        st = adc.adc_stedc_batched(ctx.h, ns, ds, os_, ws, Zs, ns, o, None)
        if st != adc.ADC_OK:
            raise adc.AdcError(st, "adc_stedc_batched")

    for _ in range(max(1, warmup)):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = {"workload": "256 tridiagonal matrices, N ~ U{200..4000} (sum %d), half Toeplitz(2,1), half "
                       "random U(-1,1)/U(0,1), seed 4, DC leaf 32, dense update" % sum(ns),
           "value": 256.0 / dt, "unit": "matrices/s", "s_per_batch": dt, "steps": steps}
    # correctness of the timed result: residual of every matrix on the device
    worst = 0.0
    for (a, b), w, Zt, n in zip(mats, ws, Zs, ns):
        ad, bd = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        Z = Zt.t()
        TZ = ad[:, None] * Z
        TZ[:-1] += bd[:, None] * Z[1:]
        TZ[1:] += bd[:, None] * Z[:-1]
        tn = float(np.max(np.abs(a) + np.concatenate([[0], np.abs(b)]) + np.concatenate([np.abs(b), [0]])))
        worst = max(worst, float(torch.linalg.norm(TZ - Z * w[None, :])) / (n * tn))
    out["max_resid"] = worst
    if sequential:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for d_, o_, w_, Z_, n in zip(ds, os_, ws, Zs, ns):
            st = adc.adc_stedc(ctx.h, n, d_, o_, w_, Z_, n, None, 0, o, None)
            if st != adc.ADC_OK:
                raise adc.AdcError(st, "adc_stedc")
        torch.cuda.synchronize()
        out["sequential_matrices_per_s"] = 256.0 / (time.perf_counter() - t0)
    del Zs
    torch.cuda.empty_cache()
    return out


def run_batched_hss(torch, adc, ctx, steps):
    """16 matrices large enough for HSS merges, N ~ U{4000..8000} (seed 11),
    alternately Toeplitz(2,1) and random U(-1,1)/U(0,1), the headline
    options: one adc_stedc_batched call (those matrices are solved together,
    level-batched with the HSS route where it applies) against the same
    matrices through adc_stedc one at a time.  Median of `steps` timed calls
    after one untimed call each; every matrix's residual checked."""
    from paper_1510_04591_amd import workloads
    rng = np.random.default_rng(11)
    sizes = [int(x) for x in rng.integers(4000, 8001, 16)]
    mats = [workloads.toeplitz(n) if i % 2 == 0 else workloads.random_uniform(n, 60 + i)
            for i, n in enumerate(sizes)]
    ds = [torch.from_numpy(a).cuda() for a, _ in mats]
    os_ = [torch.from_numpy(b).cuda() for _, b in mats]
    ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in sizes]
    Zs = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n in sizes]
    o = adc.opts(**HEADLINE)

    def batched():
        rep = adc.adc_report()
        st = adc.adc_stedc_batched(ctx.h, sizes, ds, os_, ws, Zs, sizes, o, rep)
        if st != adc.ADC_OK:
            raise adc.AdcError(st, "adc_stedc_batched")
        return rep

    def one_by_one():
        for d_, o_, w_, Z_, n in zip(ds, os_, ws, Zs, sizes):
            st = adc.adc_stedc(ctx.h, n, d_, o_, w_, Z_, n, None, 0, o, None)
            if st != adc.ADC_OK:
                raise adc.AdcError(st, "adc_stedc")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(steps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    t_seq = timed(one_by_one)
    t_b = timed(batched)
    rep = batched().as_dict()
    torch.cuda.synchronize()
    worst = 0.0
    for (a, b), w, Zt, n in zip(mats, ws, Zs, sizes):
        ad, bd = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        Z = Zt.t()
        TZ = ad[:, None] * Z
        TZ[:-1] += bd[:, None] * Z[1:]
        TZ[1:] += bd[:, None] * Z[:-1]
        tn = float(np.max(np.abs(a) + np.concatenate([[0], np.abs(b)]) + np.concatenate([np.abs(b), [0]])))
        worst = max(worst, float(torch.linalg.norm(TZ - Z * w[None, :])) / (n * tn))
    del Zs
    torch.cuda.empty_cache()
    return {"workload": "16 tridiagonal matrices, N ~ U{4000..8000} (sum %d), alternately Toeplitz(2,1) and "
                        "random U(-1,1)/U(0,1), seed 11, headline HSS options" % sum(sizes),
            "value": 16.0 / t_b, "unit": "matrices/s", "s_per_batch": t_b, "steps": steps,
            "one_by_one_matrices_per_s": 16.0 / t_seq, "hss_merges": rep["hss_merges"], "max_resid": worst}


def recorded_traffic(kernel, table=None):
    """Bytes per launch of `kernel` from the counter record, or None when a
    source it depends on has changed since the counters were taken."""
    import hashlib
    rec = (TRAFFIC if table is None else table).get(kernel)
    if rec is None:
        return None
    for fn, want in rec["sources"].items():
        path = os.path.join(ROOT, "paper_1510_04591_amd", "csrc", fn)
        try:
            got = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
        except OSError:
            return None
        if want is None or got != want:
            return None
    return rec["bytes_per_launch"]


def run_c5(torch, adc, ctx, steps):
    """Learned rank predictor at full size: collect boundary ranks from the
    training families (Toeplitz N = 4096 and 32768, random uniform N = 8192
    seed 2, four matrices of the 256-matrix batch) with HSS forced on every
    merge, train the MLP on the GPU, then solve N = 32768 matrices with
    prescribed spectra (uniform, geometric, clusters; not seen in training)
    with the sample count from eq. (bounds) and from the MLP, the latter also
    with the rank-saturation guard."""
    from paper_1510_04591_amd import workloads
    out = train_predictor(torch, adc, ctx, full=True)
    out["spectra"] = {}
    N = 32768
    for kind in ("uniform", "geometric", "clusters"):
        a, b = workloads.prescribed_tridiagonal(kind, N)
        lam, _ = workloads.spectrum(kind, N)
        res = {}
        for name, mode, sg in (("bound", adc.ADC_RANK_BOUND, 0), ("mlp", adc.ADC_RANK_MLP, 0),
                               ("mlp_sat_guard", adc.ADC_RANK_MLP, 1)):
            o = adc.opts(dc_leaf=32, hss_leaf=128, hss_min_k=2048, hss_levels=-1, hss_min_flops=0, rank_mode=mode,
                         sat_guard=sg)
            res[name] = timed_config(torch, adc, ctx, a, b, o, steps=max(steps, 1), exact=np.sort(lam))
        out["spectra"][kind] = res
        print(f"# C5 {kind}: " + ", ".join(f"{k} {v['median_s']:.4f} s (s={v['samples']}, retries {v['retries']}, "
                                           f"saturated {v['saturated_merges']}, orth {v['validation']['orth']:.1e})"
                                           for k, v in res.items()), flush=True)
    return out


FAMILIES = ("clement", "legendre", "laguerre", "hermite", "toeplitz")


def family_matrix(kind, n):
    """Order-n matrix of one of the five families of Example 3 and its exact
    eigenvalues where a closed form is known (else None)."""
    from paper_1510_04591_amd import workloads
    if kind == "clement":
        a, b = workloads.clement(n - 1)
        return a, b, np.arange(-(n - 1), n, 2, dtype=np.float64)
    if kind == "toeplitz":
        a, b = workloads.toeplitz(n)
        return a, b, np.sort(2 + 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    a, b = getattr(workloads, kind)(n)
    return a, b, None


def run_families(torch, adc, ctx, sizes, steps):
    """Example 3 / Table 5 setting: each family at each size solved with the
    headline HSS options and with the dense update; median seconds of
    `steps` timed solves after one untimed one, residual and orthogonality of
    the HSS result, eigenvalue error where the spectrum has a closed form."""
    hss_opts = adc.opts(**HEADLINE)
    dense_opts = adc.opts(dc_leaf=32, force_dense=1)
    out = {}
    for kind in FAMILIES:
        out[kind] = {}
        for n in sizes:
            a, b, exact = family_matrix(kind, n)
            ad, bd = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
            w = torch.empty(n, dtype=torch.float64, device="cuda")
            Zt = torch.empty((n, n), dtype=torch.float64, device="cuda")
            row = {}
            for name, o in (("dense", dense_opts), ("hss", hss_opts)):
                times = []
                for it in range(steps + 1):
                    rep = adc.adc_report()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st = adc.adc_stedc(ctx.h, n, ad, bd, w, Zt, n, None, 0, o, rep)
                    torch.cuda.synchronize()
                    if st != adc.ADC_OK:
                        raise adc.AdcError(st, "adc_stedc", rep.as_dict())
                    if it > 0:
                        times.append(time.perf_counter() - t0)
                row[name] = float(np.median(times))
            r = rep.as_dict()
            v = validate(torch, a, b, w, Zt.t(), exact if exact is not None else w.cpu().numpy())
            if exact is None:
                v.pop("eig_err_rel")
            row.update(speedup=row["dense"] / row["hss"], hss_merges=r["hss_merges"], samples=r["samples"],
                       max_rank=r["max_rank"], fallbacks=r["hss_fallbacks"], K_top=r["K_per_level"][0],
                       validation=v)
            out[kind][str(n)] = row
            print(f"# {kind} n={n}: dense {row['dense']:.4f} s, HSS {row['hss']:.4f} s, "
                  f"x{row['speedup']:.2f}, K top {row['K_top']}, rank {row['max_rank']}, "
                  f"resid {v['resid']:.1e} orth {v['orth']:.1e}", flush=True)
            del Zt
    return out


def timed_config(torch, adc, ctx, a, b, o, steps=3, warm=1, exact=None):
    """Median seconds of `steps` synchronised solves after `warm` untimed ones,
    the last report, and the validation of every timed result (residual,
    orthogonality, and eigenvalues against `exact`, or else against Sturm
    counts at sampled indices)."""
    from oracle import sturm
    n = len(a)
    ad, bd = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    Zt = torch.empty((n, n), dtype=torch.float64, device="cuda")
    tn = float(np.max(np.abs(a) + np.concatenate([[0], np.abs(b)]) + np.concatenate([np.abs(b), [0]])))
    if exact is None:
        ks = np.unique(np.array([0, 1, n // 7, n // 3, n // 2, 2 * n // 3, n - 2, n - 1]))
        ref_ks = sturm.eigenvalues_by_index(a, b, ks)
    times, vals, r = [], [], None
    for it in range(warm + steps):
        rep = adc.adc_report()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = adc.adc_stedc(ctx.h, n, ad, bd, w, Zt, n, None, 0, o, rep)
        torch.cuda.synchronize()
        if st != adc.ADC_OK:
            raise adc.AdcError(st, "adc_stedc", rep.as_dict())
        if it < warm:
            continue
        times.append(time.perf_counter() - t0)
        r = rep.as_dict()
        if exact is not None:
            v = validate(torch, a, b, w, Zt.t(), exact)
        else:
            v = validate(torch, a, b, w, Zt.t(), w.cpu().numpy())
            v["eig_err_rel"] = float(np.max(np.abs(w.cpu().numpy()[ks] - ref_ks))) / tn
        vals.append(v)
    del Zt
    torch.cuda.empty_cache()
    v = {key: max(x[key] for x in vals) for key in vals[0]}
    v["steps_validated"] = len(vals)
    return {"median_s": float(np.median(times)), "steps": steps, "warmup": warm, "hss_merges": r["hss_merges"],
            "hss_per_level": r["hss_per_level"], "K_top": r["K_per_level"][0], "samples": r["samples"],
            "max_rank": r["max_rank"], "retries": r["retries"], "fallbacks": r["hss_fallbacks"],
            "saturated_merges": r["hss_saturated"],
            "hss_compress_s": r["t_phase"][6], "hss_multiply_s": r["t_phase"][8], "validation": v}


def gpu_time_at(torch, adc, ctx, n):
    """HSS-ADC (headline options) and dense DC at order n: the GPU beside the
    CPU sample of the same size."""
    from paper_1510_04591_amd import workloads
    a, b = workloads.toeplitz(n)
    exact = np.sort(2 + 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    h = timed_config(torch, adc, ctx, a, b, adc.opts(**HEADLINE), exact=exact)
    d = timed_config(torch, adc, ctx, a, b, adc.opts(dc_leaf=32, force_dense=1), exact=exact)
    return {"hss_adc_s": h["median_s"], "dense_dc_s": d["median_s"], "n": n}


def train_predictor(torch, adc, ctx, full=False):
    """Collect boundary ranks from the training families with HSS forced on
    every merge (Toeplitz N = 4096, random uniform N = 4096 seed 2, four
    matrices of the batch; with `full` also Toeplitz 32768 and random 8192)
    and train the MLP on the GPU."""
    from paper_1510_04591_amd import workloads
    Xs, ys = [], []
    if full:
        train = [workloads.toeplitz(4096), workloads.toeplitz(32768), workloads.random_uniform(8192, 2)]
    else:
        train = [workloads.toeplitz(4096), workloads.random_uniform(4096, 2)]
    train += [workloads.batched(8, 4)[i] for i in (0, 1, 5, 6)]
    for a, b in train:
        n = len(a)
        w = torch.empty(n, dtype=torch.float64, device="cuda")
        Z = torch.empty((n, n), dtype=torch.float64, device="cuda")
        for leaf in ((32, 64, 128) if n <= 8192 else (128,)):
            o = adc.opts(dc_leaf=32, hss_leaf=leaf, hss_min_k=max(2 * leaf, 256 if n > 8192 else 0), hss_levels=-1,
                         hss_min_flops=0)
            cap = 1 << 17
            X = torch.empty((cap, 16), dtype=torch.float32, device="cuda")
            y = torch.empty(cap, dtype=torch.float32, device="cuda")
            st, rows = adc.adc_mlp_collect(ctx.h, n, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), w, Z, n,
                                           o, cap, X, y)
            if st != adc.ADC_OK:
                raise adc.AdcError(st, "adc_mlp_collect")
            Xs.append(X[:rows].clone())
            ys.append(y[:rows].clone())
        del Z
    X = torch.cat(Xs)
    y = torch.cat(ys)
    perm = torch.from_numpy(np.random.default_rng(0).permutation(X.shape[0])).cuda()
    X, y = X[perm].contiguous(), y[perm].contiguous()
    if adc.adc_mlp_init(ctx.h, 7) != adc.ADC_OK:
        raise RuntimeError("adc_mlp_init")
    t0 = time.perf_counter()
    st, loss = adc.adc_mlp_train(ctx.h, X.shape[0], X, y, 150, 64, 1e-3)
    if st != adc.ADC_OK:
        raise adc.AdcError(st, "adc_mlp_train")
    torch.cuda.empty_cache()
    return {"training_rows": int(X.shape[0]), "train_loss": loss, "target_var": float(torch.var(y)),
            "train_s": time.perf_counter() - t0}


def run_extra(torch, adc, ctx, args):
    """The other configurations, each timed (median of 3 after one untimed
    solve) and every timed result validated."""
    from paper_1510_04591_amd import workloads
    out = {}
    N = 32768
    # random N = 8192, HSS leaf 64, ID tolerance 1e-14, HSS at K >= 2048
    a, b = workloads.random_uniform(8192, 2)
    out["random_8192_leaf64"] = timed_config(
        torch, adc, ctx, a, b, adc.opts(dc_leaf=32, hss_leaf=64, id_tol=1e-14, hss_min_k=2048, hss_levels=-1,
                                        hss_min_flops=0))
    print(f"# random 8192: {out['random_8192_leaf64']['median_s']:.4f} s", flush=True)
    # the headline matrix with HSS at exactly the top three merge levels
    a, b = workloads.toeplitz(N)
    exact = np.sort(2 + 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)))
    out["toeplitz_32768_top3"] = timed_config(
        torch, adc, ctx, a, b, adc.opts(dc_leaf=32, hss_leaf=128, hss_levels=3, hss_min_k=2048, hss_min_flops=0,
                                        oversample=16), exact=exact)
    print(f"# toeplitz 32768, HSS at the top three levels: {out['toeplitz_32768_top3']['median_s']:.4f} s",
          flush=True)
    # the learned rank predictor on the prescribed uniform spectrum
    tr = train_predictor(torch, adc, ctx)
    a, b = workloads.prescribed_tridiagonal("uniform", N)
    lam, _ = workloads.spectrum("uniform", N)
    c5 = {"training": tr}
    for name, kw in (("bound", dict(rank_mode=adc.ADC_RANK_BOUND)), ("mlp", dict(rank_mode=adc.ADC_RANK_MLP)),
                     ("mlp_sat_guard", dict(rank_mode=adc.ADC_RANK_MLP, sat_guard=1))):
        o = adc.opts(dc_leaf=32, hss_leaf=128, hss_min_k=2048, hss_levels=-1, hss_min_flops=0, **kw)
        c5[name] = timed_config(torch, adc, ctx, a, b, o, exact=np.sort(lam))
        print(f"# prescribed uniform 32768, {name}: {c5[name]['median_s']:.4f} s, s={c5[name]['samples']}, "
              f"retries {c5[name]['retries']}, saturated {c5[name]['saturated_merges']}, "
              f"orth {c5[name]['validation']['orth']:.1e}", flush=True)
    out["prescribed_uniform_32768"] = c5
    # Example 3 / Table 5 at its largest order: the five families against dense DC
    out["families_25000"] = run_families(torch, adc, ctx, [25000], 3)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1510_04591_amd import adc, workloads
    if args.calibrate_copy:
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                          "copies": 3}), flush=True)
        return
    if args.c5:
        ctx = adc.Context(0)
        print(json.dumps({"c5": run_c5(torch, adc, ctx, args.steps)}), flush=True)
        ctx.close()
        return
    if args.families:
        ctx = adc.Context(0)
        sizes = [int(x) for x in args.family_sizes.split(",")]
        print(json.dumps({"families": run_families(torch, adc, ctx, sizes, max(args.steps, 1))}), flush=True)
        ctx.close()
        return
    if args.batched_only:
        ctx = adc.Context(0)
        print(json.dumps({"batched": run_batched(torch, adc, ctx, args.steps, args.warmup),
                          "batched_hss": run_batched_hss(torch, adc, ctx, max(args.steps, 3))}), flush=True)
        ctx.close()
        return

    N = args.n
    a, b = workloads.toeplitz(N)
    k = np.arange(1, N + 1)
    exact = np.sort(2 + 2 * np.cos(k * np.pi / (N + 1)))
    ad = torch.from_numpy(a).cuda()
    bd = torch.from_numpy(b).cuda()
    ctx = adc.Context(0)
    w = torch.empty(N, dtype=torch.float64, device="cuda")
    Zt = torch.empty((N, N), dtype=torch.float64, device="cuda")
    hss_opts = adc.opts(**dict(HEADLINE, hss_leaf=args.hss_leaf, id_tol=args.id_tol))
    dense_opts = adc.opts(dc_leaf=32, force_dense=1)

    def solve(o):
        rep = adc.adc_report()
        st = adc.adc_stedc(ctx.h, N, ad, bd, w, Zt, N, None, 0, o, rep)
        if st != adc.ADC_OK:
            raise adc.AdcError(st, "adc_stedc", rep.as_dict())
        return rep.as_dict()

    def run(o, steps, warm):
        """warm untimed solves, then `steps` solves each bracketed by device
        synchronisation; every step's result validated outside its span."""
        for _ in range(warm):
            solve(o)
        torch.cuda.synchronize()
        times, reps, vals = [], [], []
        ref = None
        identical = 0
        for i in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = solve(o)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            reps.append(r)
            if args.no_validate:
                continue
            if i == 0:
                vals.append(validate(torch, a, b, w, Zt.t(), exact))
                ref = (w.clone(), Zt.clone())
            elif torch.equal(w, ref[0]) and torch.equal(Zt, ref[1]):
                identical += 1
            else:
                vals.append(validate(torch, a, b, w, Zt.t(), exact))
        v = None
        if vals:
            v = {key: max(x[key] for x in vals) for key in vals[0]}
            v["steps_validated"] = steps
            v["steps_bit_identical_to_first"] = identical
            v["steps_validated_in_full"] = len(vals)
        del ref
        torch.cuda.empty_cache()
        return float(np.sum(times)) / steps, times, reps, v

    out = {}
    val = {}
    if args.mode in ("both", "dense"):
        t_dense, times_d, reps_d, v = run(dense_opts, args.dense_steps, args.dense_warmup)
        out["dense"] = (t_dense, reps_d, times_d)
        if v:
            val["dense"] = v
        print(f"# dense DC: {t_dense:.4f} s/step (median {np.median(times_d):.4f}) {val.get('dense', '')}", flush=True)
    if args.mode in ("both", "hss"):
        t_hss, times_h, reps_h, v = run(hss_opts, args.steps, args.warmup)
        out["hss"] = (t_hss, reps_h, times_h)
        if v:
            val["hss"] = v
        print(f"# HSS-ADC: {t_hss:.4f} s/step (median {np.median(times_h):.4f}) {val.get('hss', '')}", flush=True)

    head = "hss" if "hss" in out else "dense"
    t_head, reps, times_head = out[head]
    names = ["leaves", "deflation", "secular", "loewner_v", "dense_gemm", "hss_sampling", "hss_compress",
             "hss_check", "hss_multiply", "order_pack"]
    ph = np.sum([r["t_phase"] for r in reps], axis=0)
    pb = np.sum([r["phase_bytes"] for r in reps], axis=0)
    # dominant kernel: the largest total time among the kernels whose
    # algorithmic flops or bytes the library counts; each launch is
    # bracketed by HIP events on the library's stream
    kt = np.sum([r["kern_time"] for r in reps], axis=0)
    kf = np.sum([r["kern_flops"] for r in reps], axis=0)
    kb = np.sum([r["kern_bytes"] for r in reps], axis=0)
    kl = np.sum([r["kern_launches"] for r in reps], axis=0)
    kn = adc.adc_report.KERNELS
    counted = [i for i in range(len(kn)) if kl[i] > 0 and (kf[i] > 0 or kb[i] > 0)]
    dom = max(counted, key=lambda i: kt[i])
    launches = int(kl[dom])
    avg_dur = kt[dom] / launches
    if kf[dom] / max(kb[dom], 1.0) > PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
        achieved = kf[dom] / launches / avg_dur / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None}
    else:
        achieved = kb[dom] / launches / avg_dur / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof["traffic"] = recorded_traffic(kn[dom], TRAFFIC if head == "hss" else TRAFFIC_DENSE)
    roof["kernel"] = kn[dom]
    roof["launches_per_step"] = launches / len(reps)
    roof["avg_launch_ms"] = 1e3 * avg_dur
    if head == "hss" and ph[8] > 0 and pb[8] > 0:
        # the whole HSS multiply phase (Algorithm 3 with the check's probe
        # products) against the least traffic of the update products
        roof["alg3_phase"] = {"model_bytes_per_step": float(pb[8] / len(reps)),
                              "ms_per_step": float(1e3 * ph[8] / len(reps)),
                              "achieved_gbs": float(pb[8] / ph[8] / 1e9),
                              "frac": float(pb[8] / ph[8] / 1e9 / PEAK_HBM_GBS),
                              "kernel_bytes_per_step": float(sum(kb[i] for i in (0, 1, 7)) / len(reps))}
    kernels = {kn[i]: {"ms_per_step": 1e3 * kt[i] / len(reps), "launches_per_step": kl[i] / len(reps),
                       "avg_launch_us": 1e6 * kt[i] / max(kl[i], 1),
                       "tflops": (kf[i] / kt[i] / 1e12) if kf[i] > 0 else None,
                       "gbs": (kb[i] / kt[i] / 1e9) if kb[i] > 0 else None}
               for i in range(len(kn)) if kl[i] > 0}

    r0 = reps[-1]
    res = {
        "metric": METRIC,
        "value": t_head,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps if head == "hss" else args.dense_steps,
        "warmup": args.warmup if head == "hss" else args.dense_warmup,
        "ms_per_step": 1e3 * t_head,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"toeplitz(2,1) N={N}, DC leaf 32, HSS on merges with K>=2048 and dense update >=2.5e10 flops, HSS leaf {args.hss_leaf}, p=16, ID tolerance {args.id_tol:g}",
                   "update": head, "n": N, "K_per_level": r0["K_per_level"],
                   "hss_per_level": r0["hss_per_level"], "max_rank": r0["max_rank"],
                   "samples": r0["samples"], "retries": r0["retries"], "fallbacks": r0["hss_fallbacks"],
                   "saturated_merges": r0["hss_saturated"]},
        "median_step_s": float(np.median(times_head)),
        "dense_dc_s": out["dense"][0] if "dense" in out else None,
        "dense_dc_median_s": float(np.median(out["dense"][2])) if "dense" in out else None,
        "dense_dc_steps": args.dense_steps if "dense" in out else None,
        "speedup_vs_dense": (out["dense"][0] / out["hss"][0]) if ("dense" in out and "hss" in out) else None,
        "phases_s": {n_: float(ph[i] / len(reps)) for i, n_ in enumerate(names)},
        "validation": val,
        "roofline": roof,
        "kernels": kernels,
    }
    del Zt
    torch.cuda.empty_cache()
    if not args.no_extra and args.mode == "both":
        res["configs"] = run_extra(torch, adc, ctx, args)
    if not args.no_batched:
        res["batched"] = run_batched(torch, adc, ctx, max(args.steps, 3), 1)
        print(f"# batched: {res['batched']['value']:.1f} matrices/s", flush=True)
        res["batched_hss"] = run_batched_hss(torch, adc, ctx, 3)
        print(f"# batched with HSS: {res['batched_hss']['value']:.1f} matrices/s "
              f"(one by one {res['batched_hss']['one_by_one_matrices_per_s']:.1f})", flush=True)
    if not args.no_cpu:
        cb = cpu_baseline()
        cb["gpu_s_same_size"] = gpu_time_at(torch, adc, ctx, cb["measured_n"])
        res["cpu_baseline"] = cb
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
