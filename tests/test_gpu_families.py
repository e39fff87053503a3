"""The matrix families of the paper's Example 3 (Clement, Legendre-type,
Laguerre-type, Hermite-type) through the whole path, dense and with HSS at
every merge of deflated size >= 2048: eigenvalues against closed forms,
Sturm counts at sampled indices, residual and orthogonality on the device."""
import numpy as np
import pytest
import torch

from oracle import dc as odc, sturm
from paper_1510_04591_amd import adc, workloads
from conftest import cuda

pytestmark = pytest.mark.gpu


def device_checks(a, b, w, Z):
    """||T Z - Z diag(w)||_F / (n ||T||_1) and ||Z^T Z - I||_max on the GPU."""
    ad, bd = cuda(a), cuda(b)
    TZ = ad[:, None] * Z
    TZ[:-1] += bd[:, None] * Z[1:]
    TZ[1:] += bd[:, None] * Z[:-1]
    n = len(a)
    res = float(torch.linalg.norm(TZ - Z * w[None, :])) / (n * odc.tnorm1(a, b))
    G = Z.t() @ Z
    G.diagonal().sub_(1.0)
    return res, float(G.abs().max())


CASES = {
    "clement": (lambda n: workloads.clement(n - 1), 6000),
    "legendre": (workloads.legendre, 6000),
    "laguerre": (workloads.laguerre, 6000),
    "hermite": (workloads.hermite, 6000),
}


@pytest.mark.parametrize("family", list(CASES))
@pytest.mark.parametrize("update", ["dense", "hss"])
def test_family(ctx, family, update):
    gen, n = CASES[family]
    a, b = gen(n)
    n = len(a)
    print(f"{family} n={n} {update}", flush=True)
    kw = dict(force_dense=1) if update == "dense" else dict(hss_levels=-1, hss_min_k=2048, hss_min_flops=0, hss_leaf=128)
    w, Z, rep = adc.eigh_tridiagonal(ctx, cuda(a), cuda(b), **kw)
    torch.cuda.synchronize()
    tn = odc.tnorm1(a, b)
    wh = w.cpu().numpy()
    assert np.all(np.diff(wh) >= 0)
    if family == "clement":
        m = n - 1
        exact = np.arange(-m, m + 1, 2, dtype=np.float64)
        assert np.max(np.abs(wh - exact)) <= 1e-13 * tn
    else:
        # Gauss nodes from numpy overflow at these orders: Sturm counts instead
        ks = np.array([0, 1, n // 3, n // 2, n - 2, n - 1])
        assert np.max(np.abs(wh[ks] - sturm.eigenvalues_by_index(a, b, ks))) <= 1e-13 * tn
    res, orth = device_checks(a, b, w, Z)
    print(f"  resid {res:.2e} orth {orth:.2e} K top {rep['K_per_level'][0]} hss merges {rep['hss_merges']}",
          flush=True)
    assert res <= 1e-13 and orth <= 1e-12
    if update == "hss":
        assert rep["hss_merges"] >= 1 and rep["hss_fallbacks"] == 0
