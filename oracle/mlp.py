"""Learned HSS rank predictor: features, the 16-64-64-1 MLP and Adam (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper sets the HSS sample count from the a-priori bound of eq. (bounds)
(Section 4.1): a rank per boundary between neighbouring leaf segments, the
maximum over the boundaries, plus oversampling.  The predictor keeps that
structure and replaces the bound by a learned per-boundary estimate of
log2 of the rank that the interpolative decompositions actually find.  The
features, the network and the training rule are this project's definitions
(the paper has no learned component); they are written out here in FP64.

Features of one interior leaf boundary p = bounds[b+1] of a merge of size K
with poles d (ascending), gam_i = lam_i - d_i, mu_i = d_{i+1} - lam_i
(mu_{K-1} = inf) and neighbouring segments [lo, p), [p, hi) with
lo = bounds[b], hi = bounds[b+2]; span = lam_{K-1} - d_0;
dist(q) = min(|lam_q - d_{q-1}|, |d_q - lam_{q-1}|) from the differences of
eq. (d-lambda); cl(x) = log2(x) clamped to [-64, 64] (-64 for x <= 0):

   0  log2(K) / 16                      8  std_j cl(g_j/span) / 8
   1  log2(p - lo) / 8                  9  mean_j cl(min(gam_j, mu_j)/span) / 32
   2  log2(hi - p) / 8                 10  min_j  cl(min(gam_j, mu_j)/span) / 32
   3  cl(span / dist(p)) / 32          11  fraction of g_j < 1e-10 span
   4  cl(span / min_q dist(q)) / 32    12  p / K
   5  min_j cl(g_j/span) / 32          13  log2(number of leaves) / 8
   6  mean_j cl(g_j/span) / 32         14  cl((d_{hi-1} - d_lo)/span) / 32
   7  max_j cl(g_j/span) / 32          15  cl(dist(p) / (d_p - d_{p-1})) / 32

with g_j = d_{j+1} - d_j over the pole gaps j in [lo, hi-1), the gam/mu
statistics over j in [lo, hi), and q over the rows lo < q < hi.  Feature 3
is the ratio R of eq. (bounds).

Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3 with
W1 64x16, W2 64x64, W3 1x64; parameters packed as W1, b1, W2, b2, W3, b3
(row-major W[out, in]), 5313 values.  Loss: mean squared error of y against
the target log2(rank).  Training: Adam (Kingma and Ba 2015) over minibatches
taken in the given order.
"""
import math

import numpy as np

NF = 16
H = 64
SIZES = [(H, NF), (H,), (H, H), (H,), (1, H), (1,)]
NPARAM = sum(int(np.prod(s)) for s in SIZES)  # 5313


def _cl(x):
    x = np.asarray(x, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        lg = np.where(x > 0, np.log2(np.where(x > 0, x, 1.0)), -64.0)
    lg = np.where(np.isnan(x), -64.0, lg)
    return np.clip(lg, -64.0, 64.0)


def _dist(d, gam, mu, q):
    """min(|lam_q - d_{q-1}|, |d_q - lam_{q-1}|) by eq. (d-lambda)."""
    x = (d[q] - d[q - 1]) + gam[q]
    y = mu[q - 1]
    return min(abs(x), abs(y))


def features(d, gam, mu, bounds):
    """Feature matrix (nb x 16, FP64) of the interior boundaries of `bounds`
    (len nb + 2, first 0, last K)."""
    d = np.asarray(d, np.float64)
    gam = np.asarray(gam, np.float64)
    mu = np.asarray(mu, np.float64)
    K = len(d)
    bounds = [int(x) for x in bounds]
    nb = len(bounds) - 2
    span = (d[K - 1] + gam[K - 1]) - d[0]
    F = np.zeros((max(nb, 0), NF))
    for b in range(nb):
        lo, p, hi = bounds[b], bounds[b + 1], bounds[b + 2]
        dp = _dist(d, gam, mu, p)
        dmin = min(_dist(d, gam, mu, q) for q in range(lo + 1, hi))
        g = d[lo + 1:hi] - d[lo:hi - 1]
        lg = _cl(g / span)
        t = _cl(np.minimum(gam[lo:hi], mu[lo:hi]) / span)
        f = F[b]
        f[0] = math.log2(K) / 16
        f[1] = math.log2(p - lo) / 8
        f[2] = math.log2(hi - p) / 8
        f[3] = _cl(span / dp) / 32
        f[4] = _cl(span / dmin) / 32
        if len(g):
            f[5] = lg.min() / 32
            f[6] = lg.mean() / 32
            f[7] = lg.max() / 32
            f[8] = math.sqrt(max(np.mean(lg * lg) - lg.mean() ** 2, 0.0)) / 8
            f[11] = np.count_nonzero(g < 1e-10 * span) / len(g)
        f[9] = t.mean() / 32
        f[10] = t.min() / 32
        f[12] = p / K
        f[13] = math.log2(nb + 1) / 8
        f[14] = _cl((d[hi - 1] - d[lo]) / span) / 32
        f[15] = _cl(dp / (d[p] - d[p - 1])) / 32
    return F


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def forward(theta, X):
    """y (B,) = MLP(X (B x 16)) in FP64."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return (h2 @ W3.T + b3)[:, 0]


def loss_grad(theta, X, y):
    """Mean squared error over the B rows and its gradient (packed like
    theta), by the chain rule through the three layers."""
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    B = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = (h2 @ W3.T + b3)[:, 0]
    r = out - y
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B                      # d loss / d out
    gW3 = dy[None, :] @ h2                # 1 x 64
    gb3 = np.array([dy.sum()])
    dh2 = dy[:, None] * W3                # B x 64
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_train(theta, X, y, epochs, batch, lr, beta1=0.9, beta2=0.999, eps=1e-8, state=None):
    """Adam over minibatches of `batch` rows taken in order (the last one may
    be shorter), `epochs` passes.  Returns (theta, state, mean squared error
    of the last epoch's minibatches before their updates, averaged over all
    rows)."""
    theta = np.array(theta, np.float64)
    if state is None:
        state = {"m": np.zeros_like(theta), "v": np.zeros_like(theta), "t": 0}
    m, v = state["m"], state["v"]
    B = X.shape[0]
    last = 0.0
    for e in range(epochs):
        sse = 0.0
        for i0 in range(0, B, batch):
            xb, yb = X[i0:i0 + batch], y[i0:i0 + batch]
            loss, g = loss_grad(theta, xb, yb)
            sse += loss * xb.shape[0]
            state["t"] += 1
            t = state["t"]
            m[:] = beta1 * m + (1 - beta1) * g
            v[:] = beta2 * v + (1 - beta2) * g * g
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            theta -= lr * mh / (np.sqrt(vh) + eps)
        last = sse / B
    return theta, state, last


def predicted_rank(yhat, margin=4, floor=8, cap=100, scale=1.25):
    """Rank of a merge from the per-boundary predictions of log2(rank):
    ceil(scale 2^max) + margin, clamped to [floor, cap]."""
    if len(yhat) == 0:
        return floor
    r = int(math.ceil(scale * 2.0 ** float(np.max(yhat)))) + margin
    return max(floor, min(cap, r))


def boundary_targets(lo, hi, kr, kc, bounds):
    """Observed rank at each interior boundary: the largest row or column ID
    rank among the non-root HSS nodes whose index range starts or ends there
    (heap order, node 0 the root).  Returns log2 of it (rank at least 1)."""
    out = []
    for b in range(1, len(bounds) - 1):
        p = bounds[b]
        r = 1
        for i in range(1, len(lo)):
            if lo[i] == p or hi[i] == p:
                r = max(r, int(kr[i]), int(kc[i]))
        out.append(math.log2(r))
    return np.array(out)
