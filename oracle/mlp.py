"""Learned second-pass proposal: a small MLP that predicts, per (slice,
cluster), the log of a sampling density from first-pass statistics and
geometry.  The paper's second pass samples columns by g(j) = max C_j - min C_j
because a light whose results vary over the slice's pixels is important
(Sec. 5); its conclusion names image-space-guided sampling as future work.
This network estimates that importance from the same sparse observations.

Readings (the paper has no network):
* features f (12 per row), from the first pass of slice s and column j
  (t = R + G + B per observed entry, mu_s = mean t over the slice's first
  pass) and geometry; see ``features``;
* network y = W3 h2 + b3, h2 = bf16(gelu(W2 h1 + b2)), h1 = bf16(gelu(W1 f + b1)),
  128 hidden units, GELU in its tanh form (Hendrycks & Gimpel), weights used
  rounded to bfloat16 (round to nearest even), FP32/FP64 accumulation;
* training target p*_j ~ sigma_j + 3 mean(sigma) per slice, sigma_j the
  standard deviation of t over the full column (the variance the paper uses
  as importance), mixed with three times its mean in uniform mass: sampling
  by sigma + 0.01 mean(sigma) concentrates the second pass as much as g does
  and completed no better than g, while the mix of 3 gave the smallest pixel
  error of the mixes 0.01 to 30 and the uniform density on mid slices at 5%;
  loss KL(p* || softmax(y)) summed over the slice; Adam (Kingma & Ba) on FP32
  master weights;
* deployment: column weights w_j = max(1, floor(2^24 exp(y_j - max y)));
  any non-finite y falls back to the plain g weights.

Pinned by: central finite differences of the FP64 backward with rounding
off, the closed-form softmax-KL gradient, a hand-computed Adam step and GELU
values (tests/test_oracle_mlp.py).
"""
import numpy as np

N_IN = 12
N_HID = 128
TWO24 = float(1 << 24)
TARGET_MIX = 3.0       # uniform mass of the target density, in units of mean(sigma)
SQRT_2_OVER_PI = np.sqrt(2.0 / np.pi)


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r.astype(np.uint32).view(np.float32)).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(SQRT_2_OVER_PI * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = SQRT_2_OVER_PI * (x + 0.044715 * x ** 3)
    th = np.tanh(u)
    du = SQRT_2_OVER_PI * (1.0 + 3 * 0.044715 * x ** 2)
    return 0.5 * (1.0 + th) + 0.5 * x * (1.0 - th * th) * du


def init_params(seed):
    """He-style initialisation (float32 master weights)."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.normal(0, np.sqrt(2.0 / N_IN), (N_HID, N_IN)),
        "b1": np.zeros(N_HID),
        "W2": rng.normal(0, np.sqrt(2.0 / N_HID), (N_HID, N_HID)),
        "b2": np.zeros(N_HID),
        "W3": rng.normal(0, np.sqrt(1.0 / N_HID), (1, N_HID)),
        "b3": np.zeros(1),
    }
    return {k: v.astype(np.float32) for k, v in p.items()}


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(p):
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k in PARAM_ORDER])


def unflatten(v):
    shapes = {"W1": (N_HID, N_IN), "b1": (N_HID,), "W2": (N_HID, N_HID), "b2": (N_HID,), "W3": (1, N_HID),
              "b3": (1,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(v[o:o + n]).reshape(shapes[k])
        o += n
    return out


def forward(p, F, rounding=True):
    """F: (R, 12) features -> y (R,), cache.  With rounding, weights and the
    two hidden activations are rounded to bfloat16 as the kernels do."""
    rnd = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    W1, W2, W3 = rnd(p["W1"]), rnd(p["W2"]), rnd(p["W3"])
    b1, b2, b3 = (np.asarray(p[k], np.float64) for k in ("b1", "b2", "b3"))
    F = np.asarray(F, np.float64)
    z1 = F @ W1.T + b1
    h1 = rnd(gelu(z1))
    z2 = h1 @ W2.T + b2
    h2 = rnd(gelu(z2))
    y = h2 @ W3[0] + b3[0]
    return y, dict(F=F, z1=z1, h1=h1, z2=z2, h2=h2, W1=W1, W2=W2, W3=W3)


def backward(c, dy):
    """Gradients of sum(dy * y) with respect to every parameter (the rounding
    points are treated as identity, i.e. straight-through)."""
    dy = np.asarray(dy, np.float64)
    g = {"W3": (dy @ c["h2"])[None, :], "b3": np.array([dy.sum()])}
    dh2 = dy[:, None] * c["W3"][0][None, :]
    dz2 = dh2 * gelu_grad(c["z2"])
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ c["W2"]
    dz1 = dh1 * gelu_grad(c["z1"])
    g["W1"] = dz1.T @ c["F"]
    g["b1"] = dz1.sum(axis=0)
    return g


def softmax_kl(y, pstar, groups):
    """Sum over slices of KL(p* || softmax(y)) and its gradient dL/dy.
    groups: (S, n) view indices -- rows of slice s are groups[s]."""
    loss = 0.0
    dy = np.zeros_like(np.asarray(y, np.float64))
    for idx in groups:
        ys = np.asarray(y, np.float64)[idx]
        ps = np.asarray(pstar, np.float64)[idx]
        mx = ys.max()
        lse = mx + np.log(np.sum(np.exp(ys - mx)))
        logq = ys - lse
        nz = ps > 0
        loss += float(np.sum(ps[nz] * (np.log(ps[nz]) - logq[nz])))
        dy[idx] = np.exp(logq) - ps
    return loss, dy


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; t starts at 1."""
    out, mo, vo = {}, {}, {}
    for k in PARAM_ORDER:
        gk = np.asarray(g[k], np.float64)
        mo[k] = b1 * np.asarray(m[k], np.float64) + (1 - b1) * gk
        vo[k] = b2 * np.asarray(v[k], np.float64) + (1 - b2) * gk * gk
        mh = mo[k] / (1 - b1 ** t)
        vh = vo[k] / (1 - b2 ** t)
        out[k] = np.asarray(p[k], np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return out, mo, vo


def targets(tfull, n):
    """p*_j ~ sigma_j + TARGET_MIX mean(sigma) from a full slice matrix tfull (m', n')."""
    sig = np.asarray(tfull, np.float64).std(axis=0)
    w = sig + TARGET_MIX * (sig.mean() if sig.mean() > 0 else 1.0)
    return w / w.sum()


def weights_from_logits(y):
    """Integer column weights max(1, floor(2^24 exp(y - max y))) (FP32 logits)."""
    y = np.asarray(y, np.float32).astype(np.float64)
    e = np.exp(y - y.max())
    return np.maximum(1.0, np.floor(TWO24 * e)).astype(np.uint64)


def features(stats, slice_geo, clusters, cols, n1):
    """The 12 features of every column of one slice.

    stats: dict of per-column count, sum, sumsq, min, max, zeros of t over the
    first pass (FP64); slice_geo: centroid (3,), bbox diagonal, mean normal
    (3,); clusters: dict rep position (C,3), rep normal (C,3), intensity sum
    (C,), bbox diagonal (C,), member count (C,); cols: cluster ids of the
    slice's columns; n1: first-pass sample count."""
    n = cols.shape[0]
    cnt = stats["count"].astype(np.float64)
    tot = stats["sum"].sum()
    mu = tot / max(n1, 1)
    mu = mu if mu > 0 else 1e-30
    safe = np.maximum(cnt, 1.0)
    mean = stats["sum"] / safe
    var = np.maximum(0.0, stats["sumsq"] / safe - mean * mean)
    F = np.zeros((n, N_IN))
    F[:, 0] = np.log1p(mean / mu)
    F[:, 1] = np.log1p(np.sqrt(var) / mu)
    F[:, 2] = np.log1p(np.where(cnt > 0, stats["max"] - stats["min"], 0.0) / mu)
    F[:, 3] = cnt / (n1 / n)
    F[:, 4] = np.where(cnt > 0, stats["zeros"] / safe, 0.0)
    cen = np.asarray(slice_geo["centroid"], np.float64)
    diag = float(slice_geo["diag"]) + 1e-6
    mn = np.asarray(slice_geo["mean_normal"], np.float64)
    pos = clusters["pos"][cols]
    d = pos - cen
    dist = np.sqrt(np.sum(d * d, axis=1)) + 1e-6
    dirv = d / dist[:, None]
    F[:, 5] = np.log1p(clusters["bbox_diag"][cols] / dist)
    F[:, 6] = np.log1p(dist / diag)
    nn = np.sqrt(np.sum(mn * mn)) + 1e-12
    F[:, 7] = dirv @ (mn / nn)
    F[:, 8] = -np.sum(clusters["nrm"][cols] * dirv, axis=1)
    isum = clusters["intensity"][cols]
    F[:, 9] = np.log1p(isum / (isum.mean() + 1e-30))
    F[:, 10] = np.log(clusters["members"][cols].astype(np.float64))
    F[:, 11] = 1.0 - nn
    return F
