"""Two-pass random sampling of a slice matrix M (m' rows x n' columns),
Sec. 5 and the abstract.

First pass: uniformly distributed random entries.  Reading: N1 distinct
entries drawn uniformly without replacement, the count rounded half up from
a rate given in parts per million (N = floor((ppm D + 500000) / 10^6),
D = m' n').  Distinct uniform entries are the first N1 images of
0, 1, 2, ... under a keyed pseudo-random permutation of [0, D): a 4-round
balanced Feistel network (Luby-Rackoff) on 2h bits, h = ceil(b / 2),
b = max(2, ceil(log2 D)), with round function
    F_r(R) = Philox(key = (seed, s), ctr = (R, r, TAG_PASS1, 0))[0] & (2^h - 1),
    (L, R) -> (R, L xor F_r(R)),
restricted to [0, D) by cycle-walking (Black & Rogaway).  Entry e is
(i, j) = (e div n', e mod n').

PDF (Eq. pdf): pdf(i, j) ~ f(i) g(j) with f(i) = 1 and
g(j) = max(C_j) - min(C_j) over the observed entries C_j of column j.
Readings: the scalar observed per entry is t = R + G + B; g is fixed after
the first pass; a column with no observation has g = 0.  g is quantised to
integer weights w_j = 0 if g_j <= 0 else max(1, floor(2^24 g_j / max g))
(all 1 if every g is 0) so that column selection is an exact integer CDF
inversion.

Second pass (Sec. 5): select a column by g, then a row uniformly; if the
entry has not been sampled yet, evaluate it; repeat until the prescribed
number is reached.  Attempt t draws (r0, r1, .., ..) = Philox(key = (seed, s),
ctr = (t, 0, TAG_PASS2, 0)), j = least j with P_j > mulhi64(r0, P_last)
(P = inclusive prefix of w), i = mulhi64(r1, m').  It stops after N2
acceptances, N2 = min(round(ppm2 D), D - N1), or after 64 N2 + 65536
attempts (shortfall).  If N1 + N2 = D the second pass takes every
remaining entry in row-major order.

Pinned by: exhaustive bijectivity of the permutation for every D <= 4096,
exact counts, row/column marginal uniformity, pass-2 acceptance
probabilities enumerated exactly on tiny slices against frequencies over
many seeds, column frequencies proportional to w without collisions, and
the 100% case (tests/test_oracle_sampling.py).
"""
import numpy as np

from .philox import TAG_PASS1, TAG_PASS2, mulhi64, philox4x64_vec

TWO24 = float(1 << 24)
FEISTEL_ROUNDS = 4


def count_from_ppm(ppm, D):
    return (int(ppm) * int(D) + 500000) // 1000000


def feistel_half_bits(D):
    b = max(2, (int(D) - 1).bit_length())
    return (b + 1) // 2


def feistel(x, seed, s, h):
    """One application of the keyed Feistel permutation of [0, 2^(2h))."""
    x = np.asarray(x, dtype=np.uint64)
    mask = np.uint64((1 << h) - 1)
    L = x >> np.uint64(h)
    R = x & mask
    for rnd in range(FEISTEL_ROUNDS):
        F = philox4x64_vec(seed, s, R, rnd, TAG_PASS1, 0)[0] & mask
        L, R = R, L ^ F
    return (L << np.uint64(h)) | R


def pass1(seed, s, m, n, ppm):
    """First-pass entries of slice s as (i, j) int64 arrays, in draw order."""
    D = m * n
    N1 = count_from_ppm(ppm, D)
    h = feistel_half_bits(D)
    e = feistel(np.arange(N1, dtype=np.uint64), seed, s, h)
    out = e.copy()
    todo = np.nonzero(out >= np.uint64(D))[0]
    while todo.size:                     # cycle-walking
        out[todo] = feistel(out[todo], seed, s, h)
        todo = todo[out[todo] >= np.uint64(D)]
    e = out.astype(np.int64)
    return e // n, e % n


def column_stats(j, t, n):
    """Per-column count, mean, population variance, min, max of observations t."""
    cnt = np.bincount(j, minlength=n).astype(np.int64)
    sm = np.bincount(j, weights=t, minlength=n)
    sq = np.bincount(j, weights=t * t, minlength=n)
    mean = np.where(cnt > 0, sm / np.maximum(cnt, 1), 0.0)
    var = np.where(cnt > 0, np.maximum(0.0, sq / np.maximum(cnt, 1) - mean * mean), 0.0)
    mx = np.full(n, -np.inf)
    mn = np.full(n, np.inf)
    np.maximum.at(mx, j, t)
    np.minimum.at(mn, j, t)
    mx[cnt == 0] = 0.0
    mn[cnt == 0] = 0.0
    return cnt, mean, var, mn, mx


def importance(mn, mx, cnt):
    """g(j) = max(C_j) - min(C_j); 0 for an unobserved column (Sec. 5)."""
    return np.where(cnt > 0, mx - mn, 0.0)


def weights_from_g(g, mix=0.0):
    """Integer column weights of the second pass from g (Sec. 5).

    mix = 0 is the paper's density, w_j = 0 if g_j <= 0 else
    max(1, floor(2^24 g_j / max g)).  A positive mix adds mix times the mean
    weight to every column before rescaling to at most 2^24 (a density
    proportional to g(j) + mix mean g, a comparison baseline for the learned
    proposal; the paper uses g alone):
        q_j = the paper's weights, S = sum q_j,
        c = floor(fp32(mix) S / n'),
        w_j = q_j if c = 0, else max(1, floor(2^24 (q_j + c) / (2^24 + c))),
    every quotient in FP64 over exact integers.  mix = +inf is the uniform
    density, w_j = 1.
    """
    g = np.asarray(g, np.float64)
    mix32 = float(np.float32(mix))
    if not mix32 >= 0.0:
        raise ValueError("mix must be >= 0")
    if mix32 == np.inf:
        return np.ones(g.shape, dtype=np.uint64)
    gmax = g.max() if g.size else 0.0
    if not gmax > 0.0:
        return np.ones(g.shape, dtype=np.uint64)
    q = np.where(g > 0.0, np.maximum(1.0, np.floor(TWO24 * g / gmax)), 0.0)
    if not (q > 0).any():
        return np.ones(g.shape, dtype=np.uint64)
    q = q.astype(np.uint64)
    S = int(q.sum())
    c = int(np.floor(np.float64(mix32) * np.float64(S) / np.float64(g.shape[0])))
    if c == 0:
        return q
    f = np.floor(TWO24 * (q + np.uint64(c)).astype(np.float64) / np.float64(2 ** 24 + c))
    return np.maximum(1.0, f).astype(np.uint64)


def pass2(seed, s, m, n, N1, ppm2, w, taken1, batch=4096):
    """Second-pass entries (i, j) in acceptance order, and the shortfall flag.

    w: uint64 column weights (n,); taken1: boolean (m * n,) of first-pass
    entries.  Attempts are taken strictly in order t = 0, 1, 2, ...
    """
    D = m * n
    N2 = min(count_from_ppm(ppm2, D), D - N1)
    taken = taken1.copy()
    if N2 == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), False
    if N1 + N2 == D:                      # everything left, row-major order
        e = np.nonzero(~taken)[0]
        return e // n, e % n, False
    P = np.cumsum(np.asarray(w, dtype=np.uint64), dtype=np.uint64)
    total = int(P[-1])
    cap = 64 * N2 + 65536
    acc_i, acc_j = [], []
    t0 = 0
    while len(acc_i) < N2 and t0 < cap:
        t1 = min(cap, t0 + min(batch, max(64, 2 * (N2 - len(acc_i)))))
        ts = np.arange(t0, t1, dtype=np.uint64)
        r0, r1, _, _ = philox4x64_vec(seed, s, ts, 0, TAG_PASS2, 0)
        u = mulhi64(r0, np.uint64(total))
        jj = np.searchsorted(P, u, side="right").astype(np.int64)
        ii = mulhi64(r1, np.uint64(m)).astype(np.int64)
        for a in range(t1 - t0):          # sequential acceptance
            e = ii[a] * n + jj[a]
            if not taken[e]:
                taken[e] = True
                acc_i.append(int(ii[a]))
                acc_j.append(int(jj[a]))
                if len(acc_i) == N2:
                    break
        t0 = t1
    short = len(acc_i) < N2
    return np.asarray(acc_i, np.int64), np.asarray(acc_j, np.int64), short
