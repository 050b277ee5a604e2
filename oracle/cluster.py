"""Cluster table of a light cut (Sec. 4): a cut node L_f stands for the VPLs
below it.  Its intensity is the sum of its members' intensities
(I_f = I_a + I_b, applied recursively), and it keeps the position and
normal of one member (L_f "is the same as L_a except the intensity").

Readings (the paper does not say which member represents a node):
* the representative is drawn with probability proportional to the
  member's total intensity s = R + G + B, quantised to integer weights
  w_k = max(1, floor(2^24 s_k / max s)) (all 1 if max s = 0) so that the
  draw is an exact integer CDF inversion: rep = least k with
  P_k > mulhi64(r0, P_last), P the inclusive prefix of w, r0 the first word
  of Philox(key = (seed, 0), ctr = (cluster, 0, TAG_REP, 0));
* s is summed in FP64 from the FP32 inputs, R + G then + B;
* the intensity is the FP64 sum of member RGB in member order, rounded to
  FP32; the bounding box is the exact min/max of member positions.

Pinned by: a hand-worked two-member cluster, singleton clusters (rep is the
member, intensity its own), the member sums against math.fsum, and the
draw frequencies against the weights (tests/test_oracle_cluster.py).
"""
import numpy as np

from .philox import TAG_REP, mulhi64, philox4x64

TWO24 = float(1 << 24)


def quantized_weights(s):
    """Integer weights max(1, floor(2^24 s / max s)) from non-negative FP64 s."""
    s = np.asarray(s, dtype=np.float64)
    smax = s.max() if s.size else 0.0
    if not smax > 0.0:
        return np.ones(s.shape, dtype=np.uint64)
    return np.maximum(1.0, np.floor(TWO24 * s / smax)).astype(np.uint64)


def cluster_table(vpls, offsets, members, seed):
    """Return rep (int32 VPL id), intensity (n_c, 3) float32, bbox_lo/hi (n_c, 3) float32."""
    nc = offsets.shape[0] - 1
    ir = np.asarray(vpls["ir"], np.float32).astype(np.float64)
    ig = np.asarray(vpls["ig"], np.float32).astype(np.float64)
    ib = np.asarray(vpls["ib"], np.float32).astype(np.float64)
    pos = np.stack([vpls["x"], vpls["y"], vpls["z"]], axis=1).astype(np.float32)
    rep = np.zeros(nc, dtype=np.int32)
    inten = np.zeros((nc, 3), dtype=np.float32)
    lo = np.zeros((nc, 3), dtype=np.float32)
    hi = np.zeros((nc, 3), dtype=np.float32)
    for c in range(nc):
        mem = members[offsets[c]:offsets[c + 1]]
        if mem.shape[0] == 0:
            rep[c] = -1
            continue
        s = (ir[mem] + ig[mem]) + ib[mem]
        w = quantized_weights(s)
        P = np.cumsum(w, dtype=np.uint64)
        r0 = philox4x64((seed, 0), (c, 0, TAG_REP, 0))[0]
        u = mulhi64(r0, int(P[-1]))
        k = int(np.searchsorted(P, np.uint64(u), side="right"))
        rep[c] = mem[k]
        for ch, arr in enumerate((ir, ig, ib)):
            acc = 0.0
            for v in arr[mem]:         # FP64, member order
                acc += float(v)
            inten[c, ch] = np.float32(acc)
        lo[c] = pos[mem].min(axis=0)
        hi[c] = pos[mem].max(axis=0)
    return rep, inten, lo, hi
