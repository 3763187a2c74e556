"""Clustered neural visibility cache: cluster labels and two-step light sampling.

Test infrastructure (see the package docstring).

Sec. 3.6 ("Clustering"): for scenes with more lights than output neurons, the
lights are grouped into k clusters (k-means) and output neuron j predicts the
average visibility of cluster j.

* Training (Sec. 3.6): for every training sample and every cluster, one light
  of the cluster is chosen uniformly at random and the shadow ray to it gives
  the cluster's label.
* Sampling (Sec. 3.6), two steps:
  1. WRS picks a cluster y from the inferred cluster visibilities.  Reading
     (the weight is not written out): w_j = m_j * max(v_j, floor), the
     expected number of unoccluded lights of cluster j (m_j lights), so that
     a light's chance follows its cluster's visibility whatever the cluster
     size.  P(y) = w_y / sum_j w_j.
  2. Streaming RIS (Talbot et al. 2005) over N candidates drawn uniformly
     from the m_y lights of cluster y: source pdf p(x) = P(y) / m_y (the
     paper writes it as the first reservoir's weight times 1/m_y; read here
     as the probability with which x is generated), target p_hat(x) = f_x,
     the unshadowed weight of the plain method.  Candidate k has resampling
     weight p_hat(x_k) / p(x_k); one is kept with probability proportional
     to it, and its contribution weight is
         W = (1 / p_hat(x)) * (1/N) * sum_k p_hat(x_k) / p(x_k)
           = (S * m_y) / ((N * P(y)) * f_x),   S = sum_k f_{x_k}.
     f_x V_x W is an unbiased estimate of sum_i f_i V_i whenever every
     cluster holding a light with f V > 0 has P > 0 (the floor) and p_hat > 0
     there.

Random numbers: Philox4x32-10 with counter (index lo, index hi, frame, tag),
key = seed.  Tag 0: the cluster pick uniform (the plain method's pick
uniform); tag 2 word 0: the RIS selection uniform; tag 4 + k//4, word k%4:
candidate k's index in its cluster, floor(r * m_y / 2^32); tag 32 + c//4,
word c%4: the training light of cluster c, floor(r * m_c / 2^32).

The cluster and candidate picks are integers decided by floating point, so
`sample` runs in the dtype it is given (FP32 for parity with the kernel)
with this operation order:
    w_j = fl(m_j) * max(v_j, floor);  C_j sequential;  t = u * C_{k-1}
    y = first j with C_j > t (else the last positive w_j);  P = w_y / C_{k-1}
    f_k = unshadowed weight (lighting module order);  S_k sequential
    pick = first k with S_k > u2 * S_{N-1} (else the last positive f_k)
    W = (S_{N-1} * fl(m_y)) / ((fl(N) * P) * f_x)
"""
from __future__ import annotations

import itertools

import numpy as np

from . import lighting, philox, shadow

TAG_RIS_SELECT = 2
TAG_RIS_CAND = 4
TAG_CLUSTER_LIGHT = 32


def _words(seed: int, frame: int, n: int, tag: int):
    return philox.philox4x32_10(philox._counter(np.arange(n, dtype=np.uint64), frame, tag), philox._key(seed))


def _index_in(word, m):
    """floor(word * m / 2^32) for uint32 words and counts m (integer arithmetic)."""
    return ((np.asarray(word, np.uint64) * np.asarray(m, np.uint64)) >> np.uint64(32)).astype(np.int64)


def cluster_sizes(offsets) -> np.ndarray:
    offsets = np.asarray(offsets, np.int64)
    return offsets[1:] - offsets[:-1]


def training_lights(seed: int, frame: int, n: int, offsets, members) -> np.ndarray:
    """Light of every cluster for samples 0..n-1: int64 [n, k], -1 for an empty cluster."""
    offsets = np.asarray(offsets, np.int64)
    members = np.asarray(members, np.int64)
    m = cluster_sizes(offsets)
    k = m.shape[0]
    out = np.full((n, k), -1, np.int64)
    for c in range(k):
        if m[c] == 0:
            continue
        w = _words(seed, frame, n, TAG_CLUSTER_LIGHT + c // 4)[c % 4]
        out[:, c] = members[offsets[c] + _index_in(w, m[c])]
    return out


def labels(pos, lights, spheres, choice) -> np.ndarray:
    """uint8 [n, k]: visibility of each sample's chosen light per cluster (0 for an empty cluster),
    decided in FP32 like the plain labels."""
    pos = np.asarray(pos, np.float32)
    lights = np.asarray(lights, np.float32)
    choice = np.asarray(choice, np.int64)
    out = np.zeros(choice.shape, np.uint8)
    for c in range(choice.shape[1]):
        ok = choice[:, c] >= 0
        for l in np.unique(choice[ok, c]):
            rows = np.nonzero(choice[:, c] == l)[0]
            out[rows, c] = shadow.labels_fp32(pos[rows], lights[l:l + 1], spheres)[:, 0]
    return out


def cluster_weights(vis, sizes, floor: float = lighting.VIS_FLOOR, dtype=np.float64) -> np.ndarray:
    """w [n, k] = m_j * max(v_j, floor) in dtype."""
    sizes = np.asarray(sizes).astype(dtype)
    return sizes[None, :] * lighting.clamp_visibility(vis, floor, dtype)


def candidates(seed: int, frame: int, y, offsets, members, n_cand: int) -> np.ndarray:
    """RIS candidates int64 [n, N]: uniform lights of each pixel's cluster y (-1 where y < 0)."""
    offsets = np.asarray(offsets, np.int64)
    members = np.asarray(members, np.int64)
    y = np.asarray(y, np.int64)
    n = y.shape[0]
    ys = np.where(y >= 0, y, 0)
    m = cluster_sizes(offsets)[ys]
    out = np.full((n, n_cand), -1, np.int64)
    for kk in range(n_cand):
        w = _words(seed, frame, n, TAG_RIS_CAND + kk // 4)[kk % 4]
        idx = members[offsets[ys] + _index_in(w, np.maximum(m, 1))]
        out[:, kk] = np.where((y >= 0) & (m > 0), idx, -1)
    return out


def unshadowed_at(pos, nrm, lights, idx, dtype=np.float64) -> np.ndarray:
    """f [n, N] of light idx[i, k] at point i, with the operation order of lighting.unshadowed_weight."""
    dt = np.dtype(dtype).type
    p = np.asarray(pos).astype(dtype)
    L = np.asarray(lights).astype(dtype)[np.asarray(idx, np.int64)]         # [n, N, 4]
    dx = L[..., 0] - p[:, None, 0]
    dy = L[..., 1] - p[:, None, 1]
    dz = L[..., 2] - p[:, None, 2]
    d2 = np.fmax((dx * dx + dy * dy) + dz * dz, dt(1e-6))
    if nrm is None:
        return L[..., 3] / d2
    n = np.asarray(nrm).astype(dtype)
    nd = (n[:, None, 0] * dx + n[:, None, 1] * dy) + n[:, None, 2] * dz
    return (L[..., 3] * np.fmax(nd, dt(0.0))) / (d2 * np.sqrt(d2))


def sample(vis, pos, nrm, lights, offsets, members, seed: int, frame: int, n_cand: int,
           floor: float = lighting.VIS_FLOOR, dtype=np.float32) -> dict:
    """Two-step pick per pixel.  Returns dict(idx [n] light or -1, cluster [n] or -1, W [n], P [n])."""
    dt = np.dtype(dtype).type
    offsets = np.asarray(offsets, np.int64)
    sizes = cluster_sizes(offsets)
    n = np.asarray(vis).shape[0]
    w = cluster_weights(vis, sizes, floor, dtype)
    u = philox.wrs_uniforms(seed, frame, n)
    y, P, _ = lighting.wrs_pick(w, u)
    cand = candidates(seed, frame, y, offsets, members, n_cand)
    safe = np.where(cand >= 0, cand, 0)
    f = np.where(cand >= 0, unshadowed_at(pos, nrm, lights, safe, dtype), dt(0))
    u2 = philox.uniform24(_words(seed, frame, n, TAG_RIS_SELECT)[0])
    kpick, _, S = lighting.wrs_pick(f, u2)
    ok = (kpick >= 0) & (y >= 0)
    ks = np.where(ok, kpick, 0)
    idx = np.where(ok, np.take_along_axis(cand, ks[:, None], axis=1)[:, 0], -1).astype(np.int64)
    fx = np.take_along_axis(f, ks[:, None], axis=1)[:, 0]
    my = sizes[np.where(y >= 0, y, 0)].astype(dtype)
    with np.errstate(invalid="ignore", divide="ignore"):
        W = np.where(ok, (S * my) / ((dt(n_cand) * P) * fx), dt(0)).astype(dtype)
        w_sum = np.where(ok, (S * my) / P, dt(0)).astype(dtype)    # sum of the resampling weights f_k m_y / P
    return {"idx": idx, "cluster": np.where(ok, y, -1).astype(np.int64), "W": W, "w_sum": w_sum,
            "P": np.where(y >= 0, P, dt(0))}


def expected_estimate(f, V, vhat, sizes, members_of, n_cand: int) -> float:
    """Exact E[f_x V_x W] of the two-step sampler at one point (FP64), by enumerating every cluster and
    every N-tuple of candidates (tiny cases only).  f, V: [L] per light; vhat: [k] clamped cluster
    visibilities; members_of[j]: the light indices of cluster j."""
    w = np.asarray(sizes, np.float64) * np.asarray(vhat, np.float64)
    P = w / w.sum()
    total = 0.0
    for j, mem in enumerate(members_of):
        if len(mem) == 0 or P[j] == 0:
            continue
        for tup in itertools.product(mem, repeat=n_cand):
            S = sum(f[x] for x in tup)
            if S == 0:
                continue
            # candidate tuple probability (1/m)^N; selection of x with probability f_x / S
            p_tup = (1.0 / len(mem)) ** n_cand
            for x in tup:                                  # the k-th candidate kept with prob f_x / S
                if f[x] == 0:
                    continue
                Wx = (S * len(mem)) / (n_cand * P[j] * f[x])
                total += P[j] * p_tup * (f[x] / S) * f[x] * V[x] * Wx
    return total


def kmeans(lights, k: int, iters: int = 20):
    """Lloyd's k-means of the light positions (Sec. 3.6 clusters the lights with k-means), FP64.

    Initial centroids by farthest points: light 0, then repeatedly the light farthest (squared
    distance to its nearest chosen centroid; ties to the lower index) from those chosen.  Each iteration assigns
    every light to its nearest centroid (squared distance (dx*dx + dy*dy) + dz*dz, ties to the lower
    cluster) and moves every non-empty cluster's centroid to the mean of its lights (coordinates summed
    sequentially in light order, then divided by the count); it stops after `iters` iterations or when
    no assignment changes.  Returns CSR (offsets [k+1], members [n] grouped by cluster, ascending light
    index within a cluster)."""
    P = np.asarray(lights, np.float32)[:, :3].astype(np.float64)
    n = P.shape[0]
    if not 1 <= k <= n:
        raise ValueError("need 1 <= k <= number of lights")
    def d2_to(c):
        dx, dy, dz = P[:, 0] - c[0], P[:, 1] - c[1], P[:, 2] - c[2]
        return (dx * dx + dy * dy) + dz * dz

    cent = np.empty((k, 3))
    cent[0] = P[0]
    dmin = d2_to(cent[0])
    for j in range(1, k):
        cent[j] = P[int(np.argmax(dmin))]                            # first maximum: lower index
        dmin = np.minimum(dmin, d2_to(cent[j]))
    assign = np.full(n, -1, np.int64)
    for _ in range(iters):
        dx = P[:, None, 0] - cent[None, :, 0]
        dy = P[:, None, 1] - cent[None, :, 1]
        dz = P[:, None, 2] - cent[None, :, 2]
        new = np.argmin((dx * dx + dy * dy) + dz * dz, axis=1)         # first minimum: lower cluster
        changed = np.any(new != assign)
        assign = new
        for j in range(k):
            idx = np.nonzero(assign == j)[0]
            if idx.size:
                cent[j] = np.cumsum(P[idx], axis=0)[-1] / idx.size   # sequential sums
        if not changed:
            break
    members = np.argsort(assign, kind="stable")
    offsets = np.concatenate([[0], np.cumsum(np.bincount(assign, minlength=k))])
    return offsets.astype(np.int64), members.astype(np.int64)
