"""Seeded synthetic inputs for TPO clustering jobs.

This module holds no step of the clustering method itself. It produces

* planted-partition attributed bipartite graphs (ABGs): a degree-corrected
  bipartite stochastic block model with Zipf degree weights, unique unweighted
  edges in random order, and Gaussian-mixture attributes on the target side U
  (the paper's ABG model, Section 2.1); and
* the Gaussian random matrices the method draws (the matrix G of Algorithm 1,
  the sketching matrices of the randomized SVDs), from a counter-based
  generator: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) turned into
  uniforms on (0, 1] with 53 bits and into normals with the Box-Muller
  transform.  The native library carries its own implementation of the same
  published generator; both sides are checked against each other.

Both the FP64 oracle and the GPU path take their inputs from here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ABG",
    "JobShape",
    "CONFIGS",
    "tfidf_csr",
    "planted_abg",
    "splitmix64_normals",
    "method_matrices",
    "STREAM_OMEGA_REDUCE",
    "STREAM_G",
    "STREAM_OMEGA",
]

# ---------------------------------------------------------------------------
# Counter-based normal generator (SplitMix64 -> 53-bit uniform -> Box-Muller)
# ---------------------------------------------------------------------------
_MASK64 = (1 << 64) - 1
_GOLDEN_GAMMA = 0x9E3779B97F4A7C15
_STREAM_SALT = 0x632BE59BD9B4E019

STREAM_OMEGA_REDUCE = 0  # d_U x l_r sketch for the attribute reduction
STREAM_G = 1             # d x d Gaussian matrix G of Algorithm 1
STREAM_OMEGA = 2         # 2d x k' sketch for RandomizedSVD(R, k)


def _splitmix64_next(state: int) -> tuple[int, int]:
    state = (state + _GOLDEN_GAMMA) & _MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    z = z ^ (z >> 31)
    return state, z


def splitmix64_normals(seed: int, stream: int, count: int) -> np.ndarray:
    """`count` standard normals of stream `stream` under `seed`.

    The stream's SplitMix64 state starts at seed XOR (salt * (stream + 1)).
    Each pair of 64-bit outputs (a, b) gives u1 = ((a >> 11) + 1) * 2^-53 and
    u2 = ((b >> 11) + 1) * 2^-53, both in (0, 1], and the two normals
    sqrt(-2 ln u1) cos(2 pi u2), sqrt(-2 ln u1) sin(2 pi u2), emitted in that
    order.  Scalar libm calls (math.log / math.cos / math.sin / math.sqrt) are
    used so that the native implementation can reproduce every bit.
    """
    if count < 0:
        raise ValueError("count must be >= 0")
    state = (int(seed) ^ ((_STREAM_SALT * (int(stream) + 1)) & _MASK64)) & _MASK64
    out = np.empty(count, dtype=np.float64)
    two_pi = 2.0 * math.pi
    scale = 1.0 / 9007199254740992.0  # 2^-53
    i = 0
    while i < count:
        state, a = _splitmix64_next(state)
        state, b = _splitmix64_next(state)
        u1 = ((a >> 11) + 1) * scale
        u2 = ((b >> 11) + 1) * scale
        rad = math.sqrt(-2.0 * math.log(u1))
        out[i] = rad * math.cos(two_pi * u2)
        if i + 1 < count:
            out[i + 1] = rad * math.sin(two_pi * u2)
        i += 2
    return out


@dataclass(frozen=True)
class MethodMatrices:
    """Random matrices one clustering job draws (row-major float64)."""

    omega_reduce: np.ndarray | None  # d_U x l_r, or None when no reduction
    g: np.ndarray                    # d x d
    omega: np.ndarray                # 2d x k'


def sketch_widths(d_u: int, d: int, k: int, oversample: int) -> tuple[int, int, int]:
    """(d_eff, l_r, k') for a job: the working attribute width, the width of
    the reduction sketch, and the width of the embedding sketch.

    d_eff = d_u when d <= 0 or d >= d_u (no reduction).  l_r = min(d + p, d_u),
    k' = min(k + p, 2 d_eff).  Shared by the generator and the native planner,
    which compute it independently.
    """
    d_eff = d_u if (d <= 0 or d >= d_u) else d
    l_r = min(d_eff + oversample, d_u) if d_eff < d_u else 0
    kp = min(k + oversample, 2 * d_eff)
    return d_eff, l_r, kp


def method_matrices(seed: int, d_u: int, d: int, k: int, oversample: int = 10) -> MethodMatrices:
    d_eff, l_r, kp = sketch_widths(d_u, d, k, oversample)
    om_r = None
    if l_r > 0:
        om_r = splitmix64_normals(seed, STREAM_OMEGA_REDUCE, d_u * l_r).reshape(d_u, l_r)
    g = splitmix64_normals(seed, STREAM_G, d_eff * d_eff).reshape(d_eff, d_eff)
    om = splitmix64_normals(seed, STREAM_OMEGA, 2 * d_eff * kp).reshape(2 * d_eff, kp)
    return MethodMatrices(om_r, g, om)


# ---------------------------------------------------------------------------
# Planted-partition ABG generator
# ---------------------------------------------------------------------------
@dataclass
class ABG:
    n_u: int
    n_v: int
    edge_u: np.ndarray          # int32 [E]
    edge_v: np.ndarray          # int32 [E]
    x_u: np.ndarray             # float32 [n_u, d_u]
    labels_u: np.ndarray        # int32 planted cluster of each u
    labels_v: np.ndarray        # int32 planted cluster of each v
    edge_w: np.ndarray | None = None  # float32 [E] or None (unweighted)
    meta: dict = field(default_factory=dict)

    @property
    def n_edges(self) -> int:
        return int(self.edge_u.shape[0])

    @property
    def d_u(self) -> int:
        return int(self.x_u.shape[1])


@dataclass(frozen=True)
class JobShape:
    """One clustering job: graph recipe plus method parameters."""

    name: str
    n_u: int
    n_v: int
    n_edges: int
    k: int
    zipf_a: float
    d_u: int
    d: int              # reduced width; 0 => no reduction
    gamma: int
    alpha: float = 0.5
    q: int = 20
    oversample: int = 10
    t_f: int = 5
    t_g: int = 20
    sigma: float = 1.5
    in_out_ratio: float = 8.0
    max_degree: int | None = None


CONFIGS: dict[str, JobShape] = {
    # Plain method at CPU scale: 2,000 x 3,000, 20,000 edges, k = 5, 5 hops.
    "cpu_scale": JobShape("cpu_scale", 2_000, 3_000, 20_000, k=5, zipf_a=2.1,
                          d_u=64, d=0, gamma=5),
    # Mid-size FP32 GPU path: 200k x 400k, 4M edges, k = 20, 10 hops,
    # 256 attribute columns reduced to 64.
    "mid_fp32": JobShape("mid_fp32", 200_000, 400_000, 4_000_000, k=20, zipf_a=2.0,
                         d_u=256, d=64, gamma=10),
    # Large graph: 5M x 10M, 150M edges, k = 100, 512 attributes -> 64.
    "large": JobShape("large", 5_000_000, 10_000_000, 150_000_000, k=100, zipf_a=1.9,
                      d_u=512, d=64, gamma=10, max_degree=100_000),
    # Sparse text-like attributes: 2M x 2M, 60M edges, k = 50, 4,096 TF-IDF
    # columns at 2% density (tfidf_fp8_device) handed over as FP8 E4M3 with
    # column scales, reduced to 64.
    "fp8_tfidf": JobShape("fp8_tfidf", 2_000_000, 2_000_000, 60_000_000, k=50, zipf_a=2.0,
                          d_u=4096, d=64, gamma=10, max_degree=100_000),
}


def _zipf_weights(rng: np.random.Generator, a: float, n: int) -> np.ndarray:
    return rng.zipf(a, size=n).astype(np.float64)


def _cap_weights(theta: np.ndarray, n_edges: int, max_degree: float) -> np.ndarray:
    """Clip weights so that no node's expected degree n_edges*theta/sum(theta)
    exceeds max_degree (fixed point of the clip, a few rounds suffice)."""
    t = theta.copy()
    for _ in range(50):
        cap = max_degree * t.sum() / n_edges
        if t.max() <= cap * (1 + 1e-12):
            break
        t = np.minimum(t, cap)
    return t


def planted_abg(n_u: int, n_v: int, n_edges: int, k: int, d_u: int, *,
                zipf_a: float = 2.0, sigma: float = 1.5, in_out_ratio: float = 8.0,
                max_degree: int | None = None, seed: int = 0,
                weighted: bool = False) -> ABG:
    """Degree-corrected bipartite SBM with k equal planted clusters.

    * Planted labels: c_u = i mod k and c_v = j mod k under a seeded shuffle.
    * Degree weights theta ~ Zipf(zipf_a), clipped so the largest expected
      degree is max_degree (default: a quarter of the other side, at most 1e5).
    * Each edge draws u with probability proportional to theta_u, then v's
      cluster (same as u's with probability r/(r + k - 1), r = in_out_ratio,
      else uniform over the other k - 1 clusters, so p_in/p_out = r), then v
      proportional to theta_v inside that cluster.  The first n_edges distinct
      (u, v) pairs are kept, in draw order; isolated nodes may remain.
    * Attributes: X_u = mu_{c_u} + sigma * eps with mu_c ~ N(0, I), stored
      float32.
    * weighted=True attaches log-normal edge weights (for weighted-path tests).
    """
    if k < 1 or n_u < 1 or n_v < 1:
        raise ValueError("bad sizes")
    if n_edges > n_u * n_v:
        raise ValueError("more edges than vertex pairs")
    rng = np.random.default_rng(seed)
    cu = (rng.permutation(n_u) % k).astype(np.int32)
    cv = (rng.permutation(n_v) % k).astype(np.int32)

    th_u = _zipf_weights(rng, zipf_a, n_u)
    th_v = _zipf_weights(rng, zipf_a, n_v)
    mdu = max_degree if max_degree is not None else min(max(n_v // 4, 1), 100_000)
    mdv = max_degree if max_degree is not None else min(max(n_u // 4, 1), 100_000)
    th_u = _cap_weights(th_u, n_edges, mdu)
    th_v = _cap_weights(th_v, n_edges, mdv)

    cdf_u = np.cumsum(th_u)
    cdf_u /= cdf_u[-1]
    # V nodes grouped by cluster for within-cluster sampling.
    order_v = np.argsort(cv, kind="stable")
    cum_v = np.cumsum(th_v[order_v])
    starts = np.searchsorted(cv[order_v], np.arange(k), side="left")
    ends = np.searchsorted(cv[order_v], np.arange(k), side="right")
    lo = np.where(starts > 0, cum_v[np.maximum(starts - 1, 0)], 0.0)
    hi = cum_v[np.maximum(ends - 1, 0)]
    hi = np.where(ends > starts, hi, lo)

    p_same = in_out_ratio / (in_out_ratio + k - 1) if k > 1 else 1.0
    keys_kept = np.empty(0, dtype=np.int64)
    need = n_edges
    chunks = []
    seen = None
    batch = max(int(n_edges * 1.3), 1024)
    for _ in range(1000):
        if need <= 0:
            break
        uu = np.searchsorted(cdf_u, rng.random(batch), side="right")
        uu = np.minimum(uu, n_u - 1)
        same = rng.random(batch) < p_same
        if k > 1:
            off = rng.integers(1, k, size=batch)
            cl = np.where(same, cu[uu], (cu[uu] + off) % k)
        else:
            cl = np.zeros(batch, dtype=np.int64)
        empty = ends[cl] <= starts[cl]
        tgt = lo[cl] + rng.random(batch) * (hi[cl] - lo[cl])
        pos = np.searchsorted(cum_v, tgt, side="right")
        pos = np.clip(pos, starts[cl], np.maximum(ends[cl] - 1, starts[cl]))
        vv = order_v[np.minimum(pos, n_v - 1)]
        keep = ~empty
        key = uu[keep].astype(np.int64) * n_v + vv[keep].astype(np.int64)
        # distinct within the batch, first occurrence order
        _, first = np.unique(key, return_index=True)
        key = key[np.sort(first)]
        if seen is not None:
            key = key[~np.isin(key, seen)]
        take = key[:need]
        chunks.append(take)
        seen = take if seen is None else np.concatenate([seen, take])
        need -= take.shape[0]
    if need > 0:
        raise RuntimeError("could not draw enough distinct edges")
    keys_kept = np.concatenate(chunks)
    eu = (keys_kept // n_v).astype(np.int32)
    ev = (keys_kept % n_v).astype(np.int32)

    mu = rng.standard_normal((k, d_u))
    x = mu[cu] + sigma * rng.standard_normal((n_u, d_u))
    w = None
    if weighted:
        w = rng.lognormal(0.0, 0.5, size=eu.shape[0]).astype(np.float32)
    return ABG(n_u, n_v, eu, ev, x.astype(np.float32), cu, cv, w,
               meta=dict(seed=seed, zipf_a=zipf_a, sigma=sigma, k=k,
                         in_out_ratio=in_out_ratio, max_degree_u=mdu,
                         max_degree_v=mdv))


def planted_attributes(labels: np.ndarray, d: int, *, sigma: float = 1.5, seed: int = 0) -> np.ndarray:
    """Attributes for nodes with the given planted clusters, by the recipe of
    planted_abg (X = mu_c + sigma * eps, mu_c ~ N(0, I)) from a random stream
    of their own: used for X_V when V is the target set."""
    labels = np.asarray(labels)
    rng = np.random.default_rng([seed, 0x5856])
    k = int(labels.max()) + 1 if labels.size else 0
    mu = rng.standard_normal((k, d))
    x = mu[labels] + sigma * rng.standard_normal((labels.shape[0], d))
    return x.astype(np.float32)


def quantize_e4m3(x: np.ndarray):
    """Per-column FP8 E4M3 (OCP e4m3fn) encoding of an attribute matrix: scale
    s_j = max_i |x_ij| / 448 (the largest finite E4M3 magnitude; 1 for an
    all-zero column), codes = round-to-nearest-even of x_ij / s_j.  Returns
    (codes uint8 [n, d], s float32 [d], the encoded values code * s in
    float64: what a consumer of the codes and scales sees)."""
    import torch

    x = np.asarray(x, dtype=np.float32)
    amax = np.abs(x).max(axis=0) if x.shape[0] else np.zeros(x.shape[1], np.float32)
    scale = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    t = torch.from_numpy(np.ascontiguousarray(x / scale[None, :])).clamp(-448.0, 448.0)
    q = t.to(torch.float8_e4m3fn)
    codes = q.view(torch.uint8).numpy().copy()
    values = q.to(torch.float64).numpy() * scale.astype(np.float64)[None, :]
    return codes, scale, values


def _tfidf_rows(labels, d_u: int, *, device, density: float, topic_frac: float, zipf_s: float,
                lognormal_sigma: float, seed: int):
    """The TF-IDF row recipe shared by tfidf_fp8_device and tfidf_csr: returns
    values(r0, r1), the dense float32 rows [r0, r1) on `device`."""
    import torch

    labels = labels.to(device=device, dtype=torch.int64)
    n = labels.numel()
    k = int(labels.max().item()) + 1 if n else 1
    nnz = max(1, int(round(density * d_u)))
    gh = torch.Generator().manual_seed(int(seed) * 7919 + 17)
    ranks = torch.arange(1, d_u + 1, dtype=torch.float64) ** (-zipf_s)
    p = torch.empty(d_u, dtype=torch.float64)
    p[torch.randperm(d_u, generator=gh)] = ranks / ranks.sum()
    w = torch.log(1.0 / p).to(torch.float32).to(device)
    p_bg = p.to(torch.float32).to(device)
    t = max(1, d_u // k)
    topics = (torch.randperm(d_u, generator=gh).repeat((k * t + d_u - 1) // d_u)[: k * t].view(k, t)).to(device)
    g = torch.Generator(device=device)

    def values(r0, r1):
        g.manual_seed(int(seed) * 1_000_003 + r0)
        m = r1 - r0
        lab = labels[r0:r1]
        from_topic = torch.rand(m, nnz, generator=g, device=device) < topic_frac
        tcol = topics[lab][torch.arange(m, device=device)[:, None],
                           torch.randint(0, t, (m, nnz), generator=g, device=device)]
        bcol = torch.multinomial(p_bg, m * nnz, replacement=True, generator=g).view(m, nnz)
        col = torch.where(from_topic, tcol, bcol)
        wts = torch.exp(lognormal_sigma * torch.randn(m, nnz, generator=g, device=device))
        tf = torch.zeros(m, d_u, device=device)
        tf.scatter_add_(1, col, wts)
        val = tf * w[None, :]
        return val / val.norm(dim=1, keepdim=True).clamp_min(1e-30)

    return values, n


def tfidf_fp8_device(labels, d_u: int, *, device, density: float = 0.02, topic_frac: float = 0.5,
                     zipf_s: float = 1.1, lognormal_sigma: float = 0.5, seed: int = 0, chunk: int = 131_072):
    """Sparse TF-IDF-like attributes for nodes with planted clusters, drawn
    on a GPU with torch and encoded as FP8 E4M3 with one scale per column.

    * Each row draws round(density * d_u) words with replacement: with
      probability topic_frac from its cluster's topic (d_u // k columns of a
      seeded permutation, wrapping), else from a background Zipf(zipf_s) law
      over a seeded permutation of the columns.
    * Each draw carries a log-normal weight exp(lognormal_sigma * N(0, 1));
      value = (sum of the word's weights in the row) * w_j, with
      w_j = log(1 / p_j) (the background probability's inverse document
      frequency); rows scaled to unit L2 norm.
    * Column scale s_j = max_i x_ij / 448; codes = E4M3 round to nearest even
      of x_ij / s_j (the quantize_e4m3 recipe).
    Rows are drawn in chunks from per-chunk seeds, twice (column maxima, then
    codes), so the n x d_u float matrix never exists whole.  Returns (codes
    uint8 [n, d_u], scales float32 [d_u]) on the device."""
    import torch

    values, n = _tfidf_rows(labels, d_u, device=device, density=density, topic_frac=topic_frac, zipf_s=zipf_s,
                            lognormal_sigma=lognormal_sigma, seed=seed)
    colmax = torch.zeros(d_u, device=device)
    for r0 in range(0, n, chunk):
        colmax = torch.maximum(colmax, values(r0, min(n, r0 + chunk)).amax(dim=0))
    scale = torch.where(colmax > 0, colmax / 448.0, torch.ones_like(colmax)).to(torch.float32)
    codes = torch.empty(n, d_u, dtype=torch.uint8, device=device)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        q = (values(r0, r1) / scale[None, :]).clamp(-448.0, 448.0).to(torch.float8_e4m3fn)
        codes[r0:r1] = q.view(torch.uint8)
    return codes, scale


def tfidf_csr(labels, d_u: int, *, device, density: float = 0.02, topic_frac: float = 0.5, zipf_s: float = 1.1,
              lognormal_sigma: float = 0.5, seed: int = 0, chunk: int = 131_072):
    """The same TF-IDF rows as tfidf_fp8_device, kept sparse and in FP32:
    returns (rowptr int64 [n + 1], col int32 [nnz], val float32 [nnz]) on
    `device`, columns ascending within a row."""
    import torch

    values, n = _tfidf_rows(labels, d_u, device=device, density=density, topic_frac=topic_frac, zipf_s=zipf_s,
                            lognormal_sigma=lognormal_sigma, seed=seed)
    counts, cols, vals = [], [], []
    for r0 in range(0, n, chunk):
        v = values(r0, min(n, r0 + chunk))
        nz = v != 0
        counts.append(nz.sum(dim=1))
        idx = nz.nonzero(as_tuple=True)
        cols.append(idx[1].to(torch.int32))
        vals.append(v[idx])
    cnt = torch.cat(counts) if counts else torch.zeros(0, dtype=torch.int64, device=device)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(cnt, 0)
    col = torch.cat(cols) if cols else torch.zeros(0, dtype=torch.int32, device=device)
    val = torch.cat(vals) if vals else torch.zeros(0, dtype=torch.float32, device=device)
    return rowptr, col.contiguous(), val.contiguous()


def e4m3_value(code: int) -> float:
    """The OCP E4M3 (e4m3fn) value of one byte from the format's definition:
    sign bit, 4 exponent bits with bias 7, 3 mantissa bits; exponent 0 is
    subnormal (m / 8 * 2^-6); 0x7F and 0xFF are NaN; no infinities."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 7
    if e == 0xF and m == 7:
        return float("nan")
    if e == 0:
        return s * (m / 8.0) * 2.0 ** -6
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def target_v(abg: ABG, x_v: np.ndarray) -> ABG:
    """The same graph with V as the target set: the two sides exchanged
    (every edge (u, v) read as (v, u)) and x_v as the target's attributes."""
    if x_v.shape[0] != abg.n_v:
        raise ValueError("x_v needs one row per node of V")
    return ABG(abg.n_v, abg.n_u, abg.edge_v.copy(), abg.edge_u.copy(), np.ascontiguousarray(x_v, np.float32),
               abg.labels_v, abg.labels_u, None if abg.edge_w is None else abg.edge_w.copy(),
               meta=dict(abg.meta, target="V"))


def planted_abg_device(n_u: int, n_v: int, n_edges: int, k: int, d_u: int, *, device,
                       zipf_a: float = 2.0, sigma: float = 1.5, in_out_ratio: float = 8.0,
                       max_degree: int | None = None, seed: int = 0):
    """The planted model of planted_abg drawn on a GPU with torch, for sizes
    where the host generator is too slow (hundreds of millions of edges).
    Same recipe (Zipf degree weights capped at max_degree, p_in/p_out =
    in_out_ratio, the first n_edges distinct pairs in draw order, X = mu_c +
    sigma * eps), different random streams: the graphs are not the host
    generator's.  Returns device tensors (edge_u, edge_v int32, x_u float32
    n_u x d_u, labels_u, labels_v int64)."""
    import torch

    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 1000003 + 17)
    cu = torch.from_numpy((rng.permutation(n_u) % k).astype(np.int64)).to(device)
    cv_np = (rng.permutation(n_v) % k).astype(np.int64)
    th_u = _zipf_weights(rng, zipf_a, n_u)
    th_v = _zipf_weights(rng, zipf_a, n_v)
    mdu = max_degree if max_degree is not None else min(max(n_v // 4, 1), 100_000)
    mdv = max_degree if max_degree is not None else min(max(n_u // 4, 1), 100_000)
    th_u = _cap_weights(th_u, n_edges, mdu)
    th_v = _cap_weights(th_v, n_edges, mdv)
    cdf_u = torch.from_numpy(np.cumsum(th_u) / th_u.sum()).to(device)
    order_v = np.argsort(cv_np, kind="stable")
    cum_v_np = np.cumsum(th_v[order_v])
    starts = np.searchsorted(cv_np[order_v], np.arange(k), side="left")
    ends = np.searchsorted(cv_np[order_v], np.arange(k), side="right")
    lo = np.where(starts > 0, cum_v_np[np.maximum(starts - 1, 0)], 0.0)
    hi = np.where(ends > starts, cum_v_np[np.maximum(ends - 1, 0)], lo)
    cum_v = torch.from_numpy(cum_v_np).to(device)
    lo_t, hi_t = torch.from_numpy(lo).to(device), torch.from_numpy(hi).to(device)
    st_t = torch.from_numpy(starts).to(device)
    en_t = torch.from_numpy(np.maximum(ends - 1, starts)).to(device)
    order_v_t = torch.from_numpy(order_v.astype(np.int64)).to(device)
    p_same = in_out_ratio / (in_out_ratio + k - 1) if k > 1 else 1.0
    kept = None
    for _ in range(20):
        batch = int(n_edges * 1.25) + 1024
        uu = torch.searchsorted(cdf_u, torch.rand(batch, generator=gen, device=device, dtype=torch.float64),
                                right=True).clamp_(max=n_u - 1)
        same = torch.rand(batch, generator=gen, device=device) < p_same
        if k > 1:
            off = torch.randint(1, k, (batch,), generator=gen, device=device)
            cl = torch.where(same, cu[uu], (cu[uu] + off) % k)
        else:
            cl = torch.zeros(batch, dtype=torch.int64, device=device)
        tgt = lo_t[cl] + torch.rand(batch, generator=gen, device=device, dtype=torch.float64) * (hi_t[cl] - lo_t[cl])
        pos = torch.searchsorted(cum_v, tgt, right=True)
        pos = torch.minimum(torch.maximum(pos, st_t[cl]), en_t[cl])
        vv = order_v_t[pos]
        key = uu * n_v + vv
        del uu, same, cl, tgt, pos, vv
        key = key if kept is None else torch.cat([kept, key])
        # distinct keys, first occurrence order
        sk, perm = torch.sort(key, stable=True)
        first = torch.ones_like(sk, dtype=torch.bool)
        first[1:] = sk[1:] != sk[:-1]
        pos_first = torch.sort(perm[first]).values
        kept = key[pos_first]
        del sk, perm, first, pos_first, key
        if kept.numel() >= n_edges:
            kept = kept[:n_edges]
            break
    if kept.numel() < n_edges:
        raise RuntimeError("could not draw enough distinct edges")
    eu = (kept // n_v).to(torch.int32)
    ev = (kept % n_v).to(torch.int32)
    del kept
    mu = torch.randn(k, d_u, generator=gen, device=device)
    x = torch.randn(n_u, d_u, generator=gen, device=device).mul_(sigma).add_(mu[cu])
    return eu, ev, x, cu, torch.from_numpy(cv_np).to(device)


def config_abg(shape: JobShape, seed: int = 0) -> ABG:
    return planted_abg(shape.n_u, shape.n_v, shape.n_edges, shape.k, shape.d_u,
                       zipf_a=shape.zipf_a, sigma=shape.sigma,
                       in_out_ratio=shape.in_out_ratio,
                       max_degree=shape.max_degree, seed=seed)


@dataclass(frozen=True)
class ServingRequest:
    """One request of the serving stream: its arrival time, the index of its
    graph in the pool, and its method parameters."""

    arrival: float
    graph: int
    k: int
    d: int
    params: dict


def serving_stream(n_requests: int, rate: float, pool: int, seed: int = 0, *,
                   n_min: int = 1_000, n_max: int = 500_000, deg=(10.0, 30.0), k_range=(2, 64),
                   d_choices=(32, 128, 256)):
    """The serving workload: Poisson arrivals at `rate` jobs/s of independent
    planted-partition jobs.  Graph shapes: |U| log-uniform in [n_min, n_max],
    |V| = 1.5 |U|, average degree uniform in `deg`, k uniform in k_range,
    attribute width d_U from d_choices reduced to min(d_U, 64), 5 hops,
    alpha 0.5.  `pool` distinct graphs are described (shapes and seeds);
    requests draw one of them each.  Returns (shapes, requests): shapes[i] =
    (n_u, n_v, n_edges, k, d_u, seed) of pool graph i."""
    rng = np.random.default_rng(seed)
    shapes = []
    for i in range(pool):
        n_u = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        n_v = int(round(1.5 * n_u))
        n_edges = int(round(n_u * rng.uniform(*deg)))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        d_u = int(rng.choice(d_choices))
        shapes.append((n_u, n_v, n_edges, k, d_u, seed * 7919 + i))
    t = 0.0
    reqs = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate)
        g = int(rng.integers(0, pool))
        n_u, n_v, n_edges, k, d_u, _ = shapes[g]
        d = min(d_u, 64)
        params = dict(k=k, alpha=0.5, gamma=5, d=d if d < d_u else 0, q=20, oversample=10, t_f=5, t_g=20,
                      seed=g)
        reqs.append(ServingRequest(t, g, k, d, params))
    return shapes, reqs
