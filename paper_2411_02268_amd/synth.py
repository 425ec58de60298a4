"""Seeded synthetic graphs (inputs only; none of the method's arithmetic lives here).

Every generator returns an undirected graph as a symmetric CSR triple
``(offsets int64[n+1], indices int32[nnz], weights uint32[nnz])`` with rows sorted
by column, no self-loops and no duplicate entries.  A weight is a function of the
unordered vertex pair and the seed, so w(i,j) == w(j,i) by construction.

The paper evaluates on SuiteSparse web, social, road and k-mer graphs made
undirected with unit weights (Section 5.1.3, Table 1); those graphs are not
available here.  These generators stand in for them:

* ``planted_exact``   planted partition with exactly d_in intra and d_out inter
                      edges per vertex (ground-truth modularity is a closed form);
* ``rmat``            R-MAT (Graph500 style) skewed graph, social-network-like;
* ``chung_lu``        power-law expected degrees (exponent 2.1), web-like;
* ``planted_batch``   thousands of small planted graphs of uneven size;
* ``serving_stream``  a Poisson request stream of R-MAT graphs;
* ``road_like``, ``kmer_like``  the low-degree classes (road networks, k-mer graphs:
                      about 2.1 CSR entries per vertex, unit weights).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


@dataclass
class CSR:
    offsets: np.ndarray  # int64 [n+1]
    indices: np.ndarray  # int32 [nnz]
    weights: np.ndarray  # uint32 [nnz]

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def total_weight(self) -> int:
        return int(self.weights.sum(dtype=np.uint64))


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014), vectorised over uint64."""
    x = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        x += np.uint64(0x9E3779B97F4A7C15)
        x ^= x >> np.uint64(30)
        x *= np.uint64(0xBF58476D1CE4E5B9)
        x ^= x >> np.uint64(27)
        x *= np.uint64(0x94D049BB133111EB)
        x ^= x >> np.uint64(31)
    return x


def pair_weights(lo: np.ndarray, hi: np.ndarray, seed: int, wmax: int) -> np.ndarray:
    """Weight in [1, wmax] drawn from a hash of the unordered pair (lo < hi)."""
    if wmax <= 1:
        return np.ones(lo.shape[0], dtype=np.uint32)
    key = (lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64)
    with np.errstate(over="ignore"):
        key ^= _splitmix64(np.array([seed], dtype=np.uint64))[0]
    h = _splitmix64(key)
    return (np.uint64(1) + h % np.uint64(wmax)).astype(np.uint32)


def _pairs_torch(n: int, lo: np.ndarray, hi: np.ndarray, seed: int, wmax: int, device: str) -> CSR:
    """The w=None branch of csr_from_undirected with its integer sorts in torch on
    `device`: the same unique pairs, the same (row, column) order and the same pair
    weights (integer sorting is a total order), in a fraction of numpy's time for
    graphs of hundreds of millions of entries."""
    import torch
    key = torch.unique(torch.from_numpy(lo * n + hi).to(device))  # sorted unique pairs
    klo, khi = (key // n).cpu().numpy(), (key % n).cpu().numpy()
    wk = torch.from_numpy(pair_weights(klo, khi, seed, wmax).astype(np.int64)).to(device)
    del klo, khi
    both = torch.cat([key, (key % n) * n + key // n])
    del key
    both, order = torch.sort(both)
    wt = torch.cat([wk, wk])[order]
    del order, wk
    counts = torch.bincount(both // n, minlength=n).cpu().numpy().astype(np.int64)
    dst = (both % n).to(torch.int32).cpu().numpy()
    del both
    wt = wt.to(torch.int32).cpu().numpy().view(np.uint32)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return CSR(offsets, dst, wt)


def csr_from_undirected(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray | None = None,
                        seed: int = 0, wmax: int = 1, device: str | None = None) -> CSR:
    """Symmetric CSR from an undirected edge sample: self-loops dropped, duplicate
    pairs collapsed (not summed), weights from ``pair_weights`` unless given.
    device (w=None only): run the sorts in torch on that device (same result)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    if w is None and device is not None:
        del u, v
        return _pairs_torch(n, lo, hi, seed, wmax, device)
    if w is None:
        # unique pairs, both directions, sorted by (row, column); the weight is a
        # symmetric hash of the pair, so it is computed after sorting
        key = np.unique(lo * n + hi)
        both = np.concatenate([key, (key % n) * n + key // n])
        both.sort()
        src, dst = both // n, both % n
        wt = pair_weights(np.minimum(src, dst), np.maximum(src, dst), seed, wmax)
    else:
        w = np.asarray(w, dtype=np.uint32)[keep]
        key, first = np.unique(lo * n + hi, return_index=True)
        lo, hi, ww = key // n, key % n, w[first]
        src = np.concatenate([lo, hi])
        dst = np.concatenate([hi, lo])
        wt = np.concatenate([ww, ww])
        order = np.argsort(src * n + dst, kind="stable")
        src, dst, wt = src[order], dst[order], wt[order]
    counts = np.bincount(src, minlength=n).astype(np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return CSR(offsets, dst.astype(np.int32), wt.astype(np.uint32))


def relabel(n: int, rng: np.random.Generator) -> np.ndarray:
    """A seeded random vertex permutation (Graph500 practice): new id = perm[old id]."""
    return rng.permutation(n).astype(np.int64)


# ----------------------------------------------------------------------------------
# planted partition with exact degrees
# ----------------------------------------------------------------------------------

def planted_exact(n_comm: int = 20, comm_size: int = 500, half_intra: int = 6,
                  inter_shifts=(1, 2), seed: int = 1, shuffle: bool = True):
    """Planted partition: every vertex has exactly 2*half_intra intra-community and
    2*len(inter_shifts) inter-community edges, weight 1.

    Intra edges: a random circulant inside each community (vertex pi[p] joined to
    pi[(p+t) mod size] for t = 1..half_intra).  Inter edges: for every shift s a
    random bijection between community c and community (c+s) mod n_comm.
    With 20 communities of 500, 6 and shifts (1, 2) this is the 12-intra/4-inter
    graph whose ground-truth modularity is 12/16 - 20/20**2 = 0.70 exactly.
    Returns (CSR, truth) where truth[v] is v's planted community.
    """
    if comm_size <= 2 * half_intra:
        raise ValueError("community too small for the circulant")
    rng = np.random.default_rng(seed)
    n = n_comm * comm_size
    us, vs = [], []
    base = np.arange(n_comm, dtype=np.int64) * comm_size
    for c in range(n_comm):
        pi = base[c] + rng.permutation(comm_size)
        for t in range(1, half_intra + 1):
            us.append(pi)
            vs.append(np.roll(pi, -t))
    for s in inter_shifts:
        for c in range(n_comm):
            d = (c + s) % n_comm
            us.append(base[c] + np.arange(comm_size))
            vs.append(base[d] + rng.permutation(comm_size))
    u = np.concatenate(us)
    v = np.concatenate(vs)
    truth = np.repeat(np.arange(n_comm, dtype=np.int32), comm_size)
    if shuffle:
        perm = relabel(n, rng)
        u, v = perm[u], perm[v]
        t2 = np.empty(n, dtype=np.int32)
        t2[perm] = truth
        truth = t2
    g = csr_from_undirected(n, u, v, wmax=1)
    return g, truth


# ----------------------------------------------------------------------------------
# R-MAT
# ----------------------------------------------------------------------------------

def rmat(scale: int = 20, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, wmax: int = 8, seed: int = 2, shuffle: bool = True,
         device: str | None = None) -> CSR:
    """R-MAT (Chakrabarti, Zhan & Faloutsos 2004) with 2**scale vertices and
    edge_factor * 2**scale undirected edge samples, no noise.  Self-loops dropped,
    duplicates collapsed, weights uniform in [1, wmax] per pair, seeded relabel."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = edge_factor * n
    u = np.zeros(m, dtype=np.int64)
    v = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for bit in range(scale):
        r = rng.random(m, dtype=np.float32)
        ubit = r >= ab                      # quadrants c, d: row bit set
        vbit = ((r >= a) & (r < ab)) | (r >= abc)   # quadrants b, d: column bit set
        u |= ubit.astype(np.int64) << bit
        v |= vbit.astype(np.int64) << bit
        del r, ubit, vbit
    if shuffle:
        perm = relabel(n, rng)
        u, v = perm[u], perm[v]
    return csr_from_undirected(n, u, v, seed=seed, wmax=wmax, device=device)


# ----------------------------------------------------------------------------------
# Chung-Lu power law
# ----------------------------------------------------------------------------------

def chung_lu_weights(n: int, avg_deg: float, gamma: float) -> np.ndarray:
    """Expected degrees w_i = A (i + i0)^(-1/(gamma-1)) with max w_0 = sqrt(n*avg)
    (structural cutoff) and mean avg; i0 found by bisection."""
    alpha = 1.0 / (gamma - 1.0)
    wmax = math.sqrt(n * avg_deg)
    idx = np.arange(n, dtype=np.float64)

    def mean_for(i0):
        return float(np.mean(wmax * (i0 / (idx + i0)) ** alpha))

    lo, hi = 1e-6, float(n)
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) < avg_deg:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    return wmax * (i0 / (idx + i0)) ** alpha


def _alias_table(p: np.ndarray):
    """Walker/Vose alias table for sampling index i with probability p[i]."""
    n = p.shape[0]
    q = p * (n / p.sum())
    prob = np.zeros(n, dtype=np.float64)
    alias = np.zeros(n, dtype=np.int64)
    small = list(np.nonzero(q < 1.0)[0])
    large = list(np.nonzero(q >= 1.0)[0])
    while small and large:
        s = small.pop()
        l_ = large.pop()
        prob[s] = q[s]
        alias[s] = l_
        q[l_] = q[l_] + q[s] - 1.0
        (small if q[l_] < 1.0 else large).append(l_)
    for rest in large + small:
        prob[rest] = 1.0
        alias[rest] = rest
    return prob, alias


def chung_lu(n: int = 1 << 24, avg_deg: float = 32.0, gamma: float = 2.1, wmax: int = 4,
             seed: int = 3, shuffle: bool = True, samples: int | None = None,
             device: str | None = None) -> CSR:
    """Chung-Lu graph: n*avg_deg/2 edge samples, both endpoints drawn in proportion
    to the expected degrees; self-loops dropped, duplicates collapsed, weights
    uniform in [1, wmax] per pair, seeded relabel."""
    rng = np.random.default_rng(seed)
    wts = chung_lu_weights(n, avg_deg, gamma)
    prob, alias = _alias_table(wts)
    m = int(samples if samples is not None else n * avg_deg / 2)
    ends = []
    for _ in range(2):
        i = rng.integers(0, n, size=m, dtype=np.int64)
        r = rng.random(m)
        ends.append(np.where(r < prob[i], i, alias[i]))
        del i, r
    u, v = ends
    if shuffle:
        perm = relabel(n, rng)
        u, v = perm[u], perm[v]
    return csr_from_undirected(n, u, v, seed=seed, wmax=wmax, device=device)


# ----------------------------------------------------------------------------------
# batched planted graphs
# ----------------------------------------------------------------------------------

def planted_uneven(n: int, cmin: int, cmax: int, d_in_half: int, d_out: int,
                   rng: np.random.Generator):
    """One planted graph with n vertices: community sizes log-uniform in
    [cmin, cmax] drawn until n is reached (a remainder below cmin joins the last
    community), a random circulant of degree 2*d_in_half inside each community and
    d_out random inter-community stubs per vertex paired at random (same-community
    and duplicate pairs are dropped).  Returns (CSR, truth)."""
    sizes = []
    left = n
    while left > 0:
        s = int(round(math.exp(rng.uniform(math.log(cmin), math.log(cmax)))))
        s = min(s, left)
        if left - s < cmin and left - s > 0:
            s = left
        sizes.append(s)
        left -= s
    if len(sizes) > 1 and sizes[-1] < cmin:
        sizes[-2] += sizes[-1]
        sizes.pop()
    truth = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    us, vs = [], []
    for st, sz in zip(starts, sizes):
        pi = st + rng.permutation(sz)
        h = min(d_in_half, (sz - 1) // 2)
        for t in range(1, h + 1):
            us.append(pi)
            vs.append(np.roll(pi, -t))
    stubs = rng.permutation(np.repeat(np.arange(n, dtype=np.int64), d_out))
    if stubs.shape[0] % 2:
        stubs = stubs[:-1]
    a, b = stubs[0::2], stubs[1::2]
    ok = truth[a] != truth[b]
    us.append(a[ok])
    vs.append(b[ok])
    u = np.concatenate(us)
    v = np.concatenate(vs)
    perm = relabel(n, rng)
    u, v = perm[u], perm[v]
    t2 = np.empty(n, dtype=np.int32)
    t2[perm] = truth
    return csr_from_undirected(n, u, v, wmax=1), t2


def _planted_one(args):
    seed, nmin, nmax, cmin, cmax = args
    rng = np.random.default_rng(seed)
    n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    return planted_uneven(n, cmin, cmax, 6, 4, rng)[0]


def planted_batch_truth(g: int, nmin: float = 1e3, nmax: float = 2e5, cmin: int = 20,
                        cmax: int = 2000, base_seed: int = 4000):
    """Graph g of ``planted_batch`` (same arguments) with its planted communities:
    (CSR, truth)."""
    rng = np.random.default_rng(base_seed + g)
    n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    return planted_uneven(n, cmin, cmax, 6, 4, rng)


def planted_batch(count: int = 4096, nmin: float = 1e3, nmax: float = 2e5, cmin: int = 20,
                  cmax: int = 2000, base_seed: int = 4000, workers: int = 1):
    """`count` planted graphs; graph g uses seed base_seed + g and has a vertex count
    log-uniform in [nmin, nmax] with intra:inter degree 12:4.  workers > 1 builds the
    graphs in that many fresh processes (same result)."""
    jobs = [(base_seed + g, nmin, nmax, cmin, cmax) for g in range(count)]
    if workers <= 1:
        return [_planted_one(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_planted_one, jobs, chunksize=max(1, count // (8 * workers)))


# ----------------------------------------------------------------------------------
# serving stream
# ----------------------------------------------------------------------------------

def rmat_torch(scale: int, edge_factor: int = 8, seed: int = 2, wmax: int = 8, a: float = 0.57,
               b: float = 0.19, c: float = 0.19, device: str = "cuda"):
    """R-MAT built entirely with torch on `device` (for streams of many distinct
    graphs): the recipe of rmat() -- edge_factor * 2**scale samples, quadrant
    probabilities a, b, c, d, a seeded relabel, self-loops dropped, duplicates
    collapsed, weights uniform in [1, wmax] per pair -- drawn from torch's seeded
    generator (a different random stream from rmat's).  Returns device tensors
    (offsets int64[n+1], indices int32[nnz], weights int32[nnz] holding uint32 bits),
    rows sorted by column."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    n = 1 << scale
    m = edge_factor * n
    u = torch.zeros(m, dtype=torch.int64, device=device)
    v = torch.zeros(m, dtype=torch.int64, device=device)
    ab, abc = a + b, a + b + c
    for bit in range(scale):
        r = torch.rand(m, generator=gen, device=device)
        u |= (r >= ab).to(torch.int64) << bit
        v |= (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64) << bit
        del r
    perm = torch.randperm(n, generator=gen, device=device)
    u, v = perm[u], perm[v]
    keep = u != v
    lo, hi = torch.minimum(u, v)[keep], torch.maximum(u, v)[keep]
    del u, v, keep, perm
    key = torch.unique(lo * n + hi)
    del lo, hi
    w = torch.randint(1, wmax + 1, (key.numel(),), generator=gen, device=device, dtype=torch.int64)
    both = torch.cat([key, (key % n) * n + key // n])
    wt = torch.cat([w, w])
    del key, w
    both, order = torch.sort(both)
    wt = wt[order].to(torch.int32)
    off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(torch.bincount(both // n, minlength=n), 0)
    idx = (both % n).to(torch.int32)
    return off, idx, wt


def serving_stream(count: int = 2000, smin: int = 14, smax: int = 21, deg: int = 16,
                   rate_hz: float = 100.0, seed: int = 5):
    """Poisson arrivals (exponential gaps at ``rate_hz``) of R-MAT requests with
    2**s vertices, s uniform in [smin, smax], deg*2**s/2 edge samples, weights in
    [1, 8].  Returns a list of (arrival_seconds, scale, graph_seed); graphs are
    built lazily with ``rmat(scale, deg // 2, seed=graph_seed)``."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps) - gaps[0]
    scales = rng.integers(smin, smax + 1, size=count)
    seeds = rng.integers(1, 2**31 - 1, size=count)
    return [(float(t[i]), int(scales[i]), int(seeds[i])) for i in range(count)]


# ----------------------------------------------------------------------------------
# low-degree classes: road networks and k-mer graphs (about 2.1 CSR entries per vertex)
# ----------------------------------------------------------------------------------

def road_like(side: int = 1024, p_keep: float = 0.6, max_sub: int = 6, seed: int = 4,
              device: str | None = None) -> CSR:
    """A road-network stand-in: a side x side grid of intersections whose street
    segments (grid edges) are kept with probability p_keep, each kept segment drawn as
    a chain through a uniform 0..max_sub intermediate points of degree 2.  Unit
    weights.  Ids keep the geometry's locality, as map data does: intersections in
    row-major order, then every segment's points in segment order.  With the defaults
    about 4.6 vertices per intersection and 2.09 CSR entries per vertex."""
    rng = np.random.default_rng(seed)
    S = side * side
    r, c = np.divmod(np.arange(S, dtype=np.int64), side)
    right = np.nonzero(c < side - 1)[0]
    down = np.nonzero(r < side - 1)[0]
    a = np.concatenate([right, down])
    b = np.concatenate([right + 1, down + side])
    keep = rng.random(a.shape[0]) < p_keep
    a, b = a[keep], b[keep]
    order = np.argsort(a * S + b, kind="stable")
    a, b = a[order], b[order]
    ksub = rng.integers(0, max_sub + 1, size=a.shape[0])
    first = S + np.concatenate([[0], np.cumsum(ksub)[:-1]])  # id of each segment's first point
    n = S + int(ksub.sum())
    # segment e is the path a_e, first_e, ..., first_e + k_e - 1, b_e
    seg = np.repeat(np.arange(a.shape[0]), ksub + 1)
    pos = np.arange(seg.shape[0]) - np.repeat(np.cumsum(ksub + 1) - (ksub + 1), ksub + 1)
    u = np.where(pos == 0, a[seg], first[seg] + pos - 1)
    v = np.where(pos == ksub[seg], b[seg], first[seg] + pos)
    return csr_from_undirected(n, u, v, seed=seed, wmax=1, device=device)


def kmer_like(n: int = 1 << 20, mean_len: float = 16.0, p_branch: float = 0.9, seed: int = 5,
              device: str | None = None) -> CSR:
    """A k-mer graph stand-in (de Bruijn graphs of sequences are mostly unbranched
    paths): the vertices, in random order, cut into chains of geometric length (mean
    mean_len), each chain end joined with probability p_branch to a uniformly random
    vertex (a branch point).  Unit weights; ids random, as k-mer hashes are.  With
    the defaults about 2.1 CSR entries per vertex."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n).astype(np.int64)
    lens = []
    total = 0
    while total < n:
        x = rng.geometric(1.0 / mean_len, size=max(16, int(1.2 * (n - total) / mean_len)))
        lens.append(x)
        total += int(x.sum())
    lens = np.concatenate(lens)
    ends = np.minimum(np.cumsum(lens), n)
    ends = ends[: int(np.searchsorted(ends, n)) + 1]
    starts = np.concatenate([[0], ends[:-1]])
    inner = np.ones(n, dtype=bool)  # position p joins p + 1 unless a chain ends at p
    inner[ends - 1] = False
    pidx = np.nonzero(inner[:-1])[0]
    u, v = [perm[pidx]], [perm[pidx + 1]]
    for e in (starts, ends - 1):
        join = rng.random(e.shape[0]) < p_branch
        u.append(perm[e[join]])
        v.append(rng.integers(0, n, size=int(join.sum())))
    return csr_from_undirected(n, np.concatenate(u), np.concatenate(v), seed=seed, wmax=1, device=device)


# ----------------------------------------------------------------------------------
# small hand graphs used by tests
# ----------------------------------------------------------------------------------

def from_edges(n: int, edges, weights=None, self_loops=None) -> CSR:
    """CSR from an explicit undirected edge list (u, v) plus optional self-loops
    {v: weight}; a self-loop appears once in its row."""
    edges = list(edges)
    if weights is None:
        weights = [1] * len(edges)
    rows = [[] for _ in range(n)]
    for (u, v), w in zip(edges, weights):
        if u == v:
            rows[u].append((u, int(w)))
        else:
            rows[u].append((v, int(w)))
            rows[v].append((u, int(w)))
    for v, w in (self_loops or {}).items():
        rows[v].append((v, int(w)))
    offsets = np.zeros(n + 1, dtype=np.int64)
    idx, wt = [], []
    for i, r in enumerate(rows):
        r.sort()
        offsets[i + 1] = offsets[i] + len(r)
        idx.extend(j for j, _ in r)
        wt.extend(w for _, w in r)
    return CSR(offsets, np.asarray(idx, dtype=np.int32), np.asarray(wt, dtype=np.uint32))


def random_small(n: int, p: float, wmax: int, seed: int, loops: bool = False) -> CSR:
    """Erdos-Renyi G(n, p) with weights in [1, wmax]; optional random self-loops."""
    rng = np.random.default_rng(seed)
    edges, ws = [], []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < p:
                edges.append((i, j))
                ws.append(int(rng.integers(1, wmax + 1)))
    sl = {}
    if loops:
        for i in range(n):
            if rng.random() < 0.3:
                sl[i] = int(rng.integers(1, wmax + 1))
    return from_edges(n, edges, ws, sl)
