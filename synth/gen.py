"""Seeded generators for the synthetic workloads.

Randomness: numpy's PCG64 generator (O'Neill, 2014) seeded per workload, so
every instance is reproducible from its seed.  Pins of one edge are distinct
(drawn with rejection of repeats inside the edge), listed in ascending vertex
order; the vertex side is the exact transpose (incident edges ascending).

Workloads (shapes follow the paper's benchmark tables: edge sizes from 2 to
tens, skewed degrees with hub vertices of up to millions of incidences):
  plain      n=10,000, m=20,000, |e| ~ U{2..8}, pins uniform, w ~ U{1..1000}
  power-law  n=2,000,000, m=5,000,000, |e| ~ Zipf(2.0) on {2..64}, pin ranks
             ~ Zipf(1.1) over 1..n mapped to ids by a seeded permutation,
             w = floor(2^(20 U)) clamped to [1, 2^20]
  hub        n=1,000,000, m=4,000,000, |e| ~ U{2..16}, one hub vertex in
             exactly m/4 edges, other pins uniform over the rest, all w = 1
  batched    instances with n ~ round(exp(U[ln 100, ln 50,000])), m = 2n,
             |e| ~ U{2..12}, w ~ U{1..1000}
  served     requests with kappa ~ log-uniform [1e3, 1e7], |e| ~ U{2..32},
             m = round(kappa/17), n = max(32, round(m/2)), w ~ U{1..1e6}
  delaunay   graph (every edge 2 pins): Delaunay triangulation of n = 2^20
             uniform points in the unit square, all w = 1
  rgg        graph: random geometric graph on n = 2^20 uniform points in the
             unit square, an edge between points closer than
             r = 0.55 sqrt(ln n / n) (mean degree about 0.95 ln n), all w = 1
  Graph vertex ids are the points' generation order (no spatial order); edges
  are listed by (smaller, larger) endpoint.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Hypergraph:
    n: int
    m: int
    e_off: np.ndarray    # int32[m+1]
    e_pins: np.ndarray   # int32[kappa]
    v_off: np.ndarray    # int32[n+1]
    v_edges: np.ndarray  # int32[kappa]
    w: np.ndarray        # uint32[m]

    @property
    def kappa(self) -> int:
        return int(self.e_off[-1]) if self.m > 0 else 0

    def sizes(self) -> np.ndarray:
        return np.diff(self.e_off.astype(np.int64))

    def degrees(self) -> np.ndarray:
        return np.diff(self.v_off.astype(np.int64))


def transpose(n: int, e_off: np.ndarray, e_pins: np.ndarray):
    """Vertex side of the dual form: v_off[n+1], v_edges[kappa] (stable)."""
    m = e_off.shape[0] - 1
    sizes = np.diff(e_off.astype(np.int64))
    eid = np.repeat(np.arange(m, dtype=np.int64), sizes)
    key = np.sort(e_pins.astype(np.int64) * (1 << 32) + eid)   # by vertex, then edge id
    v_edges = (key & 0xFFFFFFFF).astype(np.int32)
    deg = np.bincount(e_pins, minlength=n).astype(np.int64) if e_pins.size else np.zeros(n, np.int64)
    v_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=v_off[1:])
    return v_off.astype(np.int32), v_edges


def _offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    if off[-1] >= 2 ** 31:
        raise ValueError("kappa exceeds int32 range")
    return off


def _draw_distinct(rng, sizes, off, sample):
    """Draw pins for every slot with `sample(k)`, redrawing repeats in an edge."""
    m = sizes.shape[0]
    total = int(off[-1])
    pins = sample(total).astype(np.int64)
    eid = np.repeat(np.arange(m, dtype=np.int64), sizes)
    todo = np.arange(m, dtype=np.int64)
    while todo.size:
        tsz = sizes[todo]
        tot = int(tsz.sum())
        if tot == 0:
            break
        starts = off[todo]
        excl = np.zeros(todo.size, dtype=np.int64)
        np.cumsum(tsz[:-1], out=excl[1:])
        idx = np.repeat(starts - excl, tsz) + np.arange(tot, dtype=np.int64)
        key = eid[idx] * (1 << 32) + pins[idx]
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dup_sorted = np.zeros(tot, dtype=bool)
        dup_sorted[1:] = sk[1:] == sk[:-1]
        dup_slots = idx[order[dup_sorted]]
        if dup_slots.size == 0:
            break
        pins[dup_slots] = sample(dup_slots.size)
        todo = np.unique(eid[dup_slots])
    return pins


def _sort_within_edges(m, sizes, pins):
    eid = np.repeat(np.arange(m, dtype=np.int64), sizes)
    key = np.sort(eid * (1 << 32) + pins.astype(np.int64))
    return key & 0xFFFFFFFF


def from_edge_lists(n: int, edges, w) -> Hypergraph:
    """Build the dual form from explicit pin lists (order kept as given)."""
    sizes = np.array([len(e) for e in edges], dtype=np.int64)
    off = _offsets(sizes)
    pins = np.array([p for e in edges for p in e], dtype=np.int32).reshape(-1)
    v_off, v_edges = transpose(n, off.astype(np.int32), pins)
    return Hypergraph(n, len(edges), off.astype(np.int32), pins, v_off, v_edges,
                      np.asarray(w, dtype=np.uint32).reshape(-1))


def _assemble(n, sizes, pins, w) -> Hypergraph:
    m = sizes.shape[0]
    off = _offsets(sizes)
    pins = _sort_within_edges(m, sizes, pins).astype(np.int32)
    v_off, v_edges = transpose(n, off.astype(np.int32), pins)
    return Hypergraph(n, m, off.astype(np.int32), pins, v_off, v_edges,
                      np.asarray(w, dtype=np.uint32))


def random_instance(seed: int, n: int, m: int, smin: int = 2, smax: int = 8,
                    wmin: int = 1, wmax: int = 1000, empty_frac: float = 0.0) -> Hypergraph:
    """Uniform pins without repeats; |e| ~ U{smin..smax}; w ~ U{wmin..wmax}.

    `empty_frac` turns that fraction of edges into empty edges (size 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    smax = min(smax, n)
    smin = min(smin, smax)
    sizes = rng.integers(smin, smax + 1, size=m).astype(np.int64)
    if empty_frac > 0 and m > 0:
        sizes[rng.random(m) < empty_frac] = 0
    off = _offsets(sizes)
    pins = _draw_distinct(rng, sizes, off, lambda k: rng.integers(0, max(n, 1), size=k))
    w = rng.integers(wmin, wmax + 1, size=m, dtype=np.uint64).astype(np.uint32)
    return _assemble(n, sizes, pins, w)


def config_plain(seed: int = 1001) -> Hypergraph:
    """n=10,000, m=20,000, |e| ~ U{2..8}, w ~ U{1..1000}."""
    return random_instance(seed, 10_000, 20_000, 2, 8, 1, 1000)


def _zipf_table(lo: int, hi: int, s: float) -> np.ndarray:
    k = np.arange(lo, hi + 1, dtype=np.float64)
    p = k ** (-s)
    c = np.cumsum(p)
    return c / c[-1]


def config_power_law(seed: int = 1002, n: int = 2_000_000, m: int = 5_000_000) -> Hypergraph:
    """Zipf(2.0) sizes on {2..64}; Zipf(1.1) vertex popularity; log-uniform w."""
    rng = np.random.Generator(np.random.PCG64(seed))
    size_cdf = _zipf_table(2, 64, 2.0)
    sizes = (2 + np.searchsorted(size_cdf, rng.random(m), side="right")).astype(np.int64)
    sizes = np.minimum(sizes, 64)
    off = _offsets(sizes)
    rank_cdf = _zipf_table(1, n, 1.1)
    perm = rng.permutation(n).astype(np.int64)

    def sample(k):
        r = np.searchsorted(rank_cdf, rng.random(k), side="right")
        return perm[np.minimum(r, n - 1)]

    pins = _draw_distinct(rng, sizes, off, sample)
    w = np.floor(np.exp2(20.0 * rng.random(m)))
    w = np.clip(w, 1, 2 ** 20).astype(np.uint32)
    return _assemble(n, sizes, pins, w)


def config_hub_stress(seed: int = 1003, n: int = 1_000_000, m: int = 4_000_000) -> Hypergraph:
    """|e| ~ U{2..16}; one hub in exactly m/4 edges; all weights 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(2, 17, size=m).astype(np.int64)
    off = _offsets(sizes)
    hub = int(rng.integers(0, n))
    hub_edges = rng.choice(m, size=m // 4, replace=False)

    def sample(k):  # uniform over V \ {hub}
        u = rng.integers(0, n - 1, size=k)
        return u + (u >= hub)

    pins = _draw_distinct(rng, sizes, off, sample)
    pins[off[hub_edges]] = hub   # the hub takes the first slot; others avoid it
    w = np.ones(m, dtype=np.uint32)
    g = _assemble(n, sizes, pins, w)
    g.hub = hub
    return g


@dataclasses.dataclass
class Batch:
    """Independent instances in one concatenated dual form (instance-local ids).

    base arrays have count+1 entries (int64): v_base (vertex offset into
    v_off-space), e_base (edge offset), pin_base (incidence offset),
    word_base (first bitmap word of each instance).  Instance i owns
    e_off[e_base[i] + i : e_base[i+1] + i + 1] (m_i + 1 entries), and likewise
    v_off; ids inside are local to the instance."""
    count: int
    n: np.ndarray        # int64[count]
    m: np.ndarray        # int64[count]
    v_base: np.ndarray
    e_base: np.ndarray
    pin_base: np.ndarray
    word_base: np.ndarray
    e_off: np.ndarray    # int32[sum(m)+count], per-instance local offsets
    e_pins: np.ndarray
    v_off: np.ndarray    # int32[sum(n)+count]
    v_edges: np.ndarray
    w: np.ndarray
    seeds: np.ndarray    # uint32[count]

    def instance(self, i: int) -> Hypergraph:
        n, m = int(self.n[i]), int(self.m[i])
        eo = self.e_off[self.e_base[i] + i: self.e_base[i + 1] + i + 1]
        vo = self.v_off[self.v_base[i] + i: self.v_base[i + 1] + i + 1]
        p0, p1 = self.pin_base[i], self.pin_base[i + 1]
        return Hypergraph(n, m, eo, self.e_pins[p0:p1], vo, self.v_edges[p0:p1],
                          self.w[self.e_base[i]:self.e_base[i + 1]])


def batch_from_instances(graphs, seeds) -> Batch:
    count = len(graphs)
    n = np.array([g.n for g in graphs], dtype=np.int64)
    m = np.array([g.m for g in graphs], dtype=np.int64)
    k = np.array([g.kappa for g in graphs], dtype=np.int64)
    words = (m + 31) // 32

    def base(a):
        b = np.zeros(count + 1, dtype=np.int64)
        np.cumsum(a, out=b[1:])
        return b

    return Batch(count, n, m, base(n), base(m), base(k), base(words),
                 np.concatenate([g.e_off for g in graphs]).astype(np.int32),
                 np.concatenate([g.e_pins for g in graphs]).astype(np.int32),
                 np.concatenate([g.v_off for g in graphs]).astype(np.int32),
                 np.concatenate([g.v_edges for g in graphs]).astype(np.int32),
                 np.concatenate([g.w for g in graphs]).astype(np.uint32),
                 np.asarray(seeds, dtype=np.uint32))


def config_batched(seed: int = 1004, count: int = 4096, n_lo: int = 100,
                   n_hi: int = 50_000) -> Batch:
    """count instances; n log-uniform in [n_lo, n_hi]; m = 2n; |e| ~ U{2..12}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(np.int64)
    sub = rng.integers(0, 2 ** 63, size=count)
    graphs = [random_instance(int(sub[i]), int(ns[i]), int(2 * ns[i]), 2, 12, 1, 1000)
              for i in range(count)]
    return batch_from_instances(graphs, np.arange(count, dtype=np.uint32))


def edge_side_instance(seed: int, n: int, m: int, smin: int = 2, smax: int = 32,
                       wmin: int = 1, wmax: int = 1_000_000) -> Hypergraph:
    """random_instance's edge side alone: the same sizes, distinct pins and
    weights from the same seed, pins left in draw order (any order is valid)
    and no vertex side (v_off, v_edges empty): requests that carry only the
    edge side need no transpose."""
    rng = np.random.Generator(np.random.PCG64(seed))
    smax = min(smax, n)
    smin = min(smin, smax)
    sizes = rng.integers(smin, smax + 1, size=m).astype(np.int64)
    off = _offsets(sizes)
    pins = _draw_distinct(rng, sizes, off, lambda k: rng.integers(0, max(n, 1), size=k))
    w = rng.integers(wmin, wmax + 1, size=m, dtype=np.uint64).astype(np.uint32)
    return Hypergraph(n, m, off.astype(np.int32), pins.astype(np.int32),
                      np.zeros(0, np.int32), np.zeros(0, np.int32), w)


def _served_one(args):
    sub, n, m, vertex_side = args
    if vertex_side:
        return random_instance(sub, n, m, 2, 32, 1, 1_000_000)
    return edge_side_instance(sub, n, m, 2, 32, 1, 1_000_000)


def config_served_pool(seed: int = 1005, count: int = 1024, k_lo: float = 1e3,
                       k_hi: float = 1e7, vertex_side: bool = True, processes: int = 1):
    """Request pool: kappa log-uniform, |e| ~ U{2..32}, m = round(kappa/17),
    n = max(32, round(m/2)), w ~ U{1..1e6}.  vertex_side=False draws only the
    edge side (edge_side_instance, same sizes, pins and weights); processes >
    1 draws the instances in that many worker processes (same result)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kap = np.exp(rng.uniform(math.log(k_lo), math.log(k_hi), size=count))
    ms = np.maximum(1, np.rint(kap / 17.0)).astype(np.int64)
    ns = np.maximum(32, np.rint(ms / 2.0)).astype(np.int64)
    sub = rng.integers(0, 2 ** 63, size=count)
    jobs = [(int(sub[i]), int(ns[i]), int(ms[i]), vertex_side) for i in range(count)]
    if processes <= 1:
        return [_served_one(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(processes) as pool:
        return pool.map(_served_one, jobs, chunksize=4)


def poisson_arrivals(seed: int, rate: float, duration: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    est = int(rate * duration * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=est))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, size=est))])
    return t[t < duration]


# ---------------------------------------------------------------------------
# Graphs (every edge has exactly two pins), the shapes of the paper's graph
# experiments (Section 6.3): Delaunay triangulations and random geometric
# graphs of random points in the unit square, matched with uniform weights.

def from_pairs(n: int, pairs: np.ndarray, w) -> Hypergraph:
    """Graph from an int64[m, 2] array of distinct endpoints per row."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    m = pairs.shape[0]
    pins = np.sort(pairs, axis=1).astype(np.int32).reshape(-1)
    off = (2 * np.arange(m + 1, dtype=np.int64)).astype(np.int32)
    v_off, v_edges = transpose(n, off, pins)
    return Hypergraph(n, m, off, pins, v_off, v_edges, np.asarray(w, dtype=np.uint32).reshape(-1))


def _unique_pairs(a: np.ndarray, b: np.ndarray, n: int) -> np.ndarray:
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo.astype(np.int64) * n + hi)
    return np.stack([key // n, key % n], axis=1)


def config_delaunay(seed: int = 1006, n: int = 1 << 20) -> Hypergraph:
    """Delaunay triangulation of n uniform random points (unit square)."""
    from scipy.spatial import Delaunay
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    a = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 0]])
    b = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 2]])
    pairs = _unique_pairs(a, b, n)
    return from_pairs(n, pairs, np.ones(pairs.shape[0], dtype=np.uint32))


def rgg_pairs(pts: np.ndarray, r: float) -> np.ndarray:
    """All pairs of points closer than r, by a grid of r-sized cells: each
    point meets the points of its own cell (higher index only) and of four
    of the eight neighbouring cells, so every close pair is seen once."""
    n = pts.shape[0]
    G = max(1, int(math.floor(1.0 / r)))
    cx = np.minimum((pts[:, 0] * G).astype(np.int64), G - 1)
    cy = np.minimum((pts[:, 1] * G).astype(np.int64), G - 1)
    cell = cx * G + cy
    order = np.argsort(cell, kind="stable")
    scell = cell[order]
    start = np.searchsorted(scell, np.arange(G * G + 1))
    out = []
    for dx, dy in ((0, 0), (1, -1), (1, 0), (1, 1), (0, 1)):
        nx, ny = cx[order] + dx, cy[order] + dy
        ok = (nx >= 0) & (nx < G) & (ny >= 0) & (ny < G)
        nc = np.where(ok, nx * G + ny, 0)
        lo = np.where(ok, start[nc], 0)
        hi = np.where(ok, start[nc + 1], 0)
        if dx == 0 and dy == 0:
            lo = np.maximum(lo, np.arange(n) + 1)   # same cell: later points only
        cnt = np.maximum(hi - lo, 0)
        src = np.repeat(np.arange(n), cnt)
        first = np.repeat(lo - np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt)
        dst = first + np.arange(cnt.sum())
        i, j = order[src], order[dst]
        d2 = ((pts[i] - pts[j]) ** 2).sum(axis=1)
        keep = d2 < r * r
        out.append(np.stack([i[keep], j[keep]], axis=1))
    allp = np.concatenate(out) if out else np.zeros((0, 2), np.int64)
    return _unique_pairs(allp[:, 0], allp[:, 1], n)


def config_rgg(seed: int = 1007, n: int = 1 << 20) -> Hypergraph:
    """Random geometric graph: n uniform points, r = 0.55 sqrt(ln n / n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, 2))
    r = 0.55 * math.sqrt(math.log(n) / n)
    pairs = rgg_pairs(pts, r)
    return from_pairs(n, pairs, np.ones(pairs.shape[0], dtype=np.uint32))


# ---------------------------------------------------------------------------
# List order.  The generators above list pins and incident edges in ascending
# order; the interface accepts any order inside a list.  These helpers draw a
# seeded random order inside every list (the sets are unchanged).

def _shuffle_segments(rng, off: np.ndarray, vals: np.ndarray) -> np.ndarray:
    off = np.asarray(off, dtype=np.int64)
    sizes = np.diff(off)
    seg = np.repeat(np.arange(sizes.shape[0], dtype=np.int64), sizes)
    order = np.lexsort((rng.random(vals.shape[0]), seg))
    return np.ascontiguousarray(np.asarray(vals)[order])


def shuffle_lists(g: Hypergraph, seed: int) -> Hypergraph:
    """The same hypergraph with pins in a random order inside every edge and
    incident edges in a random order inside every vertex list."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = Hypergraph(g.n, g.m, g.e_off.copy(), _shuffle_segments(rng, g.e_off, g.e_pins),
                     g.v_off.copy(), _shuffle_segments(rng, g.v_off, g.v_edges), g.w.copy())
    return out


def shuffle_batch(b: Batch, seed: int) -> Batch:
    """shuffle_lists applied to every instance of a batch."""
    graphs = [shuffle_lists(b.instance(i), seed + i) for i in range(b.count)]
    return batch_from_instances(graphs, b.seeds)
