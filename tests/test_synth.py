"""Shape checks of the seeded input generators (scaled-down workloads)."""
import numpy as np

import synth


def _well_formed(g, smin, smax):
    sizes = g.sizes()
    assert g.e_off[0] == 0 and g.e_off[-1] == g.kappa and np.all(sizes >= 0)
    assert sizes.min() >= smin and sizes.max() <= smax
    assert g.e_pins.min() >= 0 and g.e_pins.max() < g.n
    eid = np.repeat(np.arange(g.m), sizes)
    key = eid.astype(np.int64) * g.n + g.e_pins
    assert np.unique(key).size == g.kappa                 # pins distinct within an edge
    # the vertex side is the exact transpose of the edge side
    vid = np.repeat(np.arange(g.n), g.degrees())
    key_v = g.v_edges.astype(np.int64) * g.n + vid
    assert np.array_equal(np.sort(key), np.sort(key_v))
    assert g.v_off[-1] == g.kappa


def test_plain_config_shape():
    g = synth.config_plain()
    assert (g.n, g.m) == (10_000, 20_000)
    _well_formed(g, 2, 8)
    assert g.w.min() >= 1 and g.w.max() <= 1000
    again = synth.config_plain()
    assert np.array_equal(g.e_pins, again.e_pins) and np.array_equal(g.w, again.w)


def test_power_law_shape_scaled():
    g = synth.config_power_law(seed=5, n=40_000, m=100_000)
    _well_formed(g, 2, 64)
    deg = g.degrees()
    assert deg.max() > 20 * deg.mean()            # skewed degrees with hubs
    assert (deg == 0).mean() > 0.1                # many unused vertices
    assert g.w.min() >= 1 and g.w.max() <= 2 ** 20
    assert 5.0 < g.sizes().mean() < 7.0           # Zipf(2) on {2..64}: mean about 5.95


def test_hub_shape_scaled():
    g = synth.config_hub_stress(seed=6, n=20_000, m=80_000)
    _well_formed(g, 2, 16)
    assert g.degrees()[g.hub] == 20_000
    assert np.all(g.w == 1)


def test_batch_layout():
    b = synth.config_batched(seed=8, count=12, n_lo=50, n_hi=500)
    assert b.count == 12 and np.all(b.m == 2 * b.n)
    for i in range(b.count):
        g = b.instance(i)
        _well_formed(g, 2, 12)
        assert g.e_off.shape[0] == g.m + 1 and g.v_off.shape[0] == g.n + 1


def test_poisson_arrivals():
    t = synth.gen.poisson_arrivals(1, 2000.0, 5.0)
    assert np.all(np.diff(t) > 0) and t[-1] < 5.0
    assert abs(t.size - 10_000) < 500


def test_delaunay_graph_shape():
    """A Delaunay triangulation of points in general position has
    3n - 3 - h edges (h = hull vertices, Euler's formula); every edge has two
    distinct pins and no edge repeats."""
    from scipy.spatial import ConvexHull
    n = 3000
    g = synth.config_delaunay(seed=9, n=n)
    _well_formed(g, 2, 2)
    rng = np.random.Generator(np.random.PCG64(9))
    h = len(ConvexHull(rng.random((n, 2))).vertices)
    assert g.m == 3 * n - 3 - h
    pairs = g.e_pins.reshape(-1, 2).astype(np.int64)
    assert np.unique(pairs[:, 0] * n + pairs[:, 1]).size == g.m
    assert np.all(g.w == 1)


def test_rgg_pairs_brute_force():
    rng = np.random.Generator(np.random.PCG64(3))
    pts = rng.random((1500, 2))
    r = 0.06
    got = synth.rgg_pairs(pts, r)
    d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    i, j = np.nonzero(np.triu(d2 < r * r, 1))
    assert np.array_equal(got, np.stack([i, j], axis=1))


def test_rgg_graph_shape():
    n = 1 << 14
    g = synth.config_rgg(seed=10, n=n)
    _well_formed(g, 2, 2)
    mean_deg = 2 * g.m / n
    assert abs(mean_deg - 0.95 * np.log(n)) < 1.5   # pi (0.55)^2 ln n, less at the border


def test_shuffle_lists_keeps_sets_and_results():
    """Shuffling the order inside every list keeps each edge's pin set and
    each vertex's edge set, and the oracle's results do not change."""
    import oracle
    g = synth.random_instance(12, 300, 900, 1, 9, 1, 4, empty_frac=0.02)
    s = synth.shuffle_lists(g, 3)
    assert np.array_equal(s.e_off, g.e_off) and np.array_equal(s.v_off, g.v_off)
    assert not np.array_equal(s.e_pins, g.e_pins)
    for e in range(g.m):
        a, b = g.e_off[e], g.e_off[e + 1]
        assert sorted(g.e_pins[a:b]) == sorted(s.e_pins[a:b])
    for v in range(g.n):
        a, b = g.v_off[v], g.v_off[v + 1]
        assert sorted(g.v_edges[a:b]) == sorted(s.v_edges[a:b])
    for seed in (1, 2):
        assert np.array_equal(oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)[0],
                              oracle.greedy(s.n, s.m, s.e_off, s.e_pins, s.w, seed)[0])
        for reseed in (False, True):
            a = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed,
                                 reseed=reseed)
            b = oracle.local_max(s.n, s.m, s.e_off, s.e_pins, s.v_off, s.v_edges, s.w, seed,
                                 reseed=reseed)
            assert np.array_equal(a[0], b[0]) and a[1]["rounds"] == b[1]["rounds"]


def test_shuffle_batch_per_instance():
    b = synth.config_batched(seed=3, count=5, n_hi=300)
    s = synth.shuffle_batch(b, 1)
    assert np.array_equal(s.pin_base, b.pin_base) and np.array_equal(s.seeds, b.seeds)
    for i in range(b.count):
        gi, si = b.instance(i), s.instance(i)
        for e in range(gi.m):
            a, c = gi.e_off[e], gi.e_off[e + 1]
            assert sorted(gi.e_pins[a:c]) == sorted(si.e_pins[a:c])
