"""GPU parity of the graph layout (hgm_opts.pairs = 1, every edge two pins).

Graphs are hypergraphs whose edges all have two pins, so the oracle is the
same: the bitmap equals the oracle's greedy bitmap and the per-round counts
equal its round simulator, bit for bit, with and without the pair layout.
Inputs follow the paper's graph experiments (Section 6.3): Delaunay
triangulations and random geometric graphs with uniform weights, plus random
weighted graphs.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

VARIANTS = ["auto", "crcw"]


@pytest.fixture(scope="module")
def hgm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_22976_amd as lib
    lib.load()
    return lib


def _check(hgm, g, seed, variant, reseed=False, **kw):
    import torch
    ebits, ref = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed,
                                  reseed=reseed)
    if not reseed:
        gb, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
        assert np.array_equal(gb, ebits)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    for pairs in (True, False):
        bits, st = hgm.match(dg, seed, hgm.make_opts(variant, reseed=reseed, pairs=pairs, **kw))
        torch.cuda.synchronize()
        got = bits.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ebits), f"bitmap differs (pairs={pairs}, {variant}, m={g.m})"
        assert st["rounds"] == ref["rounds"]
        assert np.array_equal(st["live_edges"], ref["live_edges"])
        assert np.array_equal(st["live_pins"], ref["live_pins"])
        assert np.array_equal(st["matched_per_round"], ref["matched_per_round"])
        sel = oracle.bits_to_bool(got, g.m)
        assert st["matched"] == int(sel.sum())
        assert st["weight"] == int(g.w[sel].astype(np.uint64).sum())
        assert np.array_equal(st["matched_pins"], 2 * ref["matched_per_round"])
    return st


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind", ["delaunay", "rgg"])
def test_small_geometric_graphs(hgm, variant, kind):
    g = (synth.config_delaunay if kind == "delaunay" else synth.config_rgg)(seed=31, n=5000)
    for seed in (1, 2, 0xFFFFFFFF):
        print(f"graph {kind} n={g.n} m={g.m} variant={variant} seed={seed}", flush=True)
        _check(hgm, g, seed, variant)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("case", range(5))
def test_random_weighted_graphs(hgm, variant, case):
    n, m, wmax = [(2, 1, 5), (50, 300, 3), (1000, 257, 1000), (3000, 20_000, 2 ** 32 - 1),
                  (20_000, 60_000, 1)][case]
    g = synth.random_instance(case * 31 + 7, n, m, 2, 2, 1, wmax)
    print(f"random graph case={case} n={n} m={m} variant={variant}", flush=True)
    _check(hgm, g, 5, variant)


@pytest.mark.parametrize("variant", VARIANTS)
def test_graph_reseed(hgm, variant):
    g = synth.config_rgg(seed=32, n=4000)
    print(f"graph reseed m={g.m} variant={variant}", flush=True)
    _check(hgm, g, 3, variant, reseed=True)


@pytest.mark.parametrize("variant", VARIANTS)
def test_graph_degenerate(hgm, variant):
    for n, edges in [(0, []), (4, []), (2, [[0, 1]]), (3, [[0, 1], [1, 2], [0, 2]]),
                     (6, [[0, 1], [2, 3], [4, 5]])]:
        g = synth.from_edge_lists(n, edges, np.arange(1, len(edges) + 1))
        print(f"graph degenerate n={n} edges={edges} variant={variant}", flush=True)
        _check(hgm, g, 1, variant)


@pytest.mark.parametrize("weights", ["equal", "random"])
def test_hub_heavy_graphs_take_the_edge_form(hgm, weights):
    """Graphs whose incidences sit mostly on high-degree vertices, so AUTO
    takes the edge-centric round 0 in the pair layout: a star (every edge
    meets the centre: one match), two stars joined by an edge between their
    centres, and the complete bipartite graph K(80, 80) (every vertex of
    degree 80; several rounds)."""
    rng = np.random.default_rng(17)
    k = 3000
    star = np.stack([np.zeros(k, dtype=np.int64), np.arange(1, k + 1)], 1)
    two = np.concatenate([star, np.stack([np.full(k, k + 1), np.arange(k + 2, 2 * k + 2)], 1),
                          [[0, k + 1]]])
    a, c = np.meshgrid(np.arange(80), np.arange(80, 160), indexing="ij")
    kbip = np.stack([a.reshape(-1), c.reshape(-1)], 1)
    for name, pairs, n in (("star", star, k + 1), ("two stars", two, 2 * k + 2),
                           ("K(80,80)", kbip, 160)):
        m = len(pairs)
        w = np.ones(m, dtype=np.int64) if weights == "equal" else rng.integers(1, 1000, m)
        g = synth.from_pairs(n, pairs, w)
        deg = np.diff(g.v_off)
        assert 2 * int(deg[deg >= 64].sum()) >= g.kappa   # AUTO's edge-form condition
        print(f"hub-heavy graph {name} m={m} weights={weights}", flush=True)
        st = _check(hgm, g, 3, "auto")
        if name == "star":
            assert st["matched"] == 1 and st["rounds"] == 1


def test_path_graph_pairs_rounds(hgm):
    """Increasing weights along a path: ceil(m / 2) rounds, one match every
    two rounds from the heavy end; with the pair layout too."""
    m = 101
    g = synth.from_pairs(m + 1, np.stack([np.arange(m), np.arange(1, m + 1)], 1), np.arange(1, m + 1))
    st = _check(hgm, g, 1, "crcw", rounds_per_sync=7)
    assert st["rounds"] == 51


def test_pairs_validation(hgm):
    import torch
    g = synth.random_instance(4, 100, 300, 2, 2, 1, 9)
    g.e_pins[7] = g.e_pins[6]        # an edge with a repeated pin
    g.v_off, g.v_edges = synth.transpose(g.n, g.e_off, g.e_pins)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    with pytest.raises(hgm.HgmError) as ex:
        hgm.match(dg, 1, hgm.make_opts("crcw", pairs=True, validate=True))
    assert ex.value.code == hgm.HGM_E_CSR
    torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["delaunay", "rgg"])
def test_full_size_graphs(hgm, kind):
    """n = 2^20: the sizes of the paper's delaunay_n20 and rgg_n_2_20_s0."""
    g = (synth.config_delaunay if kind == "delaunay" else synth.config_rgg)()
    print(f"full {kind} n={g.n} m={g.m}", flush=True)
    _check(hgm, g, 1, "auto")
