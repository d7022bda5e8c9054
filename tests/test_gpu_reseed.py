"""GPU parity of the per-round reseeded order (hgm_opts.reseed = 1).

Round r ranks live edges by (w, H(H(seed, r), e)); the result is no longer the
greedy matching of one fixed order, but it is still exactly determined by
(instance, seed): the oracle's round simulator with the same per-round
priorities gives the one correct bitmap and per-round counts, compared here
bit for bit.  Each output is also checked to be a maximal matching.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.fixtures import disjoint, path_graph, star

pytestmark = pytest.mark.gpu

VARIANTS = ["crcw", "auto", "crew"]


@pytest.fixture(scope="module")
def hgm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_22976_amd as lib
    lib.load()
    return lib


def _check(hgm, g, seed, variant, **kw):
    import torch
    ebits, ref = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed,
                                  reseed=True)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    bits, st = hgm.match(dg, seed, hgm.make_opts(variant, reseed=True, **kw))
    torch.cuda.synchronize()
    got = bits.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ebits), f"bitmap differs ({variant}, m={g.m}, seed={seed})"
    sel = oracle.bits_to_bool(got, g.m)
    assert st["matched"] == int(sel.sum())
    assert st["weight"] == int(g.w[sel].astype(np.uint64).sum())
    assert st["rounds"] == ref["rounds"]
    assert np.array_equal(st["live_edges"], ref["live_edges"])
    assert np.array_equal(st["live_pins"], ref["live_pins"])
    assert np.array_equal(st["matched_per_round"], ref["matched_per_round"])
    assert oracle.check_matching(g.n, g.m, g.e_off, g.e_pins, got)
    assert oracle.check_maximal(g.n, g.m, g.e_off, g.e_pins, got)
    return got, st


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("seed", [1, 2, 0xFFFFFFFF])
def test_plain_config_reseed(hgm, variant, seed):
    g = synth.config_plain()
    print(f"reseed plain variant={variant} seed={seed}", flush=True)
    _check(hgm, g, seed, variant)


SWEEP = [  # (n, m, smin, smax, wmin, wmax, empty_frac)
    (1, 1, 1, 1, 1, 5, 0.0), (10, 255, 1, 4, 1, 3, 0.0), (50, 257, 2, 5, 1, 1, 0.1),
    (2000, 1000, 2, 8, 1, 2 ** 32 - 1, 0.0), (300, 4097, 1, 12, 1, 7, 0.02),
    (20_000, 10_000, 2, 64, 1, 1000, 0.0), (5000, 30_000, 0, 6, 0, 0, 0.05),
    (100_000, 20_000, 2, 40, 1, 10 ** 6, 0.0),
]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("case", range(len(SWEEP)))
def test_random_sweep_reseed(hgm, variant, case):
    n, m, smin, smax, wmin, wmax, ef = SWEEP[case]
    g = synth.random_instance(case * 104729 + 3, n, m, smin, smax, wmin, wmax, ef)
    for seed in (0, 7):
        print(f"reseed sweep case={case} variant={variant} seed={seed}", flush=True)
        _check(hgm, g, seed, variant)


@pytest.mark.parametrize("variant", VARIANTS)
def test_degenerate_reseed(hgm, variant):
    for n, edges in [(0, []), (5, []), (0, [[], [], []]), (4, [[], [0, 1], [], [1, 2, 3]]),
                     (2, [[0], [1], [0, 1]])]:
        g = synth.from_edge_lists(n, edges, np.ones(len(edges), dtype=np.uint32))
        print(f"reseed degenerate n={n} edges={edges} variant={variant}", flush=True)
        _check(hgm, g, 9, variant)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("rps", [1, 4])
def test_path_reseed(hgm, variant, rps):
    """Increasing distinct weights along a path: 101 rounds whatever the
    priorities, so every round's maximum and test must use the same round
    seed (a mismatch matches nothing and runs into the round limit).  Equal
    weights: the order is the per-round hash alone."""
    g = path_graph(201)
    got, st = _check(hgm, g, 4, variant, rounds_per_sync=rps, max_rounds=400)
    assert st["rounds"] == 101
    g.w[:] = 1
    _check(hgm, g, 4, variant, rounds_per_sync=rps, max_rounds=400)


@pytest.mark.parametrize("variant", VARIANTS)
def test_star_and_disjoint_reseed(hgm, variant):
    got, st = _check(hgm, star(3000, seed=2), 5, variant)
    assert st["rounds"] == 1 and st["matched"] == 1
    got, st = _check(hgm, disjoint(1000, 5, seed=3), 5, variant)
    assert st["rounds"] == 1 and st["matched"] == 1000


def test_reseed_differs_from_fixed_order(hgm):
    """With equal weights the reseeded run must not silently use the fixed
    order: on this instance the two orders give different matchings."""
    import torch
    g = synth.random_instance(11, 3000, 6000, 2, 6, 1, 1)
    seed = 1
    fixed, _ = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed)
    resd, _ = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed,
                               reseed=True)
    assert not np.array_equal(fixed, resd)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    a, _ = hgm.match(dg, seed, hgm.make_opts("crcw"))
    b, _ = hgm.match(dg, seed, hgm.make_opts("crcw", reseed=True))
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy().view(np.uint32), fixed)
    assert np.array_equal(b.cpu().numpy().view(np.uint32), resd)


@pytest.fixture(scope="module")
def power_law():
    return synth.config_power_law()


@pytest.mark.parametrize("variant", VARIANTS)
def test_power_law_full_reseed(hgm, power_law, variant):
    """The large power-law workload (n = 2M, m = 5M) at full size."""
    g = power_law
    print(f"reseed power-law n={g.n} m={g.m} kappa={g.kappa} variant={variant}", flush=True)
    _check(hgm, g, 1, variant)


@pytest.mark.parametrize("variant", VARIANTS)
def test_hub_stress_full_reseed(hgm, variant):
    """The hub-stress workload (n = 1M, m = 4M, all weights 1, one vertex in
    a quarter of the edges) at full size: the order is the per-round hash
    alone, and the hub is split into pieces in the vertex-centric rounds."""
    g = synth.config_hub_stress()
    print(f"reseed hub-stress n={g.n} m={g.m} kappa={g.kappa} variant={variant}", flush=True)
    _check(hgm, g, 1, variant)


def _batch_reseed_check(hgm, b, variant, **kw):
    """Every instance of a reseeded batch equals the oracle's reseeded round
    simulator with the instance's own seed, and hgm_match on the instance
    alone with that seed."""
    import torch
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    bits, st = hgm.match_batch(db, hgm.make_opts(variant, reseed=True, **kw))
    torch.cuda.synchronize()
    got = bits.cpu().numpy().view(np.uint32)
    R = 0
    live_pins = {}
    for i in range(b.count):
        g = b.instance(i)
        seed = int(b.seeds[i])
        exp, ref = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed,
                                    reseed=True)
        seg = got[int(b.word_base[i]):int(b.word_base[i + 1])]
        assert np.array_equal(seg, exp), f"instance {i} (seed {seed}, m={g.m}) differs"
        for r, p in enumerate(ref["live_pins"]):
            live_pins[r] = live_pins.get(r, 0) + int(p)
        R = max(R, ref["rounds"])
    assert st["rounds"] == R
    assert np.array_equal(st["live_pins"], np.array([live_pins[r] for r in range(R)]))
    return got


@pytest.mark.parametrize("variant", VARIANTS)
def test_batch_reseed(hgm, variant):
    """A batch of uneven instances (some with equal weights, so the per-round
    hash decides, one empty) with per-round priorities."""
    graphs, seeds = [], []
    for i in range(40):
        n = int(np.exp(np.random.default_rng(i).uniform(np.log(5), np.log(4000))))
        wmax = 1 if i % 3 == 0 else 1000
        graphs.append(synth.random_instance(700 + i, n, 2 * n, 2, 8, 1, wmax))
        seeds.append((i * 2654435761) & 0xFFFFFFFF)
    graphs.append(synth.from_edge_lists(3, [], []))
    seeds.append(5)
    b = synth.batch_from_instances(graphs, seeds)
    print(f"reseed batch count={b.count} variant={variant}", flush=True)
    got = _batch_reseed_check(hgm, b, variant)
    # the same instances alone give the same bitmaps
    import torch
    for i in (0, 1, 7, 39):
        g = b.instance(i)
        dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
        alone, _ = hgm.match(dg, int(b.seeds[i]), hgm.make_opts(variant, reseed=True))
        torch.cuda.synchronize()
        seg = got[int(b.word_base[i]):int(b.word_base[i + 1])]
        assert np.array_equal(alone.cpu().numpy().view(np.uint32), seg)


def test_batch_reseed_path_rounds(hgm):
    """Paths with increasing weights in a batch take many rounds (the path of
    201 edges 101): round seeds must follow the round index in every
    instance, through several host synchronisations."""
    graphs = [path_graph(201), path_graph(40), star(500, seed=3)]
    for g in graphs[:2]:
        g.w[:] = 1 + (np.arange(g.m) % 3)
    b = synth.batch_from_instances(graphs, [3, 4, 5])
    for variant in VARIANTS:
        _batch_reseed_check(hgm, b, variant, rounds_per_sync=3)
