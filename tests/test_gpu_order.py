"""GPU parity with pins and incident edges in a random order inside every
list.  The interface accepts any order inside a list (the matching depends
only on the sets), while the generators emit ascending ids; these tests run
every variant, the per-round priorities, the graph layout, batches and the
server on shuffled lists, bit-exact against the oracle on the same input and
against the unshuffled input's result."""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_22976_amd as lib
    lib.load()
    return lib


def _run(hgm, g, seed, variant, **kw):
    import torch
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    bits, st = hgm.match(dg, seed, hgm.make_opts(variant, **kw))
    torch.cuda.synchronize()
    return bits.cpu().numpy().view(np.uint32), st


def _instances():
    hub = synth.config_hub_stress(seed=77, n=20_000, m=80_000)   # hub degree 20,000: split
    return {"random": synth.random_instance(31, 20_000, 40_000, 2, 24, 1, 1000),
            "hub": hub,
            "power-law": synth.config_power_law(seed=78, n=50_000, m=120_000)}


@pytest.fixture(scope="module")
def shuffled():
    out = {}
    for name, g in _instances().items():
        s = synth.shuffle_lists(g, 5)
        assert not np.array_equal(s.e_pins, g.e_pins) and not np.array_equal(s.v_edges, g.v_edges)
        out[name] = (g, s)
    return out


@pytest.mark.parametrize("name", ["random", "hub", "power-law"])
@pytest.mark.parametrize("variant", ["auto", "crcw", "crew"])
def test_shuffled_lists_fixed_order(hgm, shuffled, name, variant):
    g, s = shuffled[name]
    seed = 1
    print(f"shuffled {name} m={g.m} kappa={g.kappa} variant={variant}", flush=True)
    exp = oracle.greedy(s.n, s.m, s.e_off, s.e_pins, s.w, seed)[0]
    assert np.array_equal(exp, oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)[0])
    _, ref = oracle.local_max(s.n, s.m, s.e_off, s.e_pins, s.v_off, s.v_edges, s.w, seed)
    got, st = _run(hgm, s, seed, variant, hub_threshold=4096 if name == "hub" else 0)
    assert np.array_equal(got, exp)
    assert st["rounds"] == ref["rounds"]
    assert np.array_equal(st["live_pins"], ref["live_pins"])
    assert np.array_equal(st["matched_per_round"], ref["matched_per_round"])


@pytest.mark.parametrize("name", ["random", "hub", "power-law"])
@pytest.mark.parametrize("variant", ["auto", "crcw", "crew"])
def test_shuffled_lists_reseed(hgm, shuffled, name, variant):
    g, s = shuffled[name]
    seed = 9
    exp, ref = oracle.local_max(s.n, s.m, s.e_off, s.e_pins, s.v_off, s.v_edges, s.w, seed,
                                reseed=True)
    exp_g, _ = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed,
                                reseed=True)
    assert np.array_equal(exp, exp_g)
    got, st = _run(hgm, s, seed, variant, reseed=True)
    assert np.array_equal(got, exp)
    assert st["rounds"] == ref["rounds"]
    assert np.array_equal(st["live_pins"], ref["live_pins"])


def test_shuffled_lists_validate(hgm, shuffled):
    """Validation accepts any order inside the lists (the vertex side is
    checked to be the transpose as a set)."""
    g, s = shuffled["power-law"]
    got, _ = _run(hgm, s, 3, "auto", validate=True)
    assert np.array_equal(got, oracle.greedy(s.n, s.m, s.e_off, s.e_pins, s.w, 3)[0])


def test_shuffled_pairs(hgm):
    """Graph layout with the two pins of every edge in a random order."""
    pts = np.random.Generator(np.random.PCG64(8)).random((30_000, 2))
    pairs = synth.rgg_pairs(pts, 0.012)
    g = synth.from_pairs(30_000, pairs, np.ones(pairs.shape[0], dtype=np.uint32))
    s = synth.shuffle_lists(g, 6)
    swapped = s.e_pins.reshape(-1, 2)[:, 0] > s.e_pins.reshape(-1, 2)[:, 1]
    assert swapped.any() and not swapped.all()
    for seed, reseed in ((1, False), (2, True)):
        exp, ref = oracle.local_max(s.n, s.m, s.e_off, s.e_pins, s.v_off, s.v_edges, s.w, seed,
                                    reseed=reseed)
        for variant in ("auto", "crcw"):
            got, st = _run(hgm, s, seed, variant, pairs=True, reseed=reseed)
            assert np.array_equal(got, exp), (variant, reseed)
            assert st["rounds"] == ref["rounds"]


@pytest.mark.parametrize("variant", ["auto", "crcw", "crew"])
def test_shuffled_batch(hgm, variant):
    import torch
    b = synth.shuffle_batch(synth.config_batched(seed=19, count=64, n_hi=5000), 11)
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    bits, _ = hgm.match_batch(db, hgm.make_opts(variant))
    torch.cuda.synchronize()
    got = bits.cpu().numpy().view(np.uint32)
    for i in range(b.count):
        g = b.instance(i)
        w0, w1 = int(b.word_base[i]), int(b.word_base[i + 1])
        exp = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, int(b.seeds[i]))[0]
        assert np.array_equal(got[w0:w1], exp), (variant, i)


@pytest.mark.parametrize("edge_side_only", [False, True])
def test_shuffled_server(hgm, edge_side_only):
    pool = [synth.shuffle_lists(g, 40 + i) for i, g in
            enumerate(synth.config_served_pool(seed=56, count=24, k_lo=1e3, k_hi=2e5))]
    srv = hgm.Server(1 << 30, workers=2, edge_side_only=edge_side_only)
    try:
        for i, g in enumerate(pool):
            srv.submit(g, 500 + i, req_id=i)
        got = []
        t0 = time.time()
        while len(got) < len(pool):
            got += srv.poll(cap=64, timeout_s=0.5)
            assert time.time() - t0 < 120
    finally:
        srv.close()
    for r in got:
        g = pool[r["id"]]
        assert r["status"] == 0
        exp = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 500 + r["id"])[0]
        assert np.array_equal(r["bits"], exp), r["id"]
