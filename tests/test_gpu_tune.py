"""GPU tests of the schedule autotuner and of non-default schedules.

Any schedule (launch shapes, hub and solo bounds, clear form, first batch of
rounds) must give the one correct bitmap: the oracle's, with its per-round
counts.  The tuner times candidate schedules on the device, checks each
candidate's bitmap against the starting one's, and stores its choice in a
cache file that hgm_tuned_opts reads back."""
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


SCHEDULES = [
    dict(edge_grid=512, blocks_per_cu=2),
    dict(edge_grid=4096, blocks_per_cu=16, clear_ratio=2),
    dict(edge_grid=1, blocks_per_cu=1, clear_ratio=1 << 20),
    dict(hot_degree=1, hub_threshold=64, first_batch_pct=1),
    dict(hot_degree=1 << 30, clear_ratio=32, first_batch_pct=400),
]


@pytest.mark.parametrize("variant", ["auto", "crcw", "crew"])
@pytest.mark.parametrize("sched", range(len(SCHEDULES)))
def test_schedules_keep_parity(hgm, variant, sched):
    import torch
    g = synth.random_instance(61 + sched, 20000, 60000, 2, 12, 1, 1000)
    seed = 3
    exp, cnt, wt = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
    _, ref = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    print(f"schedule {SCHEDULES[sched]} variant={variant}", flush=True)
    bits, st = hgm.match(dg, seed, hgm.make_opts(variant, **SCHEDULES[sched]))
    torch.cuda.synchronize()
    assert np.array_equal(bits.cpu().numpy().view(np.uint32), exp)
    assert st["matched"] == cnt and st["weight"] == wt and st["rounds"] == ref["rounds"]
    assert np.array_equal(st["live_pins"], ref["live_pins"])


@pytest.mark.parametrize("sched", range(len(SCHEDULES)))
def test_batch_schedules_keep_parity(hgm, sched):
    import torch
    b = synth.config_batched(seed=300 + sched, count=48, n_lo=30, n_hi=4000)
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    kw = dict(SCHEDULES[sched])
    kw["solo_max_kappa"] = [0, 2000, -1, 1 << 16, 500][sched]
    print(f"batch schedule {kw}", flush=True)
    bits, st = hgm.match_batch(db, hgm.make_opts("auto", **kw))
    torch.cuda.synchronize()
    got = bits.cpu().numpy().view(np.uint32)
    for i in range(b.count):
        g = b.instance(i)
        exp = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, int(b.seeds[i]))[0]
        assert np.array_equal(got[int(b.word_base[i]):int(b.word_base[i + 1])], exp), i


def test_tune_and_cache(hgm, tmp_path):
    """hgm_tune on one instance: every candidate gave the same bitmap, the
    chosen schedule is stored in the cache and read back for an instance of
    the same bucket, and the matching under it equals the oracle."""
    import torch
    g = synth.random_instance(71, 50000, 120000, 2, 10, 1, 1000)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    cache = str(tmp_path / "tune.txt")
    best, rep = hgm.tune(dg, 5, hgm.make_opts("auto"), reps=1, cache=cache)
    print(f"tuned {rep}", flush=True)
    assert rep["identical"] and rep["evaluations"] >= 10
    assert rep["ms_best"] <= rep["ms_default"] * 1.0001
    text = open(cache).read()
    assert " match v0 p0 r0 " in text and "grid=" in text
    back = hgm.tuned_opts(dg, hgm.make_opts("auto"), cache=cache)
    assert back is not None and hgm.opts_dict(back) == hgm.opts_dict(best)
    other = synth.random_instance(72, 50000, 120000, 2, 10, 1, 1000)   # same bucket
    do = hgm.DeviceHypergraph.from_host(other, "cuda:0")
    assert hgm.tuned_opts(do, hgm.make_opts("auto"), cache=cache) is not None
    assert hgm.tuned_opts(do, hgm.make_opts("crew"), cache=cache) is None   # other bucket
    bits, st = hgm.match(dg, 5, best)
    torch.cuda.synchronize()
    assert np.array_equal(bits.cpu().numpy().view(np.uint32),
                          oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 5)[0])


def test_tune_batch(hgm, tmp_path):
    import torch
    b = synth.config_batched(seed=81, count=200, n_lo=50, n_hi=20000)
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    cache = str(tmp_path / "tune.txt")
    best, rep = hgm.tune_batch(db, hgm.make_opts("auto"), reps=1, cache=cache)
    print(f"tuned batch {rep}", flush=True)
    assert rep["identical"]
    assert hgm.tuned_batch_opts(db, hgm.make_opts("auto"), cache=cache) is not None
    bits, _ = hgm.match_batch(db, best)
    torch.cuda.synchronize()
    got = bits.cpu().numpy().view(np.uint32)
    for i in range(0, b.count, 7):
        g = b.instance(i)
        exp = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, int(b.seeds[i]))[0]
        assert np.array_equal(got[int(b.word_base[i]):int(b.word_base[i + 1])], exp), i
