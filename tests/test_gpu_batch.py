"""GPU parity of hgm_match_batch: every instance's bitmap segment equals the
oracle's greedy matching for that instance and seed, and equals hgm_match on
the instance alone; the aggregate per-round counts equal the sum of the
instances' oracle round counts.  Batches run with the one-workgroup solo part
for small instances at its default bound (SOLO 0), with a low bound so that
solo and round-kernel instances mix (2000 pins), and without it (-1)."""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

VARIANTS = ["auto", "crcw", "crew"]
SOLO = [0, 2000, -1]


@pytest.fixture(scope="module")
def hgm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_22976_amd as lib
    lib.load()
    return lib


def _segments(b, bits):
    out = []
    for i in range(b.count):
        w0, w1 = int(b.word_base[i]), int(b.word_base[i + 1])
        out.append(bits[w0:w1])
    return out


def _oracle_batch(b):
    per, rounds = [], []
    for i in range(b.count):
        g = b.instance(i)
        seed = int(b.seeds[i])
        bits, cnt, wt = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
        _, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed)
        per.append((bits, cnt, wt))
        rounds.append(st)
    return per, rounds


def _agg(rounds, key):
    R = max([st["rounds"] for st in rounds] + [0])
    tot = np.zeros(R, dtype=np.int64)
    for st in rounds:
        a = st[key]
        tot[:a.size] += a
    return tot


def _check_batch(hgm, b, variant, per=None, rounds=None, **kw):
    import torch
    if per is None:
        per, rounds = _oracle_batch(b)
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    bits, st = hgm.match_batch(db, hgm.make_opts(variant, **kw))
    torch.cuda.synchronize()
    got = bits.cpu().numpy().view(np.uint32)
    segs = _segments(b, got)
    for i, (exp, _, _) in enumerate(per):
        assert np.array_equal(segs[i], exp), f"instance {i} differs ({variant})"
    assert st["matched"] == sum(p[1] for p in per)
    assert st["weight"] == sum(p[2] for p in per)
    assert st["rounds"] == max([r["rounds"] for r in rounds] + [0])
    assert np.array_equal(st["live_edges"], _agg(rounds, "live_edges"))
    assert np.array_equal(st["live_pins"], _agg(rounds, "live_pins"))
    assert np.array_equal(st["matched_per_round"], _agg(rounds, "matched_per_round"))
    return got


@pytest.mark.parametrize("solo", SOLO)
@pytest.mark.parametrize("variant", VARIANTS)
def test_small_batch(hgm, variant, solo):
    b = synth.config_batched(seed=77, count=96, n_lo=20, n_hi=3000)
    print(f"batch count={b.count} m_total={int(b.e_base[-1])} variant={variant} solo={solo}",
          flush=True)
    _check_batch(hgm, b, variant, solo_max_kappa=solo)


@pytest.mark.parametrize("solo", SOLO)
@pytest.mark.parametrize("variant", VARIANTS)
def test_degenerate_batches(hgm, variant, solo):
    rng = np.random.default_rng(3)
    gs = [synth.from_edge_lists(0, [], []),                          # empty instance
          synth.random_instance(5, 40, 70, 2, 4, 1, 9),
          synth.from_edge_lists(3, [[], [0, 1], []], [4, 5, 6]),     # empty edges
          synth.from_edge_lists(5, [], []),                          # vertices, no edges
          synth.random_instance(6, 7, 33, 1, 3, 0, 2, empty_frac=0.2),
          synth.from_edge_lists(1, [[0]], [3])]
    seeds = rng.integers(0, 2 ** 32, size=len(gs)).astype(np.uint32)
    b = synth.batch_from_instances(gs, seeds)
    print(f"degenerate batch variant={variant} solo={solo}", flush=True)
    _check_batch(hgm, b, variant, solo_max_kappa=solo)
    one = synth.batch_from_instances([gs[1]], seeds[:1])
    _check_batch(hgm, one, variant, solo_max_kappa=solo)


@pytest.mark.parametrize("solo", SOLO)
@pytest.mark.parametrize("variant", VARIANTS)
def test_skewed_batch(hgm, variant, solo):
    """One large instance among thousands of tiny and empty ones, in three
    orders (large first, in the middle, last): the setup's workgroups each
    take an equal range of edges and of vertices, so one range spans dozens
    of tiny instances and the empty ones between them, while many ranges
    fall inside the large one; every instance's segment must still equal the
    oracle."""
    rng = np.random.default_rng(11)
    big = synth.random_instance(21, 60_000, 150_000, 2, 12, 1, 1000)
    tiny = []
    for k in range(3000):
        kind = k % 5
        if kind == 0:
            tiny.append(synth.from_edge_lists(0, [], []))                       # nothing
        elif kind == 1:
            tiny.append(synth.from_edge_lists(int(rng.integers(1, 4)), [], []))  # vertices only
        else:
            n = int(rng.integers(2, 9))
            tiny.append(synth.random_instance(1000 + k, n, int(rng.integers(1, 6)), 1, min(3, n),
                                              0, 5))
    for at in (0, 1500, 3000):
        gs = tiny[:at] + [big] + tiny[at:]
        seeds = rng.integers(0, 2 ** 32, size=len(gs)).astype(np.uint32)
        b = synth.batch_from_instances(gs, seeds)
        print(f"skewed batch: large instance at {at}, variant={variant} solo={solo}",
              flush=True)
        _check_batch(hgm, b, variant, solo_max_kappa=solo)


@pytest.mark.parametrize("solo", [0, -1])
@pytest.mark.parametrize("variant", ["auto", "crew"])
@pytest.mark.parametrize("threshold", [0, 64, 300])
def test_dense_batch_takes_the_edge_form(hgm, threshold, variant, solo):
    """Dense instances (every vertex of degree about 100), so AUTO's round 0
    takes the edge-centric form over the batch; with a low hub threshold the
    high-degree vertices become hubs reduced in each workgroup's table
    (AUTO) or split into pieces in every round (CREW)."""
    rng = np.random.default_rng(23)
    gs = []
    for k in range(24):
        n = int(rng.integers(60, 140))
        gs.append(synth.random_instance(500 + k, n, 2000, 2, 8, 1, int(rng.integers(1, 1000))))
    gs.append(synth.random_instance(600, 3000, 500, 2, 4, 1, 9))   # a sparse one among them
    seeds = rng.integers(0, 2 ** 32, size=len(gs)).astype(np.uint32)
    b = synth.batch_from_instances(gs, seeds)
    deg = np.concatenate([np.diff(b.instance(i).v_off) for i in range(b.count)])
    assert 2 * int(deg[deg >= 64].sum()) >= int(b.pin_base[-1])   # AUTO's edge-form condition
    print(f"dense batch hub_threshold={threshold} variant={variant} solo={solo}", flush=True)
    _check_batch(hgm, b, variant, hub_threshold=threshold, solo_max_kappa=solo)


def test_batch_equals_single_calls(hgm):
    import torch
    b = synth.config_batched(seed=5, count=40, n_lo=100, n_hi=5000)
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    bits, _ = hgm.match_batch(db, hgm.make_opts("auto"))
    segs = _segments(b, bits.cpu().numpy().view(np.uint32))
    for i in range(b.count):
        g = b.instance(i)
        dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
        one, _ = hgm.match(dg, int(b.seeds[i]), hgm.make_opts("auto"))
        torch.cuda.synchronize()
        assert np.array_equal(one.cpu().numpy().view(np.uint32), segs[i]), i


def test_batch_workload_sample(hgm):
    """512 instances with the batched workload's distribution (n log-uniform
    in [100, 50,000], m = 2n, |e| ~ U{2..12}, seeds = instance index)."""
    b = synth.config_batched(seed=1004, count=512)
    print(f"batched workload sample: m_total={int(b.e_base[-1])} "
          f"kappa_total={int(b.pin_base[-1])}", flush=True)
    per, rounds = _oracle_batch(b)
    for variant, solo in (("auto", 0), ("crcw", -1), ("crew", 30000), ("auto", 2000)):
        print(f"batched workload sample variant={variant} solo={solo}", flush=True)
        _check_batch(hgm, b, variant, per, rounds, solo_max_kappa=solo)


@pytest.mark.parametrize("variant", VARIANTS)
def test_solo_instances_beyond_lds(hgm, variant):
    """Instances with more vertices than one LDS tile of the solo part (it
    then forms and tests each round's maximum tile by tile: 2, 3 and 8
    tiles) among instances that fit one tile, one with more pins than the
    solo bound and one with more than 8 tiles' worth of vertices (both taken
    by the round kernels)."""
    lds = hgm.load().hgm_solo_lds_vertices()
    assert lds >= 4096
    gs, seeds = [], []
    sizes = [lds + 1, lds // 2, 2 * lds + 100, lds // 3, lds, 5 * lds]
    for k, n in enumerate(sizes):
        gs.append(synth.random_instance(900 + k, n, 2 * n, 2, 10, 1, 1 if k == 4 else 1000))
        seeds.append(31 * k + 1)
    gs.append(synth.random_instance(940, 8 * lds - 2000, 2 * lds, 2, 6, 1, 1000))  # 8 tiles
    seeds.append(77)
    gs.append(synth.random_instance(941, 9 * lds, lds, 2, 6, 1, 1000))     # beyond 8 tiles
    seeds.append(78)
    gs.append(synth.random_instance(950, 3 * lds, 12 * lds, 2, 10, 1, 1000))
    seeds.append(99)
    b = synth.batch_from_instances(gs, np.array(seeds, dtype=np.uint32))
    kap = np.diff(b.pin_base)
    bound = int(kap[:-1].max())
    assert kap[-1] > bound           # the last one runs in the round kernels
    print(f"solo beyond LDS: lds_verts={lds} variant={variant}", flush=True)
    _check_batch(hgm, b, variant, solo_max_kappa=bound)


@pytest.mark.parametrize("solo", SOLO)
def test_batch_round_limit(hgm, solo):
    """A path with increasing weights needs 101 rounds: with max_rounds 50
    the batch fails with HGM_E_ROUND_LIMIT whichever part runs it, and with
    max_rounds 101 it completes."""
    from tests.fixtures import path_graph
    import torch
    gs = [synth.random_instance(3, 300, 600, 2, 5, 1, 50), path_graph(201)]
    b = synth.batch_from_instances(gs, np.array([1, 2], dtype=np.uint32))
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    with pytest.raises(hgm.HgmError) as ei:
        hgm.match_batch(db, hgm.make_opts("auto", max_rounds=50, solo_max_kappa=solo))
    assert ei.value.code == hgm.HGM_E_ROUND_LIMIT
    torch.cuda.synchronize()
    _check_batch(hgm, b, "auto", max_rounds=101, solo_max_kappa=solo)


def test_solo_part_is_used(hgm):
    """Timing statistics show the solo kernel once per call when instances
    fit its bound, and the round kernels alone when it is off.  The default
    bound follows the batch's total pins (here the 2^12 floor): the small
    instances go to the solo part, the larger ones to the round kernels."""
    import torch
    b = synth.config_batched(seed=78, count=64, n_lo=20, n_hi=2000)
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    _, st = hgm.match_batch(db, hgm.make_opts("auto", solo_max_kappa=1 << 20), timing=True)
    assert st["kernel_launches"]["solo"] == 1 and st["kernel_ms"]["solo"] > 0
    assert st["kernel_launches"]["test"] == 0     # every instance ran in the solo part
    kap = np.diff(b.pin_base)
    assert kap.sum() // 1024 < 4096 and (kap <= 4096).any() and (kap > 4096).any()
    _, st = hgm.match_batch(db, hgm.make_opts("auto"), timing=True)
    assert st["kernel_launches"]["solo"] == 1 and st["kernel_launches"]["test"] > 0
    _, st = hgm.match_batch(db, hgm.make_opts("auto", solo_max_kappa=-1), timing=True)
    assert st["kernel_launches"]["solo"] == 0 and st["kernel_launches"]["test"] > 0
    torch.cuda.synchronize()


def test_batch_full_workload(hgm):
    """The full batched workload that bench.py times (4,096 instances, sum of
    kappa about 4.8e8, one launch): a seeded sample of instances, with the
    largest and the smallest, equals the oracle bit for bit; every instance's
    segment passes the greedy certificate (which only the oracle's matching
    passes) and is a maximal matching, checked over the whole concatenation
    with instance-global vertex ids; the totals add up."""
    import torch
    b = synth.config_batched(seed=1004, count=4096)
    kap = np.diff(b.pin_base)
    print(f"full batched workload: m_total={int(b.e_base[-1])} kappa_total={int(kap.sum())}",
          flush=True)
    db = hgm.DeviceBatch.from_host(b, "cuda:0")
    bits, st = hgm.match_batch(db, hgm.make_opts("auto"))
    torch.cuda.synchronize()
    got = bits.cpu().numpy().view(np.uint32)
    del db, bits
    torch.cuda.empty_cache()
    segs = _segments(b, got)

    rng = np.random.Generator(np.random.PCG64(4096))
    sample = set(rng.choice(b.count, 10, replace=False).tolist())
    sample |= {int(np.argmax(kap)), int(np.argmin(kap))}
    for i in sorted(sample):
        g = b.instance(i)
        exp = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, int(b.seeds[i]))[0]
        assert np.array_equal(segs[i], exp), f"instance {i} differs"
    # Every instance: the greedy certificate (a matching in which every
    # unmatched edge has a matched neighbour ranked above it) holds for
    # exactly one edge set, the greedy matching of the instance's order.
    t0 = time.time()
    for i in range(b.count):
        g = b.instance(i)
        assert oracle.check_greedy_certificate(g.n, g.m, g.e_off, g.e_pins, g.w,
                                               int(b.seeds[i]), segs[i]), f"instance {i}"
    print(f"greedy certificate on all {b.count} instances: {time.time() - t0:.1f} s", flush=True)

    matched = np.concatenate([oracle.bits_to_bool(segs[i], int(b.m[i])) for i in range(b.count)])
    sizes = np.concatenate([np.diff(b.e_off[b.e_base[i] + i: b.e_base[i + 1] + i + 1])
                            for i in range(b.count)])
    assert sizes.min() > 0   # |e| >= 2 in this workload (reduceat below needs non-empty edges)
    gp = b.e_pins + np.repeat(b.v_base[:-1].astype(np.int32), kap)   # instance-global vertex ids
    mp = gp[np.repeat(matched, sizes)]
    n_total = int(b.v_base[-1])
    assert np.bincount(mp, minlength=n_total).max() <= 1              # vertex-disjoint
    covered = np.zeros(n_total, dtype=bool)
    covered[mp] = True
    starts = np.zeros(sizes.size, dtype=np.int64)
    np.cumsum(sizes[:-1], out=starts[1:])
    hit = np.logical_or.reduceat(covered[gp], starts)
    assert np.all(matched | hit)                                      # maximal
    assert st["matched"] == int(matched.sum())
    assert st["weight"] == int(b.w[matched].astype(np.uint64).sum())
