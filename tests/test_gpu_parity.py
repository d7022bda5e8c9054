"""GPU parity: hgm_match (through the C ABI) against the oracle.

The matching is integer work with exactly one correct result per (instance,
seed), so every comparison is bit-exact: the bitmap equals the oracle's greedy
bitmap, and the per-round counts (live edges, live pins, matched edges) and
the round count equal the oracle's round simulator.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from tests.fixtures import disjoint, golden_files, path_graph, read_golden, star

pytestmark = pytest.mark.gpu

VARIANTS = ["crcw", "crew", "auto"]


@pytest.fixture(scope="module")
def hgm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_22976_amd as lib
    lib.load()   # raises if the HIP library is missing: no fallback
    return lib


def _run(hgm, g, seed, variant="auto", **kw):
    import torch
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    bits, st = hgm.match(dg, seed, hgm.make_opts(variant, **kw))
    torch.cuda.synchronize()
    return bits.cpu().numpy().view(np.uint32), st


def _expect(g, seed):
    bits, cnt, wt = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
    lbits, ref = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed)
    assert np.array_equal(bits, lbits)
    return bits, cnt, wt, ref


def _check(hgm, g, seed, variant, expect=None, **kw):
    bits, cnt, wt, ref = expect or _expect(g, seed)
    got, st = _run(hgm, g, seed, variant, **kw)
    assert np.array_equal(got, bits), f"bitmap differs ({variant}, m={g.m}, seed={seed})"
    assert st["matched"] == cnt and st["weight"] == wt
    assert st["rounds"] == ref["rounds"]
    assert np.array_equal(st["live_edges"], ref["live_edges"])
    assert np.array_equal(st["live_pins"], ref["live_pins"])
    assert np.array_equal(st["matched_per_round"], ref["matched_per_round"])
    return st


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("seed", [1, 2])
def test_plain_config(hgm, variant, seed):
    g = synth.config_plain()
    print(f"plain n={g.n} m={g.m} variant={variant} seed={seed}", flush=True)
    _check(hgm, g, seed, variant)


SWEEP = [  # (n, m, smin, smax, wmax, empty_frac)
    (1, 1, 1, 1, 5, 0.0), (3, 1, 2, 3, 5, 0.0), (10, 255, 1, 4, 3, 0.0),
    (50, 256, 2, 5, 1, 0.0), (50, 257, 2, 5, 1000, 0.1), (2000, 1000, 2, 8, 2 ** 32 - 1, 0.0),
    (300, 4097, 1, 12, 7, 0.02), (20_000, 10_000, 2, 64, 1000, 0.0), (100, 5000, 2, 3, 1, 0.0),
    (5000, 30_000, 0, 6, 0, 0.05), (100_000, 20_000, 2, 40, 10 ** 6, 0.0),
]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("case", range(len(SWEEP)))
def test_random_sweep(hgm, variant, case):
    n, m, smin, smax, wmax, ef = SWEEP[case]
    wmin = 0 if wmax == 0 else 1
    g = synth.random_instance(case * 7919 + 17, n, m, smin, smax, wmin, max(wmax, 0), ef)
    for seed in (0, 3, 0xFFFFFFFF):
        print(f"sweep case={case} n={n} m={m} variant={variant} seed={seed}", flush=True)
        _check(hgm, g, seed, variant)


@pytest.mark.parametrize("variant", VARIANTS)
def test_empty_and_degenerate(hgm, variant):
    for n, edges in [(0, []), (5, []), (0, [[], [], []]), (4, [[], [0, 1], [], [1, 2, 3]]),
                     (1, [[0]]), (2, [[0], [1], [0, 1]])]:
        g = synth.from_edge_lists(n, edges, np.arange(1, len(edges) + 1))
        print(f"degenerate n={n} edges={edges} variant={variant}", flush=True)
        _check(hgm, g, 1, variant)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("rps", [1, 3, 7])
def test_path_many_rounds(hgm, variant, rps):
    g = path_graph(61)
    st = _check(hgm, g, 1, variant, rounds_per_sync=rps)
    assert st["rounds"] == 31


@pytest.mark.parametrize("variant", VARIANTS)
def test_star_and_disjoint(hgm, variant):
    _check(hgm, star(3000, seed=2), 5, variant)
    _check(hgm, disjoint(1000, 5, seed=3), 5, variant)


@pytest.mark.parametrize("path", golden_files("lemma2_tight"))
@pytest.mark.parametrize("variant", VARIANTS)
def test_lemma2_fixture(hgm, path, variant):
    g, seed, ex = read_golden(path)
    got, st = _run(hgm, g, seed, variant)
    assert np.flatnonzero(oracle.bits_to_bool(got, g.m)).tolist() == ex["matched_ids"]
    assert st["weight"] == ex["weight"][0] and st["rounds"] == ex["rounds"][0]


def _seed_with_zero_hash(e):
    """Seed s with H(s, e) = 0, by running MurmurHash3's 4-byte steps backwards."""
    M = 0xFFFFFFFF
    inv = lambda c: pow(c, -1, 1 << 32)
    rotl = lambda x, r: ((x << r) | (x >> (32 - r))) & M
    rotr = lambda x, r: ((x >> r) | (x << (32 - r))) & M
    h = 0  # fmix32(0) = 0, so the pre-finaliser value is 0
    h ^= 4
    h = ((h - 0xE6546B64) * inv(5)) & M
    h = rotr(h, 13)
    k = (e * 0xCC9E2D51) & M
    k = rotl(k, 15)
    k = (k * 0x1B873593) & M
    return h ^ k


@pytest.mark.parametrize("variant", VARIANTS)
def test_edge_with_key_zero(hgm, variant):
    """An edge with weight 0 and hash 0 has packed key 0, the value used for
    'no live edge'; it must still be matched when it wins."""
    g = synth.random_instance(99, 40, 60, 2, 3, 0, 0)   # all weights 0
    e0 = 17
    seed = _seed_with_zero_hash(e0)
    assert int(oracle.priorities(seed, g.m)[e0]) == 0
    _check(hgm, g, seed, variant)
    iso = synth.from_edge_lists(6, [[0, 1], [2, 3], [4, 5]], [0, 0, 0])
    seed1 = _seed_with_zero_hash(1)
    got, _ = _run(hgm, iso, seed1, variant)
    assert oracle.bits_to_bool(got, 3).tolist() == [True, True, True]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("wval", [0, 1, 12345, 0xFFFFFFFF])
def test_uniform_weights(hgm, variant, wval):
    """All weights equal (cardinality matching): round 0's vertex pass builds
    keys without gathering the weights.  The same instance with one weight
    changed must take the gathering path and follow it (the changed edge is
    the heaviest, so it is matched)."""
    g = synth.random_instance(123, 3000, 8000, 2, 9, 1, 1)
    g.w[:] = wval
    print(f"uniform weights w={wval} variant={variant}", flush=True)
    _check(hgm, g, 5, variant)
    if wval < 0xFFFFFFFF:
        g.w[4321] = wval + 1
        bits, _, _, _ = _expect(g, 5)
        assert oracle.bits_to_bool(bits, g.m)[4321]
        _check(hgm, g, 5, variant)


@pytest.mark.parametrize("threshold", [1, 4, 64, 100_000])
def test_crew_hub_split(hgm, threshold):
    g = synth.config_hub_stress(seed=21, n=5000, m=40_000)
    print(f"hub split threshold={threshold}", flush=True)
    _check(hgm, g, 1, "crew", hub_threshold=threshold)


@pytest.mark.parametrize("threshold", [1, 4, 64, 100_000])
def test_auto_vertex_form_hub_split(hgm, threshold):
    """AUTO on a degree profile without many hot incidences takes the
    vertex-centric round 0, whose hub pieces depend on the threshold."""
    g = synth.config_hub_stress(seed=22, n=50_000, m=40_000)   # non-hub degree ~7
    print(f"auto vertex form threshold={threshold}", flush=True)
    _check(hgm, g, 2, "auto", hub_threshold=threshold)
    import torch
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    _, st = hgm.match(dg, 2, hgm.make_opts("auto", hub_threshold=threshold), timing=True)
    torch.cuda.synchronize()
    assert st["kernel_launches"]["vertex_max"] == 1 and st["kernel_launches"]["scatter"] == 0


@pytest.mark.parametrize("threshold", [1, 64, 1000, 100_000])
def test_auto_edge_form_hub_table(hgm, threshold):
    """AUTO's edge-centric round 0 on skewed degrees reduces hub pins in a
    per-workgroup LDS table of at most 512 hubs: threshold 1 overflows it
    (the rest take the global path), 100,000 leaves it empty."""
    import torch
    g = synth.config_power_law(seed=23, n=40_000, m=100_000)
    deg = g.degrees()
    print(f"auto edge form threshold={threshold} hubs={(deg > threshold).sum()}", flush=True)
    _check(hgm, g, 7, "auto", hub_threshold=threshold)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    _, st = hgm.match(dg, 7, hgm.make_opts("auto", hub_threshold=threshold), timing=True)
    torch.cuda.synchronize()
    assert st["kernel_launches"]["scatter"] == 1 and st["kernel_launches"]["vertex_max"] == 0


def _hub_on_path(path_edges=201, hub_edges=20_000, seed=5):
    """A path with increasing weights (one match every two rounds from the top
    end) and a hub whose lighter 3-pin edges {hub, leaf, path vertex} die as
    their path vertex is matched: the hub stays open for ~100 rounds while its
    live list shrinks every round."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_path = path_edges + 1
    hub = n_path
    edges = [[i, i + 1] for i in range(path_edges)]
    w = list(1000 + np.arange(path_edges))
    on = rng.integers(0, n_path, size=hub_edges)
    for k in range(hub_edges):
        edges.append([hub, hub + 1 + k, int(on[k])])
    w += list(rng.integers(1, 1000, size=hub_edges))
    return synth.from_edge_lists(hub + 1 + hub_edges, edges, np.array(w))


@pytest.mark.parametrize("threshold", [4, 64, 100_000])
def test_crew_list_compaction_many_rounds(hgm, threshold):
    g = _hub_on_path()
    print(f"hub on path threshold={threshold}", flush=True)
    st = _check(hgm, g, 3, "crew", hub_threshold=threshold, max_rounds=1000)
    assert st["rounds"] >= 100


def test_round_limit(hgm):
    import torch
    g = path_graph(40)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    with pytest.raises(hgm.HgmError) as ex:
        hgm.match(dg, 1, hgm.make_opts("crcw", max_rounds=5))
    assert ex.value.code == hgm.HGM_E_ROUND_LIMIT
    bits, st = hgm.match(dg, 1, hgm.make_opts("crcw", max_rounds=20, rounds_per_sync=6))
    torch.cuda.synchronize()
    assert st["rounds"] == 20


def _expect_csr_error(hgm, g, variant="crcw"):
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    with pytest.raises(hgm.HgmError) as ex:
        hgm.match(dg, 1, hgm.make_opts(variant, validate=True))
    assert ex.value.code == hgm.HGM_E_CSR


def test_validation_rejects_malformed(hgm):
    import copy
    base = synth.random_instance(5, 100, 200, 2, 6, 1, 50)
    _run(hgm, base, 1, "crcw", validate=True)   # valid input passes
    _run(hgm, base, 1, "crew", validate=True)
    g = copy.deepcopy(base); g.e_pins[7] = g.n             # pin out of range
    _expect_csr_error(hgm, g)
    g = copy.deepcopy(base); g.e_pins[1] = g.e_pins[0]     # repeated pin in edge 0
    _expect_csr_error(hgm, g)
    g = copy.deepcopy(base); g.e_off[5], g.e_off[6] = g.e_off[6], g.e_off[5]  # not monotone
    _expect_csr_error(hgm, g)
    g = copy.deepcopy(base); g.v_edges[3] = (g.v_edges[3] + 1) % g.m  # not the transpose
    _expect_csr_error(hgm, g, "crew")
    g = copy.deepcopy(base)  # vertex-side incidence listed twice, another one dropped
    v = int(np.argmax(np.diff(g.v_off) >= 2))
    a = g.v_off[v]
    g.v_edges[a + 1] = g.v_edges[a]
    _expect_csr_error(hgm, g, "crew")


@pytest.mark.parametrize("variant", VARIANTS)
def test_repeatable_and_workspace_reuse(hgm, variant):
    import torch
    g1 = synth.random_instance(7, 5000, 20_000, 2, 10, 1, 100)
    g2 = synth.random_instance(8, 3000, 9000, 2, 5, 1, 3)
    d1 = hgm.DeviceHypergraph.from_host(g1, "cuda:0")
    d2 = hgm.DeviceHypergraph.from_host(g2, "cuda:0")
    opts = hgm.make_opts(variant)
    ws = hgm.alloc_workspace(d1, opts)
    ws.fill_(0xA5)
    e1 = oracle.greedy(g1.n, g1.m, g1.e_off, g1.e_pins, g1.w, 4)[0]
    e2 = oracle.greedy(g2.n, g2.m, g2.e_off, g2.e_pins, g2.w, 4)[0]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(3):
            b1, _ = hgm.match(d1, 4, opts, workspace=ws)
            b2, _ = hgm.match(d2, 4, opts, workspace=ws)
            stream.synchronize()
            assert np.array_equal(b1.cpu().numpy().view(np.uint32), e1)
            assert np.array_equal(b2.cpu().numpy().view(np.uint32), e2)


# ---------------------------------------------------------------------------
# Full-size workloads (the benchmark's configuration: default options)

@pytest.fixture(scope="module")
def power_law():
    print("generating power-law instance", flush=True)
    g = synth.config_power_law()
    return g, _expect(g, 1)


@pytest.fixture(scope="module")
def hub_stress():
    print("generating hub-stress instance", flush=True)
    g = synth.config_hub_stress()
    return g, _expect(g, 1)


@pytest.mark.parametrize("variant", VARIANTS)
def test_power_law_full(hgm, power_law, variant):
    g, ex = power_law
    print(f"power-law full n={g.n} m={g.m} kappa={g.kappa} variant={variant}", flush=True)
    _check(hgm, g, 1, variant, expect=ex)


@pytest.mark.parametrize("variant", VARIANTS)
def test_hub_stress_full(hgm, hub_stress, variant):
    g, ex = hub_stress
    print(f"hub-stress full n={g.n} m={g.m} kappa={g.kappa} variant={variant}", flush=True)
    _check(hgm, g, 1, variant, expect=ex)


@pytest.mark.parametrize("shift", [12, 14])
def test_full_bins(hgm, power_law, hub_stress, shift):
    """The binned next-round maximum (bins of 2^shift vertices) on both
    full-size instances."""
    for g, ex in (power_law, hub_stress):
        print(f"full n={g.n} m={g.m} bin_shift={shift}", flush=True)
        _check(hgm, g, 1, "auto", expect=ex, bin_shift=shift)


def test_concurrent_calls_on_two_streams(hgm):
    """Two host threads call hgm_match at once, each on its own stream and
    workspace (with per-kernel timing on, which keeps a per-thread event
    pool): every result equals the oracle's."""
    import threading
    import torch
    gs = [synth.random_instance(400 + i, 20_000, 60_000, 2, 10, 1, 50) for i in range(2)]
    exp = [oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 9)[0] for g in gs]
    dgs = [hgm.DeviceHypergraph.from_host(g, "cuda:0") for g in gs]
    errors = []

    def worker(i):
        try:
            stream = torch.cuda.Stream()
            opts = hgm.make_opts("auto")
            ws = hgm.alloc_workspace(dgs[i], opts)
            for _ in range(20):
                bits, st = hgm.match(dgs[i], 9, opts, workspace=ws, stream=stream.cuda_stream,
                                     timing=True)
                stream.synchronize()
                got = bits.cpu().numpy().view(np.uint32)
                if not np.array_equal(got, exp[i]):
                    errors.append(f"thread {i}: bitmap differs")
                    return
        except Exception as ex:   # reported below, on the main thread
            errors.append(f"thread {i}: {ex!r}")

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors


@pytest.mark.parametrize("tail", [0, 1 << 30])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("rps", [0, 1, 3])
def test_timing_statistics(hgm, variant, rps, tail):
    """The per-kernel timing that bench.py reports: one test and one retire
    launch per live round (the retire that finds the next live set belongs
    to its round); round 0's maximum once (CRCW: the edge scatter; CREW and
    AUTO here: the vertex pass), and CREW's vertex pass once more in every
    later round; per-round times add up to the kernel times outside setup.
    Launches past the last live round are not counted.  With the tail (here
    taking over from round 1), the rounds from the one it took over run in
    one tail launch, whose time belongs to that round."""
    import torch
    g = synth.random_instance(31, 20_000, 50_000, 2, 8, 1, 1000)
    ebits, _, _, ref = _expect(g, 3)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    bits, st = hgm.match(dg, 3, hgm.make_opts(variant, rounds_per_sync=rps, tail_pins=tail),
                         timing=True)
    torch.cuda.synchronize()
    assert np.array_equal(bits.cpu().numpy().view(np.uint32), ebits)
    R = st["rounds"]
    assert R == ref["rounds"] and R >= 3
    n = st["kernel_launches"]
    t0 = R if tail == 0 else n["test"]    # rounds before the tail took over
    assert n["test"] == t0 and n["retire"] == t0
    if tail == 0:
        assert n["tail"] == 0
    else:
        assert 1 <= t0 < R and n["tail"] >= 1
    if variant == "crcw":
        assert n["scatter"] == 1 and n["vertex_max"] == 0
    elif variant == "crew":   # with the tail, also the pass that forms its first round
        assert n["scatter"] == 0 and n["vertex_max"] == t0 + (tail != 0)
    else:   # uniform random degrees: AUTO takes the vertex-centric round 0
        assert n["scatter"] == 0 and n["vertex_max"] == 1
    assert n["setup"] >= 1
    ms = st["kernel_ms"]
    assert all(v >= 0 for v in ms.values()) and ms["test"] > 0 and ms["retire"] > 0
    assert st["round_ms"].size == R and np.all(st["round_ms"][:t0 + (tail != 0)] > 0)
    rounds_total = sum(v for k, v in ms.items() if k != "setup")
    assert abs(float(st["round_ms"].sum()) - rounds_total) <= 1e-3 * rounds_total + 1e-4
