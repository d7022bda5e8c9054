"""Pins for the oracle: checks against facts fixed by the paper and by
mathematics, independent of the oracle's own code.

* Hash: published MurmurHash3_x86_32 test vectors; an explicit inverse built
  from modular inverses round-trips (so H(seed, .) is a bijection).
* Greedy: the greedy certificate (matching + every rejected edge blocked by a
  higher matched neighbour), which characterises the greedy set uniquely;
  Lemma 1's 1/d bound against brute-force optima; Lemma 2's tight instance.
* Local max: equals greedy for a strict order (induction down the key order),
  closed forms on paths, stars and disjoint edges, statistics invariants.
* Planted mistakes in a result are caught by the certificate.
"""
import numpy as np
import pytest

import oracle
from synth import from_edge_lists, random_instance
from tests.fixtures import disjoint, golden_files, path_graph, read_golden, star

M32 = 0xFFFFFFFF


# ---------------------------------------------------------------------------
# Hash

# (data, seed, MurmurHash3_x86_32) from the widely published test-vector list.
MURMUR_VECTORS = [
    (b"", 0, 0x00000000),
    (b"", 1, 0x514E28B7),
    (b"", 0xFFFFFFFF, 0x81F16F39),
    (b"\x00\x00\x00\x00", 0, 0x2362F9DE),
    (b"\xff\xff\xff\xff", 0, 0x76293B50),
    (b"!Ce\x87", 0, 0xF55B516B),
    (b"!Ce\x87", 0x5082EDEE, 0x2362F9DE),
    (b"a", 0x9747B28C, 0x7FA09EA6),
    (b"Hello, world!", 0x9747B28C, 0x24884CBA),
    (b"The quick brown fox jumps over the lazy dog", 0x9747B28C, 0x2FA826CD),
]


@pytest.mark.parametrize("data,seed,expect", MURMUR_VECTORS)
def test_murmur3_published_vectors(data, seed, expect):
    assert oracle.murmur3_x86_32(data, seed) == expect


def test_priority_is_murmur_of_id_bytes():
    for seed in (0, 1, 0x9747B28C):
        h = oracle.priorities(seed, 4096)
        for e in (0, 1, 2, 255, 256, 4095):
            assert int(h[e]) == oracle.murmur3_x86_32(int(e).to_bytes(4, "little"), seed)
    assert int(oracle.priorities(0, 1)[0]) == 0x2362F9DE  # published vector, id 0


def _rotr(x, r):
    return ((x >> r) | (x << (32 - r))) & M32


def _inverse_priority(h, seed):
    """Inverse of H(seed, .) on 4-byte ids, from modular inverses of the odd
    multipliers and inverses of the xor-shifts and rotations."""
    inv = lambda c: pow(c, -1, 1 << 32)
    h ^= h >> 16
    h = (h * inv(0xC2B2AE35)) & M32
    h ^= (h >> 13) ^ (h >> 26)
    h = (h * inv(0x85EBCA6B)) & M32
    h ^= h >> 16
    h ^= 4
    h = ((h - 0xE6546B64) * inv(5)) & M32
    h = _rotr(h, 13)
    k = h ^ seed
    k = (k * inv(0x1B873593)) & M32
    k = _rotr(k, 15)
    return (k * inv(0xCC9E2D51)) & M32


@pytest.mark.parametrize("seed", [0, 1, 7, 0xDEADBEEF])
def test_priority_inverse_roundtrip(seed):
    m = 50_000
    h = oracle.priorities(seed, m)
    rng = np.random.default_rng(seed)
    for e in list(range(64)) + list(rng.integers(0, m, size=2000)):
        assert _inverse_priority(int(h[e]), seed) == int(e)
    assert np.unique(h).size == m


@pytest.mark.slow
@pytest.mark.parametrize("seed", [0, 1])
def test_priority_exhaustive_bijection(seed):
    assert oracle.priority_collisions(seed) == 0


# ---------------------------------------------------------------------------
# Greedy and local max on the paper's worked example (Lemma 2 / Figure 1)

@pytest.mark.parametrize("path", golden_files("lemma2_tight"))
def test_lemma2_tight_instance(path):
    g, seed, ex = read_golden(path)
    bits, cnt, wt = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
    assert np.flatnonzero(oracle.bits_to_bool(bits, g.m)).tolist() == ex["matched_ids"]
    assert cnt == ex["count"][0] and wt == ex["weight"][0]
    bits2, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed)
    assert np.array_equal(bits, bits2)
    assert st["rounds"] == ex["rounds"][0]
    opt_w, opt_c = oracle.brute_force_max(g.n, g.m, g.e_off, g.e_pins, g.w)
    assert opt_w == ex["opt_weight"][0] and opt_c == ex["opt_count"][0]
    d = int(g.sizes().max())
    assert wt * d >= opt_w  # Lemma 1 holds, and is nearly tight here


# ---------------------------------------------------------------------------
# Lemma 1 (1/d bound) against brute force

def test_lemma1_bound_against_brute_force():
    rng = np.random.default_rng(11)
    for t in range(300):
        n = int(rng.integers(2, 11))
        m = int(rng.integers(1, 13))
        g = random_instance(1000 + t, n, m, 1, min(4, n), 1, int(rng.integers(1, 50)),
                            empty_frac=0.05)
        seed = int(rng.integers(0, 2 ** 32))
        bits, cnt, wt = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
        opt_w, opt_c = oracle.brute_force_max(g.n, g.m, g.e_off, g.e_pins, g.w)
        d = max(int(g.sizes().max()), 1)
        assert wt * d >= opt_w, (t, wt, opt_w, d)
        assert cnt * d >= opt_c, (t, cnt, opt_c, d)
        assert wt <= opt_w and cnt <= opt_c


# ---------------------------------------------------------------------------
# Greedy certificate and its power to detect wrong answers

def _check_all(g, seed, bits):
    return (oracle.check_matching(g.n, g.m, g.e_off, g.e_pins, bits)
            and oracle.check_maximal(g.n, g.m, g.e_off, g.e_pins, bits)
            and oracle.check_greedy_certificate(g.n, g.m, g.e_off, g.e_pins, g.w, seed, bits))


def test_greedy_certificate_random():
    rng = np.random.default_rng(5)
    for t in range(120):
        n = int(rng.integers(1, 400))
        m = int(rng.integers(0, 800))
        g = random_instance(2000 + t, n, m, 0 if t % 3 == 0 else 1, int(rng.integers(1, 12)),
                            0 if t % 4 == 0 else 1, int(rng.choice([1, 3, 1000, 2 ** 32 - 1])),
                            empty_frac=0.02 if t % 5 == 0 else 0.0)
        seed = int(rng.integers(0, 2 ** 32))
        bits, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
        assert _check_all(g, seed, bits), t


def test_certificate_catches_planted_mistakes():
    """Mistakes planted in a correct greedy result (on the CPU) are caught."""
    g = random_instance(77, 300, 900, 2, 6, 1, 20)
    seed = 3
    bits, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
    flags = oracle.bits_to_bool(bits, g.m)
    on, off = np.flatnonzero(flags), np.flatnonzero(~flags)
    # drop a matched edge
    f = flags.copy(); f[on[0]] = False
    assert not _check_all(g, seed, oracle.bool_to_bits(f))
    # add an unmatched edge
    f = flags.copy(); f[off[0]] = True
    assert not _check_all(g, seed, oracle.bool_to_bits(f))
    # swap: a rejected edge in, its blocking higher neighbour out
    rank = oracle.edge_rank(g.w, seed, g.m)
    e = off[0]
    pins = set(g.e_pins[g.e_off[e]:g.e_off[e + 1]].tolist())
    blockers = [x for x in on if pins & set(g.e_pins[g.e_off[x]:g.e_off[x + 1]].tolist())]
    f = flags.copy(); f[e] = True
    for x in blockers:
        f[x] = False
    assert not oracle.check_greedy_certificate(g.n, g.m, g.e_off, g.e_pins, g.w, seed,
                                               oracle.bool_to_bits(f))
    # the greedy result under a reversed order (a sign mistake) is rejected
    inv = (np.uint64(2 ** 32 - 1) - g.w.astype(np.uint64)).astype(np.uint32)
    bits_rev, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, inv, seed)
    assert not np.array_equal(bits_rev, bits)
    assert not oracle.check_greedy_certificate(g.n, g.m, g.e_off, g.e_pins, g.w, seed, bits_rev)
    # a different seed reorders equal weights
    bits_s, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed + 1)
    if not np.array_equal(bits_s, bits):
        assert not oracle.check_greedy_certificate(g.n, g.m, g.e_off, g.e_pins, g.w, seed, bits_s)


# ---------------------------------------------------------------------------
# Local max = greedy, and its statistics

def _stats_invariants(g, bits, st):
    r = st["rounds"]
    if g.m == 0:
        assert r == 0
        return
    assert st["live_edges"][0] == g.m and st["live_pins"][0] == g.kappa
    assert np.all(np.diff(st["live_edges"]) < 0)
    assert np.all(st["matched_per_round"] >= 1)
    assert int(st["matched_per_round"].sum()) == int(oracle.bits_to_bool(bits, g.m).sum())


def test_local_max_equals_greedy_many_small():
    rng = np.random.default_rng(9)
    for t in range(3000):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 60))
        g = random_instance(10_000 + t, n, m, 0 if t % 7 == 0 else 1, int(rng.integers(1, 7)),
                            0, int(rng.choice([1, 2, 5, 100])), empty_frac=0.03 if t % 5 == 0 else 0)
        seed = int(rng.integers(0, 2 ** 32))
        bg, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
        bl, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed)
        assert np.array_equal(bg, bl), t
        _stats_invariants(g, bl, st)


@pytest.mark.parametrize("n,m,smax,wmax", [(5_000, 20_000, 8, 1000), (20_000, 10_000, 32, 1),
                                           (1_000, 50_000, 4, 3), (50_000, 30_000, 16, 10 ** 6)])
def test_local_max_equals_greedy_medium(n, m, smax, wmax):
    g = random_instance(n + m, n, m, 2, smax, 1, wmax)
    for seed in (0, 1, 12345):
        bg, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
        bl, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed)
        assert np.array_equal(bg, bl)
        assert _check_all(g, seed, bg)
        _stats_invariants(g, bl, st)


# ---------------------------------------------------------------------------
# Special cases with closed forms

def test_empty_instances():
    from synth import from_edge_lists
    for n in (0, 5):
        g = from_edge_lists(n, [], [])
        bits, cnt, wt = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 1)
        assert bits.size == 0 and cnt == 0 and wt == 0
        _, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, 1)
        assert st["rounds"] == 0


def test_disjoint_edges_all_match_in_one_round():
    g = disjoint(40, 4)
    bits, cnt, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 5)
    assert cnt == 40
    _, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, 5)
    assert st["rounds"] == 1 and st["matched_per_round"].tolist() == [40]


def test_star_matches_only_the_top_edge():
    g = star(60, seed=4)
    seed = 8
    bits, cnt, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
    h = oracle.priorities(seed, g.m)
    top = max(range(g.m), key=lambda e: (int(g.w[e]), int(h[e]), e))
    assert cnt == 1 and np.flatnonzero(oracle.bits_to_bool(bits, g.m)).tolist() == [top]
    _, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed)
    assert st["rounds"] == 1


@pytest.mark.parametrize("m", [1, 2, 7, 50, 201])
def test_path_with_increasing_weights(m):
    """Only the heaviest remaining edge is a local max each round."""
    g = path_graph(m)
    bits, cnt, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 1)
    expect = list(range(m - 1, -1, -2))[::-1]
    assert np.flatnonzero(oracle.bits_to_bool(bits, g.m)).tolist() == expect
    bl, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, 1)
    assert np.array_equal(bits, bl)
    rounds = (m + 1) // 2
    assert st["rounds"] == rounds
    assert st["live_edges"].tolist() == [m - 2 * r for r in range(rounds)]
    assert st["live_pins"].tolist() == [2 * (m - 2 * r) for r in range(rounds)]
    assert st["matched_per_round"].tolist() == [1] * rounds


def test_equal_weights_follow_hash_order():
    g = random_instance(31, 200, 600, 2, 5, 1, 1)   # all weights 1
    seed = 99
    bits, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
    h = oracle.priorities(seed, g.m)
    # greedy by hash order alone, written out with a Python sort
    taken = set()
    expect = []
    for e in sorted(range(g.m), key=lambda e: int(h[e]), reverse=True):
        pins = g.e_pins[g.e_off[e]:g.e_off[e + 1]].tolist()
        if not taken.intersection(pins):
            taken.update(pins)
            expect.append(e)
    assert np.flatnonzero(oracle.bits_to_bool(bits, g.m)).tolist() == sorted(expect)


def test_empty_edges_match_in_first_round():
    from synth import from_edge_lists
    g = from_edge_lists(4, [[0, 1], [], [1, 2], [], [2, 3]], [5, 1, 9, 2, 4])
    bits, cnt, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 1)
    got = np.flatnonzero(oracle.bits_to_bool(bits, g.m)).tolist()
    assert 1 in got and 3 in got and 2 in got and 0 not in got and 4 not in got
    _, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, 1)
    assert st["matched_per_round"][0] >= 3


def test_round_limit_and_invalid_input():
    g = path_graph(10)
    with pytest.raises(RuntimeError):
        oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, 1, max_rounds=3)
    _, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, 1, max_rounds=5)
    assert st["rounds"] == 5
    bad = g.e_pins.copy(); bad[3] = g.n
    with pytest.raises(ValueError):
        oracle.greedy(g.n, g.m, g.e_off, bad, g.w, 1)


# ---------------------------------------------------------------------------
# Per-round fresh priorities (the paper's re-randomized rounds, weight first)

def test_round_priority_is_murmur_of_round_then_id():
    for seed in (0, 1, 99):
        for r in (0, 1, 7):
            rs = oracle.murmur3_x86_32(int(r).to_bytes(4, "little"), seed)
            for e in (0, 5, 1000):
                assert oracle.round_priority(seed, r, e) == oracle.murmur3_x86_32(
                    int(e).to_bytes(4, "little"), rs)


def _lm(g, seed, reseed=True, **kw):
    return oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed,
                            reseed=reseed, **kw)


def test_reseed_distinct_weights_equals_greedy():
    """With all weights distinct the tie-breaking priority never decides, so
    every round's order is the weight order and the result is greedy's."""
    rng = np.random.default_rng(21)
    for t in range(200):
        n = int(rng.integers(2, 60))
        m = int(rng.integers(1, 80))
        g = random_instance(300 + t, n, m, 1, 5, 1, 1)
        g.w = rng.permutation(np.arange(1, m + 1)).astype(np.uint32)   # distinct
        seed = int(rng.integers(0, 2 ** 32))
        bg, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
        br, st = _lm(g, seed)
        assert np.array_equal(bg, br), t
        _stats_invariants(g, br, st)


def test_reseed_matching_maximal_and_lemma1():
    rng = np.random.default_rng(22)
    for t in range(200):
        n = int(rng.integers(2, 11))
        m = int(rng.integers(1, 13))
        g = random_instance(500 + t, n, m, 1, min(4, n), 1, int(rng.choice([1, 2, 3])))
        seed = int(rng.integers(0, 2 ** 32))
        bits, st = _lm(g, seed)
        assert oracle.check_matching(g.n, g.m, g.e_off, g.e_pins, bits)
        assert oracle.check_maximal(g.n, g.m, g.e_off, g.e_pins, bits)
        flags = oracle.bits_to_bool(bits, g.m)
        wt, cnt = int(g.w[flags].sum()), int(flags.sum())
        opt_w, opt_c = oracle.brute_force_max(g.n, g.m, g.e_off, g.e_pins, g.w)
        d = max(int(g.sizes().max()), 1)
        assert wt * d >= opt_w and cnt * d >= opt_c
        _stats_invariants(g, bits, st)


def test_reseed_round_one_is_fixed_order_with_round_seed():
    """Round 0 of the reseeded run ranks by H(H(seed, 0), e): its matches are
    exactly those of a fixed-order run with seed H(seed, 0) in round 0."""
    g = random_instance(41, 3000, 9000, 2, 6, 1, 3)
    seed = 12345
    _, st = _lm(g, seed, cap=4)
    rs0 = oracle.murmur3_x86_32((0).to_bytes(4, "little"), seed)
    _, st0 = _lm(g, rs0, reseed=False, cap=4)
    assert st["matched_per_round"][0] == st0["matched_per_round"][0]
    assert st["live_edges"][1] == st0["live_edges"][1]


def test_reseed_many_small_instances_valid():
    rng = np.random.default_rng(23)
    for t in range(500):
        g = random_instance(900 + t, int(rng.integers(1, 40)), int(rng.integers(0, 60)),
                            0, 5, 1, int(rng.choice([1, 2, 10])), empty_frac=0.05)
        bits, st = _lm(g, int(rng.integers(0, 2 ** 32)))
        assert oracle.check_matching(g.n, g.m, g.e_off, g.e_pins, bits)
        assert oracle.check_maximal(g.n, g.m, g.e_off, g.e_pins, bits)
        _stats_invariants(g, bits, st)


def _murmur_id(seed, x):
    """H(seed, x) from the byte-string MurmurHash3 (pinned by published vectors)."""
    return oracle.murmur3_x86_32(int(x).to_bytes(4, "little"), seed)


def _tie_winner(seed, rnd, a, b):
    """The edge of {a, b} (equal weights) that round `rnd` ranks higher:
    larger H(H(seed, rnd), e)."""
    rs = _murmur_id(seed, rnd)
    return a if _murmur_id(rs, a) > _murmur_id(rs, b) else b


def test_reseed_round_one_tie_uses_round_one_priorities():
    """Hand-derived: h = {u,t} (w 3) is matched in round 0 and retires
    g = {y,u} (w 2), which had blocked the equal-weight pair f1 = {x,y},
    f2 = {y,z} at y.  The pair first meets at y with no heavier edge in
    round 1, so round 1's priorities H(H(seed, 1), .) decide it.  Over 40
    seeds round 0's priorities pick the other edge in 17 cases, so an oracle
    that kept round 0's order would fail here."""
    u, t, y, x, z = range(5)
    g = from_edge_lists(5, [[u, t], [y, u], [x, y], [y, z]], [3, 2, 1, 1])
    disagree = 0
    for seed in range(40):
        win = _tie_winner(seed, 1, 2, 3)
        disagree += win != _tie_winner(seed, 0, 2, 3)
        bits, st = _lm(g, seed)
        assert list(np.flatnonzero(oracle.bits_to_bool(bits, g.m))) == sorted([0, win]), seed
        assert st["rounds"] == 2
        assert list(st["live_edges"]) == [4, 2] and list(st["matched_per_round"]) == [1, 1]
        assert list(st["live_pins"]) == [8, 4]
    assert disagree > 0


def test_reseed_round_two_tie_uses_round_two_priorities():
    """Hand-derived three-round chain: Y = {p,q} (w 5) matches in round 0 and
    retires X = {t,q} (w 4); X had beaten h = {u,t} (w 3) at t, so h matches
    in round 1 and retires g = {y,u} (w 2); g had beaten the equal-weight
    pair f1 = {x,y}, f2 = {y,z} at y until then, so round 2's priorities
    H(H(seed, 2), .) decide the pair."""
    p, q, t, u, y, x, z = range(7)
    g = from_edge_lists(7, [[p, q], [t, q], [u, t], [y, u], [x, y], [y, z]], [5, 4, 3, 2, 1, 1])
    disagree = 0
    for seed in range(40):
        win = _tie_winner(seed, 2, 4, 5)
        disagree += win != _tie_winner(seed, 1, 4, 5) or win != _tie_winner(seed, 0, 4, 5)
        bits, st = _lm(g, seed)
        assert list(np.flatnonzero(oracle.bits_to_bool(bits, g.m))) == sorted([0, 2, win]), seed
        assert st["rounds"] == 3
        assert list(st["live_edges"]) == [6, 4, 2]
        assert list(st["matched_per_round"]) == [1, 1, 1]
    assert disagree > 0
