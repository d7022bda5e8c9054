"""Oracle for iterated local-max hypergraph matching.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this module;
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the GPU library.

Contents
  * ``build()``            compiles ``oracle.c`` with gcc into ``_oracle.so``.
  * ``murmur3_x86_32``     the published MurmurHash3_x86_32 (priority hash).
  * ``priorities``         H(seed, e) for every edge id.
  * ``greedy``             sequential greedy in the fixed edge order
                           (the paper's single-core Greedy baseline).
  * ``local_max``          the round-based local-max algorithm (Sequential
                           Algorithm, Algorithm 2) with per-round statistics.
  * property checks        ``check_matching`` (vertex-disjoint, definition of
                           a matching), ``check_maximal`` (definition of
                           maximal), ``check_greedy_certificate`` (the matching
                           is the greedy one for the order: see its docstring).
  * ``brute_force_max``    exhaustive maximum weight / cardinality matching for
                           tiny instances (used against Lemma 1's bound).
The edge order is the tuple (w(e), H(seed, e), e), larger first.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "_oracle.so")
_lib = None

ORACLE_OK = 0
ORACLE_E_ARG = -1
ORACLE_E_NOMEM = -2
ORACLE_E_ROUNDS = -3


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so (plain gcc, no GPU code)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall",
                               "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.oracle_murmur3_x86_32.restype = ctypes.c_uint32
    lib.oracle_murmur3_x86_32.argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.c_uint32]
    lib.oracle_priorities.restype = None
    lib.oracle_priorities.argtypes = [ctypes.c_uint32, ctypes.c_int32, P]
    lib.oracle_greedy.restype = ctypes.c_int
    lib.oracle_greedy.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_uint32, P, P, P]
    lib.oracle_round_priority.restype = ctypes.c_uint32
    lib.oracle_round_priority.argtypes = [ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_priority_collisions.restype = ctypes.c_int64
    lib.oracle_priority_collisions.argtypes = [ctypes.c_uint32]
    lib.oracle_local_max.restype = ctypes.c_int
    lib.oracle_local_max.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, P,
                                     ctypes.c_uint32, ctypes.c_int32, P, P, P, P, P,
                                     ctypes.c_int32]
    lib.oracle_local_max_reseed.restype = ctypes.c_int
    lib.oracle_local_max_reseed.argtypes = lib.oracle_local_max.argtypes
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def murmur3_x86_32(data: bytes, seed: int) -> int:
    """MurmurHash3_x86_32 of a byte string."""
    return int(_load().oracle_murmur3_x86_32(bytes(data), len(data), seed & 0xFFFFFFFF))


def priorities(seed: int, m: int) -> np.ndarray:
    """H(seed, e) for e in [0, m): hash of the id's four little-endian bytes."""
    out = np.empty(max(m, 0), dtype=np.uint32)
    if m > 0:
        _load().oracle_priorities(seed & 0xFFFFFFFF, m, _ptr(out))
    return out


def round_priority(seed: int, rnd: int, e: int) -> int:
    """H(H(seed, round), e): the reseeded order's priority."""
    return int(_load().oracle_round_priority(seed & 0xFFFFFFFF, rnd, e))


def priority_collisions(seed: int) -> int:
    """Number of repeated values of H(seed, x) over all 2^32 ids x."""
    return int(_load().oracle_priority_collisions(seed & 0xFFFFFFFF))


def n_words(m: int) -> int:
    return (m + 31) // 32


def bits_to_bool(bits: np.ndarray, m: int) -> np.ndarray:
    """Matched-edge bitmap (edge e = bit e%32 of word e//32) to a bool array."""
    b = np.asarray(bits, dtype=np.uint32)
    out = ((b[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).astype(bool).reshape(-1)
    return out[:m]


def bool_to_bits(flags: np.ndarray) -> np.ndarray:
    flags = np.asarray(flags, dtype=bool)
    m = flags.shape[0]
    pad = np.zeros(n_words(m) * 32, dtype=np.uint64)
    pad[:m] = flags
    w = pad.reshape(-1, 32) << np.arange(32, dtype=np.uint64)[None, :]
    return w.sum(axis=1).astype(np.uint32)


def greedy(n, m, e_off, e_pins, w, seed):
    """Sequential greedy.  Returns (bits uint32[ceil(m/32)], count, weight)."""
    e_off, e_pins = _i32(e_off), _i32(e_pins)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    bits = np.zeros(max(n_words(m), 1), dtype=np.uint32)
    cnt = ctypes.c_int64(0)
    wt = ctypes.c_uint64(0)
    rc = _load().oracle_greedy(n, m, _ptr(e_off), _ptr(e_pins), _ptr(w), seed & 0xFFFFFFFF,
                               _ptr(bits), ctypes.byref(cnt), ctypes.byref(wt))
    if rc != ORACLE_OK:
        raise ValueError(f"oracle_greedy failed with code {rc}")
    return bits[:n_words(m)], int(cnt.value), int(wt.value)


def local_max(n, m, e_off, e_pins, v_off, v_edges, w, seed, max_rounds=0, cap=None,
              reseed=False):
    """Round-based local max.  Returns (bits, stats dict).

    reseed=True draws fresh tie-breaking priorities every round:
    round r ranks by (w, H(H(seed, r), e), e)."""
    e_off, e_pins, v_off, v_edges = _i32(e_off), _i32(e_pins), _i32(v_off), _i32(v_edges)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    if cap is None:
        cap = m + 1
    bits = np.zeros(max(n_words(m), 1), dtype=np.uint32)
    le = np.zeros(max(cap, 1), dtype=np.int64)
    lp = np.zeros(max(cap, 1), dtype=np.int64)
    mr = np.zeros(max(cap, 1), dtype=np.int64)
    rounds = ctypes.c_int32(0)
    fn = _load().oracle_local_max_reseed if reseed else _load().oracle_local_max
    rc = fn(n, m, _ptr(e_off), _ptr(e_pins), _ptr(v_off), _ptr(v_edges),
                                  _ptr(w), seed & 0xFFFFFFFF, max_rounds, _ptr(bits),
                                  ctypes.byref(rounds), _ptr(le), _ptr(lp), _ptr(mr), cap)
    if rc == ORACLE_E_ROUNDS:
        raise RuntimeError("round limit reached")
    if rc != ORACLE_OK:
        raise ValueError(f"oracle_local_max failed with code {rc}")
    r = int(rounds.value)
    k = min(r, cap)
    return bits[:n_words(m)], {"rounds": r, "live_edges": le[:k].copy(),
                               "live_pins": lp[:k].copy(), "matched_per_round": mr[:k].copy()}


# ----------------------------------------------------------------------------
# Property checks (vectorised numpy; valid at any size).

def _edge_of_incidence(e_off):
    e_off = np.asarray(e_off, dtype=np.int64)
    sizes = np.diff(e_off)
    return np.repeat(np.arange(sizes.shape[0], dtype=np.int64), sizes)


def check_matching(n, m, e_off, e_pins, bits) -> bool:
    """Matched edges are pairwise vertex-disjoint (Preliminaries, Matching)."""
    matched = bits_to_bool(bits, m)
    eid = _edge_of_incidence(e_off)
    pins = np.asarray(e_pins, dtype=np.int64)[matched[eid]]
    if pins.size == 0:
        return True
    return int(np.bincount(pins, minlength=n).max()) <= 1


def check_maximal(n, m, e_off, e_pins, bits) -> bool:
    """No unmatched edge can be added: each has a pin covered by the matching."""
    matched = bits_to_bool(bits, m)
    eid = _edge_of_incidence(e_off)
    pins = np.asarray(e_pins, dtype=np.int64)
    covered = np.zeros(n, dtype=bool)
    covered[pins[matched[eid]]] = True
    hit = np.zeros(m, dtype=bool)
    np.logical_or.at(hit, eid, covered[pins])
    return bool(np.all(matched | hit))


def edge_rank(w, seed, m) -> np.ndarray:
    """Rank of each edge in the tuple order (w, H(seed,e), e), 0 = lowest.

    (w, h) is packed into one unsigned 64-bit word with w in the high half,
    which orders exactly as the pair; a stable sort then orders equal words
    by ascending id, the tuple's last component."""
    h = priorities(seed, m)
    wh = (np.asarray(w, dtype=np.uint64) << np.uint64(32)) | h.astype(np.uint64)
    order = np.argsort(wh, kind="stable")
    rank = np.empty(m, dtype=np.int64)
    rank[order] = np.arange(m, dtype=np.int64)
    return rank


def check_greedy_certificate(n, m, e_off, e_pins, w, seed, bits) -> bool:
    """True iff `bits` is exactly the greedy matching for the edge order.

    A set M is the greedy result for a strict order iff (i) M is a matching and
    (ii) every edge outside M shares a pin with an edge of M ranked above it:
    greedy rejects an edge exactly when an earlier (higher) chosen edge holds
    one of its pins, and by induction down the order the two conditions fix
    each edge's membership, so the set meeting both is unique.  Empty edges
    have no pins and therefore must be in M.
    """
    if not check_matching(n, m, e_off, e_pins, bits):
        return False
    matched = bits_to_bool(bits, m)
    rank = edge_rank(w, seed, m)
    eid = _edge_of_incidence(e_off)
    pins = np.asarray(e_pins, dtype=np.int64)
    cover = np.full(n, -1, dtype=np.int64)
    mi = matched[eid]
    cover[pins[mi]] = rank[eid[mi]]
    # best_cover[e] = highest rank of a matched edge at a pin of e (-1: none)
    sizes = np.diff(np.asarray(e_off, dtype=np.int64))
    best_cover = np.full(m, -1, dtype=np.int64)
    nz = sizes > 0
    if pins.size:
        starts = np.asarray(e_off, dtype=np.int64)[:-1][nz]
        best_cover[nz] = np.maximum.reduceat(cover[pins], starts)
    unmatched = ~matched
    return bool(np.all(best_cover[unmatched] > rank[unmatched]))


def brute_force_max(n, m, e_off, e_pins, w):
    """Exhaustive maximum-weight and maximum-cardinality matching (tiny m).

    Returns (max_weight, max_cardinality).  Branches on each edge in id
    order: skip it, or take it when it is disjoint from the taken set.
    """
    masks = []
    for e in range(m):
        mk = 0
        for p in e_pins[e_off[e]:e_off[e + 1]]:
            mk |= 1 << int(p)
        masks.append(mk)
    wl = [int(x) for x in w]
    best_w = 0
    best_c = 0

    def rec(i, used, tw, tc):
        nonlocal best_w, best_c
        if i == m:
            best_w = max(best_w, tw)
            best_c = max(best_c, tc)
            return
        rec(i + 1, used, tw, tc)
        if masks[i] & used == 0:
            rec(i + 1, used | masks[i], tw + wl[i], tc + 1)

    rec(0, 0, 0, 0)
    return best_w, best_c
