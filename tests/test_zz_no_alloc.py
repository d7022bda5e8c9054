"""GPU test of hgm_match_noalloc, the entry point for callers that cannot
allocate device memory: through the C ABI it must give exactly hgm_match's
bitmap and counters (the matching is integer work with one correct result),
on consecutive calls that share the per-GPU scratch array, the second on a
smaller instance, and refuse an instance larger than the array."""
import ctypes

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


def _stats(hgm, cap=4096):
    st, arrays, rms = hgm._stats_struct(cap, False)
    return st, arrays, rms


def _with_workspace(hgm, dg, seed, opts):
    bits, st = hgm.match(dg, seed, opts)
    return bits.cpu().numpy().view(np.uint32).copy(), st


def _noalloc(hgm, dg, seed, opts):
    import torch
    words = max((dg.m + 31) // 32, 1)
    bits = torch.full((words,), -1, dtype=torch.int32, device=dg.e_pins.device)
    st, arrays, rms = _stats(hgm)
    stream = torch.cuda.current_stream(dg.e_pins.device).cuda_stream
    rc = hgm.hgm_match_noalloc(dg.csr(), seed, bits.data_ptr(), opts, stream, st)
    assert rc == hgm.HGM_OK, hgm.hgm_strerror(rc)
    torch.cuda.synchronize()
    return (bits.cpu().numpy().view(np.uint32)[:(dg.m + 31) // 32].copy(),
            hgm._stats_dict(st, arrays, rms, False))


def _same(a, b):
    bits_a, st_a = a
    bits_b, st_b = b
    assert np.array_equal(bits_a, bits_b)
    for k in ("rounds", "matched", "weight"):
        assert st_a[k] == st_b[k], k
    for k in ("live_edges", "live_pins", "matched_per_round", "matched_pins"):
        assert np.array_equal(st_a[k], st_b[k]), k


@pytest.mark.parametrize("variant,extra", [("auto", {}), ("crcw", {}), ("crew", {}),
                                           ("auto", {"reseed": True})])
def test_noalloc_equals_match_twice(hgm, variant, extra):
    """Two calls in a row on one GPU, the second on a smaller instance: each
    equals hgm_match on its own workspace bit for bit (and the oracle)."""
    big = synth.random_instance(91, 60000, 120000, 2, 12, 1, 1000)
    small = synth.random_instance(92, 3000, 5000, 2, 6, 1, 50)
    opts = hgm.make_opts(variant, **extra)
    for g, seed in ((big, 5), (small, 6)):
        dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
        ws_bytes = hgm.hgm_workspace_size(dg.csr(), opts)
        assert 0 < ws_bytes <= hgm.hgm_noalloc_max_bytes()
        got = _noalloc(hgm, dg, seed, opts)
        ref = _with_workspace(hgm, dg, seed, opts)
        _same(got, ref)
        if not extra:
            expect = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)[0]
            assert np.array_equal(got[0], expect)


def test_noalloc_pairs_and_empty(hgm):
    """The graph layout, then an instance with no edges, then the graph again:
    the array left by the previous call never leaks into the next result."""
    import torch
    g = synth.random_instance(93, 20000, 40000, 2, 2, 1, 1)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    opts = hgm.make_opts("auto", pairs=True)
    first = _noalloc(hgm, dg, 3, opts)
    _same(first, _with_workspace(hgm, dg, 3, opts))
    empty = synth.from_edge_lists(5, [], [])
    de = hgm.DeviceHypergraph.from_host(empty, "cuda:0")
    bits, st = _noalloc(hgm, de, 3, hgm.make_opts("auto"))
    assert st["rounds"] == 0 and st["matched"] == 0
    again = _noalloc(hgm, dg, 3, opts)
    _same(again, first)
    torch.cuda.synchronize()


def test_noalloc_refuses_beyond_its_array(hgm):
    """An instance whose workspace exceeds the array fails with HGM_E_SIZE and
    writes nothing; timing (which creates events) is refused."""
    import torch
    cap = hgm.hgm_noalloc_max_bytes()
    m = 2_000_000
    g = synth.random_instance(94, 400000, m, 2, 3, 1, 1000)
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    opts = hgm.make_opts("crcw")
    assert hgm.hgm_workspace_size(dg.csr(), opts) > cap
    bits = torch.full(((m + 31) // 32,), 7, dtype=torch.int32, device="cuda:0")
    rc = hgm.hgm_match_noalloc(dg.csr(), 1, bits.data_ptr(), opts, 0, None)
    assert rc == hgm.HGM_E_SIZE
    torch.cuda.synchronize()
    assert int((bits != 7).sum()) == 0
    small = hgm.DeviceHypergraph.from_host(synth.random_instance(95, 100, 200, 2, 4, 1, 9),
                                           "cuda:0")
    st = hgm.HgmStats()
    st.cap = 0
    st.timing = 1
    b2 = torch.zeros(8, dtype=torch.int32, device="cuda:0")
    assert hgm.hgm_match_noalloc(small.csr(), 1, b2.data_ptr(), None, 0,
                                 st) == hgm.HGM_E_ARG
