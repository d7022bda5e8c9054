"""GPU parity of the binned next-round maximum (hgm_opts.bin_shift).

From round 1 on, in rounds where the host expects at least n / 2 surviving
pins, the retire pass writes each surviving non-hub pin's record (index in
its bin, key) to the bin of its vertex range, hub pins go through the
per-workgroup LDS table, and one workgroup per bin reduces the bin in LDS.
The bitmap and every per-round count must equal the oracle's (greedy bitmap,
round simulator counts) with bins of every allowed size, a ragged last bin,
many and few hubs (more hubs than the table holds), equal weights, key-0
edges, empty edges, per-round priorities and shuffled lists.  A vertex side
that is not the transpose of the edge side can overflow a bin: the call
returns HGM_E_CSR, writes nothing outside the bins, and the workspace serves
the next call."""
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


def _run(hgm, g, seed, ws=None, **kw):
    import torch
    dg = hgm.DeviceHypergraph.from_host(g, "cuda:0")
    bits, st = hgm.match(dg, seed, hgm.make_opts("auto", **kw), workspace=ws)
    torch.cuda.synchronize()
    return bits.cpu().numpy().view(np.uint32), st


def _check(hgm, g, seed, reseed=False, **kw):
    exp, ref = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w, seed,
                                reseed=reseed)
    if not reseed:
        gbits, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, seed)
        assert np.array_equal(gbits, exp)
    got, st = _run(hgm, g, seed, reseed=reseed, **kw)
    assert np.array_equal(got, exp), f"bitmap differs ({kw}, reseed={reseed})"
    assert st["rounds"] == ref["rounds"]
    for k in ("live_edges", "live_pins", "matched_per_round"):
        assert np.array_equal(st[k], ref[k]), k
    sel = oracle.bits_to_bool(got, g.m)
    assert st["matched"] == int(sel.sum())
    assert st["weight"] == int(g.w[sel].astype(np.uint64).sum())
    return st


@pytest.mark.parametrize("shift", [10, 12, 14, -1])
@pytest.mark.parametrize("reseed", [False, True])
def test_bins_power_law_small(hgm, shift, reseed):
    """Zipf vertex popularity (hubs above the threshold go to the LDS table,
    the rest to bins), n = 50,001: the last bin of 2^10 is ragged."""
    g = synth.config_power_law(seed=611, n=50_001, m=150_000)
    print(f"power-law small shift={shift} reseed={reseed}", flush=True)
    _check(hgm, g, 5, reseed=reseed, bin_shift=shift, hub_threshold=256)


@pytest.mark.parametrize("hub", [16, 1 << 30])
def test_bins_hub_table_full_or_absent(hgm, hub):
    """Threshold 16 makes more hubs than the LDS table holds (the others take
    the bins); 2^30 makes none (every pin in the bins)."""
    g = synth.config_power_law(seed=612, n=40_000, m=120_000)
    print(f"hub threshold {hub}", flush=True)
    _check(hgm, g, 9, bin_shift=11, hub_threshold=hub)


@pytest.mark.parametrize("reseed", [False, True])
def test_bins_equal_weights_hub_stress(hgm, reseed):
    """All weights 1 (ties broken by the priority hash), one vertex in a
    quarter of the edges."""
    g = synth.config_hub_stress(seed=613, n=200_000, m=400_000)
    print(f"hub-stress small reseed={reseed}", flush=True)
    _check(hgm, g, 3, reseed=reseed, bin_shift=12)


def test_bins_empty_and_zero_key_edges(hgm):
    """Empty edges (matched in round 0, no pins) and weight-0 edges (key 0 when
    the hash is 0 too; never above another key of the same vertex)."""
    g = synth.random_instance(614, 30_000, 120_000, 2, 10, 0, 3, empty_frac=0.05)
    print("empty and weight-0 edges", flush=True)
    _check(hgm, g, 11, bin_shift=10)


def test_bins_shuffled_lists(hgm):
    """Pins in any order within an edge, incident edges in any order within a
    vertex list."""
    g = synth.shuffle_lists(synth.config_power_law(seed=615, n=60_000, m=160_000), 77)
    print("shuffled lists", flush=True)
    _check(hgm, g, 2, bin_shift=12, hub_threshold=512)


def test_bins_overflow_is_an_error(hgm):
    """A v_off that puts every incidence on the last vertex (still a valid
    offset array, so every read stays inside v_edges) gives all other bins a
    capacity of 0: the first binned round finds them overflowing and the call
    fails with HGM_E_CSR.  The same workspace then matches the real instance
    exactly."""
    import torch
    g = synth.random_instance(616, 20_000, 60_000, 2, 8, 1, 1000)
    bad = synth.Hypergraph(g.n, g.m, g.e_off, g.e_pins,
                           np.concatenate([np.zeros(g.n, np.int32),
                                           np.array([g.kappa], np.int32)]),
                           g.v_edges, g.w)
    opts = hgm.make_opts("auto", bin_shift=10)
    dg_bad = hgm.DeviceHypergraph.from_host(bad, "cuda:0")
    ws = hgm.alloc_workspace(dg_bad, opts)
    print("overflowing bins", flush=True)
    with pytest.raises(hgm.HgmError) as ei:
        hgm.match(dg_bad, 4, opts, workspace=ws)
    assert ei.value.code == hgm.HGM_E_CSR
    torch.cuda.synchronize()
    print("same workspace, real instance", flush=True)
    _check(hgm, g, 4, ws=ws, bin_shift=10)


@pytest.mark.parametrize("tail", [1000, 1 << 30])
def test_bins_with_tail(hgm, tail):
    """Binned early rounds, then the one-workgroup tail: from round 1 on
    (bound 2^30) or for the last rounds (bound 1000)."""
    g = synth.config_power_law(seed=617, n=50_000, m=150_000)
    print(f"bins with tail {tail}", flush=True)
    st = _check(hgm, g, 6, bin_shift=11, hub_threshold=256, tail_pins=tail)
    assert st["rounds"] > 0


def test_bins_automatic_follows_degree_profile(hgm):
    """The automatic setting (the default) allocates bins for instances with
    n >= 2^17 and kappa >= 2^20 and uses them only where round 0 takes the
    vertex form; both cases equal the oracle."""
    for g in (synth.config_hub_stress(seed=618, n=150_000, m=300_000),
              synth.config_power_law(seed=619, n=150_000, m=400_000)):
        assert g.n >= 1 << 17 and g.kappa >= 1 << 20
        print(f"automatic bins n={g.n} kappa={g.kappa}", flush=True)
        _check(hgm, g, 8)
