"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2602_22976_amd as hgm
from paper_2602_22976_amd import build as hb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hb.LIB):
        hb.build(force=True)
    return hgm.load()


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(hgm_\w+)\s*\(", text)
    return sorted(set(names))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "hgm_match" in names and "hgm_workspace_size" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(hgm.EXPORTED) <= set(names)


def test_strerror_and_version(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert len(hgm.hgm_strerror(code)) > 5
    assert "unknown" in hgm.hgm_strerror(-99)
    assert hgm.hgm_version() >= 100


def _csr(n, m, kappa):
    c = hgm.HgmCsr()
    c.n, c.m, c.kappa = n, m, kappa
    fake = 0x1000
    c.e_off = c.e_pins = c.v_off = c.v_edges = c.w = fake
    return c


def test_workspace_size_layout(lib):
    small = hgm.hgm_workspace_size(_csr(10, 20, 100))
    nobins = hgm.make_opts(bin_shift=-1)
    big = hgm.hgm_workspace_size(_csr(2_000_000, 5_000_000, 30_000_000), nobins)
    assert 0 < small < big
    # two max buffers 16n, done n, two lists with their edge records (id 4,
    # pin offset 4, pin count 4, first pin 4, key 8) 48m at least; keys are
    # not stored per edge for one instance
    assert big >= 48 * 5_000_000 + 17 * 2_000_000
    assert big < 48 * 5_000_000 + 17 * 2_000_000 + 8 * 5_000_000
    rs = hgm.hgm_workspace_size(_csr(2_000_000, 5_000_000, 30_000_000),
                                hgm.make_opts(reseed=True, bin_shift=-1))
    assert rs == big
    crew = hgm.hgm_workspace_size(_csr(2_000_000, 5_000_000, 30_000_000), hgm.make_opts("crew"))
    assert crew > big
    val = hgm.hgm_workspace_size(_csr(2_000_000, 5_000_000, 30_000_000),
                                 hgm.make_opts(validate=True, bin_shift=-1))
    assert val >= big + 30_000_000 // 8 - 4096
    assert hgm.hgm_workspace_size(_csr(-1, 5, 5)) == 0
    assert hgm.hgm_workspace_size(_csr(5, 5, 2 ** 31)) == 0
    assert hgm.hgm_workspace_size(_csr(5, 5, 5), hgm.make_opts(variant=7)) == 0
    # per-round priorities with the vertex-centric rounds: the same layout
    assert hgm.hgm_workspace_size(_csr(2_000_000, 5_000_000, 30_000_000),
                                  hgm.make_opts("crew", reseed=True)) == crew
    bad = hgm.make_opts()
    bad.reseed = 2
    assert hgm.hgm_workspace_size(_csr(5, 5, 5), bad) == 0


def test_workspace_bins(lib):
    """The binned maximum's records (2-byte index and 8-byte key per pin) and
    cursors are carved only where bins can run: AUTO with the vertex side,
    offset layout, at most 1024 bins; automatically (the default) for n >=
    2^17 and kappa >= 2^20."""
    big = _csr(2_000_000, 5_000_000, 30_000_000)
    off = hgm.hgm_workspace_size(big, hgm.make_opts(bin_shift=-1))
    auto = hgm.hgm_workspace_size(big)
    assert 10 * 30_000_000 <= auto - off <= 10 * 30_000_000 + 3 * 4096 + 1024
    for rb in (12, 13, 14):  # same size for every shift that fits
        assert hgm.hgm_workspace_size(big, hgm.make_opts(bin_shift=rb)) == auto
    # 2^21 vertices in bins of 2^10 would be 1954 bins: no bins
    assert hgm.hgm_workspace_size(big, hgm.make_opts(bin_shift=10)) == off
    # CRCW, CREW, graphs and instances without the vertex side have no bins
    for variant in ("crcw", "crew"):
        assert hgm.hgm_workspace_size(big, hgm.make_opts(variant, bin_shift=12)) == \
            hgm.hgm_workspace_size(big, hgm.make_opts(variant, bin_shift=-1))
    edge_only = _csr(2_000_000, 5_000_000, 30_000_000)
    edge_only.v_off = edge_only.v_edges = None
    assert hgm.hgm_workspace_size(edge_only, hgm.make_opts(bin_shift=12)) == \
        hgm.hgm_workspace_size(edge_only, hgm.make_opts(bin_shift=-1))
    # small instances: automatic leaves bins off, an explicit shift turns them on
    small = _csr(1000, 2000, 8000)
    assert hgm.hgm_workspace_size(small) == hgm.hgm_workspace_size(
        small, hgm.make_opts(bin_shift=-1))
    assert hgm.hgm_workspace_size(small, hgm.make_opts(bin_shift=10)) >= \
        hgm.hgm_workspace_size(small) + 10 * 8000
    for bad in (1, 9, 15, -2):
        assert hgm.hgm_workspace_size(small, hgm.make_opts(bin_shift=bad)) == 0


def test_match_rejects_bad_arguments_without_gpu(lib):
    ws = 0x100000
    bits = 0x2000
    # negative sizes, huge kappa, bad option, misaligned or short workspace
    assert hgm.hgm_match(_csr(-1, 5, 5), 1, bits, ws, 1 << 30) == hgm.HGM_E_ARG
    assert hgm.hgm_match(_csr(5, 5, 2 ** 31), 1, bits, ws, 1 << 30) == hgm.HGM_E_SIZE
    assert hgm.hgm_match(_csr(5, 5, 5), 1, bits, ws, 1 << 30,
                         hgm.make_opts(variant=9)) == hgm.HGM_E_ARG
    assert hgm.hgm_match(_csr(5, 5, 5), 1, bits, ws, 16) == hgm.HGM_E_SIZE
    assert hgm.hgm_match(_csr(5, 5, 5), 1, bits, ws + 8, 1 << 30) == hgm.HGM_E_ARG
    assert hgm.hgm_match(_csr(5, 5, 5), 1, 0, ws, 1 << 30) == hgm.HGM_E_ARG
    c = _csr(5, 5, 5)
    c.e_pins = None
    assert hgm.hgm_match(c, 1, bits, ws, 1 << 30) == hgm.HGM_E_ARG
    c = _csr(5, 5, 5)
    c.v_edges = None
    assert hgm.hgm_match(c, 1, bits, ws, 1 << 30, hgm.make_opts("crew")) == hgm.HGM_E_ARG
    assert lib.hgm_match(None, 1, None, None, 0, None, None, None) == hgm.HGM_E_ARG
    st = hgm.HgmStats()
    st.cap = -1
    assert hgm.hgm_match(_csr(5, 5, 5), 1, bits, ws, 1 << 30, None, 0, st) == hgm.HGM_E_ARG
    o = hgm.make_opts(rounds_per_sync=1000)
    assert hgm.hgm_match(_csr(5, 5, 5), 1, bits, ws, 1 << 30, o) == hgm.HGM_E_ARG
    # pairs (graphs): kappa must be 2m, e_pins 8-byte aligned, e_off optional
    assert hgm.hgm_match(_csr(5, 5, 9), 1, bits, ws, 1 << 30,
                         hgm.make_opts(pairs=True)) == hgm.HGM_E_ARG
    c = _csr(5, 5, 10)
    c.e_pins = 0x1004
    assert hgm.hgm_match(c, 1, bits, ws, 1 << 30, hgm.make_opts(pairs=True)) == hgm.HGM_E_ARG
    assert hgm.hgm_match(_csr(5, 5, 10), 1, bits, ws, 1 << 30,
                         hgm.make_opts("crew", pairs=True)) == hgm.HGM_E_ARG
    bad = hgm.make_opts()
    bad.pairs = 3
    assert hgm.hgm_match(_csr(5, 5, 10), 1, bits, ws, 1 << 30, bad) == hgm.HGM_E_ARG


def test_noalloc_arguments_without_gpu(lib):
    """hgm_match_noalloc refuses before any HIP call: bad sizes and options
    as hgm_match does, a workspace beyond its fixed array (HGM_E_SIZE) and
    timing statistics (HGM_E_ARG)."""
    bits = 0x2000
    cap = hgm.hgm_noalloc_max_bytes()
    assert cap == 64 << 20
    assert hgm.hgm_match_noalloc(_csr(-1, 5, 5), 1, bits) == hgm.HGM_E_ARG
    assert hgm.hgm_match_noalloc(_csr(5, 5, 2 ** 31), 1, bits) == hgm.HGM_E_SIZE
    assert hgm.hgm_match_noalloc(_csr(5, 5, 5), 1, bits,
                                 hgm.make_opts(variant=9)) == hgm.HGM_E_ARG
    assert lib.hgm_match_noalloc(None, 1, None, None, None, None) == hgm.HGM_E_ARG
    big = _csr(2_000_000, 5_000_000, 30_000_000)
    assert hgm.hgm_workspace_size(big) > cap
    assert hgm.hgm_match_noalloc(big, 1, bits) == hgm.HGM_E_SIZE
    st = hgm.HgmStats()
    st.timing = 1
    assert hgm.hgm_match_noalloc(_csr(5, 5, 5), 1, bits, None, 0, st) == hgm.HGM_E_ARG


def test_schedule_options_without_gpu(lib):
    """Schedule fields out of range are refused; the tuner's workspace covers
    its largest candidate edge grid."""
    c = _csr(2_000_000, 5_000_000, 30_000_000)
    for kw in (dict(edge_grid=-1), dict(edge_grid=65537), dict(blocks_per_cu=33),
               dict(clear_ratio=-2), dict(hot_degree=-1), dict(first_batch_pct=401),
               dict(solo_max_kappa=-2)):
        assert hgm.hgm_workspace_size(c, hgm.make_opts(**kw)) == 0, kw
    assert hgm.hgm_workspace_size(c, hgm.make_opts(edge_grid=65536, blocks_per_cu=32)) > 0
    base = hgm.hgm_workspace_size(c)
    t = lib.hgm_tune_workspace_size(ctypes.byref(c), None)
    assert t >= base and t >= hgm.hgm_workspace_size(c, hgm.make_opts(edge_grid=4096))


def test_tune_cache_lookup_without_gpu(lib, tmp_path):
    """The cache is a text file of `key : name=value ...` lines; without a
    device the key's device part reads "unknown".  A line for the instance's
    bucket fills the schedule fields; other buckets and a missing file leave
    the options unchanged."""
    c = _csr(10_000, 20_000, 100_000)      # round(log2 kappa) = 17, mean size 5
    path = tmp_path / "cache.txt"
    path.write_text("unknown match v0 p0 r0 k17 d5 c0 : solo=1 grid=512 bpc=4 hub=1024 hot=16 "
                    "clear=2 first=25 ms_default=1 ms_tuned=0.5\n"
                    "unknown match v2 p0 r0 k17 d5 c0 : grid=4096\n")
    o = hgm.make_opts("auto")
    assert lib.hgm_tuned_opts(str(path).encode(), ctypes.byref(c), ctypes.byref(o)) == 0
    assert (o.edge_grid, o.blocks_per_cu, o.hub_threshold, o.hot_degree, o.clear_ratio,
            o.first_batch_pct) == (512, 4, 1024, 16, 2, 25)
    o = hgm.make_opts("crew")
    assert lib.hgm_tuned_opts(str(path).encode(), ctypes.byref(c), ctypes.byref(o)) == 0
    assert o.edge_grid == 4096 and o.blocks_per_cu == 0
    o = hgm.make_opts("crcw")
    assert lib.hgm_tuned_opts(str(path).encode(), ctypes.byref(c), ctypes.byref(o)) == -1
    assert o.edge_grid == 0
    assert lib.hgm_tuned_opts(str(tmp_path / "none.txt").encode(), ctypes.byref(c),
                              ctypes.byref(o)) == -1


def test_product_package_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2602_22976_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "import baselines" not in text and "from baselines" not in text, fn
                assert "oracle_" not in text, fn


def _batch(count, n, m, kappa, words):
    b = hgm.HgmBatch()
    b.count, b.n_total, b.m_total, b.kappa_total, b.words_total = count, n, m, kappa, words
    fake = 0x1000
    b.v_base = b.e_base = b.pin_base = b.word_base = fake
    b.e_off = b.e_pins = b.v_off = b.v_edges = b.w = b.seeds = fake
    return b


def test_batch_arguments_without_gpu(lib):
    ok = _batch(4, 100, 200, 800, 8)
    size = hgm.hgm_batch_workspace_size(ok)
    # plus global offsets (one instance without its tail lists)
    assert size > hgm.hgm_workspace_size(_csr(100, 200, 800), hgm.make_opts(tail_pins=-1))
    assert hgm.hgm_batch_workspace_size(_batch(-1, 1, 1, 1, 1)) == 0
    assert hgm.hgm_batch_workspace_size(_batch(1, 1, 1, 2 ** 31, 1)) == 0
    assert hgm.hgm_batch_workspace_size(_batch(1, 1, 1, 1, 2 ** 27)) == 0
    ws, bits = 0x100000, 0x2000
    assert hgm.hgm_match_batch(_batch(-1, 1, 1, 1, 1), bits, ws, 1 << 30) == hgm.HGM_E_ARG
    assert hgm.hgm_match_batch(_batch(1, 1, 1, 2 ** 31, 1), bits, ws, 1 << 30) == hgm.HGM_E_SIZE
    assert hgm.hgm_match_batch(ok, bits, ws, 64) == hgm.HGM_E_SIZE
    assert hgm.hgm_match_batch(ok, 0, ws, 1 << 30) == hgm.HGM_E_ARG
    assert hgm.hgm_match_batch(ok, bits, ws, 1 << 30, hgm.make_opts(validate=True)) == hgm.HGM_E_ARG
    # per-round priorities: each edge also keeps its instance's seed and local id
    assert hgm.hgm_batch_workspace_size(ok, hgm.make_opts(reseed=True)) >= size + 8 * 200 - 256
    assert hgm.hgm_match_batch(ok, bits, ws, 1 << 30, hgm.make_opts(pairs=True)) == hgm.HGM_E_ARG
    b = _batch(4, 100, 200, 800, 8)
    b.seeds = None
    assert hgm.hgm_match_batch(b, bits, ws, 1 << 30) == hgm.HGM_E_ARG
    b = _batch(0, 0, 5, 5, 1)   # edges but no instance
    assert hgm.hgm_match_batch(b, bits, ws, 1 << 30) == hgm.HGM_E_ARG
    assert lib.hgm_match_batch(None, None, None, 0, None, None, None) == hgm.HGM_E_ARG


def test_server_arguments_without_gpu(lib):
    h = ctypes.c_void_p()
    so = hgm.HgmServerOpts()
    assert lib.hgm_server_create(None, 1 << 20, ctypes.byref(so), ctypes.byref(h)) == hgm.HGM_E_ARG
    assert lib.hgm_server_create(0x1000, 0, ctypes.byref(so), ctypes.byref(h)) == hgm.HGM_E_ARG
    assert lib.hgm_server_create(0x1008, 1 << 20, ctypes.byref(so), ctypes.byref(h)) == hgm.HGM_E_ARG
    so.workers = -1
    assert lib.hgm_server_create(0x1000, 1 << 20, ctypes.byref(so), ctypes.byref(h)) == hgm.HGM_E_ARG
    so.workers = 0
    so.match.validate = 1
    assert lib.hgm_server_create(0x1000, 1 << 20, ctypes.byref(so), ctypes.byref(h)) == hgm.HGM_E_ARG
    so.match.validate = 0
    so.edge_side_only = 2
    assert lib.hgm_server_create(0x1000, 1 << 20, ctypes.byref(so), ctypes.byref(h)) == hgm.HGM_E_ARG
    so.edge_side_only = 1
    so.match.variant = hgm.VARIANTS["crew"]
    assert lib.hgm_server_create(0x1000, 1 << 20, ctypes.byref(so), ctypes.byref(h)) == hgm.HGM_E_ARG
    assert lib.hgm_server_submit(None, None) == hgm.HGM_E_ARG
    assert lib.hgm_server_poll(None, None, 0, 0.0) == hgm.HGM_E_ARG
    assert lib.hgm_server_info(None, None) == hgm.HGM_E_ARG
    assert lib.hgm_server_destroy(None) == hgm.HGM_E_ARG


def test_request_check_without_gpu(lib):
    """hgm_request_check (the server's pre-upload check) on host arrays:
    well-formed requests pass, and each kind of malformed offset or id is
    rejected with HGM_E_CSR before any upload."""
    import numpy as np
    import synth
    g = synth.random_instance(5, 40, 60, 0, 6, 1, 9, empty_frac=0.1)
    for vside in (True, False):
        q, keep, _ = hgm.request(g, 1, 0, vside)
        assert hgm.hgm_request_check(q, vside) == hgm.HGM_OK

    def bad(field, mutate, vside=True):
        arrays = {k: getattr(g, k).copy() for k in ("e_off", "e_pins", "v_off", "v_edges", "w")}
        mutate(arrays[field])
        h = synth.Hypergraph(g.n, g.m, **arrays)
        q, keep, _ = hgm.request(h, 1, 0, vside)
        q.kappa = g.kappa
        return hgm.hgm_request_check(q, vside)

    def set_at(i, v):
        def f(a):
            a[i] = v
        return f

    k = g.kappa
    assert bad("e_off", set_at(0, 1)) == hgm.HGM_E_CSR              # does not start at 0
    assert bad("e_off", set_at(g.m, k - 1)) == hgm.HGM_E_CSR        # does not end at kappa
    i = int(np.flatnonzero(np.diff(g.e_off) > 1)[0]) + 1
    assert bad("e_off", set_at(i, int(g.e_off[i - 1]) - 1)) == hgm.HGM_E_CSR  # decreases
    assert bad("e_pins", set_at(3, g.n)) == hgm.HGM_E_CSR           # pin out of range
    assert bad("e_pins", set_at(7, -1)) == hgm.HGM_E_CSR
    assert bad("v_off", set_at(g.n, k + 1)) == hgm.HGM_E_CSR
    assert bad("v_edges", set_at(2, g.m)) == hgm.HGM_E_CSR          # edge id out of range
    assert bad("v_edges", set_at(2, g.m), vside=False) == hgm.HGM_OK  # vertex side not read
    # size and NULL errors
    q, keep, _ = hgm.request(g, 1, 0, True)
    q.n = -1
    assert hgm.hgm_request_check(q, True) == hgm.HGM_E_ARG
    q, keep, _ = hgm.request(g, 1, 0, False)
    assert hgm.hgm_request_check(q, True) == hgm.HGM_E_ARG          # vertex side missing
    assert lib.hgm_request_check(None, 1) == hgm.HGM_E_ARG


def test_server_rejects_duplicate_live_id():
    """A caller's id that is still in flight is refused before the C call
    (its result buffers are kept under that id)."""
    import synth
    srv = hgm.Server.__new__(hgm.Server)
    srv.live = {7: None}
    srv.next_id = 8
    srv.edge_side_only = False
    with pytest.raises(ValueError):
        srv.submit(synth.random_instance(1, 10, 10), 1, req_id=7)
    srv.h = None
