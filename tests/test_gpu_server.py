"""The request server: every request's bitmap is the same in the mix as
alone (and equals the oracle), admission never exceeds the HBM budget,
requests beyond the budget wait, requests that arrive while others run are
admitted and their waves overlap on the device."""
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


@pytest.fixture(scope="module")
def pool():
    """Mixed sizes: kappa log-uniform in [1e3, 3e5], |e| ~ U{2..32}."""
    return synth.config_served_pool(seed=55, count=48, k_lo=1e3, k_hi=3e5)


def _drain(srv, n, timeout=120.0):
    got = []
    t0 = time.time()
    while len(got) < n:
        got += srv.poll(cap=64, timeout_s=0.5)
        assert time.time() - t0 < timeout, f"only {len(got)} of {n} results"
    return got


def _expected(pool):
    return [oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 1000 + i)[0]
            for i, g in enumerate(pool)]


def test_mix_equals_alone_and_oracle(hgm, pool):
    import torch
    exp = _expected(pool)
    srv = hgm.Server(1 << 30, workers=2)
    try:
        # warm-up: the workers' first device calls happen here
        srv.submit(pool[0], 1, req_id=10_000)
        _drain(srv, 1)
        # a first burst; once it has been admitted as a wave, the rest arrive
        # and form a second wave while the first is still on the device
        for i in range(24):
            srv.submit(pool[i], 1000 + i, req_id=i)
        t0 = time.time()
        while srv.info()["queued"] > 0:
            assert time.time() - t0 < 30, "first wave never admitted"
            time.sleep(0.0001)
        for i in range(24, len(pool)):
            srv.submit(pool[i], 1000 + i, req_id=i)
        res = _drain(srv, len(pool))
        info = srv.info()
    finally:
        srv.close()
    assert info["arena_peak"] <= info["arena_bytes"]
    for r in res:
        assert r["status"] == 0
        assert np.array_equal(r["bits"], exp[r["id"]]), f"request {r['id']} differs in the mix"
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    # alone: each request through hgm_match on its own
    for i in (0, 7, 30, len(pool) - 1):
        dg = hgm.DeviceHypergraph.from_host(pool[i], "cuda:0")
        bits, _ = hgm.match(dg, 1000 + i, hgm.make_opts("auto"))
        torch.cuda.synchronize()
        assert np.array_equal(bits.cpu().numpy().view(np.uint32), exp[i])
    # several waves, and at least two of them overlapped in time
    waves = {}
    for r in res:
        waves.setdefault((r["t_admit"], r["t_done"]), []).append(r["id"])
    spans = sorted(waves)
    assert len(spans) >= 2
    overlap = any(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    assert overlap, "no two waves were on the device at the same time"


def test_tiny_budget_queues_and_never_overcommits(hgm, pool):
    exp = _expected(pool)
    big = max(range(len(pool)), key=lambda i: pool[i].kappa)
    # room for about one large request at a time
    budget = 64 * pool[big].kappa + (8 << 20)
    srv = hgm.Server(budget, workers=3)
    try:
        for i, g in enumerate(pool):
            srv.submit(g, 1000 + i, req_id=i)
        res = _drain(srv, len(pool))
        info = srv.info()
    finally:
        srv.close()
    assert info["arena_peak"] <= budget
    assert all(r["status"] == 0 for r in res)
    for r in res:
        assert np.array_equal(r["bits"], exp[r["id"]])
    assert max(r["wave_size"] for r in res) < len(pool)   # the budget split the work


def test_request_larger_than_budget_fails_cleanly(hgm, pool):
    big = max(pool, key=lambda g: g.kappa)
    small = min(pool, key=lambda g: g.kappa)
    srv = hgm.Server(1 << 20, workers=1)   # 1 MiB
    try:
        srv.submit(big, 1, req_id=0)
        srv.submit(small, 2, req_id=1)
        res = {r["id"]: r for r in _drain(srv, 2)}
    finally:
        srv.close()
    assert res[0]["status"] == hgm.HGM_E_SIZE
    assert res[1]["status"] == 0
    exp = oracle.greedy(small.n, small.m, small.e_off, small.e_pins, small.w, 2)[0]
    assert np.array_equal(res[1]["bits"], exp)


def test_edge_side_only_requests(hgm, pool):
    """Requests without the vertex side (not uploaded): same bitmaps."""
    exp = _expected(pool)
    srv = hgm.Server(1 << 30, workers=3, edge_side_only=True)
    try:
        for i, g in enumerate(pool):
            srv.submit(g, 1000 + i, req_id=i)
        res = _drain(srv, len(pool))
    finally:
        srv.close()
    assert all(r["status"] == 0 for r in res)
    for r in res:
        assert np.array_equal(r["bits"], exp[r["id"]]), f"request {r['id']} differs"


def test_submit_argument_errors(hgm):
    """Requests the server refuses at submit, through the C ABI: nothing is
    queued and the server keeps serving."""
    import ctypes
    lib = hgm.load()
    srv = hgm.Server(1 << 20, workers=1)
    try:
        def submit(**kw):
            q = hgm.HgmRequest()
            q.id, q.n, q.m, q.kappa = 0, 0, 0, 0
            for k, v in kw.items():
                setattr(q, k, v)
            return lib.hgm_server_submit(srv.h, ctypes.byref(q))
        assert submit(n=-1) == hgm.HGM_E_ARG
        assert submit(kappa=1 << 31) == hgm.HGM_E_ARG
        assert submit(m=3, n=2) == hgm.HGM_E_ARG            # arrays missing
        assert submit(m=2 ** 31 - 1) == hgm.HGM_E_SIZE      # its bitmap exceeds a wave's bits
        assert lib.hgm_server_submit(None, None) == hgm.HGM_E_ARG
        assert srv.info()["submitted"] == 0
        g = synth.random_instance(3, 50, 40, 2, 5, 1, 9)
        srv.submit(g, 4, req_id=7)
        (r,) = _drain(srv, 1)
    finally:
        srv.close()
    assert r["status"] == 0
    assert np.array_equal(r["bits"], oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 4)[0])


@pytest.mark.parametrize("variant,max_batch", [("crew", 0), ("crcw", 1), ("auto", 5)])
def test_server_variants_and_wave_caps(hgm, pool, variant, max_batch):
    """The server with other round variants and wave caps (max_batch = 1:
    one request per wave): every bitmap still equals the oracle's."""
    exp = _expected(pool)
    srv = hgm.Server(1 << 30, workers=2, max_batch=max_batch, opts=hgm.make_opts(variant))
    try:
        for i, g in enumerate(pool[:16]):
            srv.submit(g, 1000 + i, req_id=i)
        res = _drain(srv, 16)
    finally:
        srv.close()
    assert all(r["status"] == 0 for r in res)
    for r in res:
        assert np.array_equal(r["bits"], exp[r["id"]]), f"request {r['id']} differs ({variant})"
    if max_batch:
        assert max(r["wave_size"] for r in res) <= max_batch


def _served_request(seed, kappa):
    """A request of the served workload's shape with about `kappa` pins:
    |e| ~ U{2..32}, m = round(kappa / 17), n = max(32, round(m / 2)),
    w ~ U{1..1e6}."""
    m = max(1, round(kappa / 17))
    return synth.random_instance(seed, max(32, round(m / 2)), m, 2, 32, 1, 1_000_000)


@pytest.mark.parametrize("edge_side_only", [True, False])
def test_large_requests_served_range(hgm, pool, edge_side_only):
    """Requests across the served workload's whole kappa range [1e3, 1e7]:
    three large ones (kappa about 1e6, 3e6 and 1e7) submitted among small
    ones; every bitmap equals the oracle's."""
    big = [_served_request(901, 1e6), _served_request(902, 3e6), _served_request(903, 1e7)]
    print("large requests kappa=" + ",".join(str(g.kappa) for g in big), flush=True)
    reqs = big[:1] + pool[:8] + big[1:2] + pool[8:16] + big[2:]
    srv = hgm.Server(4 << 30, workers=3, edge_side_only=edge_side_only)
    try:
        for i, g in enumerate(reqs):
            srv.submit(g, 7000 + i, req_id=i)
        res = _drain(srv, len(reqs), timeout=300)
        info = srv.info()
    finally:
        srv.close()
    assert info["arena_peak"] <= info["arena_bytes"]
    for r in res:
        g = reqs[r["id"]]
        assert r["status"] == 0
        exp = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 7000 + r["id"])[0]
        assert np.array_equal(r["bits"], exp), f"request {r['id']} (kappa {g.kappa}) differs"


@pytest.mark.parametrize("edge_side_only", [True, False])
def test_malformed_request_fails_alone(hgm, pool, edge_side_only):
    """A request with a pin out of range, or offsets that do not end at
    kappa, completes with HGM_E_CSR before upload; the requests submitted
    around it, which may share its wave, still equal the oracle."""
    exp = _expected(pool)
    bad_pin = synth.random_instance(4, 100, 80, 2, 6, 1, 9)
    bad_pin.e_pins = bad_pin.e_pins.copy()
    bad_pin.e_pins[5] = bad_pin.n + 3
    bad_off = synth.random_instance(5, 100, 80, 2, 6, 1, 9)
    bad_off.e_off = bad_off.e_off.copy()
    bad_off.e_off[40] = bad_off.e_off[39] - 1
    srv = hgm.Server(1 << 30, workers=1, edge_side_only=edge_side_only)
    try:
        for i in range(12):
            srv.submit(pool[i], 1000 + i, req_id=i)
        srv.submit(bad_pin, 1, req_id=100)
        srv.submit(bad_off, 1, req_id=101)
        for i in range(12, 20):
            srv.submit(pool[i], 1000 + i, req_id=i)
        res = {r["id"]: r for r in _drain(srv, 22)}
    finally:
        srv.close()
    assert res[100]["status"] == hgm.HGM_E_CSR and res[101]["status"] == hgm.HGM_E_CSR
    for i in range(20):
        assert res[i]["status"] == 0
        assert np.array_equal(res[i]["bits"], exp[i]), i
