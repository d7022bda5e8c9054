#!/usr/bin/env python3
"""Benchmark of one hgm_match step on one MI355X.

A step is one whole matching of the workload: key construction, every round
(maximum, test, retire + compaction) until no live edge remains, and the
host's termination checks.  Inputs are resident in HBM before timing starts.

Printed (one JSON line):
  value        live pin incidences processed per second, sum over rounds of
               kappa_r divided by the step time (the per-round incidence
               throughput of the method, all overheads included)
  per_round    |L_r|, kappa_r, device time and kappa_r / t_r of each round;
               work_inflation = sum kappa_r / kappa; kernel_incidences_per_s
               = sum kappa_r over the summed kernel time
  roofline     the dominant kernel's algorithmic bytes / its HIP-event time,
               against the 8 TB/s HBM peak; `traffic` (bytes per launch) from
               the committed rocprofv3 PMC summary when it matches the kernel
               source, and traffic_gbs / traffic_frac, that traffic over the
               same average launch time
  cpu_baseline the oracle's greedy on one host core (a child process pinned
               by taskset): the step's sum of kappa_r over its mean time, so
               the two values compare as times; the round simulator's rate
               beside it
  cpu_multicore the OpenMP local max of baselines/ on the host's cores (up
               to 16 threads), same unit
  batched / served  the batched-vs-plain and Poisson-served legs
Graph workloads (delaunay, rgg) run with the pair layout (two pins per edge).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "pin-incidences/s per round + hypergraphs/s batched vs plain; p50/p99 latency"

WORKLOADS = {
    "power-law": ("config_power_law", "large power-law: n=2,000,000, m=5,000,000, |e|~Zipf(2.0) "
                  "on [2,64], vertex popularity Zipf(1.1), w log-uniform [1,2^20], seed 1"),
    "hub": ("config_hub_stress", "hub-stress: n=1,000,000, m=4,000,000, |e|~U[2,16], one hub "
            "in 25% of edges, all w=1, seed 1"),
    "plain": ("config_plain", "plain: n=10,000, m=20,000, |e|~U[2,8], w~U[1,1000], seed 1"),
    "delaunay": ("config_delaunay", "graph, Delaunay triangulation of 2^20 uniform points, "
                 "m=3,145,692, all w=1, pair layout, seed 1"),
    "rgg": ("config_rgg", "graph, random geometric graph on 2^20 uniform points, "
            "r=0.55 sqrt(ln n/n), m=6,891,095, all w=1, pair layout, seed 1"),
}
GRAPH_WORKLOADS = {"delaunay", "rgg"}   # every edge has two pins: run with the pair layout


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for fn in ("kernels.hip", "internal.h"):   # device code only: traffic is per kernel launch
        with open(os.path.join(ROOT, "paper_2602_22976_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(stats, variant_rounds, n, pairs=False, reseed=False, tail_from=None):
    """Bytes each kernel class must move, from the per-round counts.

    Units per round r: E = live edges, K = their pins, M / P = matched edges
    and their pins, E' / K' = survivors into round r+1.  Counts each array
    element the step needs once (re-reads from cache are not algorithmic).
    One instance stores no per-edge key: round 0 rebuilds it from the 4-byte
    weight and the hash.  From round 1 on, each live-list slot carries the
    edge's record beside its id (pin offset 4 + pin count 4 + first pin 4,
    or the two pins 8 with the pair layout, and the round's key 8), written
    by the retire pass for every survivor.  With the pair layout (graphs) no
    edge offsets are read:
      scatter (round 0): 8 B/edge (offset 4, weight 4) + 12 B/pin (pin 4,
              atomic 8)
      test:   per edge: round 0 offsets 8 + weight 4; later rounds id 4 +
              offset and count 8 + key 8 (the first pin comes from the
              record and counts as a pin).  Per pin: pin 4 + best 8 (+ 8
              clearing next round's buffer in CRCW); per matched edge 4
              (bitmap) and per matched pin 1 (done)
      retire: per edge: id 4 (not in round 0) + offset and count 8; per
              pin: pin 4 + done 1; per survivor: id 4 + record written
              (12 + key 8, pair layout 8 + 8) + its key read (weight 4 in
              round 0 or with per-round priorities, else the record's 8).
              CRCW adds 8 per surviving pin for the fused scatter; CREW 8
              per dead edge key
      vertex max: round 0 per vertex done 1 + offsets 4 + best 8, per pin
              v_edges 4 + weight 4.  Later rounds (CREW variant) read the
              lists compacted one round earlier: per vertex 21 (adds the list
              length read and write), per listed incidence id 4 + live key 8
              (the pins live one round earlier, an upper bound since done
              vertices are skipped), per kept incidence 4
      tail:   rounds from `tail_from` on run in the one-workgroup tail,
              whose compact list slots hold id 4 + pin offset and count (or
              two pins) 8 + key 8: at takeover the list is gathered (20 B
              read and 20 B written per live edge); per round the test reads
              each slot (20 B), per pin 4 + best 8, per matched edge 4, per
              matched pin 1; the retire reads each slot again, per pin 4 +
              done 1, writes 20 B per survivor, and forms the next maximum
              with 16 B per surviving pin (a zero, then the atomic)
    """
    E = list(stats["live_edges"]) + [0]
    K = list(stats["live_pins"]) + [0]
    M = stats["matched_per_round"]
    P = stats["matched_pins"]
    R = stats["rounds"]
    out = {"scatter": 0.0, "test": 0.0, "retire": 0.0, "vertex_max": 0.0, "tail": 0.0}
    offb = 0 if pairs else 8   # e_off[e], e_off[e + 1] per edge (record: offset, count)
    recw = 8 + 8 if pairs else 12 + 8   # record written per survivor, key included
    for r in range(R):
        if tail_from is not None and r >= tail_from:
            if r == tail_from:
                out["tail"] += 40 * E[r]
            out["tail"] += (20 * E[r] + 12 * K[r] + 4 * M[r] + P[r]) + \
                           (20 * E[r] + 5 * K[r] + 20 * E[r + 1] + 16 * K[r + 1])
            continue
        crew_r = variant_rounds(r)
        crew_next = variant_rounds(r + 1)
        if r == 0 and not crew_r:
            out["scatter"] += (offb // 2 + 4) * E[0] + 12 * K[0]
        if crew_r:
            if r == 0:
                out["vertex_max"] += 13 * n + 8 * K[0]
            else:
                out["vertex_max"] += 21 * n + 12 * K[r - 1] + 4 * K[r]
        test_edge = offb + 4 if r == 0 else 4 + offb + 8
        out["test"] += test_edge * E[r] + (12 + (0 if crew_next else 8)) * K[r] + 4 * M[r] + P[r]
        keysrc = 4 if (r == 0 or reseed) else 8
        ret = ((0 if r == 0 else 4) + offb) * E[r] + 5 * K[r] + (4 + recw + keysrc) * E[r + 1]
        if crew_next:
            ret += 8 * (E[r] - E[r + 1])
        else:
            ret += 8 * K[r + 1]
        out["retire"] += ret
    return out


def load_traffic(workload, kernel, digest, launches):
    """HBM bytes per launch of `kernel` from the committed PMC summary.

    The summary holds calibrated FETCH_SIZE + WRITE_SIZE bytes per call
    (summed over the class's dispatches); per launch is that over this run's
    launch count, as for `achieved`.  None when the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("{"):
                    d = json.loads(line)
                    if d.get("kernel_source") != digest:
                        return None
                    k = d.get("kernels", {}).get(kernel)
                    if k is None or not launches:
                        return None
                    return k.get("bytes_per_call") / launches
    except (OSError, ValueError):
        return None
    return None


def copy_probe(mib):
    """A plain device copy of known size, for scaling the PMC byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 3}), flush=True)


def batched_leg(count, steps):
    """Batched vs plain hypergraphs/s on `count` instances of the batched
    workload (n log-uniform in [100, 50,000], m = 2n, |e| ~ U{2..12},
    w ~ U{1..1000}, seed of instance i = i).  Batched: one hgm_match_batch
    call for all instances.  Plain: one hgm_match call per instance on the
    same device-resident arrays (each instance's slice is a standalone CSR),
    with one reused workspace."""
    import numpy as np
    import torch
    import paper_2602_22976_amd as hgm
    import synth
    t0 = time.perf_counter()
    b = synth.config_batched(seed=1004, count=count)
    gen_s = time.perf_counter() - t0
    dev = "cuda:0"
    db = hgm.DeviceBatch.from_host(b, dev)
    opts = hgm.make_opts("auto")
    ws = hgm.alloc_batch_workspace(db, opts)
    bits = torch.empty(max(db.words_total, 1), dtype=torch.int32, device=dev)
    hgm.match_batch(db, opts, workspace=ws, bits=bits, want_stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = hgm.match_batch(db, opts, workspace=ws, bits=bits, want_stats=True)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    batch_bits = bits.clone()
    _, sti = hgm.match_batch(db, opts, workspace=ws, bits=bits, timing=True)
    off = hgm.make_opts("auto", solo_max_kappa=-1)   # the round kernels alone
    ws_off = hgm.alloc_batch_workspace(db, off)
    hgm.match_batch(db, off, workspace=ws_off, bits=bits, want_stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hgm.match_batch(db, off, workspace=ws_off, bits=bits, want_stats=False)
    torch.cuda.synchronize()
    t_rounds_only = (time.perf_counter() - t0) / steps
    same_off = bool(torch.equal(bits, batch_bits))
    del ws_off

    views = []
    wmax = 0
    for i in range(b.count):
        n, m = int(b.n[i]), int(b.m[i])
        eb, vb, pb = int(b.e_base[i]), int(b.v_base[i]), int(b.pin_base[i])
        kap = int(b.pin_base[i + 1]) - pb
        dg = hgm.DeviceHypergraph(n, m, db.e_off[eb + i: eb + i + m + 1], db.e_pins[pb: pb + kap],
                                  db.v_off[vb + i: vb + i + n + 1], db.v_edges[pb: pb + kap],
                                  db.w[eb: eb + m])
        wb0, wb1 = int(b.word_base[i]), int(b.word_base[i + 1])
        views.append((dg, int(b.seeds[i]), bits[wb0:wb1] if wb1 > wb0 else bits[:1]))
        wmax = max(wmax, hgm.hgm_workspace_size(dg.csr(), opts))
    pws = torch.empty(wmax, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dg, seed, bv in views:
        hgm.match(dg, seed, opts, workspace=pws, bits=bv, want_stats=False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = bool(torch.equal(bits, batch_bits))
    return {"instances": count, "m_total": int(b.e_base[-1]), "kappa_total": int(b.pin_base[-1]),
            "generated_s": round(gen_s, 1), "rounds": st["rounds"],
            "ms_batched": t_batch * 1e3, "ms_plain": t_plain * 1e3,
            "hypergraphs_per_s_batched": count / t_batch,
            "hypergraphs_per_s_plain": count / t_plain,
            "batched_over_plain": t_plain / t_batch, "plain_equals_batched": same,
            "solo_ms": sti["kernel_ms"]["solo"],
            "kernel_ms": {k: round(v, 3) for k, v in sti["kernel_ms"].items()},
            "ms_round_kernels_only": t_rounds_only * 1e3,
            "round_kernels_only_equal": same_off}


def served_leg(rate, duration, pool_count, budget_gb, workers, warmup_s=5.0,
               edge_side_only=True, solo_max_kappa=0):
    """Open-loop Poisson arrivals at `rate` req/s for `duration` s into the
    request server.  Requests are drawn (seeded) from a pool of pre-generated
    hypergraphs in pinned host memory (kappa log-uniform in [1e3, 1e7],
    |e| ~ U{2..32}, m = round(kappa/17), n = max(32, round(m/2)),
    w ~ U{1..1e6}); request i uses priority seed i.  Latency = completion
    minus scheduled arrival (monotonic clock), over requests arriving after
    the first `warmup_s` seconds (at most a fifth of the run)."""
    import threading
    import numpy as np
    import torch
    import paper_2602_22976_amd as hgm
    import synth
    t0 = time.perf_counter()
    views, keep = served_pool(pool_count, vertex_side=not edge_side_only)
    gen_s = time.perf_counter() - t0
    arrivals = synth.gen.poisson_arrivals(2005, rate, duration)
    pick = np.random.Generator(np.random.PCG64(3005)).integers(0, len(views), size=arrivals.size)
    srv = hgm.Server(int(budget_gb * (1 << 30)), workers=workers,
                     opts=hgm.make_opts("auto", solo_max_kappa=solo_max_kappa),
                     edge_side_only=edge_side_only)
    sched = {}
    done = []
    start = time.monotonic() + 0.05

    def feed():
        for i, (ta, k) in enumerate(zip(arrivals, pick)):
            target = start + ta
            while True:
                dt = target - time.monotonic()
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.0005))
            sched[i] = target
            srv.submit(views[k], i, req_id=i)

    th = threading.Thread(target=feed)
    th.start()
    while len(done) < arrivals.size:
        done += srv.poll(cap=1024, timeout_s=0.2)
        if not th.is_alive() and len(done) < arrivals.size and time.monotonic() > start + duration + 120:
            break
    th.join()
    info = srv.info()
    srv.close()
    end = max(r["t_done"] for r in done)
    ok = [r for r in done if r["status"] == 0]
    steady = [r for r in ok if arrivals[r["id"]] >= min(warmup_s, 0.2 * duration)]
    lat = np.array([r["t_done"] - sched[r["id"]] for r in steady])
    wait = np.array([r["t_admit"] - r["t_submit"] for r in steady])
    kap = sum(views[pick[r["id"]]].kappa for r in ok)
    return {"rate": rate, "duration_s": duration, "requests": int(arrivals.size),
            "completed": len(ok), "failed": len(done) - len(ok), "pool": pool_count,
            "pool_generated_s": round(gen_s, 1), "workers": workers, "budget_gb": budget_gb,
            "edge_side_only": edge_side_only,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "hypergraphs_per_s": len(ok) / (end - start),
            "incidences_per_s": kap / (end - start),
            "mean_wave": float(np.mean([r["wave_size"] for r in ok])),
            "queue_wait_p50_ms": float(np.percentile(wait, 50) * 1e3),
            "queue_wait_p99_ms": float(np.percentile(wait, 99) * 1e3),
            "admission_stalls": int(info["stalls"]), "stall_s": float(info["stall_s"]),
            "arena_peak_gb": info["arena_peak"] / (1 << 30)}


_POOL = {}


def served_pool(count, vertex_side=False):
    """The served workload's request pool in pinned host memory (asynchronous
    uploads): kappa log-uniform in [1e3, 1e7], |e| ~ U{2..32}, m =
    round(kappa/17), n = max(32, round(m/2)), w ~ U{1..1e6}, drawn in worker
    processes; with vertex_side False only the edge side is drawn and sent.
    Returns (views of the pinned arrays, the tensors that back them)."""
    key = (count, vertex_side)
    if key in _POOL:
        return _POOL[key]
    import numpy as np
    import torch
    import synth
    pool = synth.config_served_pool(seed=1005, count=count, vertex_side=vertex_side,
                                    processes=min(16, os.cpu_count() or 1))
    keep, views = [], []
    for g in pool:
        arrs = {}
        names = ("e_off", "e_pins", "v_off", "v_edges") if vertex_side else ("e_off", "e_pins")
        for name in names:
            t = torch.empty(getattr(g, name).size, dtype=torch.int32, pin_memory=True)
            t.numpy()[:] = getattr(g, name)
            arrs[name] = t
        t = torch.empty(g.m, dtype=torch.int32, pin_memory=True)
        t.numpy()[:] = g.w.view(np.int32)
        arrs["w"] = t
        keep.append(arrs)
        empty = np.zeros(0, np.int32)
        views.append(synth.Hypergraph(
            g.n, g.m, arrs["e_off"].numpy(), arrs["e_pins"].numpy(),
            arrs["v_off"].numpy() if vertex_side else empty,
            arrs["v_edges"].numpy() if vertex_side else empty,
            arrs["w"].numpy().view(np.uint32)))
    _POOL[key] = (views, keep)
    return views, keep


def served_capacity(pool_count, budget_gb, workers, inflight, duration, plain_s,
                    solo_max_kappa=0):
    """Saturation throughput of the request server on the served workload's
    pool: a closed loop keeps `inflight` requests submitted (request i draws
    pool entry i mod pool, priority seed i) for `duration` s, counting the
    completions after the first fifth; beside it the plain form, one request
    at a time on the same sequence: upload of its edge side from the pinned
    pool, hgm_match, bitmap back to the host, for `plain_s` s.  A sample of
    the served bitmaps is compared with the plain form's."""
    import numpy as np
    import torch
    import paper_2602_22976_amd as hgm
    views, _ = served_pool(pool_count, vertex_side=False)
    order = np.random.Generator(np.random.PCG64(4005)).permutation(len(views))
    req = lambda i: views[order[i % len(views)]]
    srv = hgm.Server(int(budget_gb * (1 << 30)), workers=workers,
                     opts=hgm.make_opts("auto", solo_max_kappa=solo_max_kappa),
                     edge_side_only=True)
    t_start = time.monotonic()
    nxt = 0
    live = 0
    done = []
    while nxt < inflight:
        srv.submit(req(nxt), nxt, req_id=nxt)
        nxt += 1
        live += 1
    while live > 0:
        res = srv.poll(cap=1024, timeout_s=0.05)
        for r in res:
            done.append((r, time.monotonic()))
            live -= 1
            if time.monotonic() - t_start < duration:
                srv.submit(req(nxt), nxt, req_id=nxt)
                nxt += 1
                live += 1
    info = srv.info()
    srv.close()
    t_end = max(t for _, t in done)
    t_win = t_start + 0.2 * duration
    win = [r for r, t in done if t >= t_win and r["status"] == 0]
    lat = np.array([r["t_done"] - r["t_submit"] for r in win])
    kap = sum(req(r["id"]).kappa for r in win)
    served = {r["id"]: r["bits"] for r, _ in done[:64]}

    # Plain form on the same request sequence.
    dev = "cuda:0"
    big_m = max(g.m for g in views)
    big_k = max(g.kappa for g in views)
    d_off = torch.empty(big_m + 1, dtype=torch.int32, device=dev)
    d_pins = torch.empty(big_k, dtype=torch.int32, device=dev)
    d_w = torch.empty(big_m, dtype=torch.int32, device=dev)
    d_bits = torch.empty((big_m + 31) // 32, dtype=torch.int32, device=dev)
    opts = hgm.make_opts("auto")
    wsz = max(hgm.hgm_workspace_size(hgm.DeviceHypergraph(
        g.n, g.m, d_off[:g.m + 1], d_pins[:g.kappa], d_off[:0], d_pins[:0], d_w[:g.m]).csr(),
        opts) for g in views)
    ws = torch.empty(wsz, dtype=torch.uint8, device=dev)
    host_bits = torch.empty((big_m + 31) // 32, dtype=torch.int32, pin_memory=True)
    _, keep = served_pool(pool_count, vertex_side=False)
    mismatch = 0
    n_plain = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < plain_s or n_plain < 8:
        g = req(n_plain)
        a = keep[order[n_plain % len(views)]]
        d_off[:g.m + 1].copy_(a["e_off"], non_blocking=True)
        d_pins[:g.kappa].copy_(a["e_pins"], non_blocking=True)
        d_w[:g.m].copy_(a["w"], non_blocking=True)
        dg = hgm.DeviceHypergraph(g.n, g.m, d_off[:g.m + 1], d_pins[:g.kappa], d_off[:0],
                                  d_pins[:0], d_w[:g.m])
        nw = (g.m + 31) // 32
        hgm.match(dg, n_plain, opts, workspace=ws, bits=d_bits[:max(nw, 1)], want_stats=False)
        host_bits[:nw].copy_(d_bits[:nw], non_blocking=True)
        torch.cuda.synchronize()
        if n_plain in served:
            mismatch += int(not np.array_equal(host_bits[:nw].numpy().view(np.uint32),
                                               served[n_plain]))
        n_plain += 1
    t_plain = time.perf_counter() - t0
    cap = len(win) / (t_end - t_win)
    plain = n_plain / t_plain
    return {"pool": len(views), "inflight": inflight, "workers": workers,
            "solo_max_kappa": solo_max_kappa,
            "duration_s": duration, "completed": len(done),
            "hypergraphs_per_s": cap, "incidences_per_s": kap / (t_end - t_win),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "admission_stalls": int(info["stalls"]),
            "plain_hypergraphs_per_s": plain, "plain_requests": n_plain,
            "served_over_plain": cap / plain,
            "plain_mismatches_in_sample": mismatch}


def ceilings(grid_per_cu=8):
    """Rates of the access patterns the round kernels use, each timed with HIP
    events on torch's current stream (median of 5 launches after one): the
    streaming read rate (1 GiB), random 8-byte and 1-byte gathers from
    buffers of 2 MiB (an XCD's L2 holds it), 16 MiB (best[] of the power-law
    workload) and 256 MiB (beyond the Infinity Cache), device-scope 64-bit
    atomic max at random addresses (plain and filtered by a read, as the
    scatter runs it) over 16 MiB, and on one address; per-launch time of
    back-to-back empty kernels of the round kernels' shape, on a stream and
    replayed from a captured HIP graph."""
    import ctypes
    import torch
    from paper_2602_22976_amd import build as hb
    if not os.path.exists(hb.PROBE_LIB):
        hb.build(force=True)
    lib = ctypes.CDLL(hb.PROBE_LIB)
    P = ctypes.c_void_p
    lib.hgm_probe_stream.argtypes = [P, ctypes.c_int64, P, P, ctypes.c_int]
    lib.hgm_probe_gather.argtypes = [P, ctypes.c_int64, ctypes.c_int, P, ctypes.c_int64, P, P,
                                     ctypes.c_int]
    lib.hgm_probe_atomic.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int, P,
                                     ctypes.c_int]
    dev = "cuda:0"
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    grid = cus * grid_per_cu
    stream = torch.cuda.current_stream().cuda_stream
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    count = 1 << 26
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    idx = torch.randint(0, 2 ** 31 - 1, (count,), dtype=torch.int64, device=dev,
                        generator=gen).to(torch.int32)

    def timed(launch):
        launch()
        times = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            launch()
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        times.sort()
        return times[2]

    out = {"grid": grid, "count": count}
    big = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    ms = timed(lambda: lib.hgm_probe_stream(big.data_ptr(), big.numel(), sink.data_ptr(), stream,
                                           grid))
    out["stream_read_GBps"] = big.numel() / (ms * 1e-3) / 1e9
    del big
    for mib in (2, 16, 256):
        buf = torch.ones(mib << 20, dtype=torch.uint8, device=dev)
        for eb in (8, 1):
            ms = timed(lambda: lib.hgm_probe_gather(buf.data_ptr(), buf.numel(), eb,
                                                    idx.data_ptr(), count, sink.data_ptr(),
                                                    stream, grid))
            out[f"gather{eb}_{mib}MiB_G_per_s"] = count / (ms * 1e-3) / 1e9
        del buf
    buf = torch.zeros((16 << 20) // 8, dtype=torch.int64, device=dev)
    for filt in (0, 1):
        buf.zero_()
        ms = timed(lambda: lib.hgm_probe_atomic(buf.data_ptr(), buf.numel(), idx.data_ptr(),
                                                count, filt, stream, grid))
        out[("filtered_" if filt else "") + "atomic_max8_16MiB_G_per_s"] = count / (ms * 1e-3) / 1e9
    n1 = 1 << 20
    ms = timed(lambda: lib.hgm_probe_atomic(buf.data_ptr(), 1, idx.data_ptr(), n1, 0, stream,
                                            grid))
    out["one_address_atomic_max8_G_per_s"] = n1 / (ms * 1e-3) / 1e9
    torch.cuda.synchronize()
    lib.hgm_probe_launches.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
    cnt = torch.zeros(65536, dtype=torch.int32, device=dev)
    for g_wg, n_launch in ((2048, 20), (2048, 100), (256, 100)):
        su, gu = ctypes.c_double(), ctypes.c_double()
        rc = lib.hgm_probe_launches(cnt.data_ptr(), sink.data_ptr(), g_wg, n_launch, 5,
                                    ctypes.byref(su), ctypes.byref(gu))
        if rc == 0:
            out[f"launch_us_stream_{g_wg}wg_x{n_launch}"] = su.value
            out[f"launch_us_graph_{g_wg}wg_x{n_launch}"] = gu.value
    return out


def scatter_forms(reps=5):
    """The per-vertex maximum the round kernels compute (best[v] = max key of
    v's records), timed in two forms on the same records (median of reps,
    HIP events on torch's current stream, each form checked equal to the
    other): filtered device atomics on a cleared best[] (the round kernels'
    form; the clear timed on its own) and propagation blocking (records
    binned by vertex range of 2^rb ids, then each range max-reduced in LDS and
    written whole; phases timed on their own).  Records: (pin, key) of
    round 0's scatter on the power-law workload (every pin), of its survivors
    (the pins of a seeded 40% of the edges, in edge order) and of hub-stress
    survivors (36% of the edges that avoid the hub, which round 0 matches);
    key = w << 32 | a seeded random 32-bit priority."""
    import ctypes
    import numpy as np
    import torch
    import synth
    from paper_2602_22976_amd import build as hb
    if not os.path.exists(hb.PROBE_LIB):
        hb.build(force=True)
    lib = ctypes.CDLL(hb.PROBE_LIB)
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.hgm_probe_scatter_atomic.argtypes = [P, P, I64, P, I64, I, P, I]
    lib.hgm_probe_scatter_binned.argtypes = [P, P, I64, P, I64, I, P, P, P, P, I, P, I]
    dev = "cuda:0"
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(11)

    def records(g, keep):
        sizes = np.diff(g.e_off.astype(np.int64))
        edge = np.repeat(np.arange(g.m, dtype=np.int64), sizes)
        sel = keep[edge]
        pri = rng.integers(0, 2 ** 32, size=g.m, dtype=np.uint64)
        key = (g.w.astype(np.uint64) << np.uint64(32)) | pri
        return g.e_pins[sel].astype(np.uint32), key[edge[sel]]

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def median(x):
        return sorted(x)[len(x) // 2]

    shapes = []
    g = synth.config_power_law()
    shapes.append(("power-law round-0 scatter", g.n, *records(g, np.ones(g.m, bool))))
    shapes.append(("power-law survivors (40% of edges)", g.n,
                   *records(g, rng.random(g.m) < 0.4)))
    del g
    g = synth.config_hub_stress()
    deg = np.bincount(g.e_pins, minlength=g.n)
    hub = int(deg.argmax())
    sizes = np.diff(g.e_off.astype(np.int64))
    has_hub = np.zeros(g.m, bool)
    has_hub[np.repeat(np.arange(g.m), sizes)[g.e_pins == hub]] = True
    shapes.append(("hub-stress survivors (36% of hub-free edges)", g.n,
                   *records(g, (rng.random(g.m) < 0.36) & ~has_hub)))
    del g, deg, has_hub, sizes
    out = []
    for name, n, vid_h, key_h in shapes:
        count = len(vid_h)
        vid = torch.from_numpy(vid_h.view(np.int32)).to(dev)
        key = torch.from_numpy(key_h.view(np.int64)).to(dev)
        best_a = torch.empty(n, dtype=torch.int64, device=dev)
        best_b = torch.empty(n, dtype=torch.int64, device=dev)
        row = {"records": name, "n": n, "count": count}
        grid = cus * 8
        clear_t, scat_t = [], []
        for _ in range(reps + 1):
            e0, e1, e2 = ev(), ev(), ev()
            e0.record()
            lib.hgm_probe_scatter_atomic(0, 0, 0, best_a.data_ptr(), n, 1, stream, grid)
            e1.record()
            lib.hgm_probe_scatter_atomic(vid.data_ptr(), key.data_ptr(), count,
                                         best_a.data_ptr(), n, 0, stream, grid)
            e2.record()
            e2.synchronize()
            clear_t.append(e0.elapsed_time(e1))
            scat_t.append(e1.elapsed_time(e2))
        row["atomic_clear_ms"] = median(clear_t[1:])
        row["atomic_scatter_ms"] = median(scat_t[1:])
        for rb in (12, 13, 14):
            nb = (n + (1 << rb) - 1) >> rb
            per_bin = torch.bincount((vid.to(torch.int64) & 0xFFFFFFFF) >> rb, minlength=nb)
            base = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
            base[1:] = torch.cumsum(per_bin, 0)
            cursor = torch.zeros(nb, dtype=torch.int32, device=dev)
            bin_v = torch.empty(count, dtype=torch.int16, device=dev)
            bin_key = torch.empty(count, dtype=torch.int64, device=dev)
            for producers in (cus, 2 * cus):
                w_t, r_t = [], []
                ok = True
                for _ in range(reps + 1):
                    e0, e1, e2 = ev(), ev(), ev()
                    e0.record()
                    rc1 = lib.hgm_probe_scatter_binned(
                        vid.data_ptr(), key.data_ptr(), count, best_b.data_ptr(), n, rb,
                        base.data_ptr(), cursor.data_ptr(), bin_v.data_ptr(), bin_key.data_ptr(),
                        1, stream, producers)
                    e1.record()
                    rc2 = lib.hgm_probe_scatter_binned(
                        vid.data_ptr(), key.data_ptr(), count, best_b.data_ptr(), n, rb,
                        base.data_ptr(), cursor.data_ptr(), bin_v.data_ptr(), bin_key.data_ptr(),
                        2, stream, producers)
                    e2.record()
                    e2.synchronize()
                    if rc1 or rc2:
                        ok = False
                        break
                    w_t.append(e0.elapsed_time(e1))
                    r_t.append(e1.elapsed_time(e2))
                tag = f"binned_rb{rb}_p{producers}"
                if not ok:
                    row[tag] = "rejected"
                    continue
                row[tag + "_write_ms"] = median(w_t[1:])
                row[tag + "_reduce_ms"] = median(r_t[1:])
                row[tag + "_equal"] = bool(torch.equal(best_a, best_b))
            del bin_v, bin_key
        print(json.dumps(row), flush=True)
        out.append(row)
        del vid, key, best_a, best_b
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# Summaries of rocprofv3 output (csv) for profiles/: kernel classes by name.

KERNEL_CLASS = [("k_retire", "retire"), ("k_bin_max", "retire"), ("k_test", "test"), ("k_max0_edge", "scatter"),
                ("k_scatter0", "scatter"), ("k_max0_vertex", "vertex_max"),
                ("k_vertex_max", "vertex_max"), ("k_solo", "solo"), ("k_tail", "tail"),
                ("k_prologue", "setup"), ("k_init", "setup"), ("k_batch_setup", "setup"),
                ("k_live0", "setup"), ("k_validate", "setup"), ("k_zero_words", "setup")]


def kernel_short_name(name):
    """'void hgm::(anonymous namespace)::k_test<true, 1, false>(hgm::Graph, ...)'
    -> 'k_test<true, 1, false>'."""
    s = name.replace("(anonymous namespace)::", "")
    s = s.split("(")[0].strip()
    if s.startswith("void "):
        s = s[5:]
    return s.replace("hgm::", "")


def kernel_class(name):
    short = kernel_short_name(name)
    for key, cls in KERNEL_CLASS:
        if key in short:
            return cls
    return None


def _csv_rows(root, suffix):
    import csv
    rows = []
    for dirpath, _, files in os.walk(root):
        for fn in files:
            if fn.endswith(suffix):
                with open(os.path.join(dirpath, fn), newline="") as f:
                    rows += list(csv.DictReader(f))
    return rows


def summarize_trace(root):
    """Markdown table of a --kernel-trace run: per kernel, dispatches, per
    call (hgm calls = k_prologue dispatches), total, mean, min and max
    duration in microseconds."""
    rows = _csv_rows(root, "kernel_trace.csv")
    per = {}
    for r in rows:
        name = r["Kernel_Name"]
        cls = kernel_class(name)
        if cls is None:
            continue
        short = kernel_short_name(name)
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        per.setdefault((short, cls), []).append(d)
    calls = max(1, sum(len(v) for (k, c), v in per.items() if k.startswith("k_prologue")))
    out = [f"calls (k_prologue dispatches): {calls}", "",
           "| kernel | class | dispatches | per call | total us per call | avg us | min us | max us |",
           "|---|---|---|---|---|---|---|---|"]
    for (k, c), v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| {k} | {c} | {len(v)} | {len(v) / calls:.1f} | {sum(v) / calls:.1f} | "
                   f"{sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} |")
    return "\n".join(out)


def _pmc_by_class(root, counter):
    kib, n = {}, {}
    for r in _csv_rows(root, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        cls = kernel_class(r["Kernel_Name"])
        if cls is None:
            continue
        kib[cls] = kib.get(cls, 0.0) + float(r["Counter_Value"])
        n[cls] = n.get(cls, 0) + 1
    return kib, n


def summarize_counters(root):
    """Markdown table of a rocprofv3 --pmc run (csv) with any counters: per
    kernel of the library, its dispatches and each counter summed over them."""
    rows = _csv_rows(root, "counter_collection.csv")
    per, disp, names = {}, {}, set()
    for r in rows:
        if kernel_class(r["Kernel_Name"]) is None:
            continue
        k = kernel_short_name(r["Kernel_Name"])
        c = r["Counter_Name"]
        names.add(c)
        per.setdefault(k, {}).setdefault(c, 0.0)
        per[k][c] += float(r["Counter_Value"])
        disp.setdefault(k, set()).add(r.get("Dispatch_Id", ""))
    cols = sorted(names)
    out = ["| kernel | dispatches | " + " | ".join(cols) + " |",
           "|---|---|" + "---|" * len(cols)]
    order = sorted(per, key=lambda k: -max(per[k].values()))
    for k in order:
        out.append(f"| {k} | {len(disp[k])} | " +
                   " | ".join(f"{per[k].get(c, 0.0):.3g}" for c in cols) + " |")
    return "\n".join(out)


def summarize_pmc(workload, fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, calls,
                  copy_mib=1024):
    """JSON line of calibrated HBM traffic per kernel class and per hgm call:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the same
    counters read for the copy probe's three copies of copy_mib MiB."""
    # the copy probe's three copies (dispatches whose kernel name says copy;
    # the fill of its source is left out)
    def total(root, counter):
        rows = [r for r in _csv_rows(root, "counter_collection.csv")
                if r.get("Counter_Name") == counter]
        copies = [r for r in rows if "copy" in r["Kernel_Name"].lower()]
        return sum(float(r["Counter_Value"]) for r in (copies or rows))
    copied_kib = 3 * copy_mib * 1024.0
    f_meas, w_meas = total(cal_fetch_dir, "FETCH_SIZE"), total(cal_write_dir, "WRITE_SIZE")
    ff, fw = copied_kib / f_meas, copied_kib / w_meas
    fk, fn = _pmc_by_class(fetch_dir, "FETCH_SIZE")
    wk, _ = _pmc_by_class(write_dir, "WRITE_SIZE")
    kernels = {}
    for cls in sorted(set(fk) | set(wk)):
        disp = fn.get(cls, 0)
        b = (fk.get(cls, 0.0) * ff + wk.get(cls, 0.0) * fw) * 1024.0
        kernels[cls] = {"dispatches": disp, "fetch_kib": fk.get(cls, 0.0),
                        "write_kib": wk.get(cls, 0.0), "launches_per_call": disp / calls,
                        "bytes_per_call": b / calls}
    return json.dumps({"kernel_source": kernel_source_digest(), "workload": workload,
                       "calls": calls, "copy_factor": {"fetch": ff, "write": fw,
                                                       "copy_probe_mib": copy_mib,
                                                       "fetch_kib_measured": f_meas,
                                                       "write_kib_measured": w_meas},
                       "kernels": kernels})


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def tuning_leg(reps=3):
    """Default vs autotuned schedule (hgm_tune / hgm_tune_batch, median of
    `reps` calls per candidate) on the power-law and hub-stress instances and
    a 1,024-instance sample of the batched workload."""
    import torch
    import paper_2602_22976_amd as hgm
    import synth
    out = {}
    for name, make in (("power-law", synth.config_power_law),
                       ("hub", synth.config_hub_stress)):
        dg = hgm.DeviceHypergraph.from_host(make(), "cuda:0")
        best, rep = hgm.tune(dg, 1, hgm.make_opts("auto"), reps=reps)
        out[name] = rep
        del dg
        torch.cuda.empty_cache()
    db = hgm.DeviceBatch.from_host(synth.config_batched(seed=1004, count=1024), "cuda:0")
    best, rep = hgm.tune_batch(db, hgm.make_opts("auto"), reps=reps)
    out["batched_1024"] = rep
    del db
    torch.cuda.empty_cache()
    return out


def cpu_baseline(g, seed, budget_s, sum_k, reseed=False):
    """The oracle on one host core: a child process pinned with taskset to
    the last core this process may use runs the greedy oracle (key
    construction, sort, scan; at least three runs, arithmetic mean) and the
    round simulator once.  `value` is the GPU step's live incidences (sum of
    kappa_r) over the greedy's mean time, so the ratio of the GPU value to it
    is the ratio of the times; the round simulator's figure is reported
    beside it."""
    import subprocess
    import tempfile
    import numpy as np
    core = sorted(os.sched_getaffinity(0))[-1]
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "instance.npz")
        np.savez(path, n=g.n, m=g.m, e_off=g.e_off, e_pins=g.e_pins, v_off=g.v_off,
                 v_edges=g.v_edges, w=g.w)
        cmd = ["taskset", "-c", str(core), sys.executable, "-m", "oracle.timing", path,
               str(seed), str(budget_s), "1" if reseed else "0"]
        out = subprocess.run(cmd, cwd=ROOT, check=True, capture_output=True, text=True).stdout
    d = json.loads(out.strip().splitlines()[-1])
    t = d["greedy_s"]
    return {"value": sum_k / t, "unit": "pin-incidences/s", "cores": 1, "kind": "oracle",
            "cpu": d["cpu"], "host_cpus": os.cpu_count(), "pinned_core": core,
            "allowed_cores": d["allowed_cores"],
            "simulator_value": d["sum_kappa_r"] / d["simulator_s"],
            "sample": (f"oracle greedy (key construction, sort, scan) on the full workload, one "
                       f"thread pinned by taskset to core {core}: {len(d['greedy_runs'])} runs, "
                       f"mean {t:.3f} s; value = the GPU step's sum of kappa_r ({sum_k}) over "
                       f"that time.  Oracle round simulator on the same core: "
                       f"{d['simulator_s']:.3f} s, {d['rounds']} rounds, sum kappa_r = "
                       f"{d['sum_kappa_r']} (simulator_value)")}


def cpu_multicore(g, seed, budget_s, reseed=False):
    """The OpenMP local max (baselines/) on the host's cores, full workload."""
    import baselines
    threads = max(1, min(16, os.cpu_count() or 1))
    baselines.local_max(g.n, g.m, g.e_off, g.e_pins, g.w, seed, reseed=reseed,
                        threads=threads)   # warm-up
    t0 = time.perf_counter()
    runs = 0
    while True:
        _, rounds, sum_k = baselines.local_max(g.n, g.m, g.e_off, g.e_pins, g.w, seed,
                                               reseed=reseed, threads=threads)
        runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    t = (time.perf_counter() - t0) / runs
    return {"value": sum_k / t, "unit": "pin-incidences/s", "cores": threads,
            "kind": "openmp local max", "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": (f"multicore CPU local max ({threads} threads) on the full workload, "
                       f"{runs} run(s) of {t:.3f} s each, {rounds} rounds, sum kappa_r = {sum_k}")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="power-law", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="auto", choices=["auto", "crcw", "crew"])
    ap.add_argument("--rounds-per-sync", type=int, default=0)
    ap.add_argument("--reseed", type=int, default=0,
                    help="1: priorities drawn afresh every round (the paper's per-round noise)")
    ap.add_argument("--hub-threshold", type=int, default=0,
                    help="degree above which a vertex is split into pieces (0 = library default)")
    ap.add_argument("--cpu-baseline", type=float, default=10.0,
                    help="seconds of oracle work for the CPU baseline (0 = skip)")
    ap.add_argument("--cpu-multicore", type=float, default=3.0,
                    help="seconds of the multicore CPU local max baseline (0 = skip)")
    ap.add_argument("--batch-count", type=int, default=4096,
                    help="instances in the batched-vs-plain leg (0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="duration of the served leg (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-pool", type=int, default=1024)
    ap.add_argument("--capacity-seconds", type=float, default=10.0,
                    help="closed-loop saturation run of the server and plain form (0 = skip)")
    ap.add_argument("--capacity-inflight", type=int, default=256)
    ap.add_argument("--tune", type=int, default=1,
                    help="1: default vs autotuned schedules (power-law, hub, batched sample)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--serve-solo-max-kappa", type=int, default=0,
                    help="solo part bound of the server's waves (0 = library default, -1 = off)")
    ap.add_argument("--serve-vertex-side", type=int, default=0,
                    help="1: requests also upload the vertex side (default: edge side only)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB: only run a plain device copy (PMC calibration) and exit")
    ap.add_argument("--summarize-trace", default=None,
                    help="rocprofv3 --kernel-trace output directory (csv): print its table")
    ap.add_argument("--summarize-counters", default=None,
                    help="rocprofv3 --pmc output directory (csv, any counters): print the "
                         "per-kernel sums")
    ap.add_argument("--summarize-pmc", nargs=4, default=None,
                    metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE output directories of the "
                         "workload and of --copy-probe 1024: print the traffic summary line")
    ap.add_argument("--calls", type=int, default=0,
                    help="hgm calls in the profiled run (for --summarize-pmc)")
    ap.add_argument("--ceilings", type=int, default=0,
                    help="1: only measure the memory-system ceilings (streaming, random "
                         "gathers, atomics) and print them as one JSON line; 2: only time "
                         "the per-vertex max by atomics against propagation blocking")
    args = ap.parse_args()

    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters))
        return
    if args.summarize_pmc:
        print(summarize_pmc(args.workload, *args.summarize_pmc, calls=max(1, args.calls)))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs on one GPU; --gpus above 1 is not supported "
              "(batches of independent instances shard across GPUs without communication, "
              "see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.ceilings == 2:
        print(json.dumps({"scatter_forms": scatter_forms()}), flush=True)
        return
    if args.ceilings:
        print(json.dumps({"ceilings": ceilings()}), flush=True)
        return

    import paper_2602_22976_amd as hgm
    import synth
    from paper_2602_22976_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build(force=True)

    fn, desc = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = getattr(synth, fn)()
    gen_s = time.perf_counter() - t0
    print(f"# workload {args.workload}: n={g.n} m={g.m} kappa={g.kappa} (generated in "
          f"{gen_s:.1f} s)", file=sys.stderr, flush=True)
    seed = 1
    dev = "cuda:0"
    dg = hgm.DeviceHypergraph.from_host(g, dev)
    pairs = args.workload in GRAPH_WORKLOADS
    if pairs and args.variant == "crew":
        print("bench.py: graph workloads run the edge-centric rounds (auto or crcw)",
              file=sys.stderr)
        sys.exit(2)
    opts = hgm.make_opts(args.variant, rounds_per_sync=args.rounds_per_sync, pairs=pairs,
                         hub_threshold=args.hub_threshold, reseed=bool(args.reseed))
    ws = hgm.alloc_workspace(dg, opts)
    bits = torch.empty(max((g.m + 31) // 32, 1), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    def step(timing=False):
        return hgm.match(dg, seed, opts, workspace=ws, bits=bits, timing=timing)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Timed region: K whole steps, synchronised on both sides.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    sum_k = int(np.sum(st["live_pins"]))
    value = sum_k / t_step

    # Same steps with HIP events around every kernel (per-kernel device time).
    tot_ms = {}
    launches = {}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = []       # each of these steps ends in a synchronisation (the stats copy)
    round_ms = None    # per-round device time, summed over the steps
    for _ in range(args.steps):
        ts = time.perf_counter()
        sti = step(timing=True)
        step_ms.append((time.perf_counter() - ts) * 1e3)
        rm = np.asarray(sti["round_ms"], dtype=np.float64)
        round_ms = rm if round_ms is None else round_ms + rm
        for k, v in sti["kernel_ms"].items():
            tot_ms[k] = tot_ms.get(k, 0.0) + v
            launches[k] = launches.get(k, 0) + sti["kernel_launches"][k]
    torch.cuda.synchronize()
    t_step_events = (time.perf_counter() - t1) / args.steps

    crew_all = args.variant == "crew"
    crew0 = crew_all or launches.get("vertex_max", 0) > 0   # AUTO's round-0 form
    tail_from = (int(round(launches.get("test", 0) / args.steps))
                 if launches.get("tail", 0) > 0 else None)
    model = algorithmic_bytes(st, lambda r: crew_all or (r == 0 and crew0), g.n, pairs,
                              bool(args.reseed), tail_from)
    cand = {k: tot_ms[k] for k in model if tot_ms.get(k, 0) > 0}
    dom = max(cand, key=cand.get)
    dom_ms = tot_ms[dom] / args.steps
    dom_launch = launches[dom] / args.steps
    achieved = model[dom] / (dom_ms * 1e-3) / 1e9
    digest = kernel_source_digest()
    traffic = load_traffic(args.workload, dom, digest, dom_launch)
    # Measured traffic rate: calibrated L2-to-fabric bytes per launch over the
    # average launch time (fabric bytes include Infinity Cache hits, so this
    # bounds the DRAM rate from above).
    traffic_gbs = (traffic / (dom_ms / dom_launch * 1e-3) / 1e9
                   if traffic is not None and dom_launch else None)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "pin-incidences/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "n": g.n, "m": g.m, "kappa": g.kappa,
                   "variant": args.variant, "hub_threshold": args.hub_threshold or None,
                   "reseed": bool(args.reseed),
                   "rounds": st["rounds"],
                   "sum_kappa_r": sum_k, "matched": st["matched"]},
        "input_incidences_per_s": g.kappa / t_step,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbs": traffic_gbs,
                     "traffic_frac": traffic_gbs / HBM_PEAK_GBS if traffic_gbs else None,
                     "kernel": dom, "launches_per_step": dom_launch,
                     "ms_per_step": dom_ms, "algorithmic_bytes_per_step": model[dom],
                     "kernel_source": digest},
        "kernel_ms_per_step": {k: v / args.steps for k, v in tot_ms.items()},
        "kernel_launches_per_step": {k: v / args.steps for k, v in launches.items()},
        "ms_per_step_with_events": t_step_events * 1e3,
        "ms_per_step_median": float(np.median(step_ms)),
        "work_inflation": sum_k / max(g.kappa, 1),
        "kernel_incidences_per_s": sum_k / (sum(tot_ms.values()) / args.steps * 1e-3),
        "per_round": {"live_edges": [int(x) for x in st["live_edges"]],
                      "live_pins": [int(x) for x in st["live_pins"]],
                      "round_ms": [round(float(x), 4) for x in round_ms / args.steps],
                      "incidences_per_s": [float(k / (t * 1e-3)) if t > 0 else None
                                           for k, t in zip(st["live_pins"],
                                                           round_ms / args.steps)]},
        "batched": None,
        "served": None,
        "cpu_baseline": None,
        "cpu_multicore": None,
    }
    if args.batch_count > 0:
        result["batched"] = batched_leg(args.batch_count, max(1, min(args.steps, 5)))
    if args.serve_seconds > 0:
        result["served"] = served_leg(args.serve_rate, args.serve_seconds, args.serve_pool,
                                      args.serve_budget_gb, args.serve_workers,
                                      edge_side_only=not args.serve_vertex_side,
                                      solo_max_kappa=args.serve_solo_max_kappa)
    if args.capacity_seconds > 0:
        result["served_capacity"] = served_capacity(args.serve_pool, args.serve_budget_gb,
                                                    args.serve_workers, args.capacity_inflight,
                                                    args.capacity_seconds,
                                                    max(2.0, args.capacity_seconds / 2),
                                                    args.serve_solo_max_kappa)
    if args.tune:
        del ws
        torch.cuda.empty_cache()
        result["tuning"] = tuning_leg()
    if args.cpu_baseline > 0:
        result["cpu_baseline"] = cpu_baseline(g, seed, args.cpu_baseline, sum_k,
                                              bool(args.reseed))
    if args.cpu_multicore > 0:
        result["cpu_multicore"] = cpu_multicore(g, seed, args.cpu_multicore, bool(args.reseed))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
