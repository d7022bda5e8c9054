"""Maximum sizes: kappa just below 2^31, the interface's limit for 32-bit
offsets and ids, on the GPU.

A random instance of that size is too slow to generate and to check against
the oracle, so the input is K vertex-disjoint copies of a small instance G0
whose edges have distinct weights.  Distinct weights decide every comparison
before the hash does, so each copy is matched exactly as G0 alone: the
expected bitmap is G0's greedy bitmap (512 edges, a whole number of words)
repeated K times, the round count is G0's, and every per-round count is K
times G0's.  The oracle computes G0's result; the copies make the sizes.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

M0, N0 = 512, 1024


@pytest.fixture(scope="module")
def hgm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_22976_amd as lib
    lib.load()
    return lib


def _g0():
    g = synth.random_instance(77, N0, M0, 2, 14, 1, 1)
    rng = np.random.Generator(np.random.PCG64(78))
    g.w[:] = (rng.permutation(M0) + 1) * 1000   # distinct weights
    return g


def _tile_offsets(off0, count, step):
    """Offsets of `count` consecutive copies of a CSR offset array (count *
    step < 2^31, so 32-bit arithmetic is exact)."""
    k = off0.size - 1
    out = np.empty(count * k + 1, dtype=np.int32)
    body = out[:-1].reshape(count, k)
    body[:] = off0[None, :-1]
    body += (np.arange(count, dtype=np.int32) * np.int32(step))[:, None]
    out[-1] = count * step
    return out


def _tile_ids(ids0, count, step):
    out = np.empty((count, ids0.size), dtype=np.int32)
    out[:] = ids0[None, :]
    out += (np.arange(count, dtype=np.int32) * np.int32(step))[:, None]
    return out.reshape(-1)


def _device_tiled(hgm, g0, K, vertex_side):
    import torch
    e_off = _tile_offsets(g0.e_off, K, g0.kappa)
    e_pins = _tile_ids(g0.e_pins, K, N0)
    w = np.tile(g0.w, K)
    dev = "cuda:0"
    t = lambda a: torch.from_numpy(a).to(dev)
    empty = torch.empty(0, dtype=torch.int32, device=dev)
    if vertex_side:
        v_off, v_edges = t(_tile_offsets(g0.v_off, K, g0.kappa)), t(_tile_ids(g0.v_edges, K, M0))
    else:
        v_off, v_edges = empty, empty
    dg = hgm.DeviceHypergraph(K * N0, K * M0, t(e_off), t(e_pins), v_off, v_edges,
                              t(w.view(np.int32)))
    del e_off, e_pins, w
    return dg


def _expect_g0(g0, seed):
    bits, cnt, wt = oracle.greedy(g0.n, g0.m, g0.e_off, g0.e_pins, g0.w, seed)
    lb, st = oracle.local_max(g0.n, g0.m, g0.e_off, g0.e_pins, g0.v_off, g0.v_edges, g0.w, seed)
    assert np.array_equal(bits, lb)
    # another seed gives the same result: the weights alone decide
    assert np.array_equal(bits, oracle.greedy(g0.n, g0.m, g0.e_off, g0.e_pins, g0.w, seed + 1)[0])
    return bits, cnt, wt, st


def _check_tiled(hgm, g0, K, variant, vertex_side):
    import torch
    seed = 5
    bits0, cnt0, wt0, st0 = _expect_g0(g0, seed)
    print(f"tiled K={K} kappa={K * g0.kappa} variant={variant} vertex_side={vertex_side}",
          flush=True)
    dg = _device_tiled(hgm, g0, K, vertex_side)
    assert dg.kappa == K * g0.kappa and dg.kappa < 2 ** 31
    bits, st = hgm.match(dg, seed, hgm.make_opts(variant))
    torch.cuda.synchronize()
    got = bits.cpu().numpy().view(np.uint32)
    assert got.size == K * (M0 // 32)
    assert np.array_equal(got.reshape(K, M0 // 32), np.broadcast_to(bits0, (K, M0 // 32)))
    assert st["matched"] == K * cnt0 and st["weight"] == K * wt0
    assert st["rounds"] == st0["rounds"]
    assert np.array_equal(st["live_edges"], K * st0["live_edges"])
    assert np.array_equal(st["live_pins"], K * st0["live_pins"])


def test_kappa_near_2_31_edge_form(hgm):
    g0 = _g0()
    K = (2 ** 31 - 1) // g0.kappa
    _check_tiled(hgm, g0, K, "crcw", vertex_side=False)


def test_kappa_2_30_auto_with_vertex_side(hgm):
    g0 = _g0()
    K = (2 ** 30) // g0.kappa
    _check_tiled(hgm, g0, K, "auto", vertex_side=True)
