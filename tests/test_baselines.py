"""The multicore CPU baseline (OpenMP local max) against the oracle: same
bitmap, round count and summed live pins, fixed and per-round orders."""
import numpy as np
import pytest

import baselines
import oracle
import synth


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_cpu_local_max_equals_oracle(threads):
    for case in range(6):
        g = synth.random_instance(900 + case, 400, 1500, 0, 7, 0, 6, 0.03)
        for reseed in (False, True):
            exp, st = oracle.local_max(g.n, g.m, g.e_off, g.e_pins, g.v_off, g.v_edges, g.w,
                                       case, reseed=reseed)
            got, rounds, sum_k = baselines.local_max(g.n, g.m, g.e_off, g.e_pins, g.w, case,
                                                     reseed=reseed, threads=threads)
            assert np.array_equal(got, exp)
            assert rounds == st["rounds"] and sum_k == int(st["live_pins"].sum())


def test_cpu_local_max_graph_and_empty():
    g = synth.config_rgg(seed=3, n=3000)
    exp, _, _ = oracle.greedy(g.n, g.m, g.e_off, g.e_pins, g.w, 2)
    got, _, _ = baselines.local_max(g.n, g.m, g.e_off, g.e_pins, g.w, 2, threads=4)
    assert np.array_equal(got, exp)
    e = synth.from_edge_lists(3, [], [])
    got, rounds, sum_k = baselines.local_max(e.n, e.m, e.e_off, e.e_pins, e.w, 1)
    assert got.size == 0 and rounds == 0 and sum_k == 0
