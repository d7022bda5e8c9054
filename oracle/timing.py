"""Timing of the oracle on the host, for the benchmark's CPU baseline.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the benchmark runs
this module as a child process pinned to one core (taskset), so that the
figure is a single-core time as in the paper's one-core Greedy baseline.

    python3 -m oracle.timing <instance.npz> <seed> <budget_s> [reseed]

reads n, m, e_off, e_pins, v_off, v_edges, w from the .npz, times the greedy
oracle (key construction, sort and scan) over at least three runs and until
`budget_s` seconds have passed, then the round simulator once, and prints one
JSON line: mean and per-run seconds of each, the CPU the process ran on and
the cores it was allowed."""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import greedy, local_max


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def main(argv):
    path, seed, budget = argv[0], int(argv[1]), float(argv[2])
    reseed = len(argv) > 3 and argv[3] == "1"
    d = np.load(path)
    n, m = int(d["n"]), int(d["m"])
    runs = []
    t_end = time.perf_counter() + budget
    while len(runs) < 3 or time.perf_counter() < t_end:
        t0 = time.perf_counter()
        greedy(n, m, d["e_off"], d["e_pins"], d["w"], seed)
        runs.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    _, st = local_max(n, m, d["e_off"], d["e_pins"], d["v_off"], d["v_edges"], d["w"], seed,
                      reseed=reseed)
    t_sim = time.perf_counter() - t0
    print(json.dumps({"greedy_s": float(np.mean(runs)), "greedy_runs": runs,
                      "simulator_s": t_sim, "rounds": st["rounds"],
                      "sum_kappa_r": int(np.sum(st["live_pins"])),
                      "cpu": cpu_model(), "allowed_cores": sorted(os.sched_getaffinity(0))}))


if __name__ == "__main__":
    main(sys.argv[1:])
