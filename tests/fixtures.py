"""Small hand-built instances and the golden-file reader shared by the tests."""
import glob
import os

import numpy as np

from synth import from_edge_lists

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(path):
    """Parse a fixture: `n`, `seed`, `edge w p...` lines and `expect key v...`."""
    n = seed = None
    edges, ws, expect = [], [], {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "n":
                n = int(tok[1])
            elif tok[0] == "seed":
                seed = int(tok[1])
            elif tok[0] == "edge":
                ws.append(int(tok[1]))
                edges.append([int(x) for x in tok[2:]])
            elif tok[0] == "expect":
                expect[tok[1]] = [int(x) for x in tok[2:]]
    return from_edge_lists(n, edges, ws), seed, expect


def golden_files(prefix=""):
    return sorted(glob.glob(os.path.join(GOLDEN, prefix + "*.txt")))


def path_graph(m, seed=1):
    """Path v0 - v1 - ... - vm; edge i = {i, i+1} with weight i+1."""
    return from_edge_lists(m + 1, [[i, i + 1] for i in range(m)], np.arange(1, m + 1))


def star(k, seed=1, wmax=50):
    """k edges {0, i} sharing centre 0, random weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return from_edge_lists(k + 1, [[0, i + 1] for i in range(k)],
                           rng.integers(1, wmax + 1, size=k))


def disjoint(k, size=3, seed=1):
    """k pairwise disjoint edges of `size` pins."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return from_edge_lists(k * size, [list(range(i * size, (i + 1) * size)) for i in range(k)],
                           rng.integers(1, 1000, size=k))
