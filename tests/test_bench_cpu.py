"""bench.py's host side, without a GPU: the one-GPU contract and the
algorithmic byte model of each kernel class (hand-computed from the per-unit
figures in its docstring)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402  (standard library only at import time)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


STATS = {"live_edges": [10, 4], "live_pins": [30, 12], "matched_per_round": [3, 4],
         "matched_pins": [9, 12], "rounds": 2}


def test_byte_model_offset_layout():
    out = bench.algorithmic_bytes(STATS, lambda r: False, n=100, pairs=False)
    # round 0 scatter: 8 B/edge + 12 B/pin
    assert out["scatter"] == 8 * 10 + 12 * 30
    # test, round 0: 12 B/edge, 20 B/pin (pin, best, clear), 4 B/matched edge,
    # 1 B/matched pin; round 1: 20 B/edge (id and record)
    assert out["test"] == (12 * 10 + 20 * 30 + 4 * 3 + 9) + (20 * 4 + 20 * 12 + 4 * 4 + 12)
    # retire, round 0: 8 B/edge, 5 B/pin, per survivor id 4 + record 20 +
    # weight 4, 8 B/surviving pin; round 1: 12 B/edge, no survivors
    assert out["retire"] == (8 * 10 + 5 * 30 + 28 * 4 + 8 * 12) + (12 * 4 + 5 * 12)
    assert out["vertex_max"] == 0


def test_byte_model_pair_layout_and_reseed():
    out = bench.algorithmic_bytes(STATS, lambda r: False, n=100, pairs=True)
    assert out["scatter"] == 4 * 10 + 12 * 30
    assert out["test"] == (4 * 10 + 20 * 30 + 4 * 3 + 9) + (12 * 4 + 20 * 12 + 4 * 4 + 12)
    assert out["retire"] == (5 * 30 + 24 * 4 + 8 * 12) + (4 * 4 + 5 * 12)
    # with per-round priorities the key of a survivor is rebuilt from its
    # weight in every round (4 B), not read from the record (8 B)
    three = {"live_edges": [10, 4, 2], "live_pins": [30, 12, 6], "matched_per_round": [3, 1, 2],
             "matched_pins": [9, 3, 6], "rounds": 3}
    fixed = bench.algorithmic_bytes(three, lambda r: False, n=100, pairs=False)
    redrawn = bench.algorithmic_bytes(three, lambda r: False, n=100, pairs=False, reseed=True)
    assert fixed["retire"] - redrawn["retire"] == 4 * 2   # round 1's two survivors
    assert fixed["test"] == redrawn["test"]


def test_byte_model_vertex_rounds():
    out = bench.algorithmic_bytes(STATS, lambda r: True, n=100, pairs=False)
    assert out["scatter"] == 0
    assert out["vertex_max"] == (13 * 100 + 8 * 30) + (21 * 100 + 12 * 30 + 4 * 12)
    # no clearing store in the test when the next round is vertex-centric;
    # the retire writes the dead edges' keys instead of scattering
    assert out["test"] == (12 * 10 + 12 * 30 + 4 * 3 + 9) + (20 * 4 + 12 * 12 + 4 * 4 + 12)
    assert out["retire"] == (8 * 10 + 5 * 30 + 28 * 4 + 8 * 6) + (12 * 4 + 5 * 12 + 8 * 4)


def test_byte_model_tail():
    """Rounds from tail_from on go to the tail: list gathered once (40 B per
    live edge), then per round test and retire over its compact slots."""
    three = {"live_edges": [10, 4, 2], "live_pins": [30, 12, 6], "matched_per_round": [3, 1, 2],
             "matched_pins": [9, 3, 6], "rounds": 3}
    full = bench.algorithmic_bytes(three, lambda r: False, n=100, pairs=False)
    out = bench.algorithmic_bytes(three, lambda r: False, n=100, pairs=False, tail_from=1)
    assert out["scatter"] == full["scatter"]
    # round 0's test and retire (which builds round 1's list) stay
    assert out["test"] == 12 * 10 + 20 * 30 + 4 * 3 + 9
    assert out["retire"] == 8 * 10 + 5 * 30 + 28 * 4 + 8 * 12
    r1 = (20 * 4 + 12 * 12 + 4 * 1 + 3) + (20 * 4 + 5 * 12 + 20 * 2 + 16 * 6)
    r2 = (20 * 2 + 12 * 6 + 4 * 2 + 6) + (20 * 2 + 5 * 6)
    assert out["tail"] == 40 * 4 + r1 + r2


def test_summarize_counters(tmp_path):
    """The per-kernel counter table of a rocprofv3 --pmc csv: sums per
    library kernel over its dispatches, other kernels left out."""
    import bench
    d = tmp_path / "run" / "host"
    d.mkdir(parents=True)
    rows = [("1", "void hgm::(anonymous namespace)::k_test<false, 1, false>(hgm::Graph)", "SQ_WAVES", "10"),
            ("1", "void hgm::(anonymous namespace)::k_test<false, 1, false>(hgm::Graph)", "SQ_WAIT_ANY", "7"),
            ("2", "void hgm::(anonymous namespace)::k_test<false, 1, false>(hgm::Graph)", "SQ_WAVES", "5"),
            ("3", "some_other_kernel(int)", "SQ_WAVES", "99")]
    with open(d / "run_counter_collection.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for r in rows:
            f.write(",".join(f'"{x}"' for x in r) + "\n")
    out = bench.summarize_counters(str(tmp_path)).splitlines()
    assert out[0] == "| kernel | dispatches | SQ_WAIT_ANY | SQ_WAVES |"
    assert out[2] == "| k_test<false, 1, false> | 2 | 7 | 15 |"
    assert len(out) == 3
