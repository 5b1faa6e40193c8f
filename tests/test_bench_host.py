"""Host logic of the benchmark (no GPU): the row count of a schedule prefix
that the oracle's baseline rate is divided into, and the traffic record's
guard against changed kernel sources."""
import json
import os
import sys
from math import comb

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def brute_prefix_rows(n, b, rounds):
    """Metric rows of the first `rounds` rounds, by listing the triplets of
    every tile (P, Q) of those rounds (Fig. 2's block anti-diagonals)."""
    nb = -(-n // b)
    rows = 0
    for r in range(rounds):
        s = nb - 1 - r if r < nb else r
        for P in range(s // 2 + 1):
            Q = s - P
            if Q >= nb:
                continue
            for i in range(P * b, min(n, P * b + b)):
                for k in range(Q * b, min(n, Q * b + b)):
                    rows += 3 * sum(1 for j in range(i + 1, k) if P * b <= j < min(n, Q * b + b))
    return rows


@pytest.mark.parametrize("n,b", [(10, 3), (33, 8), (64, 16), (50, 24), (41, 32)])
def test_prefix_rows(n, b):
    nb = -(-n // b)
    assert bench.prefix_rows(n, b, 2 * nb - 1) == 3 * comb(n, 3)
    for rounds in (1, 2, 3, nb, nb + 1):
        assert bench.prefix_rows(n, b, rounds) == brute_prefix_rows(n, b, rounds)


def test_traffic_record_needs_the_recorded_sources():
    class Inst:
        name = "chunglu_n4000_b2.2"
    path = os.path.join(ROOT, "profiles", "k_sweep_dataflow_chunglu_n4000_f64.traffic.json")
    rec = json.load(open(path))
    got = bench.recorded_traffic("k_sweep_dataflow", Inst(), rec["b"], rec["prec"])
    # equal to the record while the kernel sources hash to it, else None
    assert got in (None, rec["traffic_bytes_per_launch"])
    assert bench.recorded_traffic("k_sweep_dataflow", Inst(), rec["b"] + 1, rec["prec"]) is None
