"""Host logic of the benchmark (no GPU): the row count of a schedule prefix
that the oracle's baseline rate is divided into, the traffic record's
guard against changed kernel sources, and the record's arithmetic from
counter files."""
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


def _pmc_csv(d, rows):
    os.makedirs(d)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w") as fh:
        fh.write("Dispatch_Id,Kernel_Name,Counter_Value\n")
        for i, name, v in rows:
            fh.write(f'{i},"{name}",{v}\n')


def test_traffic_record_from_counter_files(tmp_path):
    """The record's bytes: the sweep's mean KiB per dispatch after the
    skipped ones, scaled so that the 1 GiB calibration add reads as 1 GiB;
    other kernels and other tile sizes are ignored."""
    class Inst:
        name = "sbm_n500_k10"
    sweep = "void ccp::k_sweep_dataflow<double, 16, 8, false, false>(ccp::DataflowArgs, long)"
    other = "void ccp::k_sweep_dataflow<double, 32, 4, false, false>(ccp::DataflowArgs, long)"
    sparse = "void ccp::k_sweep_dataflow<double, 16, 8, true, false>(ccp::DataflowArgs, long)"
    cal = "void at::native::elementwise_kernel<CUDAFunctorOnSelf_add<double>>(int)"
    gib_kib = 1024 * 1024
    _pmc_csv(str(tmp_path / "f"), [(1, sweep, 999.0), (2, sweep, 100.0), (3, sweep, 300.0),
                                   (4, other, 7.0), (5, sparse, 9.0), (6, cal, gib_kib / 2)])
    _pmc_csv(str(tmp_path / "w"), [(1, sweep, 999.0), (2, sweep, 50.0), (3, sweep, 50.0),
                                   (4, cal, gib_kib)])
    path = bench.write_traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), Inst(), 16, "f64", 1,
                                      out_dir=str(tmp_path))
    rec = json.load(open(path))
    assert rec["dispatches"] == 2 and rec["kernel"] == "k_sweep_dataflow<double, 16, 8, false, false>"
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["traffic_bytes_per_launch"] == (200 * 2 + 50) * 1024
    assert os.path.basename(path) == "k_sweep_dataflow_sbm_n500_f64.traffic.json"
