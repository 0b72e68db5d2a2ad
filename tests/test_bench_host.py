"""Host-side logic of bench.py (CPU only): the one-GPU contract, the algorithmic-byte model
of the priced phases, the counters' staleness guard, the whole-build traffic sum, the L2
hit-rate summary and the placement probe's rule."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_algorithmic_bytes_per_unit():
    n, m = 1 << 20, 3 * 430_000
    st = dict(n=n, m=m, kind="str", key_bytes=60 * n, frontier_total=0, frontier0=0, claims=0, lists=False,
              update_deletes=0, update_records=0)
    assert bench.algorithmic_bytes("assign", st) == 15 * n  # slot, two code reads, one code write
    assert bench.algorithmic_bytes("hash", st) == 60 * n + 8 * n + 12 * n  # bytes, offset, edge
    assert bench.algorithmic_bytes("hash", dict(st, kind="u64")) == 8 * n + 12 * n
    assert bench.algorithmic_bytes("build", st) == 12 * n + 8 * m


def test_counters_are_ignored_when_stale_or_missing():
    assert bench.counters_traffic("no_such_workload", "assign") is None
    assert bench.counters_traffic("mwhc_str_n2^31_mean60B_gamma1.23", "no_such_phase") is None
    d1, d2 = bench.sources_digest("assign"), bench.sources_digest("assign")
    assert d1 == d2 and len(d1) == 16
    assert bench.sources_digest("assign") != bench.sources_digest("hash")


def test_placement_probe_rule():
    def run(seq, requested=2):
        tries, it = [], iter(seq)
        tries.append(next(it))
        while bench.need_another_allocation(tries, requested):
            tries.append(next(it))
        return tries

    assert run([240, 280, 240, 280]) == [240, 280, 240]  # alternating layouts: back to the fast one
    assert run([280, 240, 280]) == [280, 240]
    assert run([286, 279, 286, 279]) == [286, 279]  # every layout slow: stop within 2 % of the best
    assert run([279, 286, 279, 286]) == [279, 286, 279]
    assert run([300, 300, 300, 300, 300], requested=4) == [300] * 4
    assert run([250, 300, 300, 300, 300]) == [250, 300, 300, 300]  # at most two beyond the request


def test_step_traffic_sums_every_build_kernel(monkeypatch):
    import json

    assert bench.counters_step_traffic("no_such_workload") is None
    w = "mwhc_str_n2^31_mean60B_gamma1.23"
    with open(bench.COUNTERS_FILE.format(workload=w.replace("^", ""))) as fh:
        doc = json.load(fh)
    monkeypatch.setattr(bench, "sources_digest", lambda p: doc["phases"][p]["sources_digest"])
    total = bench.counters_step_traffic(w)
    build = [v for k, v in doc["kernels"].items() if not k.startswith("k_gen_")]
    assert total == sum(v["fetch_bytes"] + v["write_bytes"] for v in build)
    # the phases' kernels are a part of the build's, the generators none of it
    assert total > sum(v["fetch_bytes"] + v["write_bytes"] for v in doc["phases"].values())
    assert total < sum(v["fetch_bytes"] + v["write_bytes"] for v in doc["kernels"].values())
    monkeypatch.setattr(bench, "sources_digest", lambda p: "0" * 16)  # any kernel source changed
    assert bench.counters_step_traffic(w) is None


def test_l2_summary_sums_dispatches_and_rates(tmp_path):
    d = tmp_path / "pmc" / "sub"
    d.mkdir(parents=True)
    head = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    rows = ["1,\"mphx::k_assign_round(uint3 const*)\",TCC_HIT_sum,1000000", "1,\"mphx::k_assign_round(uint3 const*)\",TCC_MISS_sum,3000000",
            "2,\"mphx::k_assign_round(uint3 const*)\",TCC_HIT_sum,1000000", "2,\"mphx::k_assign_round(uint3 const*)\",TCC_MISS_sum,3000000",
            "3,\"void mphx::k_apply<(mphx::ApplyMode)1>(int)\",TCC_HIT_sum,9000000",
            "3,\"void mphx::k_apply<(mphx::ApplyMode)1>(int)\",TCC_MISS_sum,1000000"]
    (d / "p_counter_collection.csv").write_text(head + "\n".join(rows) + "\n")
    out = tmp_path / "l2.txt"
    assert bench.summarize_l2(str(tmp_path / "pmc"), str(out), "t", "cmd") == 0
    table = {ln.split()[0]: ln.split() for ln in out.read_text().splitlines() if ln.startswith("k_")}
    assert table["k_assign_round"][1:] == ["2", "2.0", "6.0", "0.250"]
    assert table["k_apply"][1:] == ["1", "9.0", "1.0", "0.900"]
