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
    """The frozen per-edge model: hash 20 (u64) or key bytes + 20 (strings), build 42, frontier
    2.3, peel 51 per peeled edge, assign 16, rank 2.8; resolve and update have none."""
    n, m = 1 << 20, 3 * 430_000
    L0 = 250_000
    st = dict(n=n, m=m, kind="str", key_bytes=60 * n, frontier_total=0, frontier0=0, claims=0, lists=False,
              round0_updates=False, layer0=L0, update_deletes=0, update_records=0)
    ab = bench.algorithmic_bytes
    assert ab("hash", st) == 60 * n + 8 * n + 12 * n  # bytes, offset, edge
    assert ab("hash", dict(st, kind="u64")) == 8 * n + 12 * n
    assert ab("build", st) == 42 * n
    assert ab("assign", st) == 16 * n
    assert ab("rank", st) == 2.8 * n
    assert ab("order", st) == 8 * n
    assert ab("resolve", st) == 0 and ab("update", st) == 0
    # round 0's layer is peeled by the apply launches unless the round-0 kernel deletes it
    assert ab("frontier", st) == 2.3 * n and ab("apply", st) == 51 * n
    assert ab("frontier", dict(st, lists=True)) == 2.3 * n  # claim lists alone: apply still deletes layer 0
    s2 = dict(st, lists=True, round0_updates=True)
    assert ab("frontier", s2) == 2.3 * n + 51 * L0
    assert ab("apply", s2) == 51 * (n - L0)
    # the whole build: 134 bytes per u64 edge, 194 per 60-byte string edge (no order phase)
    phases = ("hash", "build", "frontier", "apply", "resolve", "update", "assign", "rank")
    assert abs(sum(ab(p, dict(s2, kind="u64")) for p in phases) - 134.1 * n) < 1
    assert abs(sum(ab(p, s2) for p in phases) - 194.1 * n) < 1


def test_kernel_roofline_arithmetic():
    """frac = per-edge bytes x edges per launch / average launch time / 8 TB/s."""
    n, L0 = 1 << 31, 514_000_000
    st = dict(n=n, m=3 * 880_468_296, kind="str", key_bytes=60 * n, frontier_total=0, frontier0=0, claims=0,
              lists=True, round0_updates=True, layer0=L0, update_deletes=0, update_records=0)
    row = dict(ms=184.2, launches=63, alg_bytes=bench.algorithmic_bytes("apply", st))
    rf = bench.kernel_roofline("apply", row, None)
    per_launch = 51 * (n - L0) / 63
    avg_s = 184.2e-3 / 63
    assert rf["alg_bytes_per_launch"] == round(per_launch)
    assert abs(rf["launch_avg_us"] - avg_s * 1e6) < 0.01
    assert abs(rf["frac"] - per_launch / avg_s / 8e12) < 1e-4
    assert round(rf["frac"], 2) == 0.06 and rf["traffic"] is None
    # counted traffic per launch: amplification against the model's bytes
    rf = bench.kernel_roofline("apply", row, 5.7e9)
    assert abs(rf["amplification"] - 5.7e9 / per_launch) < 0.01
    assert abs(rf["traffic_frac"] - 5.7e9 / avg_s / 8e12) < 1e-4
    # assignment: 16 bytes per edge, a launch per layer
    row = dict(ms=171.0, launches=63, alg_bytes=bench.algorithmic_bytes("assign", st))
    assert round(bench.kernel_roofline("assign", row, None)["frac"], 3) == round(16 * n / 0.171 / 8e12, 3)


def test_peel_roofline_sums_the_peel_phases():
    rows = {"hash": dict(ms=63.0, alg_bytes=10), "frontier": dict(ms=37.0, alg_bytes=4e10),
            "apply": dict(ms=155.0, alg_bytes=8e10), "resolve": dict(ms=48.0, alg_bytes=0),
            "update": dict(ms=45.0, alg_bytes=0), "assign": dict(ms=170.0, alg_bytes=3e10)}
    pr = bench.peel_roofline(rows, 6.65e11, 1 << 31)
    assert pr["phases"] == ["frontier", "apply", "resolve", "update"]
    assert pr["ms"] == 285.0 and pr["alg_bytes"] == int(1.2e11)
    assert abs(pr["alg_frac"] - 1.2e11 / 0.285 / 8e12) < 1e-4
    assert abs(pr["traffic_frac"] - 6.65e11 / 0.285 / 8e12) < 1e-4
    assert abs(pr["amplification"] - 6.65e11 / 1.2e11) < 0.01
    assert bench.peel_roofline(rows, None, 1 << 31)["traffic_frac"] is None


def test_build_windows_cut_each_build_in_dispatch_order():
    seq = ["k_gen_str_bytes", "k_zero16", "k_hash_str_words", "k_part_scatter1_x3", "k_part_accum", "k_round0_updates",
           "k_part_hist2", "k_update_accum", "k_apply", "k_claims_resolve", "k_assign_round", "k_assign_round",
           "k_pack_count", "k_scan_add", "k_gen_str_len", "k_hash_str_words", "k_part_accum", "k_round0_updates",
           "k_apply", "k_assign_round", "k_pack_count", "k_hash_str_words", "k_round0_updates"]
    rows = [(i, name, float(i)) for i, name in enumerate(seq)]
    w = bench.build_windows(rows)
    assert w["builds"] == 2  # the third build never reached its assignment
    assert w["hash_build"] == ((2 + 3 + 4) + (15 + 16)) / 2
    assert w["peel"] == ((5 + 6 + 7 + 8 + 9) + (17 + 18)) / 2
    assert w["assign_rank"] == ((10 + 11 + 12 + 13) + (19 + 20)) / 2


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
