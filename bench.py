#!/usr/bin/env python3
"""MWHC minimal-perfect-hash build throughput on one MI355X.

One step = one whole build over device-resident synthetic keys: hash the keys to a tripartite
3-hypergraph, peel it in synchronous rounds, assign g by backward substitution along the
layers in reverse round order, and build the rank table (retries included when a 2-core
remains).  The reported value is keys (= hypergraph edges) per second.

Default workload: 2^31 byte-string keys (printable ASCII, log-normal lengths with mean 60 B,
clamped to 8..512 B, distinct by construction), gamma = 123/100, generated on the device
before timing.  --config c1 / c2 select 10^6 / 2^27 u64 keys instead.

Prints one JSON line (rank 0).  Per-kernel times come from HIP events the library records on
the build's stream (option "timing"); the roofline object uses the algorithmic bytes of the
dominant kernel (accounting below) divided by its measured time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak

CONFIGS = {
    "c1": dict(kind="u64", n=1_000_000, workload="mwhc_u64_n1e6_gamma1.23"),
    "c2": dict(kind="u64", n=1 << 27, workload="mwhc_u64_n2^27_gamma1.23"),
    "c3": dict(kind="str", n=1 << 31, workload="mwhc_str_n2^31_mean60B_gamma1.23"),
}
BATCH_WORKLOAD = "mwhc_batched_65536_buckets_loguniform_100_1e6_u64_gamma1.23"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu() -> dict:
    """The host CPU the oracle ran on: model name, logical CPUs, and those this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return dict(cpu_model=model, nproc=os.cpu_count(), cpus_usable=usable)


# Algorithmic bytes per edge of each step of the path, frozen before measuring: every logical
# element counted once per required access at its element size, never at cache-line size.
#   hash    u64: key 8 + edge 12; strings: the key bytes + an 8-byte offset + edge 12
#   build   edge 12 read + three 5-byte (degree, label) records read and written (3 x 10)
#   frontier  degrees read (1.23 per edge) + first frontier written (about 1.05 per edge)
#   peel    per peeled edge: label 4, claim 2, edge 12, two 10-byte record read-modify-writes
#           20, hinge degree 1, round 4, frontier push and pop 8
#   order   round read 4 + order written 4 (the generic peel only)
#   assign  edge 12, hinge 1, two value reads and one value write of 1 byte each
#   rank    codes and used flags read 2.5, packed codes and samples written 0.3
PER_EDGE = dict(hash_u64=20.0, hash_str_fixed=20.0, build=42.0, frontier=2.3, peel=51.0, order=8.0,
                assign=16.0, rank=2.8)


def round0_deletes_in_frontier(st: dict) -> bool:
    """True when round 0's deletes run inside the round-0 kernel (claim lists with update
    lists): its layer is then peeled under the frontier timer, not by the apply launches."""
    return bool(st.get("lists", False) and st.get("round0_updates", False))


def algorithmic_bytes(phase: str, st: dict) -> float:
    """Bytes a phase must move at least once per build, from the per-edge model above.

    Each peeled edge's 51 bytes go to the kernel that deletes it: round 0's layer to the
    round-0 kernel (frontier timer) when that kernel deletes it, every other layer to the
    apply launches.  The claim resolution and the update-list accumulation are this
    implementation's own traffic and have no bytes of their own in the model.
    """
    n = st["n"]
    L0 = st.get("layer0", 0)
    if phase == "hash":
        if st["kind"] == "u64":
            return PER_EDGE["hash_u64"] * n
        return st["key_bytes"] + PER_EDGE["hash_str_fixed"] * n
    if phase == "build":
        return PER_EDGE["build"] * n
    if phase == "frontier":
        return PER_EDGE["frontier"] * n + (PER_EDGE["peel"] * L0 if round0_deletes_in_frontier(st) else 0.0)
    if phase == "apply":
        return PER_EDGE["peel"] * (n - L0 if round0_deletes_in_frontier(st) else n)
    if phase == "order":
        return PER_EDGE["order"] * n
    if phase == "assign":
        return PER_EDGE["assign"] * n
    if phase == "rank":
        return PER_EDGE["rank"] * n
    return 0.0


PEEL_PHASES = ("frontier", "apply", "resolve", "update")


def peel_roofline(phase_rows: dict, peel_traffic, n: int) -> dict:
    """The peel alone (round 0 through the last round: frontier, apply, resolve and update
    phases) against the HBM peak: its model bytes and, when counters are current, its counted
    HBM bytes per build, both over the summed kernel time of those phases."""
    rows = [phase_rows[p] for p in PEEL_PHASES if p in phase_rows]
    ms = sum(r["ms"] for r in rows)
    alg = sum(r["alg_bytes"] for r in rows)
    out = dict(phases=[p for p in PEEL_PHASES if p in phase_rows], ms=round(ms, 3), alg_bytes=int(alg),
               alg_GBps=None, alg_frac=None, traffic=None, traffic_GBps=None, traffic_frac=None,
               amplification=None, peak=HBM_PEAK_GBS, unit="GB/s",
               edges_per_s=round(n / (ms / 1e3), 1) if ms > 0 else None)
    if ms <= 0:
        return out
    a = alg / (ms / 1e3) / 1e9
    out.update(alg_GBps=round(a, 1), alg_frac=round(a / HBM_PEAK_GBS, 4))
    if peel_traffic is not None:
        t = peel_traffic / (ms / 1e3) / 1e9
        out.update(traffic=round(peel_traffic), traffic_GBps=round(t, 1), traffic_frac=round(t / HBM_PEAK_GBS, 4),
                   amplification=round(peel_traffic / alg, 2) if alg else None)
    return out


def kernel_roofline(phase: str, row: dict, traffic_per_launch) -> dict:
    """The roofline object of one phase: model bytes per launch over the average launch time
    (HIP events on the build's stream), against the HBM peak; `traffic` is the counted HBM
    bytes per launch when the counters are current."""
    per_launch = row["alg_bytes"] / row["launches"]
    avg_s = row["ms"] / 1e3 / row["launches"]
    ach = per_launch / avg_s / 1e9
    out = dict(bound="hbm", kernel=phase, achieved=round(ach, 2), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(ach / HBM_PEAK_GBS, 4),
               traffic=None if traffic_per_launch is None else round(traffic_per_launch),
               alg_bytes_per_launch=round(per_launch), launch_avg_us=round(avg_s * 1e6, 2),
               launches=row["launches"])
    if traffic_per_launch is not None:
        out["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        out["traffic_GBps"] = round(traffic_per_launch / avg_s / 1e9, 1)
        out["traffic_frac"] = round(traffic_per_launch / avg_s / 1e9 / HBM_PEAK_GBS, 4)
        out["amplification"] = round(traffic_per_launch / per_launch, 2) if per_launch else None
    return out


# Phases, the kernels each is made of, and the sources those kernels are compiled from: HBM
# counters taken on a kernel are reused only while its sources are unchanged.
PHASE_KERNELS = {
    "hash": ("k_hash_str_words", "k_hash_u64_tiles"),
    "build": ("k_part_accum",),
    "frontier": ("k_round0",),
    "apply": ("k_apply",),
    "resolve": ("k_claims_resolve",),
    "update": ("k_update_accum",),
    "assign": ("k_assign_round",),
}
PHASE_SOURCES = {
    "hash": ("keys.hip",),
    "build": ("part.hip", "scan.hip"),
    "frontier": ("peel.hip", "part.hip", "scan.hip"),
    "apply": ("peel.hip",),
    "resolve": ("part.hip", "scan.hip"),
    "update": ("part.hip", "scan.hip"),
    "assign": ("solve.hip",),
}
COUNTERS_FILE = os.path.join(ROOT, "profiles", "hbm_counters_{workload}.json")


def sources_digest(phase: str) -> str:
    import hashlib

    csrc = os.path.join(ROOT, "paper_1312_0526_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(PHASE_SOURCES[phase] + ("common.h", "launch.h")):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def need_another_allocation(tries: list, requested: int) -> bool:
    """Placement probe: allocate again until `requested` allocations were probed, then at most
    two more while the last probe is more than 2 % slower than the best seen."""
    if len(tries) < requested:
        return True
    if len(tries) >= requested + 2:
        return False
    return tries[-1] > 1.02 * min(tries)


def counters_traffic(workload: str, phase: str):
    """HBM bytes per launch of a phase from the committed counter summary, or None when there
    is none or the phase's kernel sources changed since it was taken."""
    path = COUNTERS_FILE.format(workload=workload.replace("^", ""))
    if not os.path.exists(path) or phase not in PHASE_SOURCES:
        return None
    with open(path) as fh:
        doc = json.load(fh)
    row = doc.get("phases", {}).get(phase)
    if not row or row.get("sources_digest") != sources_digest(phase) or not row.get("launches"):
        return None
    return (row["fetch_bytes"] + row["write_bytes"]) / row["launches"]


def counters_step_traffic(workload: str):
    """HBM bytes of one whole build (every kernel of the counted run except the input
    generators, which run before the timed region), or None when there is no summary or any
    phase's kernel sources changed since it was taken."""
    path = COUNTERS_FILE.format(workload=workload.replace("^", ""))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        doc = json.load(fh)
    phases = doc.get("phases", {})
    if set(phases) != set(PHASE_SOURCES) or any(phases[p].get("sources_digest") != sources_digest(p)
                                                for p in phases):
        return None
    return sum(v["fetch_bytes"] + v["write_bytes"] for k, v in doc.get("kernels", {}).items()
               if not k.startswith("k_gen_"))


def summarize_counters(fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str,
                       workload: str, command: str) -> int:
    """Writes profiles/hbm_counters_<workload>.{json,txt} from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE) of one build and two of the ceilings leg (copy calibration)."""
    import csv
    import glob

    def per_kernel(d):
        out = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
                name = name.split("(")[0].split("<")[0].split("::")[-1]
                cur = out.setdefault(name, [0.0, 0])
                cur[0] += float(r["Counter_Value"]) * 1024.0  # KiB -> bytes
                cur[1] += 1
        return out

    fk, wk = per_kernel(fetch_dir), per_kernel(write_dir)
    cf, cw = per_kernel(copy_fetch_dir), per_kernel(copy_write_dir)
    fw, ww = build_windows(dispatch_rows(fetch_dir)), build_windows(dispatch_rows(write_dir))
    copy_bytes = float(4 << 30)  # the ceilings leg copies 4 GiB: reads and writes that much
    f_scale = copy_bytes / (cf["k_copy"][0] / cf["k_copy"][1])
    w_scale = copy_bytes / (cw["k_copy"][0] / cw["k_copy"][1])
    doc = dict(workload=workload, command=command,
               calibration=dict(kernel="k_copy", bytes=copy_bytes, fetch_per_dispatch=cf["k_copy"][0] / cf["k_copy"][1],
                                write_per_dispatch=cw["k_copy"][0] / cw["k_copy"][1], fetch_scale=f_scale,
                                write_scale=w_scale),
               phases={}, kernels={})
    for k in sorted(set(fk) | set(wk)):
        doc["kernels"][k] = dict(dispatches=fk.get(k, [0, 0])[1], fetch_bytes=fk.get(k, [0, 0])[0] * f_scale,
                                 write_bytes=wk.get(k, [0, 0])[0] * w_scale)
    # the library times hash, build and frontier as one span per build, the rounds per launch
    builds = doc["kernels"].get("k_round0", {}).get("dispatches", 1)
    for ph, prefixes in PHASE_KERNELS.items():
        ks = [k for k in doc["kernels"] if any(k.startswith(p) for p in prefixes)]
        if not ks:
            continue
        per_launch = ph in ("apply", "assign")
        doc["phases"][ph] = dict(kernels=ks, sources_digest=sources_digest(ph),
                                 launches=sum(doc["kernels"][k]["dispatches"] for k in ks) if per_launch else builds,
                                 fetch_bytes=sum(doc["kernels"][k]["fetch_bytes"] for k in ks),
                                 write_bytes=sum(doc["kernels"][k]["write_bytes"] for k in ks))
    # the same build cut in dispatch order: everything between the round-0 kernel and the
    # first assignment launch is the peel, whichever kernels it is made of
    if fw["builds"] and fw["builds"] == ww["builds"]:
        doc["windows"] = dict(builds=fw["builds"], sources_digest={p: sources_digest(p) for p in PEEL_PHASES},
                              **{w: dict(fetch_bytes=fw[w] * f_scale, write_bytes=ww[w] * w_scale)
                                 for w in WINDOWS})
    path = COUNTERS_FILE.format(workload=workload.replace("^", ""))
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)
    lines = [f"# HBM traffic counters: {workload}", "", f"command: {command}", "",
             f"Calibration: the ceilings leg's 4 GiB copy (k_copy) reads FETCH_SIZE = "
             f"{doc['calibration']['fetch_per_dispatch'] / 2**30:.3f} GiB and WRITE_SIZE = "
             f"{doc['calibration']['write_per_dispatch'] / 2**30:.3f} GiB per dispatch, so fetch figures are "
             f"scaled by {f_scale:.3f} and write figures by {w_scale:.3f}.", "",
             f"{'kernel':28s} {'disp':>5s} {'fetch_GB':>10s} {'write_GB':>10s}"]
    for k, v in sorted(doc["kernels"].items(), key=lambda kv: -(kv[1]["fetch_bytes"] + kv[1]["write_bytes"])):
        if v["fetch_bytes"] + v["write_bytes"] < 1e8:
            continue
        lines.append(f"{k:28s} {v['dispatches']:5d} {v['fetch_bytes'] / 1e9:10.2f} {v['write_bytes'] / 1e9:10.2f}")
    lines += ["", "Per phase (the kernels bench.py's phase timers cover), bytes summed over dispatches:", ""]
    for ph, v in doc["phases"].items():
        lines.append(f"{ph:10s} launches {v['launches']:4d}  fetch {v['fetch_bytes'] / 1e9:9.2f} GB  "
                     f"write {v['write_bytes'] / 1e9:9.2f} GB  sources {v['sources_digest']}")
    if "windows" in doc:
        lines += ["", f"Per build in dispatch order (mean over {doc['windows']['builds']} builds): hash and record "
                  "build up to the round-0 kernel, the peel from it up to the first assignment launch, then "
                  "assignment and rank:", ""]
        for w in WINDOWS:
            v = doc["windows"][w]
            lines.append(f"{w:12s} fetch {v['fetch_bytes'] / 1e9:9.2f} GB  write {v['write_bytes'] / 1e9:9.2f} GB")
    with open(path[:-5] + ".txt", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


WINDOWS = ("hash_build", "peel", "assign_rank")


def dispatch_rows(d: str) -> list:
    """(dispatch id, kernel name, counter value in bytes) of a rocprofv3 --pmc run, in
    dispatch order."""
    import csv
    import glob

    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
            name = name.split("(")[0].split("<")[0].split("::")[-1]
            rows.append((int(r["Dispatch_Id"]), name, float(r["Counter_Value"]) * 1024.0))
    rows.sort()
    return rows


def build_windows(rows: list) -> dict:
    """Counter bytes of each build's three windows, averaged over the builds in the run: a
    build starts at its hashing kernel; the peel window opens at the round-0 kernel and closes
    at the first assignment launch.  Kernels outside any build (input generators, probes) and
    incomplete builds are left out."""
    sums = {w: 0.0 for w in WINDOWS}
    builds, cur, state = 0, None, None
    for _, name, b in rows:
        if name.startswith("k_hash_"):
            if cur is not None and state == "assign_rank":
                builds += 1
                for w in WINDOWS:
                    sums[w] += cur[w]
            cur, state = {w: 0.0 for w in WINDOWS}, "hash_build"
        elif cur is None:
            continue
        elif name.startswith("k_round0") and state == "hash_build":
            state = "peel"
        elif name.startswith("k_assign_round") and state == "peel":
            state = "assign_rank"
        elif name.startswith("k_gen_") or name.startswith("k_copy") or name.startswith("k_probe"):
            continue
        cur[state] += b
    if cur is not None and state == "assign_rank":
        builds += 1
        for w in WINDOWS:
            sums[w] += cur[w]
    return dict(builds=builds, **{w: (sums[w] / builds if builds else 0.0) for w in WINDOWS})


def counters_peel_traffic(workload: str):
    """Counted HBM bytes of one build's peel window, or None when there is no summary or a
    peel phase's kernel sources changed since it was taken."""
    path = COUNTERS_FILE.format(workload=workload.replace("^", ""))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        doc = json.load(fh)
    w = doc.get("windows")
    if not w or any(w["sources_digest"].get(p) != sources_digest(p) for p in PEEL_PHASES):
        return None
    return w["peel"]["fetch_bytes"] + w["peel"]["write_bytes"]


def summarize_l2(pmc_dir: str, out_path: str, title: str, command: str) -> int:
    """Writes a per-kernel table of a rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum run: L2
    requests that hit and missed, summed over dispatches, and the hit rate."""
    import csv
    import glob

    acc = {}
    for f in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
            name = name.split("(")[0].split("<")[0].split("::")[-1]
            row = acc.setdefault(name, {"dispatches": set(), "TCC_HIT_sum": 0.0, "TCC_MISS_sum": 0.0})
            row["dispatches"].add(r["Dispatch_Id"])
            if r["Counter_Name"] in ("TCC_HIT_sum", "TCC_MISS_sum"):
                row[r["Counter_Name"]] += float(r["Counter_Value"])
    lines = [f"# {title}", "", f"command: {command}", "",
             "L2 (TCC) requests summed over each kernel's dispatches; hit rate = hits / (hits + misses).", "",
             f"{'kernel':28s} {'disp':>5s} {'hits_M':>10s} {'misses_M':>10s} {'hit_rate':>9s}"]
    for k, v in sorted(acc.items(), key=lambda kv: -(kv[1]["TCC_HIT_sum"] + kv[1]["TCC_MISS_sum"])):
        tot = v["TCC_HIT_sum"] + v["TCC_MISS_sum"]
        if tot < 1e6:
            continue
        lines.append(f"{k:28s} {len(v['dispatches']):5d} {v['TCC_HIT_sum'] / 1e6:10.1f} {v['TCC_MISS_sum'] / 1e6:10.1f} "
                     f"{v['TCC_HIT_sum'] / tot:9.3f}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


def summarize_kernel_stats(csv_path: str, out_path: str, title: str, command: str) -> int:
    """Writes a text table of a rocprofv3 --stats kernel_stats.csv."""
    import csv

    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# {title}", "", f"command: {command}", "",
             f"{'kernel':36s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>11s} {'pct':>6s}"]
    modes = {"(mphx::ApplyMode)0": "atomic", "(mphx::ApplyMode)1": "claim list", "(mphx::ApplyMode)2": "update list"}
    for r in rows:
        name = r["Name"].replace("(anonymous namespace)::", "").replace("void ", "")
        for k, v in modes.items():
            name = name.replace(k, v)
        depth = 0
        for j, ch in enumerate(name):  # drop the parameter list: the first '(' outside <...>
            depth += ch == "<"
            depth -= ch == ">"
            if ch == "(" and depth == 0:
                name = name[:j]
                break
        name = name.replace("mphx::", "").replace("HIP_vector_type<unsigned int, 2u>", "uint2")[:36]
        lines.append(f"{name:36s} {r['Calls']:>6s} {int(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:11.2f} {float(r['Percentage']):6.2f}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


def peel_r_leg(args, mx, torch) -> dict:
    """The generic peel of random r-uniform hypergraphs (Section 2's r-hypergraphs) with 2^27
    edges, device-generated, vertices per edge just above each r's peeling threshold 1/c*_r
    (1.23 for r = 3 above 1.222, 1.33 for r = 4 above 1.295, 1.45 for r = 5 above 1.424):
    whole peels (records, rounds, canonical order) timed."""
    dev = torch.device("cuda:0")
    n = args.peel_r_n
    rows = {}
    for r, gamma in ((3, 1.23), (4, 1.33), (5, 1.45)):
        m = int(gamma * n)
        g = torch.Generator(device=dev)
        g.manual_seed(r)
        edges = torch.randint(0, m, (n, r), dtype=torch.int64, device=dev, generator=g)
        while True:  # r distinct vertices per edge: redraw the rows with a repeat
            srt = torch.sort(edges, dim=1).values
            bad = (srt[:, 1:] == srt[:, :-1]).any(dim=1)
            nb = int(bad.sum().item())
            if nb == 0:
                break
            edges[bad] = torch.randint(0, m, (nb, r), dtype=torch.int64, device=dev, generator=g)
        e32 = edges.to(torch.int32)
        del edges, srt, bad
        got = mx.peel_r(e32, m)
        torch.cuda.synchronize()
        steps = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(steps):
            got = mx.peel_r(e32, m)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        rows[f"r{r}"] = dict(edges=n, vertices=m, ms_per_peel=round(sec * 1e3, 3), edges_per_s=round(n / sec, 1),
                             rounds=got["n_rounds"], peeled=got["n_peeled"])
        log(f"[peel_r] r={r} n={n} m={m}: {sec * 1e3:.1f} ms/peel, {n / sec / 1e9:.3f} G edges/s, "
            f"{got['n_rounds']} rounds, {got['n_peeled']} peeled")
        del e32, got
        torch.cuda.empty_cache()
    return dict(workload=f"peel_r_uniform_n{n}", rows=rows)


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def golden_header(path: str) -> list:
    """Comment lines of a golden digest file (plain or gzip text), or [] when it is absent."""
    import gzip

    if not os.path.exists(path):
        return []
    opener = gzip.open if path.endswith(".gz") else open
    with opener(path, "rt") as fh:
        return [ln[1:].strip() for ln in fh if ln.startswith("#")]


def oracle_all_core_c4() -> dict:
    """The all-core oracle run behind the 65,536-bucket golden digests: one unchanged oracle
    build per bucket, buckets spread over processes; wall time and keys from its header."""
    import re

    for ln in golden_header(os.path.join(GOLDEN_DIR, "c4_buckets_65536.txt.gz")):
        m = re.match(r"(\d+) oracle processes on (\d+) host CPUs, (\d+) s wall, (\d+) keys", ln)
        if m:
            procs, cpus, wall, keys = (int(x) for x in m.groups())
            return dict(value=round(keys / wall, 1), unit="keys/s", processes=procs, host_cpus=cpus, wall_s=wall,
                        keys=keys, kind="oracle", source="tests/golden/c4_buckets_65536.txt.gz (make_fullsize.py c4)")
    return {}


def oracle_per_request_c5(np) -> dict:
    """Single-threaded oracle build times of the served workload's 60 full-size requests
    (golden digests' run; key generation excluded): p50 and p99."""
    path = os.path.join(GOLDEN_DIR, "c5_served_60.txt")
    if not os.path.exists(path):
        return {}
    secs = [float(ln.split()[-1]) for ln in open(path) if not ln.startswith("#") and ln.strip()]
    import re

    # the run's line, e.g. "16 oracle processes on 16 host CPUs, 62 s wall"
    runs = [m.group(0) for m in map(re.compile(r"\d+ oracle processes on \d+ host CPUs, \d+ s wall").search,
                                    golden_header(path)) if m]
    return dict(requests=len(secs), p50_ms=round(float(np.percentile(secs, 50)) * 1e3, 1),
                p99_ms=round(float(np.percentile(secs, 99)) * 1e3, 1), kind="oracle", cores=1,
                source="tests/golden/c5_served_60.txt (make_fullsize.py c5)" + (f": {runs[0]}" if runs else ""))


def batched_leg(args, mx, torch, np, workloads) -> dict:
    """65,536 independent u64 buckets, sizes floor(100 * 10^(4u)), one captured persistent
    launch per step; beside it the plain path on a sample of the same buckets."""
    dev = torch.device("cuda:0")
    sizes = workloads.bucket_sizes(args.batch_buckets, 100, 1_000_000, seed=0)
    off = np.zeros(len(sizes) + 1, np.uint64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    block, grid = args.batch_block, args.batch_grid
    autotune = not args.no_batch_autotune and block == 0 and grid == 0
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    tunes = []

    def setup():
        keys = mx.gen_buckets_u64(torch.from_numpy(off.view(np.int64)).to(dev))
        bb = mx.BatchBuild(off, block=block, grid=grid)
        if autotune:
            # the library's autotuner on the full batch, in this allocation (which shape wins
            # depends on the allocation's physical layout), between the two shapes that win at
            # this workload: 1024 threads x one workgroup per CU and 512 x two (the 256-thread
            # shapes ran 4-10 % slower on every sample); one timed build each
            t = bb.autotune(keys, candidates=[(1024, cus, 0), (512, 2 * cus, 0)], reps=1)
            tunes.append(t)
            log(f"[batched] autotune on the full batch: " +
                ", ".join(f"{b}x{g} {ms:.1f} ms" for (b, g), ms in zip(t["candidates"], t["ms"])) +
                f" -> {bb.tuning.block}x{bb.tuning.grid}")
        bb.capture(keys)
        bb.launch()  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bb.launch()
        torch.cuda.synchronize()
        return keys, bb, (time.perf_counter() - t0) * 1e3

    # the same physical-placement probe as the plain leg: keys and slots allocated again (after a
    # full release) while the last allocation's step is more than 2 % slower than the best seen
    keys, bb, t = setup()
    probes = [t]
    while not args.no_placement_probe and need_another_allocation(probes, args.placement_tries):
        bb.destroy_graph()
        del bb, keys
        torch.cuda.empty_cache()
        keys, bb, t = setup()
        probes.append(t)
    if len(probes) > 1:
        log(f"[batched] placement probe: {', '.join(f'{x:.1f}' for x in probes)} ms/step over {len(probes)} allocations")
    log(f"[batched] {len(sizes)} buckets, {total} keys ({total * 8 / 1e9:.1f} GB), slots "
        f"{bb.ws.numel() / 1e9:.1f} GB, max bucket {bb.max_bucket}")
    for _ in range(args.warmup):
        bb.launch()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bb.launch()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    res = bb.bucket_results()
    ok = res["status"] == 0
    ok_keys = int(sizes[ok].sum())
    sec = float(np.median(times))
    extra_tries = int(res["tries"].sum() - len(res))
    log(f"[batched] median {sec * 1000:.1f} ms/step, {ok_keys / sec / 1e9:.3f} G keys/s, "
        f"{int((~ok).sum())} failed buckets, {extra_tries} retries")
    clock = batch_clock_step(mx, torch, bb, keys)
    # the plain path (one mphf_build_u64 per bucket) on a random sample of the same buckets,
    # with one workspace and one pair of output buffers allocated before timing (sized for the
    # sample's largest bucket), so the calls time the build, not allocation
    rng = np.random.default_rng(1)
    sample = rng.choice(len(sizes), size=min(args.plain_sample, len(sizes)), replace=False)
    nmax = int(sizes[sample].max())
    mmax = 3 * mx.part_size(nmax, (123, 100))
    pws = torch.empty(mx.mphf_workspace_bytes(nmax), dtype=torch.uint8, device=dev)
    pout = (torch.empty((mmax + 31) // 32, dtype=torch.int64, device=dev),
            torch.empty((mmax + 511) // 512, dtype=torch.int64, device=dev))
    mx.mphf_build_u64(keys[int(off[sample[0]]):int(off[sample[0] + 1])], seed=0, ws=pws, out=pout)  # warm
    plain_keys = plain_sec = 0
    by_class = {}
    for b in sample:
        kb = keys[int(off[b]):int(off[b + 1])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mx.mphf_build_u64(kb, seed=0, ws=pws, out=pout)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plain_sec += dt
        plain_keys += int(sizes[b])
        c = by_class.setdefault(f"1e{int(np.log10(sizes[b]))}", [0, 0.0, 0])
        c[0] += int(sizes[b])
        c[1] += dt
        c[2] += 1
    plain_rate = plain_keys / plain_sec
    del pws, pout
    log(f"[batched] plain path on {len(sample)} sampled buckets (preallocated workspace and outputs): "
        f"{plain_rate / 1e9:.3f} G keys/s; " +
        ", ".join(f"{k}..: {v[0] / v[1] / 1e9:.3f} G keys/s over {v[2]}" for k, v in sorted(by_class.items())))
    bb.destroy_graph()
    out = dict(workload=BATCH_WORKLOAD, buckets=len(sizes), keys=total, ms_per_step=round(sec * 1000, 3),
               value=round(ok_keys / sec, 1), unit="edges/s", failed_buckets=int((~ok).sum()),
               retries=extra_tries, block=bb.tuning.block, grid=bb.tuning.grid,
               placement_probe_ms=[round(x, 1) for x in probes], autotune=tunes[-1] if tunes else None,
               plain_same_buckets=dict(value=round(plain_rate, 1), unit="edges/s", buckets=len(sample),
                                       note="one mphx_mphf_build_u64 per bucket into a preallocated workspace "
                                            "and outputs (no allocation in the timed calls)",
                                       by_size=dict((k, dict(buckets=v[2], keys_per_s=round(v[0] / v[1], 1)))
                                                    for k, v in sorted(by_class.items()))),
               speedup_vs_plain=round(ok_keys / sec / plain_rate, 2), oracle_all_core=oracle_all_core_c4(),
               phase_clock=clock)
    del bb, keys
    torch.cuda.empty_cache()
    return out


BATCH_CLOCK_PHASES = ("records", "deletes", "claim_grouping", "resolve", "other_rounds", "assign", "pack",
                      "lds_buckets", "queue")


def batch_clock_step(mx, torch, bb, keys) -> dict:
    """One untimed step more with the kernel that clocks its phases (option batch_clock): each
    phase's workgroup time averaged over the grid, and the work counts.  With two workgroups
    per compute unit their phases overlap, so the averages add up to the step but a phase's
    average is not the time the chip spends in it."""
    grid = bb.tuning.grid or torch.cuda.get_device_properties(0).multi_processor_count
    mx.batch_clock(reset=True)
    mx.set_option("batch_clock", 1)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bb.run(keys)
        torch.cuda.synchronize()
        step_ms = (time.perf_counter() - t0) * 1e3
        c = mx.batch_clock(reset=True)
    finally:
        mx.set_option("batch_clock", 0)
    per_wg = 1e3 / c["tick_hz"] / grid
    phases = {p: round(c[p] * per_wg, 2) for p in BATCH_CLOCK_PHASES}
    counts = {k: v for k, v in c.items() if k not in BATCH_CLOCK_PHASES and k not in ("tick_hz", "workgroup")}
    dels_s = phases["deletes"] / 1e3
    log(f"[batched] clocked step {step_ms:.1f} ms ({bb.tuning.block} x {grid}), workgroup time per phase: " +
        ", ".join(f"{p} {v:.1f}" for p, v in phases.items()) + f" ms; workgroup lifetime "
        f"{c['workgroup'] * per_wg:.1f} ms; {c['deletes_issued'] / max(1, c['device_keys']):.3f} deletes per "
        f"device-path key ({c['deletes_issued'] / 1e9:.2f} G, {c['deletes_issued'] / max(dels_s, 1e-9) / 1e9:.1f} G/s "
        f"over the deletes' average workgroup time), {c['list_records'] / max(1, c['device_keys']):.3f} list records "
        f"per key")
    return dict(step_ms=round(step_ms, 1), block=bb.tuning.block, grid=grid,
                workgroup_ms=round(c["workgroup"] * per_wg, 2), phases_ms=phases, counts=counts,
                note="ticks of each phase summed over workgroups / grid / tick rate (option batch_clock); "
                     "an untimed extra step with the clocked kernel")


def ceilings_leg(mx, torch) -> dict:
    """Machine ceilings of the access patterns the build is made of (the library's probe
    kernels): a streaming copy, random 8-byte atomics / loads and 1-byte stores over a
    16 GiB table (HBM-sized, far beyond the caches), and LDS-resident 8-byte atomics."""
    dev = torch.device("cuda:0")

    def best_ms(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        return best

    out = {}
    src = torch.empty(4 << 30, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    ms = best_ms(lambda: mx.probe_copy(src, dst))
    out["copy_GBps"] = round(2 * src.numel() / ms / 1e6, 1)
    del src, dst
    table = torch.zeros(16 << 30, dtype=torch.uint8, device=dev)
    count = 1 << 30
    for name, op, esz in (("atomic_add_ret_Gops", mx.PROBE_ATOMIC_ADD_RET, 8), ("atomic_add_Gops", mx.PROBE_ATOMIC_ADD, 8),
                          ("load8_Gops", mx.PROBE_LOAD8, 8), ("store1_Gops", mx.PROBE_STORE1, 1)):
        ms = best_ms(lambda: mx.probe_random(op, table, table.numel() // esz, count, seed=op))
        out[name] = round(count / ms / 1e6, 2)
    del table
    lds = torch.empty(4096 * 8192 * 8, dtype=torch.uint8, device=dev)
    ms = best_ms(lambda: mx.probe_random(mx.PROBE_LDS_ATOMIC_ADD, lds, 8192, 1 << 32, grid=4096, block=1024))
    out["lds_atomic_add_Gops"] = round((1 << 32) / ms / 1e6, 1)
    del lds
    torch.cuda.empty_cache()
    out["footprint"] = "random ops over a 16 GiB table; copy of 4 GiB; LDS tables of 8192 x 8 B"
    log(f"[ceilings] {out}")
    return out


FOOTPRINT_MB = (32, 128, 256, 512, 660, 880, 1320, 2640, 16384)


def footprint_leg(mx, torch) -> dict:
    """The random probes as a function of the table's footprint: 2^30 random 8-byte loads,
    1-byte stores, returning 8-byte atomics and 4-byte atomics over tables from inside the
    last-level cache (256 MB) to 16 GiB.  The sizes in between are those of the code array
    (m bytes at 2^31 keys: 2640 MB), one part of it (880 MB) and its 2-bit form (660 MB)."""
    dev = torch.device("cuda:0")
    table = torch.zeros(16 << 30, dtype=torch.uint8, device=dev)
    count = 1 << 30
    rows = {}
    for name, op, esz in (("load8", mx.PROBE_LOAD8, 8), ("store1", mx.PROBE_STORE1, 1),
                          ("atomic_add_ret", mx.PROBE_ATOMIC_ADD_RET, 8), ("atomic_add32", mx.PROBE_ATOMIC_ADD32, 4)):
        rates = {}
        for mb in FOOTPRINT_MB:
            slots = (mb << 20) // esz
            assert slots * esz <= table.numel()
            mx.probe_random(op, table, slots, count // 8, seed=1)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            mx.probe_random(op, table, slots, count, seed=2)
            b.record()
            b.synchronize()
            rates[str(mb)] = round(count / a.elapsed_time(b) / 1e6, 2)
        rows[name] = rates
        log(f"[footprint] {name} G/s by MB: {rates}")
    del table
    torch.cuda.empty_cache()
    return dict(unit="G operations/s", count=count, footprint_MB=list(FOOTPRINT_MB), rates=rows)


def random_ops(phase: str, st: dict) -> dict:
    """Random device-memory operations per step of a phase (atomics and gathers to arrays far
    larger than the caches), the count its measured ceiling applies to."""
    n, F, F0 = st["n"], st["frontier_total"], st["frontier0"]
    lists = st.get("lists", False)
    U = st.get("update_deletes", 0)
    L0 = st.get("layer0", 0) if round0_deletes_in_frontier(st) else 0
    if phase == "apply":
        # per edge the apply launches delete: edge-triple gather (and the state, without claim
        # lists), two returning deletes unless they went to an update list; per vertex taken
        # to degree 1: one atomicMin claim without claim lists
        if lists:
            return dict(atomics=2 * n - U, loads=n - L0)
        return dict(atomics=2 * n + (F - F0), loads=2 * n)
    if phase == "frontier":
        # with claim lists the hinge test gathers the lower-part vertices and their records;
        # when round 0 also deletes its layer, one edge gather per layer-0 edge
        return dict(atomics=0, loads=F0 + L0) if lists else dict(atomics=F0, loads=0)
    if phase == "assign":
        return dict(atomics=0, loads=2 * n, stores=n)
    return {}


LOOKUP_KEYS = 10_000_000
LOOKUP_BATCH = 1 << 16
LOOKUP_REPEATS = 10


def table2_lookups(torch, n: int, nk: int, run, out) -> dict:
    """Lookups in the paper's lookup-experiment shape (Section 5, Table 2): the first nk keys
    of the set in batches of 2^16 keys, all batches repeated 10 times back to back on the
    stream; per-batch time from HIP events.  run(b0, b1) evaluates keys [b0, b1) into
    out[b0:b1].  Checks that the values are distinct, below n, and that the batched
    evaluation equals one call over all keys."""
    batches = [(b, min(b + LOOKUP_BATCH, nk)) for b in range(0, nk, LOOKUP_BATCH)]
    run(0, nk)
    torch.cuda.synchronize()
    distinct = int(torch.unique(out).numel())
    ok = distinct == nk and int(out.min().item()) >= 0 and int(out.max().item()) < n
    whole = out.clone()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(LOOKUP_REPEATS * len(batches) + 1)]
    ev[0].record()
    j = 1
    for _ in range(LOOKUP_REPEATS):
        for b0, b1 in batches:
            run(b0, b1)
            ev[j].record()
            j += 1
    torch.cuda.synchronize()
    ok = ok and bool(torch.equal(out, whole))
    per_key = []
    for k in range(1, j):
        b0, b1 = batches[(k - 1) % len(batches)]
        per_key.append(ev[k - 1].elapsed_time(ev[k]) * 1e6 / (b1 - b0))  # ns per key
    total_ms = ev[0].elapsed_time(ev[j - 1])
    mean = sum(per_key) / len(per_key)
    sd = (sum((x - mean) ** 2 for x in per_key) / len(per_key)) ** 0.5
    rate = LOOKUP_REPEATS * nk / (total_ms / 1e3)
    del whole
    return dict(workload=f"lookup_{nk}_keys_batches_of_{LOOKUP_BATCH}", keys=nk, batch=LOOKUP_BATCH,
                batches=len(batches) * LOOKUP_REPEATS, ns_per_key=round(mean, 4), rel_std=round(sd / mean, 4),
                lookups_per_s=round(rate, 1), values_distinct_and_in_range=ok)


def lookup_leg(mx, torch, r: dict, n: int, kind: int, keys=None, data=None, offs=None,
               ceilings=None) -> dict:
    """Evaluation of the MPHF just built in the shape of Table 2 (see table2_lookups)."""
    nk = min(LOOKUP_KEYS, n)
    out = torch.empty(nk, dtype=torch.int64, device=torch.device("cuda:0"))
    codes, rank, P, seed = r["codes"], r["rank"], r["P"], r["seed_used"]

    def run(b0, b1):
        if kind == mx.KEYS_U64:
            mx.lookup_u64(codes, rank, P, seed, keys[b0:b1], out=out[b0:b1])
        else:
            mx.lookup_str(codes, rank, P, seed, data, offs[b0:b1 + 1], out=out[b0:b1])

    res = table2_lookups(torch, n, nk, run, out)
    res["paper_ns_per_key_one_core"] = "199-415 (Table 2, three CPUs, one thread)"
    rate = res["lookups_per_s"]
    # each lookup gathers three code words, one rank sample and the hinge's rank block: about
    # four random lines besides the streamed key
    if ceilings and ceilings.get("load8_Gops"):
        res["roofline"] = dict(bound="random gathers", achieved=round(4 * rate / 1e9, 2),
                               peak=ceilings["load8_Gops"], unit="G gathers/s",
                               frac=round(4 * rate / 1e9 / ceilings["load8_Gops"], 3))
    log(f"[lookup] {nk} keys in batches of {LOOKUP_BATCH} x {LOOKUP_REPEATS}: {res['ns_per_key']:.3f} ns/key "
        f"per batch (rel. sd {res['rel_std']:.3f}), {rate / 1e9:.2f} G lookups/s, "
        f"ok={res['values_distinct_and_in_range']}")
    del out
    return res


SF_SIGMA = 256


def sf_leg(args, mx, torch, n: int, kind: int, ws, keys=None, data=None, offs=None) -> dict:
    """Static function (Section 3) of the same keys: sigma = 256, key i's value a byte of
    SplitMix64 output i + 1 at state 7 (made on the device); builds timed like the plain leg,
    with the first 10^7 keys' lookups checked against their values."""
    dev = torch.device("cuda:0")
    gamma = (123, 100)
    vals = torch.empty(n, dtype=torch.int32, device=dev)
    G, M1, M2 = 0x9E3779B97F4A7C15, 0xBF58476D1CE4E5B9, 0x94D049BB133111EB

    def to_i64(x):
        return x - (1 << 64) if x >= 1 << 63 else x

    chunk = 1 << 27
    for c0 in range(0, n, chunk):
        c1 = min(c0 + chunk, n)
        z = (torch.arange(c0 + 1, c1 + 1, dtype=torch.int64, device=dev) * to_i64(G)) + 7
        z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * to_i64(M1)
        z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * to_i64(M2)
        z = z ^ ((z >> 31) & ((1 << 33) - 1))
        vals[c0:c1] = (z & (SF_SIGMA - 1)).to(torch.int32)
        del z
    words = torch.empty(max(mx.sf_words(n, SF_SIGMA, gamma), 1), dtype=torch.int64, device=dev)
    if ws.numel() < mx.sf_workspace_bytes(n, gamma, kind):  # without claim lists the values need 4n more
        ws = torch.empty(mx.sf_workspace_bytes(n, gamma, kind), dtype=torch.uint8, device=dev)

    def step():
        if kind == mx.KEYS_U64:
            return mx.sf_build_u64(keys, vals, SF_SIGMA, seed=0, gamma=gamma, ws=ws, words=words)
        return mx.sf_build_str(data, offs, vals, SF_SIGMA, seed=0, gamma=gamma, ws=ws, words=words)

    r = step()
    torch.cuda.synchronize()
    mx.phase_times(reset=True)
    t0 = time.perf_counter()
    steps = max(1, min(args.steps, 3))
    for _ in range(steps):
        r = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    phases = {k: round(v[0] / steps, 3) for k, v in mx.phase_times(reset=True).items() if v[1]}
    nk = min(LOOKUP_KEYS, n)
    if kind == mx.KEYS_U64:
        f = mx.sf_lookup_u64(r["words"], SF_SIGMA, r["P"], r["seed_used"], keys[:nk])
    else:
        f = mx.sf_lookup_str(r["words"], SF_SIGMA, r["P"], r["seed_used"], data, offs[: nk + 1])
    ok = bool(torch.equal(f, vals[:nk].to(torch.int64)))
    res = dict(workload=f"static_function_sigma{SF_SIGMA}_same_keys", sigma=SF_SIGMA, bits=mx.sf_bits(SF_SIGMA),
               ms_per_build=round(sec * 1e3, 3), keys_per_s=round(n / sec, 1), tries=r["tries"],
               rounds=r["n_rounds"], bits_per_key=round(mx.sf_bits(SF_SIGMA) * r["m"] / n, 3),
               lookups_equal_values=ok, phases_ms=phases)
    log(f"[sf] sigma {SF_SIGMA}: {sec * 1e3:.1f} ms/build, {n / sec / 1e9:.3f} G keys/s, lookups ok={ok}")
    del words, f, r
    torch.cuda.empty_cache()
    # the ranked layout of the same function (marks of the non-zero values, rank samples, the
    # fields in vertex order): same builds plus the compaction
    outs = tuple(torch.empty(max(w, 1), dtype=torch.int64, device=dev) for w in mx.sfr_sizes(n, SF_SIGMA, gamma))

    def rstep():
        if kind == mx.KEYS_U64:
            return mx.sfr_build_u64(keys, vals, SF_SIGMA, seed=0, gamma=gamma, ws=ws, out=outs)
        return mx.sfr_build_str(data, offs, vals, SF_SIGMA, seed=0, gamma=gamma, ws=ws, out=outs)

    r = rstep()
    torch.cuda.synchronize()
    mx.phase_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        r = rstep()
    torch.cuda.synchronize()
    rsec = (time.perf_counter() - t0) / steps
    rphases = {k: round(v[0] / steps, 3) for k, v in mx.phase_times(reset=True).items() if v[1]}
    if kind == mx.KEYS_U64:
        f = mx.sfr_lookup_u64(r, SF_SIGMA, keys[:nk])
    else:
        f = mx.sfr_lookup_str(r, SF_SIGMA, data, offs[: nk + 1])
    rok = bool(torch.equal(f, vals[:nk].to(torch.int64)))
    fields = int(r["rank"][-1])
    bits = r["m"] + 64 * r["rank"].numel() + fields * mx.sf_bits(SF_SIGMA)
    res["ranked"] = dict(ms_per_build=round(rsec * 1e3, 3), keys_per_s=round(n / rsec, 1), fields=fields,
                         bits_per_key=round(bits / n, 3),
                         paper_bound_bits_per_key=round(mx.sf_bits(SF_SIGMA) + r["m"] / n, 3),
                         lookups_equal_values=rok, phases_ms=rphases)
    log(f"[sf] ranked: {rsec * 1e3:.1f} ms/build, {bits / n:.3f} bits/key ({fields} fields), lookups ok={rok}")
    del vals, outs, f
    return res


def hem_leg(args, mx, torch, n: int, kind: int, keys=None, data=None, offs=None) -> dict:
    """HEM split (Section 3) of the same keys for each k in --hem-k: signatures (64-bit for u64
    keys, the whole 128-bit digest for strings), 2^k buckets by their top bits, one MWHC MPHF per bucket by the batched kernel; builds timed like
    the plain leg (steps capped at 3), then one lookup of all n keys timed with HIP events and
    checked to be a bijection onto [0, n)."""
    dev = torch.device("cuda:0")
    gamma = (123, 100)
    ws = torch.empty(max(mx.hem_workspace_bytes(n, k, gamma, kind) for k in args.hem_k), dtype=torch.uint8, device=dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    rows = {}
    for k, tune in [(k, t) for k in args.hem_k for t in args.hem_tune]:
        block, grid = (int(x) for x in tune.split("x"))
        mx.set_option("hem_block", block)
        mx.set_option("hem_grid", grid)
        if ws.numel() < mx.hem_workspace_bytes(n, k, gamma, kind):
            del ws
            ws = torch.empty(mx.hem_workspace_bytes(n, k, gamma, kind), dtype=torch.uint8, device=dev)

        def step():
            if kind == mx.KEYS_U64:
                return mx.hem_build(keys=keys, k=k, seed=0, gamma=gamma, ws=ws)
            return mx.hem_build(data=data, offs=offs, k=k, seed=0, gamma=gamma, ws=ws)

        h = step()
        torch.cuda.synchronize()
        mx.phase_times(reset=True)
        steps = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(steps):
            del h
            h = step()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        phases = {p: round(v[0] / steps, 3) for p, v in mx.phase_times(reset=True).items() if v[1]}
        B = 1 << k
        words = h["codes"].numel() + h["rank"].numel()
        bits = 64 * words + 64 * (4 * B + 3)  # codes, rank samples, three offset arrays and the seeds
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if kind == mx.KEYS_U64:
            mx.hem_lookup(h, keys=keys, out=out)
        else:
            mx.hem_lookup(h, data=data, offs=offs, out=out)
        e1.record()
        torch.cuda.synchronize()
        lk_ms = e0.elapsed_time(e1)
        # a bijection onto [0, n): every value in range and every slot hit once
        inrange = bool(int(out.min().item()) >= 0 and int(out.max().item()) < n)
        hit = torch.zeros(n, dtype=torch.uint8, device=dev)
        if inrange:
            hit.index_fill_(0, out, 1)
        ok = inrange and int(hit.sum(dtype=torch.int64).item()) == n
        del hit
        nk = min(LOOKUP_KEYS, n)

        def run(b0, b1):
            if kind == mx.KEYS_U64:
                mx.hem_lookup(h, keys=keys[b0:b1], out=out[b0:b1])
            else:
                mx.hem_lookup(h, data=data, offs=offs[b0:b1 + 1], out=out[b0:b1])

        t2 = table2_lookups(torch, n, nk, run, out[:nk])
        sizes = (h["bucket_off"][1:] - h["bucket_off"][:-1])
        rows[f"k{k}" + ("" if tune == "1024x0" else f"_{tune}")] = dict(buckets=B, block=block, grid=grid, ms_per_build=round(sec * 1e3, 3), keys_per_s=round(n / sec, 1),
                             bits_per_key=round(bits / n, 4), max_bucket=int(sizes.max().item()),
                             max_tries=h["tries"], max_rounds=h["n_rounds"], phases_ms=phases,
                             lookup_all_ms=round(lk_ms, 3), lookup_ns_per_key=round(lk_ms * 1e6 / n, 4),
                             bijection=ok, table2_lookup=t2)
        log(f"[hem] k={k} block x grid {tune}: {sec * 1e3:.1f} ms/build, {n / sec / 1e9:.3f} G keys/s, {bits / n:.3f} bits/key, "
            f"lookup {lk_ms * 1e6 / n:.3f} ns/key, bijection ok={ok}; Table 2 shape {t2['ns_per_key']:.3f} ns/key "
            f"per batch, ok={t2['values_distinct_and_in_range']}")
        del h, sizes
    mx.set_option("hem_block", 1024)
    mx.set_option("hem_grid", 0)
    del ws, out
    torch.cuda.empty_cache()
    return dict(workload="hem_split_same_keys", rows=rows)


def stream_leg(args, mx, torch) -> dict:
    """One MWHC MPHF over a u64 key set held in host memory, too large for the in-HBM build
    (the paper's 7.6e9 keys, Section 5): the streamed build (vertex records with the XOR of the
    other two endpoints, no edge ids), once with every layer in device memory and once with the
    layers spilled to host memory past a layer area of 0.3 n slots.  Whole builds are timed with
    their transfers; then every key is streamed through the evaluation and the values checked to
    form a bijection onto [0, n)."""
    dev = torch.device("cuda:0")
    n, chunk = args.stream_n, args.stream_chunk
    gamma = (123, 100)
    P = mx.part_size(n, gamma)
    m = 3 * P
    t0 = time.perf_counter()
    hk = torch.empty(n, dtype=torch.int64)
    for c0 in range(0, n, chunk):  # the u64 key generator on the device, copied down
        c1 = min(n, c0 + chunk)
        hk[c0:c1].copy_(mx.gen_keys_u64(c1 - c0, gen_seed=0, start=c0, device=dev))
    torch.cuda.synchronize()
    log(f"[stream] {n} keys ({8 * n / 1e9:.1f} GB) in pageable host memory, generated in "
        f"{time.perf_counter() - t0:.1f} s; P = {P}, m = {m} vertices")
    codes = torch.empty((m + 31) // 32, dtype=torch.int64, device=dev)
    rank = torch.empty((m + 511) // 512, dtype=torch.int64, device=dev)
    # the in-HBM build's workspace per key at 2^31 keys (claim lists on), scaled, plus the keys
    in_hbm = mx.mphf_workspace_bytes(1 << 31, gamma) / (1 << 31) * n + 8 * n
    rows = {}
    host_layers = None
    for name, slots in (("layers_in_hbm", n), ("layers_spilled", (3 * n) // 10)):
        need = mx.stream_workspace_bytes(n, gamma, chunk, slots)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        if slots < n and host_layers is None:
            host_layers = torch.empty(12 * n, dtype=torch.uint8)
            host_layers[::4096] = 0  # touch every page before timing
        mx.set_option("timing", 1)
        mx.phase_times(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = mx.mphf_build_stream_u64(hk, seed=0, gamma=gamma, chunk_keys=chunk, layer_slots=slots,
                                     host_layers=host_layers if slots < n else None, ws=ws, out=(codes, rank),
                                     device=dev)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ph = {k: round(v[0], 1) for k, v in mx.phase_times(reset=True).items() if v[1]}
        t1 = time.perf_counter()
        bad = mx.check_stream_u64(codes, rank, r["P"], r["seed_used"], hk, chunk_keys=chunk)
        t_check = time.perf_counter() - t1
        rows[name] = dict(layer_slots=slots, device_workspace_bytes=need, s_per_build=round(sec, 3),
                          keys_per_s=round(n / sec, 1), tries=r["tries"], rounds=r["n_rounds"], layer0=r["layer0"],
                          phases_ms=ph, bijection=bad == 0, bad_values=bad, check_s=round(t_check, 2))
        log(f"[stream] {name}: {sec:.2f} s/build = {n / sec / 1e9:.3f} G keys/s (device workspace {need / 1e9:.1f} GB, "
            f"tries {r['tries']}, rounds {r['n_rounds']}); phases {ph}; all {n} keys looked up in {t_check:.1f} s, "
            f"bijection ok={bad == 0}")
        del ws, r
        torch.cuda.empty_cache()
    bits = 64 * (codes.numel() + rank.numel()) / n
    del codes, rank, hk, host_layers
    return dict(workload=f"mwhc_stream_u64_n{n}_gamma1.23", n=n, vertices=m, chunk_keys=chunk,
                host_key_bytes=8 * n, in_hbm_build_bytes_estimate=int(in_hbm), bits_per_key=round(bits, 4),
                rows=rows, paper_context="Section 5: 7.6e9 keys built in under 21 h on one CPU with a disk "
                                         "(Intel i7 E5520, 32 GiB)")


def hem_host_str_leg(args, mx, torch, np, workloads) -> dict:
    """HEM split of a byte-string key set held in host memory: n-gram-like keys (log-normal
    lengths with mean 23 B, clamped to 8..512 B, distinct by construction), 128-bit signatures
    (16 bytes per key stay on the device).  Times whole builds with their transfers, then
    streams every key again, looks it up and checks that the values form a bijection."""
    dev = torch.device("cuda:0")
    n, k, chunk, batch = args.hem_host_str_n, args.hem_host_k, args.hem_host_chunk, args.hem_host_batch
    chunk_bytes = 64 * chunk
    gamma = (123, 100)
    qtab = torch.from_numpy(workloads.quantile_table(args.hem_host_str_mean).view(np.int16)).to(dev)
    t0 = time.perf_counter()
    # lengths first, to size the host byte array
    total = 0
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        _, offs = mx.gen_str_keys(c1 - c0, qtab, gen_seed=0, start=c0, device=dev)
        total += int(offs[-1].item())
        del offs
    hd = torch.empty(total + 8, dtype=torch.uint8)
    ho = torch.empty(n + 1, dtype=torch.int64)
    hd[::4096] = 0  # touch every page before timing
    ho[::512] = 0
    base = 0
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        d, o = mx.gen_str_keys(c1 - c0, qtab, gen_seed=0, start=c0, device=dev)
        ln = int(o[-1].item())
        hd[base:base + ln].copy_(d[:ln])
        ho[c0:c1 + 1].copy_(o + base)
        base += ln
        del d, o
    torch.cuda.synchronize()
    log(f"[hem_host_str] {n} string keys ({total / 1e9:.1f} GB of bytes, mean {total / n:.1f} B, and "
        f"{8 * (n + 1) / 1e9:.1f} GB of offsets) in pageable host memory, generated in {time.perf_counter() - t0:.1f} s")
    need = mx.hem_host_workspace_bytes(n, k, mx.KEYS_STR, chunk, chunk_bytes, batch, gamma)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    mx.set_option("timing", 1)

    def step():
        return mx.hem_build_host(data=hd, offs=ho, k=k, seed=0, gamma=gamma, chunk_keys=chunk,
                                 chunk_bytes=chunk_bytes, batch_keys=batch, ws=ws, device=dev)

    h = step()
    torch.cuda.synchronize()
    mx.phase_times(reset=True)
    steps = max(1, min(args.steps, 2))
    t0 = time.perf_counter()
    for _ in range(steps):
        del h
        h = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    phases = {p: round(v[0] / steps, 3) for p, v in mx.phase_times(reset=True).items() if v[1]}
    B = 1 << k
    bits = 64 * (h["codes"].numel() + h["rank"].numel()) + 64 * (4 * B + 3)
    del ws
    torch.cuda.empty_cache()
    hit = torch.zeros(n, dtype=torch.uint8, device=dev)
    ok = True
    t0 = time.perf_counter()
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        b0, b1 = int(ho[c0]), int(ho[c1])
        dd = hd[b0:b1].to(dev)
        do = (ho[c0:c1 + 1] - b0).to(dev)
        f = mx.hem_lookup(h, data=dd, offs=do)
        ok = ok and bool(int(f.min().item()) >= 0 and int(f.max().item()) < n)
        if ok:
            hit.index_fill_(0, f, 1)
        del dd, do, f
    ok = ok and int(hit.sum(dtype=torch.int64).item()) == n
    torch.cuda.synchronize()
    t_check = time.perf_counter() - t0
    del hit, h, hd, ho
    torch.cuda.empty_cache()
    log(f"[hem_host_str] k={k}: {sec:.2f} s/build = {n / sec / 1e9:.3f} G keys/s with transfers, phases {phases}, "
        f"{bits / n:.3f} bits/key; all-key lookups in {t_check:.1f} s, bijection ok={ok}")
    return dict(workload=f"hem_host_str_n{n}_mean{args.hem_host_str_mean:g}B_k{k}", keys=n, key_bytes=total,
                offset_bytes=8 * (n + 1), k=k, chunk_keys=chunk, chunk_bytes=chunk_bytes, batch_keys=batch,
                device_workspace_bytes=need, s_per_build=round(sec, 3), keys_per_s=round(n / sec, 1),
                phases_ms=phases, bits_per_key=round(bits / n, 4), bijection=ok, check_s=round(t_check, 1),
                signature_bits=128)


def hem_host_leg(args, mx, torch) -> dict:
    """HEM split of a u64 key set held in host memory (pinned when the host allows) and larger than device memory
    would allow in place: the keys stream over PCIe in chunks, only their 8-byte signatures stay
    on the device.  Times whole builds (transfers included), then streams the keys again to look
    every one up and checks that the values form a bijection onto [0, n)."""
    dev = torch.device("cuda:0")
    n, k = args.hem_host_n, args.hem_host_k
    chunk, batch = args.hem_host_chunk, args.hem_host_batch
    gamma = (123, 100)
    t0 = time.perf_counter()
    try:
        hk = torch.empty(n, dtype=torch.int64, pin_memory=True)
        memory = "pinned"
    except RuntimeError as e:  # the host may cap page-locked memory: ordinary pages then
        log(f"[hem_host] pinned allocation of {8 * n / 1e9:.1f} GB refused ({str(e).splitlines()[0]}): pageable")
        hk = torch.empty(n, dtype=torch.int64)
        hk[::512] = 0  # touch every page before timing
        memory = "pageable"
    t_pin = time.perf_counter() - t0
    t0 = time.perf_counter()
    for c0 in range(0, n, chunk):  # the u64 key generator on the device, copied down
        c1 = min(n, c0 + chunk)
        hk[c0:c1].copy_(mx.gen_keys_u64(c1 - c0, gen_seed=0, start=c0, device=dev))
    torch.cuda.synchronize()
    log(f"[hem_host] {n} keys ({8 * n / 1e9:.1f} GB) in {memory} host memory: allocated in {t_pin:.1f} s, "
        f"generated in {time.perf_counter() - t0:.1f} s")
    need = mx.hem_host_workspace_bytes(n, k, mx.KEYS_U64, chunk, 0, batch, gamma)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    in_place = mx.hem_workspace_bytes(n, k, gamma, mx.KEYS_U64) + 8 * n  # the in-HBM split: keys + its workspace
    log(f"[hem_host] device workspace {need / 1e9:.1f} GB (the in-HBM split would need {in_place / 1e9:.1f} GB)")

    mx.set_option("timing", 1)

    def step():
        return mx.hem_build_host(keys=hk, k=k, seed=0, gamma=gamma, chunk_keys=chunk, batch_keys=batch, ws=ws,
                                 device=dev)

    h = step()
    torch.cuda.synchronize()
    mx.phase_times(reset=True)
    steps = max(1, min(args.steps, 2))
    t0 = time.perf_counter()
    for _ in range(steps):
        del h
        h = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    phases = {p: round(v[0] / steps, 3) for p, v in mx.phase_times(reset=True).items() if v[1]}
    B = 1 << k
    bits = 64 * (h["codes"].numel() + h["rank"].numel()) + 64 * (4 * B + 3)
    del ws
    torch.cuda.empty_cache()
    # every key looked up, chunk by chunk from host memory; the values must hit [0, n) once each
    hit = torch.zeros(n, dtype=torch.uint8, device=dev)
    out = torch.empty(chunk, dtype=torch.int64, device=dev)
    dk = torch.empty(chunk, dtype=torch.int64, device=dev)
    ok = True
    t0 = time.perf_counter()
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        dk[: c1 - c0].copy_(hk[c0:c1], non_blocking=True)
        f = mx.hem_lookup(h, keys=dk[: c1 - c0], out=out[: c1 - c0])
        ok = ok and bool(int(f.min().item()) >= 0 and int(f.max().item()) < n)
        if ok:
            hit.index_fill_(0, f, 1)
    ok = ok and int(hit.sum(dtype=torch.int64).item()) == n
    torch.cuda.synchronize()
    t_check = time.perf_counter() - t0
    del hit, out, dk, h, hk
    torch.cuda.empty_cache()
    log(f"[hem_host] k={k}: {sec:.2f} s/build = {n / sec / 1e9:.3f} G keys/s with transfers, phases {phases}, "
        f"{bits / n:.3f} bits/key; all-key lookups from host memory in {t_check:.1f} s, bijection ok={ok}")
    return dict(workload=f"hem_host_u64_n{n}_k{k}", host_memory=memory, keys=n, key_bytes=8 * n, k=k,
                chunk_keys=chunk,
                batch_keys=batch, device_workspace_bytes=need, in_hbm_split_bytes=in_place,
                s_per_build=round(sec, 3), keys_per_s=round(n / sec, 1), phases_ms=phases,
                stream_GBps=round(8 * n / (phases.get("hash", 0) / 1e3) / 1e9, 1) if phases.get("hash") else None,
                bits_per_key=round(bits / n, 4), bijection=ok, check_s=round(t_check, 1))


SERVE_WORKLOAD = "mwhc_served_poisson_sizes_loguniform_1e3_1e8_u64_or_str_gamma1.23"


def served_leg(args, mx, torch, np, workloads) -> dict:
    """Poisson stream of builds (sizes log-uniform 1e3..1e8, u64 or string keys 50/50)
    submitted to the build server at its arrival times; rates swept around saturation."""
    dev = torch.device("cuda:0")
    max_n = args.serve_max
    keys = mx.gen_keys_u64(max_n, gen_seed=7, device=dev)
    q = torch.from_numpy(workloads.quantile_table().view(np.int16)).to(dev)
    data, offs = mx.gen_str_keys(max_n, q, gen_seed=8, device=dev)
    torch.cuda.synchronize()
    nreq = args.serve_requests
    sizes = workloads.request_sizes(nreq, 1000, max_n, seed=1)
    kinds = (workloads.stream(np.uint64(2), np.arange(1, nreq + 1, dtype=np.uint64)) & np.uint64(1)).astype(int)
    offs_slices = {}

    def submit(srv, i):
        n = int(sizes[i])
        if kinds[i] == 0:
            return srv.submit_u64(keys[:n], seed=i)
        if n not in offs_slices:
            offs_slices[n] = offs[: n + 1]
        return srv.submit_str(data, offs_slices[n], seed=i)

    mean_n = float(sizes.mean())
    # the plain path on the same requests, one build after another on one stream
    def plain(i):
        n = int(sizes[i])
        if kinds[i] == 0:
            return mx.mphf_build_u64(keys[:n], seed=i)
        return mx.mphf_build_str(data, offs[: n + 1], seed=i)

    for i in range(min(4, nreq)):
        plain(i)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for i in range(nreq):
        plain(i)
    torch.cuda.synchronize()
    plain_span = time.perf_counter() - p0
    plain_rate = float(sizes.sum()) / plain_span
    log(f"[served] plain path, same {nreq} requests back to back: {plain_span:.2f} s = "
        f"{plain_rate / 1e9:.3f} G keys/s")
    # saturation estimate: everything submitted at once
    srv = mx.Server(hbm_budget=args.serve_budget, slots=args.serve_slots, batch_max_keys=args.serve_lane_max)
    warm = [submit(srv, i) for i in range(min(8, nreq))]
    for t in warm:
        srv.wait(t)
        srv.release(t)
    t0 = mx.Server.clock()
    tickets = [submit(srv, i) for i in range(nreq)]
    res = [srv.wait(t) for t in tickets]
    for t in tickets:
        srv.release(t)
    span = max(r["t_done"] for r in res) - t0
    sat_rate = nreq / span
    sat_edges = float(sizes.sum()) / span
    log(f"[served] saturation: {nreq} builds in {span:.2f} s = {sat_rate:.1f} builds/s, "
        f"{sizes.sum() / span / 1e9:.3f} G keys/s (mean size {mean_n:.0f})")
    rows = []
    for frac in args.serve_rates:
        rate = frac * sat_rate
        arr = workloads.poisson_arrivals(nreq, rate, seed=int(frac * 1000))
        start = mx.Server.clock() + 0.01
        tickets = []
        for i in range(nreq):
            while mx.Server.clock() < start + arr[i]:
                pass
            tickets.append(submit(srv, i))
        res = [srv.wait(t) for t in tickets]
        for t in tickets:
            srv.release(t)
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        bad = sum(r["status"] != 0 for r in res)
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        row = dict(rate_frac=frac, offered_builds_per_s=round(rate, 2), builds_per_s=round(nreq / span, 2),
                   edges_per_s=round(float(sizes.sum()) / span, 1), p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                   p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3), failed=int(bad))
        rows.append(row)
        log(f"[served] rate {frac:.2f}x = {rate:.1f}/s: p50 {row['p50_ms']:.2f} ms, p99 {row['p99_ms']:.2f} ms, "
            f"{row['edges_per_s'] / 1e9:.3f} G keys/s, {bad} failed")
    st = srv.stats()
    srv.close()
    del keys, data, offs
    torch.cuda.empty_cache()
    return dict(workload=SERVE_WORKLOAD, requests_per_rate=nreq, mean_keys=round(mean_n, 1),
                slots=args.serve_slots, hbm_budget=args.serve_budget, peak_pool_in_use=st["peak_in_use"],
                saturation_builds_per_s=round(sat_rate, 2), saturation_edges_per_s=round(sat_edges, 1),
                plain_same_requests=dict(value=round(plain_rate, 1), unit="edges/s", requests=nreq,
                                         note="one mphf_build after another on one stream"),
                speedup_vs_plain=round(sat_edges / plain_rate, 2), rates=rows,
                oracle_per_request=oracle_per_request_c5(np))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", choices=sorted(CONFIGS), default="c3")
    ap.add_argument("--n", type=int, default=0, help="override the number of keys")
    ap.add_argument("--cpu-sample", type=int, default=1 << 26, help="keys in the oracle's timed sample (~15 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--placement-tries", type=int, default=2, help="allocations the placement probe makes")
    ap.add_argument("--no-placement-probe", action="store_true",
                    help="time the first allocation's physical layout, without probing the other")
    ap.add_argument("--legs", default="ceilings,plain,lookup,sf,hem,batched,served",
                    help="comma list of: ceilings, plain, lookup, sf and hem (need plain), batched, served, hem_host, "
                         "hem_host_str, stream, peel_r, footprint")
    ap.add_argument("--hem-k", type=lambda s: [int(x) for x in s.split(",")], default=[17],
                    help="bucket-count exponents of the hem leg")
    ap.add_argument("--hem-tune", type=lambda s: s.split(","), default=["1024x0"],
                    help="batched-kernel block x grid shapes of the hem leg (grid 0 = one per compute unit)")
    ap.add_argument("--peel-r-n", type=int, default=1 << 27, help="edges of the peel_r leg")
    ap.add_argument("--hem-host-n", type=int, default=1 << 34, help="keys of the hem_host leg (host memory)")
    ap.add_argument("--hem-host-k", type=int, default=20)
    ap.add_argument("--hem-host-chunk", type=int, default=1 << 27, help="keys per host-to-device chunk")
    ap.add_argument("--hem-host-batch", type=int, default=1 << 28, help="keys per gathered batch of groups")
    ap.add_argument("--stream-n", type=int, default=7_600_000_000, help="keys of the stream leg (host memory)")
    ap.add_argument("--hem-host-str-n", type=int, default=1 << 32, help="string keys of the hem_host_str leg")
    ap.add_argument("--hem-host-str-mean", type=float, default=23.0, help="mean key length of the hem_host_str leg")
    ap.add_argument("--stream-chunk", type=int, default=1 << 27, help="keys per host-to-device chunk of the stream leg")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write profiles/hbm_counters_<workload> from rocprofv3 --pmc output directories")
    ap.add_argument("--counters-command", default="", help="the command the counter runs used (recorded)")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=VALUE",
                    help="library option to set before timing (mphx_set_option), e.g. claim_lists=0")
    ap.add_argument("--summarize-l2", nargs=3, metavar=("PMC_DIR", "OUT_TXT", "TITLE"),
                    help="write a per-kernel L2 hit-rate table from a rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum run")
    ap.add_argument("--summarize-kernel-stats", nargs=3, metavar=("STATS_CSV", "OUT_TXT", "TITLE"),
                    help="write a text table of a rocprofv3 kernel_stats.csv (command from --counters-command)")
    ap.add_argument("--batch-buckets", type=int, default=65536)
    ap.add_argument("--batch-block", type=int, default=0)
    ap.add_argument("--batch-grid", type=int, default=0)
    ap.add_argument("--no-batch-autotune", action="store_true",
                    help="batched leg: skip the autotuner (block/grid from --batch-block/--batch-grid, else 1024 x one per CU)")
    ap.add_argument("--plain-sample", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests per rate of the served leg")
    ap.add_argument("--serve-max", type=int, default=100_000_000)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget", type=int, default=64 << 30)
    ap.add_argument("--serve-lane-max", type=int, default=1 << 17,
                    help="requests of at most this many keys take the server's batching lane")
    ap.add_argument("--serve-rates", type=lambda s: [float(x) for x in s.split(",")], default=[0.25, 0.5, 1.0, 2.0, 4.0],
                    help="offered rates as multiples of the measured saturation rate")
    args = ap.parse_args()
    if args.summarize_kernel_stats:
        return summarize_kernel_stats(*args.summarize_kernel_stats, command=args.counters_command)
    if args.summarize_l2:
        return summarize_l2(*args.summarize_l2, command=args.counters_command)
    if args.summarize_counters:
        return summarize_counters(*args.summarize_counters, workload=CONFIGS[args.config]["workload"],
                                  command=args.counters_command)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding "
              "of the peel is a design note, not built", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1312_0526_amd as mx
    import workloads

    cfg = dict(CONFIGS[args.config])
    n = args.n or cfg["n"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    gamma = (123, 100)
    legs = set(args.legs.split(","))
    options = {}
    for kv in args.set:
        key, value = kv.split("=", 1)
        mx.set_option(key, int(value))
        options[key] = int(value)
    ceilings = ceilings_leg(mx, torch) if "ceilings" in legs else None
    if "plain" not in legs:  # side legs only: no headline line
        side = {"ceilings": ceilings}
        if "batched" in legs:
            side["batched"] = batched_leg(args, mx, torch, np, workloads)
        if "served" in legs:
            side["served"] = served_leg(args, mx, torch, np, workloads)
        if "hem_host" in legs:
            side["hem_host"] = hem_host_leg(args, mx, torch)
        if "stream" in legs:
            side["stream"] = stream_leg(args, mx, torch)
        if "hem_host_str" in legs:
            side["hem_host_str"] = hem_host_str_leg(args, mx, torch, np, workloads)
        if "peel_r" in legs:
            side["peel_r"] = peel_r_leg(args, mx, torch)
        if "footprint" in legs:
            side["footprint"] = footprint_leg(mx, torch)
        print(json.dumps(side), flush=True)
        return 0

    # ---- inputs, generated on the device before timing --------------------------------------
    # The device memory allocator places the ~270 GB of keys and workspace in one of two physical layouts, on
    # some boxes alternating from one full allocation to the next; in one of them the random-
    # access phases (apply, the record build) run about 20 % slower.  Unless
    # --no-placement-probe, one build is timed in each of --placement-tries allocations
    # (everything released and allocated again in between), then in up to two more until the
    # last is within 2 % of the best seen; the timed steps run on that last allocation and the
    # probe times are reported.  The timed steps are the same builds either way.
    P = mx.part_size(n, gamma)
    m = 3 * P
    kind = mx.KEYS_U64 if cfg["kind"] == "u64" else mx.KEYS_STR
    qtab = None if kind == mx.KEYS_U64 else torch.from_numpy(workloads.quantile_table().view(np.int16)).to(dev)
    bufs = {}

    def allocate():
        t0 = time.perf_counter()
        if kind == mx.KEYS_U64:
            bufs["keys"] = mx.gen_keys_u64(n, gen_seed=0, device=dev)
        else:
            bufs["data"], bufs["offs"] = mx.gen_str_keys(n, qtab, gen_seed=0, device=dev)
        bufs["ws"] = torch.empty(mx.mphf_workspace_bytes(n, gamma, kind), dtype=torch.uint8, device=dev)
        bufs["codes"] = torch.empty(max((m + 31) // 32, 1), dtype=torch.int64, device=dev)
        bufs["rank"] = torch.empty(max((m + 511) // 512, 1), dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def build_once():
        out = (bufs["codes"], bufs["rank"])
        if kind == mx.KEYS_U64:
            return mx.mphf_build_u64(bufs["keys"], seed=0, gamma=gamma, ws=bufs["ws"], out=out)
        return mx.mphf_build_str(bufs["data"], bufs["offs"], seed=0, gamma=gamma, ws=bufs["ws"], out=out)

    def probe_ms():  # apply + build phase time of one build
        mx.phase_times(reset=True)
        build_once()
        torch.cuda.synchronize()
        ph = mx.phase_times(reset=True)
        return ph["apply"][0] + ph["build"][0]

    mx.set_option("timing", 1)
    t_alloc = allocate()
    placement = None
    if not args.no_placement_probe:
        tries = [probe_ms()]
        while need_another_allocation(tries, args.placement_tries):
            bufs.clear()
            torch.cuda.empty_cache()
            allocate()
            tries.append(probe_ms())
        placement = dict(apply_build_ms=[round(x, 1) for x in tries], allocations=len(tries),
                         note="one build per allocation; the timed steps use the last one")
        log(f"[bench] placement probe: apply + build {', '.join(f'{x:.1f}' for x in tries)} ms "
            f"over {len(tries)} allocations")
    keys, data, offs = bufs.get("keys"), bufs.get("data"), bufs.get("offs")
    ws, codes, rank = bufs["ws"], bufs["codes"], bufs["rank"]
    bufs.clear()
    key_bytes = 8 * n if kind == mx.KEYS_U64 else int(offs[-1].item())
    log(f"[bench] {cfg['workload']} n={n}: keys generated on device in {t_alloc:.1f} s with the workspace "
        f"({key_bytes / 1e9:.2f} GB of key bytes); workspace {ws.numel() / 1e9:.2f} GB, device memory in use "
        f"{torch.cuda.memory_allocated() / 1e9:.1f} GB")

    def step():
        if kind == mx.KEYS_U64:
            return mx.mphf_build_u64(keys, seed=0, gamma=gamma, ws=ws, out=(codes, rank))
        return mx.mphf_build_str(data, offs, seed=0, gamma=gamma, ws=ws, out=(codes, rank))

    mx.set_option("timing", 1)
    for i in range(args.warmup):
        r = step()
        log(f"[bench] warmup {i}: rounds={r['n_rounds']} tries={r['tries']}")
    torch.cuda.synchronize()
    mx.phase_times(reset=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = n / (ms_per_step / 1000.0)
    phases = mx.phase_times(reset=True)
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value / 1e9:.3f} G keys/s")

    lists_from = mx.get_option("claim_lists")
    st = dict(n=n, m=m, kind=cfg["kind"], key_bytes=key_bytes, frontier_total=r["frontier_total"],
              frontier0=r["frontier0"], claims=r["claims"], lists=lists_from > 0 and n >= (1 << lists_from),
              round0_updates=mx.get_option("update_lists") > 0, layer0=r["layer0"],
              update_deletes=r["update_deletes"], update_records=r["update_records"])
    phase_rows = {}
    for name, (ms, launches) in phases.items():
        if launches == 0:
            continue
        per_step_ms = ms / args.steps
        b = algorithmic_bytes(name, st)
        gbs = b / (per_step_ms / 1000.0) / 1e9 if per_step_ms > 0 else 0.0
        phase_rows[name] = dict(ms=round(per_step_ms, 3), launches=launches // args.steps,
                                alg_bytes=int(b), alg_GBps=round(gbs, 1))
        log(f"[bench]   {name:10s} {per_step_ms:9.3f} ms/step  {launches // args.steps:5d} launches  "
            f"{b / 1e9:8.2f} GB alg  {gbs:8.1f} GB/s")
    # the dominant kernel: the phase with the most time among those the model prices
    priced = {k: v for k, v in phase_rows.items() if v["alg_bytes"] > 0}
    dom = max(priced, key=lambda k: priced[k]["ms"])
    traffic = counters_traffic(cfg["workload"], dom) if n == cfg["n"] else None
    roofline = kernel_roofline(dom, phase_rows[dom], traffic)
    log(f"[bench] dominant kernel {dom}: {roofline['alg_bytes_per_launch'] / 1e9:.3f} GB/launch over "
        f"{roofline['launch_avg_us']:.1f} us = {roofline['achieved']:.1f} GB/s ({roofline['frac']:.4f} of peak)")
    peel = peel_roofline(phase_rows, counters_peel_traffic(cfg["workload"]) if n == cfg["n"] else None, n)
    log(f"[bench] peel alone: {peel['ms']:.1f} ms, model {peel['alg_frac']} of peak, counted {peel['traffic_frac']} "
        f"of peak (amplification {peel['amplification']})")
    # the whole step: every phase's algorithmic bytes, and the counted HBM bytes of one build,
    # over the step time (host gaps included)
    step_alg = sum(v["alg_bytes"] for v in phase_rows.values())
    step = dict(alg_bytes=int(step_alg), alg_GBps=round(step_alg / (ms_per_step / 1e3) / 1e9, 1),
                alg_frac=round(step_alg / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4), peak=HBM_PEAK_GBS,
                unit="GB/s", traffic=None, traffic_GBps=None, traffic_frac=None)
    step_traffic = counters_step_traffic(cfg["workload"]) if n == cfg["n"] else None
    if step_traffic is not None:
        t_gbs = step_traffic / (ms_per_step / 1e3) / 1e9
        step.update(traffic=round(step_traffic), traffic_GBps=round(t_gbs, 1), traffic_frac=round(t_gbs / HBM_PEAK_GBS, 4),
                    traffic_vs_copy=round(t_gbs / ceilings["copy_GBps"], 3) if ceilings else None,
                    amplification=round(step_traffic / step_alg, 2) if step_alg else None)
    log(f"[bench] step: {step['alg_GBps']:.1f} GB/s algorithmic ({step['alg_frac']:.3f} of peak), counted "
        f"{step['traffic_GBps']} GB/s ({step['traffic_frac']} of peak)")
    # the dominant phase against the measured ceilings of the random operations it is made of:
    # each class's rate over the phase time, against the probe's rate for that class alone
    ops = random_ops(dom, st)
    if ceilings and ops:
        sec = phase_rows[dom]["ms"] / 1e3
        classes = {"atomics": ("atomic_add_ret_Gops", "returning 8-byte atomics"),
                   "loads": ("load8_Gops", "8-byte gathers"), "stores": ("store1_Gops", "1-byte scattered stores")}
        per = {}
        for k, (ck, what) in classes.items():
            if ops.get(k):
                ach_ops = ops[k] / sec / 1e9
                per[k] = dict(what=what, per_step=int(ops[k]), achieved=round(ach_ops, 2), peak=ceilings[ck],
                              unit="G/s", frac=round(ach_ops / ceilings[ck], 3))
        if per:
            top = max(per.values(), key=lambda x: x["frac"])
            roofline["secondary"] = dict(bound="random device-memory operations: " + top["what"],
                                         achieved=top["achieved"], peak=top["peak"], unit="G/s", frac=top["frac"],
                                         classes=per,
                                         note="peaks = the probe kernels' rates over a 16 GiB table, each class "
                                              "alone; the phase runs its classes concurrently")

    # ---- oracle on a bounded sample of the same workload ------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        o = oracle.Oracle()
        ns = min(args.cpu_sample, n)
        if cfg["kind"] == "u64":
            hk = workloads.u64_keys(ns)
            c0 = time.perf_counter()
            rc, _ = o.mphf_build_u64(hk, seed=0)
        else:
            hd, ho = workloads.str_keys(ns)
            c0 = time.perf_counter()
            rc, _ = o.mphf_build_str(hd, ho, seed=0)
        cs = time.perf_counter() - c0
        cpu = dict(value=round(ns / cs, 1), unit="keys/s", cores=1, kind="oracle",
                   sample=f"first {ns} keys of the same generator, single-threaded C oracle, "
                          f"{cs:.1f} s (status {rc})", **host_cpu())
        log(f"[bench] oracle: {ns} keys in {cs:.2f} s = {ns / cs / 1e6:.3f} M keys/s")

    lookup = None
    if "lookup" in legs:
        lookup = lookup_leg(mx, torch, r, n, kind, keys=keys if kind == mx.KEYS_U64 else None,
                            data=None if kind == mx.KEYS_U64 else data,
                            offs=None if kind == mx.KEYS_U64 else offs, ceilings=ceilings)

    sf = None
    if "sf" in legs:  # the MPHF's tables go; its counts stay for the headline line
        r = {k: v for k, v in r.items() if not isinstance(v, torch.Tensor)}
        del codes, rank
        codes = rank = None
        torch.cuda.empty_cache()
        sf = sf_leg(args, mx, torch, n, kind, ws, keys=keys if kind == mx.KEYS_U64 else None,
                    data=None if kind == mx.KEYS_U64 else data, offs=None if kind == mx.KEYS_U64 else offs)

    del ws, codes, rank
    torch.cuda.empty_cache()
    hem = None
    if "hem" in legs:
        hem = hem_leg(args, mx, torch, n, kind, keys=keys if kind == mx.KEYS_U64 else None,
                      data=None if kind == mx.KEYS_U64 else data, offs=None if kind == mx.KEYS_U64 else offs)
    if cfg["kind"] == "u64":
        del keys
    else:
        del data, offs
    torch.cuda.empty_cache()
    # the batched and served legs read no phase times: no per-launch event pairs (they would
    # slow the plain builds that serve as their comparators and the server's workers)
    mx.set_option("timing", 0)
    batched = batched_leg(args, mx, torch, np, workloads) if "batched" in legs else None
    served = served_leg(args, mx, torch, np, workloads) if "served" in legs else None
    hem_host = hem_host_leg(args, mx, torch) if "hem_host" in legs else None
    stream = stream_leg(args, mx, torch) if "stream" in legs else None

    out = {
        "metric": "edges peeled/s (hash+peel+assign+rank), plain single-hypergraph build",
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": cfg["workload"], "n": n, "gamma": "123/100", "m": m,
                   "key_bytes": key_bytes, "rounds": r["n_rounds"], "tries": r["tries"],
                   "parallelism": "single GPU", **({"options": options} if options else {}),
                   **({"placement": placement} if placement else {})},
        "roofline": roofline,
        "peel_roofline": peel,
        "step_roofline": step,
        "cpu_baseline": cpu,
        "ceilings": ceilings,
        "phases": phase_rows,
        "lookup": lookup,
        "static_function": sf,
        "hem": hem,
        "batched": batched,
        "served": served,
        "hem_host": hem_host,
        "stream": stream,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
