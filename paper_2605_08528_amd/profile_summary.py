"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2605_08528_amd.profile_summary trace KERNEL_TRACE_CSV [--workgroups N]
    python -m paper_2605_08528_amd.profile_summary counters COUNTER_CSV [--last K]
    python -m paper_2605_08528_amd.profile_summary window KERNEL_TRACE_CSV --kernel NAME [--n 20]

``trace`` reads a ``--kernel-trace --output-format csv`` file and prints, per
kernel and launch size (workgroups), the dispatch count and the mean and
percentiles of the dispatch durations.  Dispatches of the step and
observation kernels that are followed by the road-touch counting kernel
belong to a counting pass (atomics on) and are listed apart.

``counters`` reads a ``--pmc ... --output-format csv`` counter collection and
prints, per kernel and launch size, the mean of each counter over the last
K dispatches.

``window`` prints the durations of the dispatches of one kernel that
precede its first counting pass: in bench.py's run, the first seed's
profiled eager pass, whose HIP-event mean the roofline uses.

``traffic`` reads the FETCH_SIZE and WRITE_SIZE collections of
profile_workload (two runs), scales each counter by what it reads for the
256 MiB device copy at the start of that run, and writes (``--out``) the
per-launch HBM bytes (mean over each launch's last K dispatches at the
workload's size) with the hash of the sources each kernel is built from;
bench.py reports them while that hash still matches.
"""
from __future__ import annotations

import argparse
import collections
import csv
import re

import numpy as np


def short_name(name: str) -> str:
    """Kernel name without its argument list (templates kept)."""
    n = re.sub(r"^void ", "", name)
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def trace_table(path: str, workgroups: int | None = None):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [short_name(r["Kernel_Name"]) for r in rows]
    groups = collections.defaultdict(list)
    for i, r in enumerate(rows):
        wg = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        if workgroups is not None and wg != workgroups:
            continue
        touched = i + 1 < len(rows) and names[i + 1] == "k_touch_count"
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        groups[(names[i], wg, touched)].append(us)
    out = []
    for (name, wg, touched), v in groups.items():
        a = np.array(v)
        out.append({"kernel": name, "workgroups": wg, "counting_pass": touched, "n": len(a),
                    "mean_us": float(a.mean()), "p10_us": float(np.percentile(a, 10)),
                    "p50_us": float(np.percentile(a, 50)), "p90_us": float(np.percentile(a, 90)),
                    "total_ms": float(a.sum() * 1e-3)})
    out.sort(key=lambda d: -d["total_ms"])
    return out


def before_counting(path: str, kernel: str, workgroups: int, n: int):
    """Durations (us) of the last `n` dispatches of `kernel` at `workgroups`
    that precede its first road-touch counting pass: in bench.py's sequence
    these are the dispatches of the first seed's profiled eager pass, whose
    HIP-event mean is the roofline's kernel time."""
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [short_name(r["Kernel_Name"]) for r in rows]
    seen = []
    for i, r in enumerate(rows):
        if names[i] != kernel or int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"])) != workgroups:
            continue
        if i + 1 < len(rows) and names[i + 1] == "k_touch_count":
            break
        seen.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    return np.array(seen[-n:])


def counter_table(path: str, last: int = 20):
    rows = list(csv.DictReader(open(path)))
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    order = collections.defaultdict(list)
    for r in rows:
        name = short_name(r["Kernel_Name"])
        wg = int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"])) if "Grid_Size" in r else -1
        key = (name, wg)
        did = int(r.get("Dispatch_Id", 0))
        per[key][r["Counter_Name"]].append((did, float(r["Counter_Value"])))
        order[key].append(did)
    out = []
    for key, ctrs in per.items():
        ids = sorted(set(order[key]))[-last:]
        keep = set(ids)
        vals = {}
        for cname, pairs in ctrs.items():
            sums = collections.defaultdict(float)
            for did, v in pairs:
                if did in keep:
                    sums[did] += v           # per-dispatch sum over dimension instances
            vals[cname] = float(np.mean(list(sums.values()))) if sums else float("nan")
        out.append({"kernel": key[0], "workgroups": key[1], "dispatches": len(ids), **vals})
    out.sort(key=lambda d: (d["kernel"], d["workgroups"]))
    return out


KERNEL_SOURCES = {"k_obs": ("k_obs.hip",), "k_step": ("k_step.hip",), "k_policy": ("k_policy.hip",),
                  "k_full": ("k_full.hip", "ac_layout.h"), "k_ppo": ("k_ppo.hip", "ac_layout.h")}


def kernel_family(launch: str) -> str:
    """Source family of a launch name: k_obs_policy and k_obs<...> come from
    k_obs.hip, k_step<...> from k_step.hip, and so on."""
    if launch.startswith("k_obs_full") or launch.startswith("k_actor_critic"):
        return "k_full"
    if launch.startswith("k_ppo"):
        return "k_ppo"
    for fam in ("k_obs", "k_step", "k_policy"):
        if launch.startswith(fam):
            return fam
    return ""


def kernel_source_hash(family: str) -> str:
    """Hash of the sources a kernel family is built from (its .hip file, the
    layout header it reads and the shared device header; the host-side launch
    declarations are not part of it)."""
    import hashlib
    import os
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family] + ("sf_dev.h",):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


COPY_BYTES = 256 * 2 ** 20


def copy_scale(path: str, counter: str) -> float:
    """Bytes per counter KiB: the 256 MiB copy (the run's first dispatch, a
    copyBuffer) against the counter's reading for it."""
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    first = min(int(r["Dispatch_Id"]) for r in rows)
    kib = sum(float(r["Counter_Value"]) for r in rows if int(r["Dispatch_Id"]) == first)
    return COPY_BYTES / 1024.0 / kib


def traffic_record(fetch_csv: str, write_csv: str, agents: int, last: int = 20):
    fs, ws = copy_scale(fetch_csv, "FETCH_SIZE"), copy_scale(write_csv, "WRITE_SIZE")
    f = {(d["kernel"], d["workgroups"]): d for d in counter_table(fetch_csv, last)}
    w = {(d["kernel"], d["workgroups"]): d for d in counter_table(write_csv, last)}
    out = {"fetch_scale": fs, "write_scale": ws, "copy_bytes": COPY_BYTES, "last_dispatches": last,
           "launches": {}}
    for key, d in f.items():
        fam = kernel_family(key[0])
        if not fam or key not in w:
            continue
        # the workload's launches: one workgroup per world, per 16 agents, or per agent
        name = key[0]
        prev = out["launches"].get(name)
        rec = {"kernel": fam, "workgroups": key[1], "fetch_kib": d["FETCH_SIZE"], "write_kib": w[key]["WRITE_SIZE"],
               "dispatches": d["dispatches"], "agents": agents, "source_hash": kernel_source_hash(fam)}
        if prev is None or rec["dispatches"] > prev["dispatches"]:
            out["launches"][name] = rec
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "counters", "window", "traffic"])
    ap.add_argument("--write-csv", default=None)
    ap.add_argument("--agents", type=int, default=4096)
    ap.add_argument("--out", default=None)
    ap.add_argument("--kernel", default="k_step<192, false>")
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("csv")
    ap.add_argument("--workgroups", type=int, default=None)
    ap.add_argument("--last", type=int, default=20)
    ap.add_argument("--min-total-ms", type=float, default=0.0)
    args = ap.parse_args()
    if args.mode == "trace":
        print(f"{'kernel':34s} {'wgs':>6s} {'count':>5s} {'n':>6s} {'mean us':>9s} {'p10':>8s} "
              f"{'p50':>8s} {'p90':>8s} {'total ms':>9s}")
        for d in trace_table(args.csv, args.workgroups):
            if d["total_ms"] < args.min_total_ms:
                continue
            print(f"{d['kernel']:34s} {d['workgroups']:6d} {'yes' if d['counting_pass'] else 'no':>5s} "
                  f"{d['n']:6d} {d['mean_us']:9.2f} {d['p10_us']:8.2f} {d['p50_us']:8.2f} "
                  f"{d['p90_us']:8.2f} {d['total_ms']:9.2f}")
    elif args.mode == "window":
        v = before_counting(args.csv, args.kernel, args.workgroups or 256, args.n)
        print(f"{args.kernel} at {args.workgroups or 256} workgroups: the {len(v)} dispatches before the first "
              f"counting pass: mean {v.mean():.2f} us, p50 {np.percentile(v, 50):.2f}, min {v.min():.2f}, "
              f"max {v.max():.2f}")
    elif args.mode == "traffic":
        import json
        rec = traffic_record(args.csv, args.write_csv, args.agents, args.last)
        text = json.dumps(rec, indent=1)
        if args.out:
            open(args.out, "w").write(text + "\n")
        print(text)
    else:
        for d in counter_table(args.csv, args.last):
            extra = "  ".join(f"{k}={v:.4g}" for k, v in d.items() if k not in ("kernel", "workgroups", "dispatches"))
            print(f"{d['kernel']:34s} wgs={d['workgroups']:<6d} n={d['dispatches']:<4d} {extra}")


if __name__ == "__main__":
    main()
