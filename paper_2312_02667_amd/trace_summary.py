"""Summaries of rocprofv3 output for the layer benchmark (``bench.py``), printed as the
markdown tables kept with each profile.

``trace``: per-kernel statistics of a ``--kernel-trace`` CSV, and the timed region (the
layers after the set-up ones, found by counting theta dispatches: each layer of N = 1024 runs
as two halves, two theta dispatches) with the union of each kernel class's dispatch intervals
set against the event timing that ``bench.py`` printed for the same run.

``traffic``: HBM bytes per Jacobi launch from two ``--pmc`` runs (FETCH_SIZE, WRITE_SIZE, KiB
per dispatch), each scaled by what the same counter read for ``hbm_copy_kernel`` (bench's
``--copy-calibration MIB``: MIB MiB read and MIB MiB written per dispatch).  A launch is what
``bench.py`` counts as one: a Jacobi round over all gates of the layer, i.e. two half-batch
dispatches.

    python -m paper_2312_02667_amd.trace_summary trace --csv T.csv --bench B.json \
        --precision fp32 --setup-layers 9 [--breakdown]
    python -m paper_2312_02667_amd.trace_summary traffic --fetch F.csv --write W.csv \
        --bench B.json --precision fp32 --setup-layers 9 --copy-mib 256
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources the Jacobi round kernels are built from: a counter summary is valid for the
# build whose digest it records
KERNEL_SOURCES = ("ptebd_kernels.hip", "ptebd_jacobi64.hip", "ptebd_device.h",
                  "ptebd_internal.h")
CTYPE = {"fp32": "float", "fp64": "double"}
PRECOND = ("colsort_kernel", "gram64_kernel", "potrf_kernel", "trsm_kernel", "herk_kernel",
           "xinit_kernel", "yhat_kernel", "ugemm_kernel")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def short_name(full: str) -> str:
    m = re.search(r"(\w+_kernel)(<\w+>)?\(", full)
    if m:
        return m.group(1) + (m.group(2) or "")
    return full.split("(")[0][:60]


def load_bench(path: str) -> dict:
    """The JSON line bench.py printed (the last line starting with '{')."""
    line = None
    with open(path) as f:
        for ln in f:
            if ln.startswith("{"):
                line = ln
    if line is None:
        raise SystemExit(f"no JSON line in {path}")
    return json.loads(line)


def union_ms(intervals) -> float:
    total, lo, hi = 0, None, None
    for a, b in sorted(intervals):
        if hi is None or a > hi:
            if hi is not None:
                total += hi - lo
            lo, hi = a, b
        elif b > hi:
            hi = b
    if hi is not None:
        total += hi - lo
    return total / 1e6


def timed_start(rows, precision: str, setup_layers: int, key_start) -> int:
    theta = sorted(key_start(r) for r in rows if short_name(r["Kernel_Name"]) ==
                   f"theta_kernel<{CTYPE[precision]}>")
    idx = 2 * setup_layers
    if len(theta) <= idx:
        raise SystemExit(f"{len(theta)} theta dispatches, fewer than 2 x {setup_layers} + 1")
    return theta[idx]


def is_jacobi(name: str, precision: str) -> bool:
    return name in (f"jacobi_round_kernel<{CTYPE[precision]}>", "jacobi64_round_kernel")


def cmd_trace(a) -> None:
    rows = list(csv.DictReader(open(a.csv)))
    bench = load_bench(a.bench)
    stats = defaultdict(lambda: {"calls": 0, "ns": 0, "lds": 0, "vgpr": 0, "grid": ""})
    for r in rows:
        s = stats[short_name(r["Kernel_Name"])]
        s["calls"] += 1
        s["ns"] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        s["lds"] = int(r["LDS_Block_Size"])
        s["vgpr"] = int(r["VGPR_Count"])
        s["grid"] = f"{r['Grid_Size_X']}x{r['Grid_Size_Y']}"
    print("| kernel | calls | total ms | avg us | LDS B | VGPRs | grid (threads) |")
    print("|---|---|---|---|---|---|---|")
    for name, s in sorted(stats.items(), key=lambda kv: -kv[1]["ns"])[: a.top]:
        print(f"| {name} | {s['calls']} | {s['ns'] / 1e6:.2f} | {s['ns'] / 1e3 / s['calls']:.1f} "
              f"| {s['lds']} | {s['vgpr']} | {s['grid']} |")
    t0 = timed_start(rows, a.precision, a.setup_layers, lambda r: int(r["Start_Timestamp"]))
    # the timed layers end with the last write-back (queries after them are not timed)
    t1 = max(int(r["End_Timestamp"]) for r in rows
             if short_name(r["Kernel_Name"]).startswith("writeback_kernel"))
    win = [r for r in rows if t0 <= int(r["Start_Timestamp"]) < t1]
    span = (t1 - t0) / 1e6
    cls = defaultdict(list)
    for r in win:
        n = short_name(r["Kernel_Name"])
        base = n.split("<")[0]
        if is_jacobi(n, a.precision):
            key = "jacobi"
        elif base in PRECOND:
            key = "precond"
        elif base in ("theta_kernel", "finalize_kernel", "writeback_kernel",
                      "sweep_check_kernel", "jacobi_init_kernel"):
            key = base.replace("_kernel", "")
        else:
            key = "other"
        cls[key].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    steps = bench["steps"]
    print()
    print(f"Timed region: {steps} layers, {span:.1f} ms from the first timed theta dispatch to "
          f"the end of the last write-back ({span / steps:.2f} ms per layer; bench.py's ms_per_step "
          f"{bench['ms_per_step']:.2f}).")
    print()
    print("| class | dispatches | busy ms (sum) | union ms | union / span |")
    print("|---|---|---|---|---|")
    for key in ("theta", "precond", "jacobi_init", "jacobi", "sweep_check", "finalize",
                "writeback", "other"):
        iv = cls.get(key, [])
        if not iv:
            continue
        busy = sum(b - x for x, b in iv) / 1e6
        u = union_ms(iv)
        print(f"| {key} | {len(iv)} | {busy:.2f} | {u:.2f} | {u / span:.3f} |")
    if a.breakdown:
        breakdown(win, t0, t1, span)
    jac = bench["kernels"]["jacobi"]
    u = union_ms(cls["jacobi"])
    launches = jac["launches"]
    print()
    print(f"Jacobi rounds: bench.py counts {launches} launches (a round over all gates, two "
          f"half-batch dispatches; sweeps queued past convergence, whose dispatches exit at "
          f"once, are not counted) in {jac['total_ms']:.2f} ms of event time, "
          f"{jac['total_ms'] / launches:.4f} ms per launch.  The trace: {len(cls['jacobi'])} "
          f"dispatches, union {u:.2f} ms, {u / launches:.4f} ms per counted launch "
          f"({100 * (u / jac['total_ms'] - 1):+.1f} % against the events).")


def breakdown(win, t0: int, t1: int, span: float) -> None:
    """Per-kernel unions over the timed region, and how long 0, 1, 2 or more dispatches ran
    at once (a sweep of the dispatch start and end events)."""
    per = defaultdict(list)
    for r in win:
        per[short_name(r["Kernel_Name"]).split("<")[0]].append(
            (int(r["Start_Timestamp"]), min(int(r["End_Timestamp"]), t1)))
    print()
    print("| kernel | dispatches | busy ms (sum) | union ms | union / span |")
    print("|---|---|---|---|---|")
    for name, iv in sorted(per.items(), key=lambda kv: -union_ms(kv[1])):
        busy = sum(b - x for x, b in iv) / 1e6
        u = union_ms(iv)
        print(f"| {name} | {len(iv)} | {busy:.2f} | {u:.2f} | {100 * u / span:.1f} % |")
    ev = []
    for iv in per.values():
        for x, b in iv:
            ev.append((x, 1))
            ev.append((b, -1))
    ev.sort()
    at = defaultdict(int)
    depth, last = 0, t0
    for t, d in ev:
        at[min(depth, 2)] += t - last
        depth += d
        last = t
    at[0] += t1 - last
    no_jac = span - union_ms(per.get("jacobi_round_kernel", []) +
                             per.get("jacobi64_round_kernel", []))
    print()
    print(f"Two or more dispatches run at once during {at[2] / 1e6:.1f} ms "
          f"({100 * at[2] / 1e6 / span:.1f} %), one during {at[1] / 1e6:.1f} ms, none during "
          f"{at[0] / 1e6:.1f} ms; no Jacobi round runs during {no_jac:.1f} ms.")


def counter_rows(path: str, counter: str):
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out.append(r)
    return out


def cmd_traffic(a) -> None:
    bench = load_bench(a.bench)
    res = {}
    for counter, path in (("FETCH_SIZE", a.fetch), ("WRITE_SIZE", a.write)):
        rows = counter_rows(path, counter)
        cal = [float(r["Counter_Value"]) for r in rows
               if short_name(r["Kernel_Name"]) == "hbm_copy_kernel"]
        if not cal:
            raise SystemExit(f"no hbm_copy_kernel dispatch in {path}")
        expect_kib = a.copy_mib * 1024.0
        scale = expect_kib / (sum(cal) / len(cal))
        t0 = timed_start(rows, a.precision, a.setup_layers, lambda r: int(r["Dispatch_Id"]))
        jac = [float(r["Counter_Value"]) for r in rows if int(r["Dispatch_Id"]) >= t0 and
               is_jacobi(short_name(r["Kernel_Name"]), a.precision)]
        theta = [float(r["Counter_Value"]) for r in rows if int(r["Dispatch_Id"]) >= t0 and
                 short_name(r["Kernel_Name"]) == f"theta_kernel<{CTYPE[a.precision]}>"]
        res[counter] = {"cal_kib": sum(cal) / len(cal), "scale": scale, "n": len(jac),
                        "bytes": 1024.0 * scale * sum(jac),
                        "theta_bytes": 1024.0 * scale * sum(theta), "n_theta": len(theta)}
    jk = bench["kernels"]["jacobi"]
    launches = jk["launches"]
    alg = jk["bytes"] / launches
    rd = res["FETCH_SIZE"]["bytes"] / launches
    wr = res["WRITE_SIZE"]["bytes"] / launches
    tk = bench["kernels"]["theta"]
    t_alg = tk["bytes"]
    t_hbm = res["FETCH_SIZE"]["theta_bytes"] + res["WRITE_SIZE"]["theta_bytes"]
    print(f"kernel_source_sha256: {kernel_source_digest()}")
    print(f"hbm_bytes_per_launch: {rd + wr:.6e}")
    print()
    print("| quantity | value |")
    print("|---|---|")
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        print(f"| calibration: {c} of one {a.copy_mib} MiB copy | {res[c]['cal_kib']:.0f} KiB "
              f"(scale factor {res[c]['scale']:.4f}) |")
    print(f"| Jacobi dispatches in the timed layers | {res['FETCH_SIZE']['n']} |")
    print(f"| launches counted by bench.py | {launches} |")
    print(f"| HBM read per launch (scaled) | {rd:.4e} B |")
    print(f"| HBM write per launch (scaled) | {wr:.4e} B |")
    print(f"| algorithmic bytes per launch (bench.py: the executed rounds' Gram reads and "
          f"rotation reads and writes) | {alg:.4e} B |")
    print(f"| traffic / algorithmic | {(rd + wr) / alg:.3f} |")
    print(f"| theta, {res['FETCH_SIZE']['n_theta']} timed dispatches | {t_hbm:.4e} B "
          f"({t_hbm / t_alg:.2f}x its {t_alg:.4e} algorithmic bytes) |")


def main(argv=None) -> None:
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = p.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--csv", required=True)
    t.add_argument("--bench", required=True)
    t.add_argument("--precision", default="fp32", choices=list(CTYPE))
    t.add_argument("--setup-layers", type=int, default=9)
    t.add_argument("--top", type=int, default=16)
    t.add_argument("--breakdown", action="store_true",
                   help="also per-kernel unions and concurrency over the timed region")
    w = sub.add_parser("traffic")
    w.add_argument("--fetch", required=True)
    w.add_argument("--write", required=True)
    w.add_argument("--bench", required=True)
    w.add_argument("--precision", default="fp32", choices=list(CTYPE))
    w.add_argument("--setup-layers", type=int, default=9)
    w.add_argument("--copy-mib", type=int, default=256)
    a = p.parse_args(argv)
    cmd_trace(a) if a.cmd == "trace" else cmd_traffic(a)


if __name__ == "__main__":
    main()
