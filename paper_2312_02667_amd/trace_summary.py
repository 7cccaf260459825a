"""Summaries of rocprofv3 output for the layer benchmark (``bench.py``), printed as the
markdown tables kept with each profile.

``trace``: per-kernel statistics of a ``--kernel-trace`` CSV, and the timed region (the
layers after the set-up ones, found by counting theta dispatches: each layer of N = 1024 runs
as two halves, two theta dispatches) with the union of each kernel class's dispatch intervals
set against the event timing that ``bench.py`` printed for the same run.

``counters``: rocprofv3's MFMA utilisation (MFMA busy cycles over active cycles) and the
instruction mix of the timed Jacobi and theta dispatches from one ``--pmc`` pass.

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


COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_F64",
            "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU", "SQ_INSTS_MFMA",
            "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE")


def cmd_counters(a) -> None:
    """MFMA utilisation and instruction mix of the timed Jacobi and theta dispatches from one
    --pmc pass (the profiler serializes dispatches while it counts, so each dispatch ran
    alone).  GRBM_GUI_ACTIVE is summed over the XCDs, so one XCD's active cycles are its sum
    over xcds; MFMA utilisation is the busy cycles summed over the SIMDs over (active cycles x
    SIMDs), rocprofv3's MfmaUtil."""
    per = defaultdict(dict)
    names = {}
    for r in csv.DictReader(open(a.csv)):
        d = int(r["Dispatch_Id"])
        per[d][r["Counter_Name"]] = float(r["Counter_Value"])
        names[d] = (short_name(r["Kernel_Name"]), int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
    theta_ids = sorted(d for d, n in names.items() if n[0] == f"theta_kernel<{CTYPE[a.precision]}>")
    t0 = theta_ids[2 * a.setup_layers]
    mops = "SQ_INSTS_VALU_MFMA_MOPS_F32" if a.precision == "fp32" else "SQ_INSTS_VALU_MFMA_MOPS_F64"
    print("| kernel (timed dispatches) | dispatches | MFMA flops issued | MFMA busy (MfmaUtil) | "
          "issued MFMA rate | VALU per MFMA | LDS per MFMA | LDS bank conflict cycles / active |")
    print("|---|---|---|---|---|---|---|---|")
    peak = 157.3e12 if a.precision == "fp32" else 78.6e12
    for label, pick in (("jacobi_round", lambda n: is_jacobi(n, a.precision)),
                        ("theta", lambda n: n == f"theta_kernel<{CTYPE[a.precision]}>")):
        ids = [d for d in per if d >= t0 and pick(names[d][0])]
        if not ids:
            continue
        tot = defaultdict(float)
        ns = 0
        for d in ids:
            for c, v in per[d].items():
                tot[c] += v
            ns += names[d][2] - names[d][1]
        flops = 512.0 * tot[mops]
        active = tot["GRBM_GUI_ACTIVE"] / a.xcds
        util = tot["SQ_VALU_MFMA_BUSY_CYCLES"] / (active * a.simds) if active else float("nan")
        rate = flops / (ns * 1e-9) if ns else float("nan")
        mf = tot["SQ_INSTS_MFMA"] or float("nan")
        lds_act = tot["SQ_LDS_IDX_ACTIVE"]
        conf = tot["SQ_LDS_BANK_CONFLICT"] / lds_act if lds_act else float("nan")
        print(f"| {label} | {len(ids)} | {flops:.4e} | {util:.3f} | {rate / 1e12:.1f} TFLOP/s "
              f"({rate / peak:.3f} of peak) | {tot['SQ_INSTS_VALU'] / mf:.1f} | "
              f"{tot['SQ_INSTS_LDS'] / mf:.2f} | {conf:.3f} |")
    print()
    print(f"Dispatch durations from the counter pass's own timestamps; active cycles per XCD "
          f"over the summed durations give a clock of "
          f"{sum(per[d].get('GRBM_GUI_ACTIVE', 0) for d in per if d >= t0) / a.xcds / max(1, sum(names[d][2] - names[d][1] for d in per if d >= t0)):.2f} GHz.")


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
    c = sub.add_parser("counters")
    c.add_argument("--csv", required=True)
    c.add_argument("--precision", default="fp32", choices=list(CTYPE))
    c.add_argument("--setup-layers", type=int, default=9)
    c.add_argument("--xcds", type=int, default=8)
    c.add_argument("--simds", type=int, default=1024)
    a = p.parse_args(argv)
    {"trace": cmd_trace, "traffic": cmd_traffic, "counters": cmd_counters}[a.cmd](a)


if __name__ == "__main__":
    main()
