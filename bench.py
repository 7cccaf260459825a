#!/usr/bin/env python3
"""Benchmark of the pTEBD layer on one MI355X: bond updates per second at chi = 256.

Workload: 1D brickwork random circuit, N = 1024 qubits, Haar-random SU(4) gates (seed 0),
initial state |0...0>, chi_max = 256, cutoff 1e-12, g = 0 (no PtSU, as in the paper's
timings), norm stabilization with the complement reading of eps (eps = 1 - kept sigma^2,
the reading that keeps the norm at 1 over many truncating layers; the literal reading
drives it to about 300 over these 20 layers, at the same cost).  The bulk bond dimension doubles every layer, so layers 1..9 bring the chain to
saturation (layer 9 is the first whose two-site wavefunctions are 512 x 512 and are
truncated back to 256); they are set-up, untimed.  One benchmark step is one further
brickwork layer (512 or 511 gates), every bond a 512 x 512 complex SVD truncated to 256;
``--warmup`` steps run untimed, then ``--steps`` steps are timed.  With the defaults
(warmup 1, steps 10) the circuit depth is 20.

The headline path is the mixed-precision one (FP32 contractions and Jacobi column updates,
FP64 rotation angles, singular values, eps, nu, Lambda and Lambda^{-1} divisions).  The
same workload is run on the FP64 path for the speed comparison, and the fidelity error
between the two final states is computed with the library's FP64 overlap query.  The
CPU baseline times the oracle (numpy complex128 + LAPACK) on a bounded sample of the same
bond update.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "bond updates/sec at χ=256 (mixed vs FP64 GPU) at fidelity err ≤1e-6"
EPS_READING = "complement"
PEAKS_TFLOPS = {"fp32": 157.3, "fp64": 78.6}  # dense MFMA peaks of MI355X
HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse_args(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n-sites", type=int, default=1024)
    p.add_argument("--chi", type=int, default=256)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-f1", action="store_true",
                   help="skip the canonicalize + sampling measurement")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target CPU seconds for the oracle sample")
    p.add_argument("--autotune-cache", default=os.path.join(ROOT, "paper_2312_02667_amd",
                                                              "autotune_cache.json"),
                   help="SVD schedule cache written by paper_2312_02667_amd.autotune; the entry "
                        "for the workload's shape, if any, is applied (empty: none)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="first run a plain elementwise copy kernel (MIB MiB read, MIB MiB "
                        "written) three times, a kernel of known traffic for scaling hardware "
                        "byte counters")
    return p.parse_args(argv)


def setup_layers(chi: int) -> int:
    """Layers until every bulk bond update works on a (2 chi) x (2 chi) theta."""
    return int(math.ceil(math.log2(chi))) + 1


def run_path(precision, layers, n_setup, warmup, steps, n_sites, chi, stream,
             autotune_cache=""):
    import torch

    from paper_2312_02667_amd import autotune, ptebd

    m = ptebd.MPS(n_sites, chi, precision, stream=stream)
    tuned = None
    if autotune_cache:
        key, params = autotune.apply(m, autotune_cache, chi, len(layers[-1][0]))
        tuned = {"cache": os.path.relpath(autotune_cache, ROOT), "key": key, "params": params}
        log(f"[{precision}] autotuned SVD schedule {key}: {params}")
    for i in range(n_setup + warmup):
        bonds, gates = layers[i]
        st = m.apply_layer(bonds, gates, chi_max=chi, cutoff=1e-12, eps_reading=EPS_READING)
        log(f"[{precision}] layer {i + 1} (untimed): {st['device_ms']:.1f} ms, "
            f"max sweeps {st['max_sweeps']}")
    torch.cuda.synchronize()
    m.set_profiling(True)
    n_updates = 0
    per_layer = []
    t0 = time.perf_counter()
    for i in range(n_setup + warmup, n_setup + warmup + steps):
        bonds, gates = layers[i]
        st = m.apply_layer(bonds, gates, chi_max=chi, cutoff=1e-12, eps_reading=EPS_READING)
        n_updates += len(bonds)
        per_layer.append({"layer": i + 1, "device_ms": st["device_ms"],
                          "max_sweeps": st["max_sweeps"],
                          "mean_sweeps": float(np.mean(st["sweeps"])),
                          "sum_eps": float(np.sum(st["eps"])),
                          "n_unconverged": st["n_unconverged"]})
        log(f"[{precision}] layer {i + 1} (timed): {st['device_ms']:.1f} ms, "
            f"max sweeps {st['max_sweeps']}, mean {np.mean(st['sweeps']):.2f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kstats = m.kernel_stats()
    m.set_profiling(False)
    return m, {"value": n_updates / elapsed, "elapsed_s": elapsed, "updates": n_updates,
               "ms_per_step": 1e3 * elapsed / steps, "kernels": kstats, "layers": per_layer,
               "autotune": tuned, "svd_params": m.svd_params()}


def measured_traffic(kernel_name: str, precision: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    summary, valid only while the kernel source is the one the counters were taken on."""
    import hashlib
    import re
    summary = os.path.join(ROOT, "profiles", f"{kernel_name}_{precision}_N1024_chi256.md")
    src = os.path.join(ROOT, "paper_2312_02667_amd", "csrc", "ptebd_kernels.hip")
    try:
        text = open(summary).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m_hash = re.search(r"kernel_source_sha256: ([0-9a-f]+)", text)
    m_val = re.search(r"hbm_bytes_per_launch: ([0-9.eE+-]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != digest:
        return None
    return float(m_val.group(1))


def roofline(kstats, precision):
    name = max(kstats, key=lambda k: kstats[k]["total_ms"])
    ks = kstats[name]
    secs = ks["total_ms"] / 1e3
    launches = max(ks["launches"], 1)
    if ks["flops"] > 0:
        achieved = ks["flops"] / secs / 1e12
        peak = PEAKS_TFLOPS[precision]
        out = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
               "frac": achieved / peak}
    else:
        achieved = ks["bytes"] / secs / 1e9
        out = {"bound": "hbm", "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s",
               "frac": achieved / HBM_GBS}
    traffic = measured_traffic("jacobi_round", precision) if name == "jacobi" else None
    if name == "jacobi" and "frac" in out:
        # the Jacobi kernel forms each complex product with three real MFMA products, so the
        # MFMA units execute three quarters of the algorithmic (8 per complex multiply-add) flops
        out["mfma_issued_frac"] = 0.75 * out["frac"]
    out.update({"traffic": traffic, "kernel": name, "launches": ks["launches"],
                "avg_launch_ms": ks["total_ms"] / launches,
                "flops_per_launch": ks["flops"] / launches,
                "bytes_per_launch": ks["bytes"] / launches})
    return out


def cpu_baseline(chi: int, seconds: float):
    """The oracle's bond update timed on a bounded sample of saturated chi bonds."""
    from oracle import ptebd_oracle as po
    from paper_2312_02667_amd import inputs

    n = 2 * int(math.ceil(math.log2(chi))) + 8
    g, l = inputs.random_vidal_state(n, chi, seed=1)
    base = po.VidalMPS(g, l)
    full = [q for q in range(n - 1)
            if len(base.lam[q]) == len(base.lam[q + 1]) == len(base.lam[q + 2]) == chi]
    rng = np.random.default_rng(7)
    gates = [inputs.haar_unitary(rng) for _ in range(64)]
    count = 0
    t0 = time.perf_counter()
    while True:
        q = full[count % len(full)]
        m = base.copy()
        po.bond_update(m, q, gates[count % len(gates)], chi, 1e-12, stabilize=True,
                       eps_reading=EPS_READING)
        count += 1
        el = time.perf_counter() - t0
        if el >= seconds or count >= 4096:
            break
    try:
        from threadpoolctl import threadpool_info
        threads = max([x.get("num_threads", 1) for x in threadpool_info()
                       if x.get("user_api") == "blas"] or [1])
    except Exception:  # noqa: BLE001
        threads = 1
    return {"value": count / el, "unit": "bond updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{count} bond updates of a {2 * chi}x{2 * chi} complex theta truncated to "
                      f"{chi} (numpy complex128, LAPACK gesdd, {threads} BLAS threads, "
                      f"{len(os.sched_getaffinity(0))} cores visible) on a synthetic saturated "
                      f"Vidal state, {el:.1f} s"}


def measure_f1(precision: str, n_sites: int, chi: int, depth: int, n_samples: int, seed: int):
    """The measurement step after the last layer (Algorithm 1): canonicalize a truncated
    Haar-circuit state, then draw n_samples bit strings by perfect sampling.  Returns wall
    times and the sampling kernel's achieved rate (algorithmic flops / event time)."""
    import torch

    from paper_2312_02667_amd import inputs, ptebd

    layers = inputs.brickwork_circuit(n_sites, depth, seed)
    m = ptebd.MPS(n_sites, chi, precision)
    for bonds, gates in layers:
        m.apply_layer(bonds, gates, chi_max=chi, cutoff=1e-12, eps_reading=EPS_READING)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nrm = m.canonicalize(cutoff=1e-12)
    t_can = time.perf_counter() - t0
    u = np.random.default_rng(seed + 1).random((n_samples, n_sites))
    m.sample(u[:16])                      # warm-up (buffers, code objects)
    m.set_profiling(True)
    t0 = time.perf_counter()
    bits = m.sample(u)
    t_samp = time.perf_counter() - t0
    ks = m.kernel_stats()["sample"]
    m.set_profiling(False)
    m.close()
    peak = PEAKS_TFLOPS[precision]
    ach = ks["flops"] / (ks["total_ms"] / 1e3) / 1e12 if ks["total_ms"] > 0 else 0.0
    return {"workload": f"N={n_sites} chi_max={chi} Haar SU(4) brickwork depth {depth} "
                        f"(eps reading {EPS_READING}), then canonicalize and {n_samples} "
                        f"samples",
            "canonicalize_s": t_can, "norm_before": nrm,
            "sample_s": t_samp, "samples_per_s": n_samples / t_samp,
            "sample_kernel_ms": ks["total_ms"], "sample_launches": ks["launches"],
            "sample_roofline": {"bound": "mfma", "achieved": ach, "peak": peak,
                                "unit": "TFLOP/s", "frac": ach / peak},
            "mean_bit": float(bits.mean())}


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build does not "
              f"shard the chain over several GPUs.", file=sys.stderr)
        return 2
    import torch

    from paper_2312_02667_amd import inputs

    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    if args.copy_calibration > 0:
        # an elementwise kernel that reads MIB MiB and writes MIB MiB (dst = 2 * src)
        n_el = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {args.copy_calibration} MiB read + write (torch.mul)")
        del src, dst
    chi, n = args.chi, args.n_sites
    n_setup = setup_layers(chi)
    depth = n_setup + args.warmup + args.steps
    layers = inputs.brickwork_circuit(n, depth, args.seed)
    log(f"workload N={n} chi={chi} depth={depth} (setup {n_setup}, warmup {args.warmup}, "
        f"timed {args.steps})")

    mixed_m, mixed = run_path(args.precision, layers, n_setup, args.warmup, args.steps, n, chi,
                              stream, args.autotune_cache)
    result = {
        "metric": METRIC, "value": mixed["value"], "unit": "bond updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"1D brickwork Haar-SU(4) random circuit, N={n}, chi_max={chi}, "
                               f"cutoff 1e-12, g=0, eps reading {EPS_READING}; "
                               f"step = one saturated layer "
                               f"({(n - 1 + 1) // 2} or {(n - 1) // 2} bond updates of "
                               f"{2 * chi}x{2 * chi} theta); depth {depth}",
                   "n_sites": n, "chi_max": chi, "depth": depth, "seed": args.seed,
                   "precision": args.precision},
        "roofline": roofline(mixed["kernels"], args.precision),
        "autotune": mixed["autotune"],
        "svd_params": mixed["svd_params"],
        "kernels": mixed["kernels"],
        "layers": mixed["layers"],
    }
    result["norm"] = mixed_m.norm()
    result["norm_estimate"] = mixed_m.norm_estimate()
    result["fidelity_estimate"] = mixed_m.fidelity_estimate()
    if not args.no_fp64 and args.precision != "fp64":
        f64_m, f64 = run_path("fp64", layers, n_setup, args.warmup, args.steps, n, chi, stream,
                              args.autotune_cache)
        ov = mixed_m.overlap(f64_m)
        n1, n2 = mixed_m.norm(), f64_m.norm()
        err_f = 1.0 - abs(ov) ** 2 / (n1 ** 2 * n2 ** 2)
        result["fp64_gpu"] = {"value": f64["value"], "ms_per_step": f64["ms_per_step"],
                              "roofline": roofline(f64["kernels"], "fp64"),
                              "autotune": f64["autotune"], "svd_params": f64["svd_params"],
                              "layers": f64["layers"]}
        result["speedup_vs_fp64_gpu"] = mixed["value"] / f64["value"]
        result["err_F_vs_fp64_gpu"] = err_f
        log(f"err_F(mixed vs fp64) = {err_f:.3e}")
        f64_m.close()
    if not args.no_f1:
        log("measurement step: canonicalize + perfect sampling (N=100, chi=64) ...")
        result["f1"] = measure_f1(args.precision, 100, 64, 20, 8192, args.seed)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        result["cpu_baseline"] = cpu_baseline(chi, args.cpu_seconds)
    else:
        result["cpu_baseline"] = None
    mixed_m.close()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
