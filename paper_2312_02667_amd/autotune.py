"""Autotuner for the batched SVD's tile shape and schedule, with a JSON cache.

The Jacobi SVD of a layer has per-handle controls (``ptebd_set_svd_params``): the width of
the Jacobi column blocks (16 or, on the FP32 path, 32 columns: the tile shape of the Gram and
update products and of the inner 2b x 2b eigenproblem), the number of inner sweeps per block
pair and the cosine above which another one follows, the ordering of each rotated pair's
columns by norm, the split of a large batch over two streams, and (FP32) the Cholesky
preconditioning.  Which choice is fastest depends on the shape of the work: the theta size
(twice the bond dimension) and how many gates one batch holds.  The tuner times candidate
schedules on one fixed input of that shape and keeps the fastest one that

* converges (no gate reaches the sweep cap), and
* stays within the fidelity budget: after the timed layers its state's fidelity error
  against the same layers on the FP64 path, err_F = 1 - |<a|b>|^2 / (<a|a> <b|b>), is at most
  ERR_F_TOL and at most ERR_F_SLACK times that of the default schedule (every candidate
  computes the same SVD; only the rounding path differs),

then stores it in a JSON cache keyed by precision, theta size and batch-size bucket.  The
layers use the complement eps reading, the one the benchmark runs.
``lookup`` / ``apply`` read the cache back for a handle.

The search is coordinate descent from the defaults: each control in turn takes every value
of its candidate list with the others held, and the best point found so far is kept; two
passes.  The search itself (``search``) only sees an evaluation function, so it runs without
a GPU; ``measure_schedule`` is the GPU evaluation over the C ABI, on the saturated layers of a
Haar brickwork chain (``chain_spec``) or of the lattice and batched-mix workloads
(``workload_spec``, inputs from ``workloads``).

Command line (one MI355X)::

    python -m paper_2312_02667_amd.autotune --n-sites 1024 --chi 256 --precision fp32 \\
        --cache paper_2312_02667_amd/autotune_cache.json
    python -m paper_2312_02667_amd.autotune --workload lattice
"""

from __future__ import annotations

import argparse
import json
import math
import os
import time

# The controls the tuner may move and their candidate values.  tol_factor and max_sweeps
# are accuracy controls and stay at the caller's values.
SEARCH_SPACE = {
    "block_cols": (16, 32),
    "inner_sweeps": (1, 2, 3),
    "inner_repeat": (3e-3, 1e-2, 3e-2),
    "sort_pairs": (0, 1),
    "streams": (1, 2),
    "precondition": (0, 1),
}

# A candidate's err_F against the FP64 path after the timed layers: at most ERR_F_TOL and at
# most ERR_F_SLACK times the default schedule's (plus ERR_F_FLOOR, the FP64 overlap's own
# resolution).  FP32: 1e-7 over three saturated layers keeps an 11-layer run well inside
# 1e-6; FP64 candidates are compared with the FP64 default at its rounding level.
ERR_F_TOL = {"fp32": 1e-7, "fp64": 1e-12}
ERR_F_SLACK = 4.0
ERR_F_FLOOR = 1e-13

EPS_READING = "complement"

CACHE_VERSION = 2


def cache_key(precision: str, chi: int, n_gates: int) -> str:
    """Theta of a saturated bond is (2 chi) x (2 chi); batches are bucketed by powers of 2."""
    bucket = 1 << max(0, int(math.ceil(math.log2(max(1, n_gates)))))
    return f"{precision}/theta{2 * int(chi)}/gates{bucket}"


def _space_for(precision: str) -> dict:
    space = dict(SEARCH_SPACE)
    if precision != "fp32":
        space.pop("precondition")  # the FP64 path is not preconditioned
        space.pop("block_cols")    # nor built with 32-column blocks
    return space


def _canon(params: dict, space: dict) -> tuple:
    return tuple((k, params[k]) for k in sorted(space))


def search(evaluate, defaults: dict, space: dict, passes: int = 2, min_gain: float = 0.01):
    """Coordinate descent.  ``evaluate(params) -> dict(ms=float, ok=bool, ...)``; ``ok`` is
    False for a candidate that did not converge or moved the bond weights.  A candidate
    replaces the best point only when it is faster by more than the fraction ``min_gain``
    (run-to-run noise of a layer's device time is below 1 %), so the defaults stay unless
    something is clearly better.  Returns (best_params, best_result, history) with history a
    list of (params, result)."""
    seen = {}
    history = []

    def run(p):
        key = _canon(p, space)
        if key not in seen:
            r = evaluate(dict(p))
            seen[key] = r
            history.append((dict(p), r))
        return seen[key]

    best = {k: defaults[k] for k in space}
    best_r = run(best)
    if not best_r["ok"]:
        raise RuntimeError("the default schedule itself failed the checks")
    for _ in range(passes):
        improved = False
        for name, values in space.items():
            for v in values:
                if v == best[name]:
                    continue
                cand = dict(best)
                cand[name] = v
                # inner_repeat only matters when a second inner sweep can follow
                if cand["inner_sweeps"] == 1 and name == "inner_repeat":
                    continue
                r = run(cand)
                if r["ok"] and r["ms"] < best_r["ms"] * (1.0 - min_gain):
                    best, best_r, improved = cand, r, True
        if not improved:
            break
    return best, best_r, history


def load_cache(path: str) -> dict:
    if not path or not os.path.exists(path):
        return {"version": CACHE_VERSION, "entries": {}}
    with open(path) as f:
        data = json.load(f)
    if data.get("version") != CACHE_VERSION or not isinstance(data.get("entries"), dict):
        raise ValueError(f"{path}: not an autotuner cache of version {CACHE_VERSION}")
    return data


def save_cache(path: str, data: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)


def lookup(cache: dict, precision: str, chi: int, n_gates: int):
    """The cached schedule for this shape, or None."""
    e = cache.get("entries", {}).get(cache_key(precision, chi, n_gates))
    return dict(e["params"]) if e else None


def apply(mps, cache_path: str, chi: int, n_gates: int):
    """Set the cached schedule on a handle; returns (key, params) or (key, None) if the cache
    holds nothing for the shape (the handle keeps its schedule)."""
    key = cache_key(mps.precision, chi, n_gates)
    params = lookup(load_cache(cache_path), mps.precision, chi, n_gates)
    if params:
        mps.set_svd_params(**params)
    return key, params


def accept(err_f: float, default_err_f: float, precision: str, n_unconverged: int) -> bool:
    """A candidate counts only if it converged and its fidelity error against the FP64 path
    is within the budget and close to the default schedule's."""
    return (n_unconverged == 0 and err_f <= ERR_F_TOL[precision]
            and err_f <= ERR_F_SLACK * default_err_f + ERR_F_FLOOR)


def measure_schedule(n_sites, caps, precision: str, setup: list, timed: list,
                     repeats: int = 1):
    """Build the GPU evaluation for ``search`` over any batch of states: ``setup`` and
    ``timed`` are lists of ``apply_layer`` keyword sets (bonds, gates, chi_max, state_idx).
    Each candidate runs on a fresh handle: the set-up layers with the default schedule (the
    path is deterministic, so every candidate starts from the same bits), then the timed
    layers with the candidate's.  The same timed layers applied to the set-up states on the
    FP64 path give the reference for err_F (the largest over the states).  The result holds
    the summed device time of the timed layers (the least over ``repeats``), the largest sweep
    count, err_F and whether the checks passed.  Returns (evaluate, defaults)."""
    from . import ptebd

    n_states = len(n_sites)

    def fresh():
        h = ptebd.MPS(n_sites, caps, precision)
        for kw in setup:
            h.apply_layer(**kw, eps_reading=EPS_READING)
        return h

    m = fresh()
    defaults = m.svd_params()
    fp64 = ptebd.MPS(n_sites, caps, "fp64")
    for s in range(n_states):
        fp64.import_state(*m.export(s), s)
    m.close()
    for kw in timed:
        fp64.apply_layer(**kw, eps_reading=EPS_READING)
    n64 = [fp64.norm(s) for s in range(n_states)]
    ref = {}

    def evaluate(params):
        best_ms, sweeps, unconv, err = None, 0, 0, 0.0
        for _ in range(max(1, repeats)):
            h = fresh()
            h.set_svd_params(**params)
            ms = 0.0
            for kw in timed:
                st = h.apply_layer(**kw, eps_reading=EPS_READING)
                ms += st["device_ms"]
                sweeps = max(sweeps, int(st["max_sweeps"]))
                unconv += int(st["n_unconverged"])
            err = max(1.0 - abs(h.overlap(fp64, s, s)) ** 2 / (h.norm(s) ** 2 * n64[s] ** 2)
                      for s in range(n_states))
            h.close()
            best_ms = ms if best_ms is None else min(best_ms, ms)
        if not ref:
            ref["err"] = err  # the first evaluation is the default schedule
        ok = accept(err, ref["err"], precision, unconv)
        return {"ms": best_ms, "ok": ok, "max_sweeps": sweeps, "err_F": err,
                "n_unconverged": unconv}

    return evaluate, {k: defaults[k] for k in SEARCH_SPACE if k in defaults}


def chain_spec(n_sites: int, chi: int, seed: int = 0, timed_layers: int = 3) -> dict:
    """A Haar brickwork chain of n_sites driven (default schedule) to the layer where every
    bulk bond is at chi, then ``timed_layers`` saturated layers."""
    from . import inputs

    setup = max(1, int(math.ceil(math.log2(max(2, chi))))) + 1
    layers = [dict(bonds=b, gates=g, chi_max=chi)
              for b, g in inputs.brickwork_circuit(n_sites, setup + timed_layers, seed)]
    return {"n_sites": [n_sites], "caps": [chi], "setup": layers[:setup],
            "timed": layers[setup:],
            "workload": f"Haar brickwork, N={n_sites}, chi={chi}, {timed_layers} saturated "
                        f"layers of {len(layers[setup]['bonds'])} gates, seed {seed}"}


def workload_spec(workload: str, timed_layers: int) -> dict:
    """The lattice or batched-mix workload (``workloads``): the compiled lattice layers up to
    the 40th as set-up (its largest bonds are at 512 from about the 21st) and the next
    ``timed_layers`` timed; the mix's first 10 of 16 layers as set-up (every state's bulk
    bonds at its cap) and the next ``timed_layers`` timed."""
    from . import workloads

    n_sites, caps, calls = workloads.layer_calls(workload)
    first = 39 if workload == "lattice" else 10
    if first + timed_layers > len(calls):
        raise ValueError(f"the {workload} workload has {len(calls)} layers")
    timed = calls[first:first + timed_layers]
    return {"n_sites": n_sites, "caps": caps, "setup": calls[:first], "timed": timed,
            "workload": f"{workload} workload, {len(n_sites)} state(s), caps up to {max(caps)}, "
                        f"layers {first + 1}..{first + timed_layers} timed "
                        f"(up to {max(len(kw['bonds']) for kw in timed)} gates)"}


def tune_spec(spec: dict, precision: str, cache_path: str, repeats: int = 1, passes: int = 2,
              log=print, min_gain: float = 0.01) -> dict:
    """Tune one workload shape on the GPU and store the result in the cache under the key of
    its largest cap and largest timed layer; returns the entry."""
    evaluate, defaults = measure_schedule(spec["n_sites"], spec["caps"], precision,
                                          spec["setup"], spec["timed"], repeats)
    space = _space_for(precision)

    def logged(p):
        r = evaluate(p)
        log(json.dumps({"params": p, **r}))
        return r

    best, best_r, history = search(logged, defaults, space, passes, min_gain)
    base_r = history[0][1]
    n_gates = max(len(kw["bonds"]) for kw in spec["timed"])
    entry = {
        "params": best,
        "ms": best_r["ms"],
        "default_ms": base_r["ms"],
        "default_params": history[0][0],
        "min_gain": min_gain,
        "workload": f"{spec['workload']}; eps reading {EPS_READING}; err_F against the same "
                    f"layers on the FP64 path",
        "evaluated": [{"params": p, "ms": r["ms"], "ok": r["ok"],
                       "err_F": r["err_F"], "max_sweeps": r["max_sweeps"]}
                      for p, r in history],
        "time": time.strftime("%Y-%m-%d %H:%M:%S"),
    }
    cache = load_cache(cache_path)
    cache["entries"][cache_key(precision, max(spec["caps"]), n_gates)] = entry
    save_cache(cache_path, cache)
    return entry


def tune(n_sites: int, chi: int, precision: str, cache_path: str, seed: int = 0,
         timed_layers: int = 3, repeats: int = 1, passes: int = 2, log=print,
         min_gain: float = 0.01) -> dict:
    """Tune the saturated layers of a Haar brickwork chain (``chain_spec``)."""
    return tune_spec(chain_spec(n_sites, chi, seed, timed_layers), precision, cache_path,
                     repeats, passes, log, min_gain)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", choices=("chain", "lattice", "mix"), default="chain")
    ap.add_argument("--n-sites", type=int, default=1024)
    ap.add_argument("--chi", type=int, nargs="+", default=[256])
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--cache", default=os.path.join(os.path.dirname(__file__),
                                                    "autotune_cache.json"))
    ap.add_argument("--timed-layers", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=1)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--min-gain", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    if a.workload == "chain":
        specs = [chain_spec(a.n_sites, chi, a.seed, a.timed_layers) for chi in a.chi]
    else:
        specs = [workload_spec(a.workload, a.timed_layers)]
    for spec in specs:
        e = tune_spec(spec, a.precision, a.cache, a.repeats, a.passes,
                      log=lambda s: print(s, flush=True), min_gain=a.min_gain)
        print(json.dumps({"workload": spec["workload"], "best": e["params"], "ms": e["ms"],
                          "default_ms": e["default_ms"]}), flush=True)


if __name__ == "__main__":
    main()
