"""Autotuner logic on the CPU: cache keys, the coordinate search (with a stand-in evaluation
of known optimum), rejection of candidates that fail the checks, and the JSON cache."""

import json

import numpy as np
import pytest

from paper_2312_02667_amd import autotune

DEFAULTS = {"block_cols": 16, "inner_sweeps": 2, "inner_repeat": 1e-2, "sort_pairs": 1,
            "streams": 2, "precondition": 1}


def test_cache_key_buckets():
    assert autotune.cache_key("fp32", 256, 512) == "fp32/theta512/gates512"
    assert autotune.cache_key("fp32", 256, 511) == "fp32/theta512/gates512"
    assert autotune.cache_key("fp64", 64, 5) == "fp64/theta128/gates8"
    assert autotune.cache_key("fp32", 32, 1) == "fp32/theta64/gates1"
    assert autotune.cache_key("fp32", 32, 0) == "fp32/theta64/gates1"


def _separable(opt, weights=None):
    """Cost with its minimum at opt: each control off its optimum adds its weight."""
    calls = []

    def evaluate(p):
        calls.append(dict(p))
        ms = 100.0 + sum((weights or {}).get(k, 5.0) * (p[k] != opt[k]) for k in opt)
        return {"ms": ms, "ok": True, "err_F": 0.0, "max_sweeps": 5}
    return evaluate, calls


def test_search_reaches_the_optimum_from_the_defaults():
    space = autotune._space_for("fp32")
    opt = {"block_cols": 32, "inner_sweeps": 3, "inner_repeat": 3e-2, "sort_pairs": 0,
           "streams": 1, "precondition": 1}
    evaluate, calls = _separable(opt)
    best, best_r, history = autotune.search(evaluate, DEFAULTS, space)
    assert best == opt
    assert best_r["ms"] == 100.0
    assert calls[0] == DEFAULTS                       # the default schedule comes first
    assert len({tuple(sorted(c.items())) for c in calls}) == len(calls)  # no repeats


def test_search_skips_fp64_preconditioning_and_wide_blocks():
    space = autotune._space_for("fp64")
    assert "precondition" not in space and "block_cols" not in space
    d = {k: v for k, v in DEFAULTS.items() if k not in ("precondition", "block_cols")}
    evaluate, calls = _separable({**d, "streams": 1})
    best, _, _ = autotune.search(evaluate, d, space)
    assert best["streams"] == 1
    assert all("precondition" not in c and "block_cols" not in c for c in calls)


def test_acceptance_uses_the_fidelity_budget():
    """Converged, within ERR_F_TOL and within ERR_F_SLACK x the default's err_F."""
    tol = autotune.ERR_F_TOL["fp32"]
    assert autotune.accept(1e-9, 1e-9, "fp32", 0)
    assert not autotune.accept(1e-9, 1e-9, "fp32", 1)               # an SVD hit the cap
    assert not autotune.accept(2 * tol, 2 * tol, "fp32", 0)         # over the budget
    assert not autotune.accept(5e-9, 1e-9, "fp32", 0)               # 5x the default's error
    assert autotune.accept(3.9e-9, 1e-9, "fp32", 0)
    assert autotune.accept(1e-14, 0.0, "fp64", 0)                   # FP64 overlap resolution


def test_failed_candidates_are_never_chosen():
    space = autotune._space_for("fp32")

    def evaluate(p):
        # the fastest schedule does not converge
        bad = p["inner_sweeps"] == 1
        return {"ms": 50.0 if bad else 100.0 - p["streams"], "ok": not bad,
                "err_F": 0.0, "max_sweeps": 30 if bad else 6}
    best, best_r, _ = autotune.search(evaluate, DEFAULTS, space)
    assert best["inner_sweeps"] != 1 and best_r["ok"]


def test_the_default_must_pass():
    with pytest.raises(RuntimeError):
        autotune.search(lambda p: {"ms": 1.0, "ok": False}, DEFAULTS,
                        autotune._space_for("fp32"))


def test_inner_repeat_is_not_varied_with_one_inner_sweep():
    space = autotune._space_for("fp32")
    opt = dict(DEFAULTS, inner_sweeps=1)
    evaluate, calls = _separable(opt, weights={"inner_sweeps": 20.0})
    best, _, _ = autotune.search(evaluate, DEFAULTS, space)
    assert best["inner_sweeps"] == 1
    moved = [c for c in calls if c["inner_sweeps"] == 1 and c["inner_repeat"] != best["inner_repeat"]]
    assert not moved


class _FakeMPS:
    precision = "fp32"

    def __init__(self):
        self.set = []

    def set_svd_params(self, **kw):
        self.set.append(kw)


def test_cache_roundtrip_lookup_and_apply(tmp_path):
    path = str(tmp_path / "cache.json")
    cache = autotune.load_cache(path)
    assert cache == {"version": autotune.CACHE_VERSION, "entries": {}}
    params = dict(DEFAULTS, streams=1)
    cache["entries"][autotune.cache_key("fp32", 256, 512)] = {"params": params, "ms": 1.0}
    autotune.save_cache(path, cache)
    again = autotune.load_cache(path)
    assert autotune.lookup(again, "fp32", 256, 511) == params
    assert autotune.lookup(again, "fp32", 128, 512) is None
    m = _FakeMPS()
    key, got = autotune.apply(m, path, 256, 512)
    assert key == "fp32/theta512/gates512" and got == params and m.set == [params]
    m2 = _FakeMPS()
    assert autotune.apply(m2, path, 64, 512)[1] is None and m2.set == []


def test_cache_of_another_version_is_refused(tmp_path):
    path = tmp_path / "old.json"
    path.write_text(json.dumps({"version": 0, "entries": {}}))
    with pytest.raises(ValueError):
        autotune.load_cache(str(path))


def test_noise_level_gains_do_not_move_the_schedule():
    space = autotune._space_for("fp32")

    def evaluate(p):
        # every other schedule 0.5 % faster than the defaults: below the 1 % threshold
        return {"ms": 100.0 if p == DEFAULTS else 99.5, "ok": True, "err_F": 0.0,
                "max_sweeps": 6}
    best, _, _ = autotune.search(evaluate, DEFAULTS, space)
    assert best == DEFAULTS
    best, _, _ = autotune.search(evaluate, DEFAULTS, space, min_gain=0.0)
    assert best != DEFAULTS


def test_committed_cache_is_valid():
    """The cache shipped with the package (applied by the benchmark) loads, every entry's
    schedule lies in the search space of its precision, and the benchmark's shape has one."""
    import os
    path = os.path.join(os.path.dirname(autotune.__file__), "autotune_cache.json")
    cache = autotune.load_cache(path)
    assert cache["entries"]
    for key, e in cache["entries"].items():
        precision = key.split("/")[0]
        space = autotune._space_for(precision)
        assert set(e["params"]) == set(space), key
        for k, v in e["params"].items():
            assert v in space[k], (key, k, v)
        assert e["ms"] <= e["default_ms"] and e["evaluated"], key
    assert autotune.lookup(cache, "fp32", 256, 512) is not None
    assert autotune.lookup(cache, "fp64", 256, 511) is not None


def test_workload_specs_and_their_cache_keys():
    """The lattice and batched-mix workloads as tuning inputs: set-up and timed layers in
    order, and the keys their runs look up (largest cap, largest layer's gate bucket)."""
    from paper_2312_02667_amd import workloads

    for name, first, key in (("lattice", 39, "fp32/theta1024/gates32"),
                             ("mix", 10, "fp32/theta512/gates8192")):
        n_sites, caps, calls = workloads.layer_calls(name)
        spec = autotune.workload_spec(name, 3)
        assert spec["n_sites"] == n_sites and spec["caps"] == caps
        assert len(spec["setup"]) == first and len(spec["timed"]) == 3
        assert np.array_equal(spec["timed"][0]["bonds"], calls[first]["bonds"])
        n_gates = max(len(c["bonds"]) for c in calls)
        assert autotune.cache_key("fp32", max(caps), n_gates) == key
        assert max(len(kw["bonds"]) for kw in spec["timed"]) <= n_gates
    with pytest.raises(ValueError):
        autotune.workload_spec("mix", 7)     # 10 set-up + 7 timed > 16 layers
    chain = autotune.chain_spec(64, 16, seed=1, timed_layers=2)
    assert len(chain["setup"]) == 5 and len(chain["timed"]) == 2
    assert all(kw["chi_max"] == 16 for kw in chain["setup"] + chain["timed"])
