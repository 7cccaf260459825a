"""The autotuner end to end on the GPU at a small shape: every evaluated schedule runs the same
saturated layers through the C ABI, the default one first, and the chosen schedule is stored
and applied back to a handle."""

import pytest

from paper_2312_02667_amd import autotune, ptebd
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def test_tune_small_chain(tmp_path):
    path = str(tmp_path / "cache.json")
    entry = autotune.tune(40, 16, "fp32", path, seed=3, timed_layers=2, passes=1, log=say)
    ev = entry["evaluated"]
    assert ev[0]["lambda_dev"] == 0.0 and ev[0]["ok"]           # the default, first
    assert all(e["ms"] > 0 for e in ev)
    assert entry["ms"] <= entry["default_ms"]
    assert set(entry["params"]) == set(autotune._space_for("fp32"))
    # schedules differ only in rounding: every accepted one keeps Lambda within tolerance
    assert all(e["lambda_dev"] <= autotune.LAMBDA_TOL["fp32"] for e in ev if e["ok"])
    m = ptebd.MPS(40, 16, "fp32")
    try:
        key, params = autotune.apply(m, path, 16, 20)
        assert key == "fp32/theta32/gates32" and params == entry["params"]
        got = m.svd_params()
        assert all(got[k] == pytest.approx(v) for k, v in params.items())
    finally:
        m.close()
