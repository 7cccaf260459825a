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
    assert ev[0]["ok"] and ev[0]["params"]["block_cols"] == 16    # the default, first
    assert all(e["ms"] > 0 for e in ev)
    assert entry["ms"] <= entry["default_ms"]
    assert set(entry["params"]) == set(autotune._space_for("fp32"))
    assert any(e["params"]["block_cols"] == 32 for e in ev)      # the tile shape is searched
    # schedules differ only in rounding: every accepted one is within the fidelity budget
    # against the FP64 path and near the default's error
    for e in ev:
        if e["ok"]:
            assert e["err_F"] <= autotune.ERR_F_TOL["fp32"]
            assert e["err_F"] <= autotune.ERR_F_SLACK * ev[0]["err_F"] + autotune.ERR_F_FLOOR
    m = ptebd.MPS(40, 16, "fp32")
    try:
        key, params = autotune.apply(m, path, 16, 20)
        assert key == "fp32/theta32/gates32" and params == entry["params"]
        got = m.svd_params()
        assert all(got[k] == pytest.approx(v) for k, v in params.items())
    finally:
        m.close()
