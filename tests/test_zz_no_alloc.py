"""The allocation-free batched SVD (fixed device scratch array) against the allocating one:
same inputs, same results, on two calls in a row (the second smaller, so it runs on what the
first left in the shared array), in both precisions."""

import numpy as np
import pytest

from paper_2312_02667_amd import ptebd
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _inputs(seed, batch, m, n):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((batch, m, n)) + 1j * rng.standard_normal((batch, m, n))
    # graded columns, as the truncated two-site wavefunctions have
    return a * np.logspace(0, -5, n)[None, None, :]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_svd_matches_allocating_svd(precision):
    tol = 1e-13 if precision == "fp64" else 1e-6
    for call, (batch, m, n) in enumerate(((2, 300, 200), (1, 96, 150))):
        a = _inputs(10 + call, batch, m, n)
        say(f"noalloc svd {precision} call {call}: batch {batch}, {m} x {n}")
        s0, u0, vh0, sw0, c0 = ptebd.svd_batched(a, precision)
        s1, u1, vh1, sw1, c1 = ptebd.svd_batched(a, precision, noalloc=True)
        assert c0 == c1 == ptebd.OK
        assert np.array_equal(sw0, sw1)
        scale = s0[:, :1]
        assert np.max(np.abs(s1 - s0) / scale) <= tol
        k = min(m, n)
        # vectors of singular values above 1e-3 sigma_1 (the rest are compared through the
        # reconstruction below)
        keep = s0 > 1e-3 * scale
        for b in range(batch):
            kk = int(keep[b].sum())
            assert np.max(np.abs(u1[b][:, :kk] - u0[b][:, :kk])) <= 1e3 * tol
            assert np.max(np.abs(vh1[b][:kk] - vh0[b][:kk])) <= 1e3 * tol
            rec = (u1[b] * s1[b][None, :k]) @ vh1[b]
            assert np.linalg.norm(rec - a[b]) <= 1e2 * tol * np.linalg.norm(a[b])
        say(f"  max |ds|/s1 = {np.max(np.abs(s1 - s0) / scale):.2e}, "
            f"bitwise s equal: {np.array_equal(s0, s1)}")
