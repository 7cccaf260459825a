"""The benchmark's own workload against the FP64 oracle, layer by layer: N = 1024, the
Haar-SU(4) brickwork circuit of depth 20 (seed 0), chi_max = 256, cutoff 1e-12, nu on the
complement reading, the mixed (FP32) path.  Layers 10..20 truncate every bulk bond (512 x 512
theta to 256).  After each of them the fidelity error

    err_F = 1 - |<oracle|gpu>|^2 / (<oracle|oracle> <gpu|gpu>)

must stay <= 1e-6, the accuracy condition of the benchmark's metric (checked also after the
untruncated layers 5 and 9), and each gate's discarded weight must agree with the oracle's.
Bond dimensions are compared loosely: before saturation a bond keeps every sigma above the
cutoff, and the FP32 path resolves sigma only to about u sqrt(R) sigma_1 ~ 1e-6 sigma_1, the
size of its cutoff floor 2^-19 sigma_1, so a value at the floor may be kept on one side and
dropped on the other (its weight, ~4e-12, is far below what err_F can see).  The oracle applies a
layer's gates at once through a thread pool (they act on disjoint sites, Sec. II.C) with one
BLAS thread each; the overlap is the library's FP64 query on the oracle state imported into an
FP64 handle (pinned against the oracle's own overlap in test_gpu_layer)."""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import ptebd_oracle as po
from paper_2312_02667_amd import inputs, ptebd
from tests.gpu_util import oracle_cutoff, say

pytestmark = pytest.mark.gpu


def test_benchmark_workload_against_oracle_per_layer():
    from threadpoolctl import threadpool_limits

    n, chi, depth = 1024, 256, 20
    layers = inputs.brickwork_circuit(n, depth, seed=0)
    ref = po.product_state(n)
    m = ptebd.MPS(n, chi, "fp32")
    probe = ptebd.MPS(n, chi, "fp64")
    errs, eps_diff, dim_diffs = [], 0.0, 0
    with threadpool_limits(limits=1, user_api="blas"), ThreadPoolExecutor(16) as pool:
        for li, (bonds, gates) in enumerate(layers):
            st = m.apply_layer(bonds, gates, chi_max=chi, cutoff=1e-12, eps_reading="complement")
            assert st["n_unconverged"] == 0
            stats, trig = po.apply_layer(ref, bonds, gates, chi_max=chi,
                                         cutoff=oracle_cutoff(1e-12, "fp32"),
                                         eps_reading="complement", map_fn=pool.map)
            assert st["triggered"] == trig
            dg, dr = np.array(m.bond_dims()), np.array(ref.bond_dims())
            nd = int(np.sum(dg != dr))
            dim_diffs += nd
            assert nd <= 0.02 * n and int(np.max(np.abs(dg - dr))) <= 2, (li + 1, nd)
            if li + 1 not in (5, 9) and li + 1 < 10:
                continue
            probe.import_state(ref.gam, ref.lam)
            err = 1.0 - abs(m.overlap(probe)) ** 2 / (m.norm() ** 2 * probe.norm() ** 2)
            de = float(np.max(np.abs(np.asarray(st["eps"]) - np.array([x["eps"] for x in stats]))))
            say(f"layer {li + 1}: err_F {err:.3e}, largest per-gate |d eps| {de:.2e}, bonds with "
                f"another dimension {nd}")
            assert err <= 1e-6, (li + 1, err)
            if li + 1 >= 10:
                errs.append(err)
                eps_diff = max(eps_diff, de)
            # eps = 1 - kept sigma^2 per gate; FP32 sigma carries ~u sqrt(R) sigma_1 (6.5e-6
            # the largest difference measured over the 20 layers)
            assert de <= 3e-5, (li + 1, de)
    say(f"largest err_F over layers 10..20: {max(errs):.3e}; largest per-gate |d eps| "
        f"{eps_diff:.2e}; bond dimensions differing, summed over layers: {dim_diffs}")
    m.close()
    probe.close()
