"""Parity at the benchmark's full size and launch configuration: N = 1024, chi = 256, one
brickwork layer of 512 gates in one apply_layer call, on a synthetic saturated Vidal state.
The oracle recomputes sampled bond updates one by one from the same input; compared are the
new bond dimension, Lambda[q+1], eps, nu and the gauge-invariant two-site tensor
Lambda[q] Gamma'[q] Lambda'[q+1] Gamma'[q+1] Lambda[q+2]."""

import numpy as np
import pytest

from oracle import ptebd_oracle as po
from paper_2312_02667_amd import inputs, ptebd
from tests.gpu_util import oracle_cutoff, say

pytestmark = pytest.mark.gpu

N, CHI = 1024, 256
SAMPLED = [0, 2, 6, 8, 300, 512, 1014, 1016, 1022]  # chain ends (ragged) and bulk (512x512)

# per-precision bounds: sigma abs error / sigma_1, relative Frobenius error of the two-site
# tensor (FP32: theta and the Jacobi updates rounded at 2^-24 over ~10 sweeps of 31 rounds)
TOL = {"fp64": dict(lam=1e-11, th=1e-10, eps=1e-11), "fp32": dict(lam=2e-5, th=2e-5, eps=2e-6)}


@pytest.fixture(scope="module")
def saturated():
    say("generating the synthetic saturated state N=1024, chi=256")
    g, l = inputs.random_vidal_state(N, CHI, seed=5)
    rng = np.random.default_rng(55)
    bonds = inputs.brickwork_bonds(N, 1)
    gates = np.stack([inputs.haar_unitary(rng) for _ in bonds])
    return g, l, bonds, gates


def _two_site(gq, lam_l, lam_m, gq1, lam_r):
    a = lam_l[:, None, None] * gq * lam_m[None, None, :]
    b = gq1 * lam_r[None, None, :]
    return np.einsum("asm,mtc->astc", a, b)


@pytest.mark.parametrize("reading", ["literal", "complement"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_layer_sampled_bonds(saturated, precision, reading):
    """Both eps readings: literal is the library default, complement the benchmark's."""
    g, l, bonds, gates = saturated
    m = ptebd.MPS(N, CHI, precision)
    say(f"import ({precision}, {reading})")
    m.import_state(g, l)
    say(f"apply one layer of {len(bonds)} gates ({precision})")
    st = m.apply_layer(bonds, gates, chi_max=CHI, cutoff=1e-12, eps_reading=reading)
    assert st["n_unconverged"] == 0
    tol = TOL[precision]
    for q in SAMPLED:
        i = int(np.where(bonds == q)[0][0])
        local = po.VidalMPS([g[q], g[q + 1]], [l[q], l[q + 1], l[q + 2]])
        ref = po.bond_update(local, 0, gates[i], CHI, oracle_cutoff(1e-12, precision),
                             stabilize=True, eps_reading=reading)
        say(f"  q={q}: theta {2 * len(l[q])}x{2 * len(l[q + 2])}, k={ref['k']}")
        assert st["k"][i] == ref["k"]
        s1 = ref["sigma"][0]
        lam_gpu = m.get_lambda(q + 1)
        # relative to the largest new Schmidt value nu sigma_1 (the complement reading
        # rescales this unnormalized synthetic state's sigma by nu = 1/|kept sigma|)
        assert np.max(np.abs(lam_gpu - local.lam[1])) <= tol["lam"] * local.lam[1][0]
        if reading == "literal":
            assert abs(st["eps"][i] - ref["eps"]) <= tol["eps"] * s1 ** 2 * 10
        else:
            # eps = 1 - sum of the kept sigma^2: |d eps| <= 2 sum_j sigma_j |d sigma_j|
            assert abs(st["eps"][i] - ref["eps"]) <= 2 * tol["lam"] * s1 * float(np.sum(ref["sigma"]))
        th_ref = _two_site(local.gam[0], l[q], local.lam[1], local.gam[1], l[q + 2])
        th_gpu = _two_site(m.export_site(q), l[q], lam_gpu, m.export_site(q + 1), l[q + 2])
        err = np.linalg.norm(th_gpu - th_ref) / np.linalg.norm(th_ref)
        say(f"    two-site rel. error {err:.2e}")
        assert err <= tol["th"]
    m.close()
