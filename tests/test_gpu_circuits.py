"""Circuit-level properties on the GPU: the mixed path against the FP64 oracle at chi = 256,
batched independent states against separate runs, determinism, and checkpoint round-trip."""

import numpy as np
import pytest

from oracle import ptebd_oracle as po
from paper_2312_02667_amd import inputs, ptebd
from tests.gpu_util import say, to_oracle

pytestmark = pytest.mark.gpu


def test_mixed_path_against_oracle_at_chi_256():
    """N = 40, depth 14, chi_max = 256, Haar SU(4): bulk bonds saturate (512x512 theta from
    layer 9); err_F of the FP32 path against the FP64 oracle must stay <= 1e-6."""
    n, depth, chi = 40, 14, 256
    layers = inputs.brickwork_circuit(n, depth, seed=3)
    ref = po.product_state(n)
    m = ptebd.MPS(n, chi, "fp32")
    for li, (bonds, gates) in enumerate(layers):
        m.apply_layer(bonds, gates, chi_max=chi, cutoff=1e-12)
        po.apply_layer(ref, bonds, gates, chi_max=chi, cutoff=1e-12)
        if li + 1 >= 9:
            err = po.fidelity_error(ref, to_oracle(m))
            say(f"layer {li + 1}: err_F(fp32 GPU vs FP64 oracle) = {err:.3e}")
            assert err <= 1e-6
    assert m.bond_dims() == ref.bond_dims()
    m.close()


def test_batched_states_match_separate_runs():
    """Three circuits of different N and chi_max in one handle (one launch per layer over all
    of them) give bitwise the same states as three separate handles."""
    specs = [(30, 16, 0), (45, 32, 1), (24, 64, 2)]
    depth = 10
    circuits = [inputs.brickwork_circuit(n, depth, seed=seed, circuit_id=7) for n, _, seed in specs]
    batched = ptebd.MPS([n for n, _, _ in specs], [c for _, c, _ in specs], "fp32")
    singles = [ptebd.MPS(n, c, "fp32") for n, c, _ in specs]
    chi_max = 16
    for layer in range(depth):
        sidx, bonds, gates = [], [], []
        for s, circ in enumerate(circuits):
            b, g = circ[layer]
            sidx += [s] * len(b)
            bonds.append(b)
            gates.append(g)
            singles[s].apply_layer(b, g, chi_max=chi_max)
        batched.apply_layer(np.concatenate(bonds), np.concatenate(gates), chi_max=chi_max,
                            state_idx=np.array(sidx, np.int32))
    for s in range(len(specs)):
        gb, lb = batched.export(s)
        gs, ls = singles[s].export()
        for x, y in zip(lb, ls):
            assert np.array_equal(x, y)
        for x, y in zip(gb, gs):
            assert np.array_equal(x, y)
    batched.close()
    for x in singles:
        x.close()


def test_deterministic_and_checkpoint_roundtrip():
    n, depth, chi = 32, 12, 16
    layers = inputs.brickwork_circuit(n, depth, seed=9)
    a = ptebd.MPS(n, chi, "fp32")
    b = ptebd.MPS(n, chi, "fp32")
    for bonds, gates in layers:
        a.apply_layer(bonds, gates, chi_max=chi, ptsu_steps=1)
        b.apply_layer(bonds, gates, chi_max=chi, ptsu_steps=1)
    ga, la = a.export()
    gb, lb = b.export()
    assert all(np.array_equal(x, y) for x, y in zip(la, lb))
    assert all(np.array_equal(x, y) for x, y in zip(ga, gb))
    # checkpoint: 6 layers, export, import into a fresh handle, 6 more layers
    c = ptebd.MPS(n, chi, "fp32")
    for bonds, gates in layers[:6]:
        c.apply_layer(bonds, gates, chi_max=chi, ptsu_steps=1)
    gc, lc = c.export()
    d = ptebd.MPS(n, chi, "fp32")
    d.import_state(gc, lc)
    for bonds, gates in layers[6:]:
        d.apply_layer(bonds, gates, chi_max=chi, ptsu_steps=1)
    gd, ld = d.export()
    assert all(np.array_equal(x, y) for x, y in zip(la, ld))
    assert all(np.array_equal(x, y) for x, y in zip(ga, gd))
    for x in (a, b, c, d):
        x.close()
