"""Pins of the benchmark circuit families (App. A) and of the 2D path compilation.

The compiled circuits are checked against the physical circuits applied gate by gate to a
state vector (long-range couplings included), against Table I's compiled depths, and against
closed forms of the gates (matrix exponentials) and the spin symmetry of the HVA circuit.
"""

import os

import numpy as np
import pytest
import scipy.linalg

from oracle import statevector as sv
from paper_2312_02667_amd import circuits as c

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_compiled_depths.txt")


def run_physical(n, physical, one_d=False):
    psi = sv.zero_state(n)
    for layer in physical:
        singles, pairs = (layer if one_d else layer[1:])
        for q, u in singles.items():
            psi = sv.apply_one(psi, n, q, u)
        for qa, qb, g in pairs:
            psi = sv.apply_pair(psi, n, qa, qb, g)
    return psi


def test_random_rotation_is_the_exponential():
    rng = np.random.default_rng(3)
    for _ in range(5):
        state = rng.bit_generator.state
        u = c.random_rotation(rng)
        rng2 = np.random.default_rng()
        rng2.bit_generator.state = state
        th, a, f = rng2.uniform(0, 2 * np.pi), rng2.uniform(0, np.pi), rng2.uniform(0, 2 * np.pi)
        h = np.sin(a) * np.cos(f) * c.X + np.sin(a) * np.sin(f) * c.Y + np.cos(a) * c.Z
        np.testing.assert_allclose(u, scipy.linalg.expm(-1j * th * h), atol=1e-13)
        np.testing.assert_allclose(u.conj().T @ u, np.eye(2), atol=1e-13)


def test_eswap_is_the_exponential_and_singlet():
    for th in (0.3, 1.7, 5.9):
        np.testing.assert_allclose(c.eswap(th), scipy.linalg.expm(-0.5j * th * c.SWAP), atol=1e-13)
    u = c.singlet_preparation()
    np.testing.assert_allclose(u.conj().T @ u, np.eye(4), atol=1e-15)
    np.testing.assert_allclose(u[:, 0], np.array([0, 1, -1, 0]) / np.sqrt(2), atol=1e-15)


@pytest.mark.parametrize("n,depth", [(7, 6), (6, 5), (2, 3)])
def test_rqc_1d_compiles_to_the_physical_circuit(n, depth):
    phys = c.rqc_1d_physical(n, depth, seed=4)
    assert [sorted(p[0] for p in layer[1]) for layer in phys[:2]] == \
        [list(range(0, n - 1, 2)), list(range(1, n - 1, 2))]
    psi = sv.run_circuit(n, c.rqc_1d(n, depth, seed=4))
    np.testing.assert_allclose(psi, run_physical(n, phys, one_d=True), atol=1e-12)


def test_pqc_1d_stays_a_total_singlet():
    n, depth = 8, 6
    phys = c.pqc_1d_physical(n, depth, seed=2)
    psi = sv.run_circuit(n, c.pqc_1d(n, depth, seed=2))
    np.testing.assert_allclose(psi, run_physical(n, phys, one_d=True), atol=1e-12)
    # eSWAP commutes with the total spin, so the singlet-dimer product stays in S = 0:
    # S_tot^2 psi = 0 (S = sigma / 2).
    s2 = np.zeros_like(psi)
    for pa in (c.X, c.Y, c.Z):
        spsi = np.zeros_like(psi)
        for q in range(n):
            spsi += 0.5 * sv.apply_one(psi, n, q, pa)
        for q in range(n):
            s2 += 0.5 * sv.apply_one(spsi, n, q, pa)
    assert np.linalg.norm(s2) < 1e-12
    assert np.linalg.norm(psi) == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("lx,ly", [(4, 4), (3, 4), (4, 3), (2, 5), (5, 2)])
def test_rqc_2d_compiles_to_the_physical_circuit(lx, ly):
    n = lx * ly
    phys = c.rqc_2d_physical(lx, ly, 8, seed=5)
    compiled = c.rqc_2d(lx, ly, 8, seed=5)
    for bonds, gates in compiled:
        assert np.all(np.diff(bonds) >= 2) and bonds.min() >= 0 and bonds.max() <= n - 2
    psi = sv.run_circuit(n, compiled)
    np.testing.assert_allclose(psi, run_physical(n, phys), atol=1e-11)


def test_pqc_2d_compiles_to_the_physical_circuit():
    lx, ly = 3, 4
    n = lx * ly
    phys = c.pqc_2d_physical(lx, ly, 8, seed=6)
    assert [layer[0] for layer in phys] == [0, 1, 2, 3, 0, 1, 2, 3]
    psi = sv.run_circuit(n, c.pqc_2d(lx, ly, 8, seed=6))
    np.testing.assert_allclose(psi, run_physical(n, phys), atol=1e-11)
    with pytest.raises(ValueError):
        c.pqc_2d_physical(4, 5, 4, seed=0)


def test_lattice_couplings_edges():
    # odd extents leave the edge qubits of that direction idle (App. A, L_x = L_y = 5)
    assert len(c.lattice_couplings(5, 5, 0)) == 10 and len(c.lattice_couplings(5, 5, 1)) == 10
    assert len(c.lattice_couplings(5, 5, 2)) == 10 and len(c.lattice_couplings(5, 5, 3)) == 10
    used_c = {q for p in c.lattice_couplings(5, 5, 2) for q in p}
    assert all(4 * 5 + y not in used_c for y in range(5))       # column x = 4 idle in C
    used_d = {q for p in c.lattice_couplings(5, 5, 3) for q in p}
    assert all(y not in used_d for y in range(5))               # column x = 0 idle in D


@pytest.mark.parametrize("lx,ly", [(4, 4), (4, 6), (5, 5), (12, 12), (32, 32), (3, 7), (6, 2)])
def test_cd_pair_depth_closed_form(lx, ly):
    # App. A: a C + D pair of physical layers becomes 3 (L_y - 1) + 2 compiled layers
    assert c.cd_compiled_depth(lx, ly) == 3 * (ly - 1) + 2


def test_table1_compiled_depths():
    rows = np.loadtxt(GOLDEN, dtype=int)
    for n, lx, ly, d, compiled in rows:
        assert n == lx * ly
        if (n, d) == (25, 60):
            assert c.compiled_depth_2d(lx, ly, 48) == compiled
            assert c.compiled_depth_2d(lx, ly, 60) == 240
        else:
            assert c.compiled_depth_2d(lx, ly, d) == compiled
    # the generated circuit has that depth plus at most two trailing product-gate layers
    layers = c.rqc_2d(4, 6, 28, seed=0)
    assert 133 <= len(layers) <= 135
    assert len(c.pqc_2d(4, 6, 28, seed=0)) == 133


def test_compile_2d_with_asymmetric_gates():
    # CZ and eSWAP are symmetric under exchange of their qubits; Haar gates are not, so this
    # pins the orientation of every routed coupling.
    from paper_2312_02667_amd import inputs
    lx, ly = 3, 4
    n = lx * ly
    rng = np.random.default_rng(11)
    phys = []
    for layer in range(8):
        kind = layer % 4
        singles = {q: inputs.haar_unitary(rng, 2, special=False) for q in range(0, n, 3)}
        phys.append((kind, singles, [(a, b, inputs.haar_unitary(rng))
                                     for a, b in c.lattice_couplings(lx, ly, kind)]))
        if kind >= 2:   # the reverse orientation of the same coupling
            phys.append((kind, {}, [(b, a, inputs.haar_unitary(rng))
                                    for a, b in c.lattice_couplings(lx, ly, kind)]))
    psi = sv.run_circuit(n, c.compile_2d(lx, ly, phys))
    np.testing.assert_allclose(psi, run_physical(n, phys), atol=1e-11)
