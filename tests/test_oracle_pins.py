"""Pins of the CPU oracle against what the paper and mathematics fix (no GPU needed).

Every test here checks the oracle against something other than itself: the brute-force
state vector, the dense Schmidt decomposition, closed forms (Theorem 1's single-bond case,
nu = (1-eps)^(-1/2)), the inequalities of Theorem 1 / Lemma 2 / Theorem 3, Theorem 4's step
count, textbook special cases, and explicit dense projector contractions.
"""

import numpy as np
import pytest

from oracle import ptebd_oracle as po
from oracle import statevector as sv
from paper_2312_02667_amd import inputs
from tests.dense_tools import dense_with_projectors, vidal_from_dense

CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], np.complex128)
HAD = np.array([[1, 1], [1, -1]], np.complex128) / np.sqrt(2.0)
I2 = np.eye(2, dtype=np.complex128)


# ----------------------------------------------------------------------------- generators

def test_haar_gates_are_unitary_and_haar_distributed():
    rng = np.random.default_rng(123)
    us = [inputs.haar_unitary(rng, 4, special=True) for _ in range(4000)]
    for u in us[:200]:
        assert np.linalg.norm(u.conj().T @ u - np.eye(4)) <= 1e-14 * 10
        assert abs(np.linalg.det(u) - 1.0) <= 1e-13
    p = np.array([abs(u[0, 0]) ** 2 for u in us])
    # |U_00|^2 of Haar U(n) is Beta(1, n-1): mean 1/n, second moment 2/(n(n+1))
    assert abs(p.mean() - 0.25) < 0.015
    assert abs((p ** 2).mean() - 0.1) < 0.01


def test_brickwork_layout():
    assert list(inputs.brickwork_bonds(10, 1)) == [0, 2, 4, 6, 8]
    assert list(inputs.brickwork_bonds(10, 2)) == [1, 3, 5, 7]
    assert list(inputs.brickwork_bonds(5, 1)) == [0, 2]
    assert list(inputs.brickwork_bonds(5, 2)) == [1, 3]


# ----------------------------------------------------------------------------- gate convention

def test_gate_convention_cnot_control_is_left_site():
    # |1 0> --CNOT(control = left site q)--> |1 1>, in both the state vector and the MPS.
    x = np.array([[0, 1], [1, 0]], np.complex128)
    flip_left = np.kron(x, I2)
    psi = sv.zero_state(2)
    psi = sv.apply_gate(psi, 2, 0, flip_left)
    psi = sv.apply_gate(psi, 2, 0, CNOT)
    assert abs(psi[3] - 1.0) < 1e-15
    mps = po.product_state(2)
    po.apply_layer(mps, [0], [flip_left], chi_max=4)
    po.apply_layer(mps, [0], [CNOT], chi_max=4)
    assert np.allclose(po.to_dense(mps), psi, atol=1e-14)
    assert np.allclose(po.expect_z(mps), [-1.0, -1.0], atol=1e-14)


def test_swap_moves_excitation():
    x = np.array([[0, 1], [1, 0]], np.complex128)
    mps = po.product_state(3)
    po.apply_layer(mps, [0], [np.kron(x, I2)], chi_max=4)
    po.apply_layer(mps, [0], [SWAP], chi_max=4)
    po.apply_layer(mps, [1], [SWAP], chi_max=4)
    assert np.allclose(po.expect_z(mps), [1.0, 1.0, -1.0], atol=1e-14)


# ----------------------------------------------------------------------------- special cases

def test_bell_pair_schmidt_values():
    # CNOT (H x I)|00> = (|00> + |11>)/sqrt2: Lambda = (1/sqrt2, 1/sqrt2), entropy ln 2.
    mps = po.product_state(2)
    stats, _ = po.apply_layer(mps, [0], [CNOT @ np.kron(HAD, I2)], chi_max=4)
    lam = mps.lam[1]
    assert np.allclose(lam, [2 ** -0.5, 2 ** -0.5], atol=1e-15)
    ent = -np.sum(lam ** 2 * np.log(lam ** 2))
    assert abs(ent - np.log(2.0)) < 1e-14
    assert stats[0]["eps"] == 0.0 and stats[0]["nu"] == 1.0


def test_two_sites_reduce_to_plain_svd():
    # N = 2: one bond; theta is the 2x2 amplitude matrix of U|00>; Lambda = its singular values.
    rng = np.random.default_rng(5)
    u = inputs.haar_unitary(rng)
    mps = po.product_state(2)
    po.apply_layer(mps, [0], [u], chi_max=4)
    s_ref = np.linalg.svd(u[:, 0].reshape(2, 2), compute_uv=False)
    assert np.allclose(mps.lam[1], s_ref, atol=1e-15)


def test_product_gates_keep_bond_dimension_one():
    rng = np.random.default_rng(6)
    mps = po.product_state(6)
    for layer in (1, 2, 1):
        bonds = inputs.brickwork_bonds(6, layer)
        gates = [np.kron(inputs.haar_unitary(rng, 2, False), inputs.haar_unitary(rng, 2, False))
                 for _ in bonds]
        po.apply_layer(mps, bonds, gates, chi_max=8)
    assert mps.bond_dims() == [1] * 7


# ----------------------------------------------------------------------------- exact evolution

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_untruncated_circuit_matches_statevector(seed):
    """Small-circuit check: N=10, depth 8, chi_max=32 (exact), Haar U(4): oracle vs brute force."""
    n, depth = 10, 8
    layers = inputs.brickwork_circuit(n, depth, seed, special=False)
    psi = sv.run_circuit(n, layers)
    mps = po.product_state(n)
    for bonds, gates in layers:
        stats, trig = po.apply_layer(mps, bonds, gates, chi_max=32, cutoff=1e-12)
        assert not trig
        for st in stats:
            assert st["eps"] <= 1e-20 and st["nu"] == 1.0
    dense = po.to_dense(mps)
    assert 1.0 - sv.fidelity(psi, dense) <= 1e-12
    assert abs(po.norm(mps) - 1.0) <= 1e-12
    assert np.max(np.abs(po.expect_z(mps) - sv.expect_z(psi, n))) <= 1e-12
    # exact TEBD keeps the canonical form: every Lambda is the state's Schmidt spectrum
    for i in range(1, n):
        ref = sv.schmidt_values(psi, n, i)
        lam = mps.lam[i]
        assert np.allclose(lam, ref[: len(lam)], atol=1e-12)
        assert np.all(ref[len(lam):] <= 1e-10)
    assert po.canon_distance(mps) <= 1e-11


# ----------------------------------------------------------------------------- truncation closed forms

def _canonical_random_state(n, seed, depth=4):
    layers = inputs.brickwork_circuit(n, depth, seed, special=True)
    psi = sv.run_circuit(n, layers)
    g, l = vidal_from_dense(psi, n)
    return psi, po.VidalMPS(g, l)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_single_bond_truncation_closed_form(seed):
    """Canonical input, one gate, truncation at one bond: the kept state is the orthogonal
    projection onto the top-k Schmidt subspace, so ||Psi_T||^2 = 1 - eps and 1 - F_2 = eps;
    with nu = (1-eps)^(-1/2) the norm is restored to 1 exactly."""
    n = 8
    psi, mps = _canonical_random_state(n, seed)
    rng = np.random.default_rng(100 + seed)
    u = inputs.haar_unitary(rng)
    q = 3
    exact = sv.apply_gate(psi, n, q, u)
    for stabilize in (False, True):
        m = mps.copy()
        stats, _ = po.apply_layer(m, [q], [u], chi_max=3, cutoff=1e-12, stabilize=stabilize)
        eps = stats[0]["eps"]
        assert eps > 1e-4
        d = po.to_dense(m)
        nrm2 = np.vdot(d, d).real
        if stabilize:
            assert abs(stats[0]["nu"] - (1 - eps) ** -0.5) < 1e-15
            assert abs(nrm2 - 1.0) < 1e-12
        else:
            assert abs(nrm2 - (1.0 - eps)) < 1e-12
        f2 = abs(np.vdot(exact, d)) ** 2 / nrm2
        assert abs((1.0 - f2) - eps) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_parallel_compression_theorems(seed):
    """Random canonical MPS, every bond truncated at once (Sec. III.B):
    explicit projector contraction == oracle compression; Theorem 1 (||Psi - Psi_T||^2 <= 2 eps,
    F_2 >= 1 - 2 eps), Lemma 2 (1 - sqrt(2 eps) <= n <= 1), Theorem 3 bounds on n*."""
    n = 10
    psi, mps = _canonical_random_state(n, seed, depth=5)
    chi_keep = 5
    comp = mps.copy()
    info = po.parallel_compress(comp, chi_keep, stabilize=False)
    keep = {i: min(chi_keep, len(mps.lam[i])) for i in range(1, n)}
    ref = dense_with_projectors(mps.gam, mps.lam, keep)
    d = po.to_dense(comp)
    assert np.allclose(d, ref, atol=1e-12)
    eps = sum(info["eps"].values())
    assert 0 < eps
    diff2 = np.vdot(psi - d, psi - d).real
    nrm = np.sqrt(np.vdot(d, d).real)
    f2 = abs(np.vdot(psi, d)) ** 2 / nrm ** 2
    assert diff2 <= 2 * eps + 1e-12
    assert f2 >= 1 - 2 * eps - 1e-12
    assert 1 - np.sqrt(2 * eps) - 1e-12 <= nrm <= 1 + 1e-12
    assert f2 >= 1 - 2 * sum(np.sqrt(e) for e in info["eps"].values()) - 1e-12
    assert abs(po.norm(comp) - nrm) < 1e-12
    # Theorem 3
    stab = mps.copy()
    info_s = po.parallel_compress(stab, chi_keep, stabilize=True)
    prod_nu = np.prod(list(info_s["nu"].values()))
    n_star = po.norm(stab)
    assert abs(n_star - nrm * prod_nu) < 1e-12
    lower = (1 - np.sqrt(2 * eps)) * prod_nu
    assert lower - 1e-12 <= n_star <= prod_nu + 1e-12
    assert lower <= 1 + 1e-12 and prod_nu >= 1 - 1e-12


def test_layer_truncation_equals_projected_exact_layer():
    """Truncating inside the bond update == exact layer, then projector on the updated bonds."""
    n = 10
    psi, mps = _canonical_random_state(n, 7, depth=4)
    rng = np.random.default_rng(77)
    bonds = inputs.brickwork_bonds(n, 1)
    gates = [inputs.haar_unitary(rng) for _ in bonds]
    exact = mps.copy()
    po.apply_layer(exact, bonds, gates, chi_max=64, cutoff=0.0)
    trunc = mps.copy()
    po.apply_layer(trunc, bonds, gates, chi_max=4, cutoff=0.0, stabilize=False)
    keep = {int(q) + 1: min(4, len(exact.lam[int(q) + 1])) for q in bonds}
    ref = dense_with_projectors(exact.gam, exact.lam, keep)
    assert np.allclose(po.to_dense(trunc), ref, atol=1e-12)


# ----------------------------------------------------------------------------- tSU / PtSU

def test_ptsu_preserves_state_and_norm():
    n = 10
    psi, mps = _canonical_random_state(n, 11, depth=5)
    po.parallel_compress(mps, 4, stabilize=True)
    before = po.to_dense(mps)
    m = mps.copy()
    for _ in range(3):
        po.ptsu_step(m, cutoff=1e-14)
        after = po.to_dense(m)
        assert np.allclose(after, before, atol=1e-12 * np.max(np.abs(before)) * 10)
    assert abs(po.norm(m) - po.norm(mps)) < 1e-12


def test_ipmc_trigger_runs_ptsu_only_when_compressed():
    n = 8
    layers = inputs.brickwork_circuit(n, 6, 3)
    a = po.product_state(n)
    b = po.product_state(n)
    for bonds, gates in layers:
        _, trig_a = po.apply_layer(a, bonds, gates, chi_max=64, ptsu_steps=0)
        _, trig_b = po.apply_layer(b, bonds, gates, chi_max=64, ptsu_steps=2)
        assert not trig_a and not trig_b
    for x, y in zip(a.gam, b.gam):
        assert np.array_equal(x, y)
    c = po.product_state(n)
    d = po.product_state(n)
    any_trig = False
    for bonds, gates in layers:
        _, t1 = po.apply_layer(c, bonds, gates, chi_max=3, ptsu_steps=0)
        _, t2 = po.apply_layer(d, bonds, gates, chi_max=3, ptsu_steps=1)
        any_trig |= t1
    assert any_trig
    assert po.canon_distance(d) < po.canon_distance(c)


# ----------------------------------------------------------------------------- queries

def test_canon_distance_hand_example():
    # N=2 product state: Gamma[0] = (2, 0), Gamma[1] = (1, 0), Lambda[1] = 0.3.
    # alpha = |Gamma0|^2 = 4, gamma = 1 -> C = (|4-1| + |1-1| + |1/4-1| + |1-1|)/4 = 0.9375
    g0 = np.array([2.0, 0.0]).reshape(1, 2, 1)
    g1 = np.array([1.0, 0.0]).reshape(1, 2, 1)
    mps = po.VidalMPS([g0, g1], [np.ones(1), np.array([0.3]), np.ones(1)])
    assert abs(po.canon_distance(mps) - 0.9375) < 1e-15


def test_queries_match_dense():
    n = 8
    ga, la = inputs.random_vidal_state(n, 6, seed=1)
    gb, lb = inputs.random_vidal_state(n, 5, seed=2)
    a = po.VidalMPS(ga, la)
    b = po.VidalMPS(gb, lb)
    da, db = po.to_dense(a), po.to_dense(b)
    assert abs(po.overlap(a, b) - np.vdot(da, db)) < 1e-12 * max(1, abs(np.vdot(da, db)))
    assert abs(po.norm(a) - np.linalg.norm(da)) < 1e-12
    assert np.max(np.abs(po.expect_z(a) - sv.expect_z(da, n))) < 1e-12


def test_canonicalize_matches_schmidt_decomposition():
    n = 9
    ga, la = inputs.random_vidal_state(n, 8, seed=4)
    a = po.VidalMPS(ga, la)
    dense = po.to_dense(a)
    c, nrm = po.canonicalize(a)
    assert abs(nrm - np.linalg.norm(dense)) < 1e-12 * nrm
    assert np.allclose(po.to_dense(c) * nrm, dense, atol=1e-12 * nrm)
    for i in range(1, n):
        ref = sv.schmidt_values(dense / nrm, n, i)
        assert np.allclose(c.lam[i], ref[: len(c.lam[i])], atol=1e-12)
    assert po.canon_distance(c) < 1e-12


@pytest.mark.parametrize("n_sites", [20, 24])
def test_theorem4_ptsu_restores_canonical_form(n_sites):
    """Sec. III.D protocol: random MPS (entries a+ib, a,b~U[-1,1]), canonicalize, truncate
    every bond to chi/2, renormalize, then PtSU steps.  C falls and the canonical form is
    exact after N/2 steps (Theorem 4)."""
    chi = 16
    curves = []
    for seed in range(3):
        m = inputs.random_mps_tensors(n_sites, chi, seed)
        raw = po.VidalMPS(m, [np.ones(len(x)) for x in
                              [np.ones(1)] + [np.ones(t.shape[2]) for t in m]])
        can, _ = po.canonicalize(raw)
        po.parallel_compress(can, chi // 2, stabilize=False)
        po.scale_norm(can, 1.0 / po.norm(can))
        curve = [po.canon_distance(can)]
        for _ in range(n_sites // 2):
            po.ptsu_step(can, cutoff=1e-15)
            curve.append(po.canon_distance(can))
        assert abs(po.norm(can) - 1.0) < 1e-10
        curves.append(curve)
    curves = np.array(curves)
    mean = curves.mean(axis=0)
    assert mean[0] > 1e-3
    assert np.all(curves[:, -1] <= 1e-10)
    assert np.all(np.diff(mean[: n_sites // 4]) < 0)


def test_relative_eps_reading():
    """On a normalized canonical input the relative and the literal eps coincide; on any
    input the relative reading keeps each updated bond's local two-site norm."""
    n = 8
    psi, mps = _canonical_random_state(n, 21)
    rng = np.random.default_rng(210)
    u = inputs.haar_unitary(rng)
    a, b = mps.copy(), mps.copy()
    sa, _ = po.apply_layer(a, [3], [u], chi_max=3)
    sb, _ = po.apply_layer(b, [3], [u], chi_max=3, eps_reading="relative")
    assert abs(sa[0]["eps"] - sb[0]["eps"]) < 1e-14
    # non-normalized input: scale the state by 1.3, local norm^2 of theta is 1.69
    c = mps.copy()
    po.scale_norm(c, 1.3)
    theta = po.two_site_theta(c, 3, u)
    before = np.sum(np.abs(theta) ** 2)
    st, _ = po.apply_layer(c, [3], [u], chi_max=3, eps_reading="relative")
    assert abs(np.sum(c.lam[4] ** 2) - before) < 1e-12 * before
    assert abs(st[0]["eps"] - np.sum(st[0]["sigma"][3:] ** 2) / before) < 1e-14


@pytest.mark.parametrize("scale", [1.0, 0.8, 1.25])
def test_eps_readings_on_a_scaled_canonical_state(scale):
    """All three readings of Theorem 1's local error agree on a normalized canonical input.
    On the same state scaled by c (theta's singular values scale by c, eps_c is the canonical
    discarded weight), the updated bond's sum Lambda^2 is closed-form:
    literal c^2 (1 - eps_c) / (1 - c^2 eps_c) (> c^2 when c > 1: norm 1 repels);
    relative c^2 (the local norm is kept); complement 1 (nu rescales to unit norm)."""
    n = 8
    _, mps = _canonical_random_state(n, 22)
    u = inputs.haar_unitary(np.random.default_rng(220))
    base = mps.copy()
    sc, _ = po.apply_layer(base, [3], [u], chi_max=3)
    eps_c = sc[0]["eps"]
    assert 1e-4 < eps_c < 0.5
    expect = {"literal": scale ** 2 * (1 - eps_c) / (1 - scale ** 2 * eps_c),
              "relative": scale ** 2, "complement": 1.0}
    for reading, want in expect.items():
        m = mps.copy()
        m.lam[4] = scale * m.lam[4]        # the state, and theta at q = 3, scale by c
        st, _ = po.apply_layer(m, [3], [u], chi_max=3, eps_reading=reading)
        assert abs(np.sum(m.lam[4] ** 2) - want) < 1e-12
        if scale == 1.0:
            assert abs(st[0]["eps"] - eps_c) < 1e-13
    with pytest.raises(ValueError):
        po.apply_layer(mps.copy(), [3], [u], chi_max=3, eps_reading="other")


def _dense_schmidt(psi, n, cut):
    """Schmidt values of a state vector across the cut after site ``cut - 1``."""
    return np.linalg.svd(np.asarray(psi).reshape(2 ** cut, 2 ** (n - cut)), compute_uv=False)


@pytest.mark.parametrize("reading", ["literal", "complement"])
def test_nu_only_on_compressed_layers(reading):
    """Algorithm 1 compresses (IPMC: projector truncation, then nu, then PtSU) only when the
    layer's new bond dimension exceeds chi ("if chi~ > chi"); otherwise the TEBD result is kept
    as it is.  A canonical state with bond 1 scaled by c1 = 0.9 and bond 4 by c4 = 1.3 is the
    unit-norm canonical state times c1 c4, and after gates at q = 0 and q = 3 the local
    two-site wavefunctions carry the singular values c1 s1 and c4 s4, where c1 c4 s_i are the
    dense state's Schmidt values across the cut (unit-norm s_i).  So:
      * untriggered (chi_max = 16): Lambda[1] = c1 s1 and Lambda[4] = c4 s4, unscaled, nu = 1;
      * triggered (chi_max = 3, only bond 4 truncated): Lambda[4] = nu4 * the top 3 of c4 s4,
        and the untruncated bond 1 is multiplied by its own nu1 as well: under the complement
        reading nu1 = 1 / c1, under the literal one nu1 = 1 (nothing discarded)."""
    n, c1, c4 = 8, 0.9, 1.3
    _, mps = _canonical_random_state(n, 23)
    u = inputs.haar_unitary(np.random.default_rng(230))
    v = inputs.haar_unitary(np.random.default_rng(231))
    base = mps.copy()
    base.lam[1] = c1 * base.lam[1]
    base.lam[4] = c4 * base.lam[4]
    after = sv.apply_gate(sv.apply_gate(po.to_dense(base), n, 3, u), n, 0, v)
    loc = {4: _dense_schmidt(after, n, 4) / c1, 1: _dense_schmidt(after, n, 1) / c4}
    m = base.copy()
    st, trig = po.apply_layer(m, [3, 0], [u, v], chi_max=16, eps_reading=reading)
    assert not trig
    assert [x["nu"] for x in st] == [1.0, 1.0]
    for bond, scale in ((4, c4), (1, c1)):
        k = len(m.lam[bond])
        assert np.max(np.abs(m.lam[bond] - loc[bond][:k])) < 1e-13
        assert abs(np.sum(m.lam[bond] ** 2) - scale ** 2) < 1e-12
    m = base.copy()
    st, trig = po.apply_layer(m, [3, 0], [u, v], chi_max=3, eps_reading=reading)
    assert trig and st[0]["r"] > 3 and st[1]["r"] <= 3
    for idx, bond in enumerate((4, 1)):
        sref = loc[bond]
        k = len(m.lam[bond])
        kept2 = float(np.sum(sref[:k] ** 2))
        eps = float(np.sum(sref[k:] ** 2)) if reading == "literal" else 1.0 - kept2
        assert abs(st[idx]["eps"] - eps) < 1e-12
        nu = (1.0 - eps) ** -0.5
        assert abs(st[idx]["nu"] - nu) < 1e-12
        assert np.max(np.abs(m.lam[bond] - nu * sref[:k])) < 1e-12
    if reading == "complement":
        assert abs(st[1]["nu"] - 1.0 / c1) < 1e-12
        assert abs(np.sum(m.lam[4] ** 2) - 1.0) < 1e-12
    else:
        assert abs(st[1]["nu"] - 1.0) < 1e-12


def test_norm_stabilization_ablation_rqc_1d():
    """Sec. IV.B, numerical stability (the norm-vs-depth figure): without nu the norm of a truncated RQC-1D decays
    monotonically and exponentially; with nu under the complement reading it stays near 1.
    Under the literal reading the stabilized norm leaves that band within the same circuit
    (norm 1 is a repelling fixed point, see the scaled-state pin above)."""
    from paper_2312_02667_amd import circuits
    n, depth, chi = 21, 160, 4
    layers = circuits.rqc_1d(n, depth, seed=8)
    states = {"none": po.product_state(n), "complement": po.product_state(n),
              "literal": po.product_state(n)}
    norms = {k: [] for k in states}
    for bonds, gates in layers:
        po.apply_layer(states["none"], bonds, gates, chi_max=chi, stabilize=False)
        po.apply_layer(states["complement"], bonds, gates, chi_max=chi, eps_reading="complement")
        if states["literal"] is not None:
            try:
                po.apply_layer(states["literal"], bonds, gates, chi_max=chi)
            except po.AnnihilatedError:      # a discarded weight reached 1
                states["literal"] = None
        for k, m in states.items():
            norms[k].append(np.inf if m is None else po.norm(m))
    none = np.array(norms["none"])
    assert np.all(np.diff(none) <= 1e-12)                  # monotone decay
    assert none[-1] < 1e-5
    # exponential: the decay rate of log n over the second and the last quarter agree
    q = depth // 4
    r2 = (np.log(none[2 * q]) - np.log(none[q])) / q
    r4 = (np.log(none[-1]) - np.log(none[3 * q])) / (depth - 1 - 3 * q)
    assert r2 < 0 and r4 < 0 and 0.5 < r4 / r2 < 2.0
    comp = np.array(norms["complement"])
    assert np.all((comp > 0.8) & (comp < 1.25))
    lit = np.array(norms["literal"])
    assert lit.max() > 1.5


def _dense_conditional_sample(psi, n, u):
    """Draws bits site by site from the exact conditional probabilities of the dense state."""
    p = np.abs(psi) ** 2
    bits = np.zeros(n, np.uint8)
    block = p.reshape(1, -1)
    for q in range(n):
        block = block.reshape(2, -1)
        p0, p1 = block[0].sum(), block[1].sum()
        b = 0 if u[q] < p0 / (p0 + p1) else 1
        bits[q] = b
        block = block[b]
    return bits


@pytest.mark.parametrize("seed", [0, 1])
def test_sampling_matches_dense_conditional_sampling(seed):
    """Perfect sampling on the canonicalized MPS equals inverse-CDF sampling from the exact
    conditional probabilities of the state vector, bit for bit, for the same uniforms."""
    n = 8
    m = po.product_state(n)
    for bonds, gates in inputs.brickwork_circuit(n, 6, seed):
        po.apply_layer(m, bonds, gates, chi_max=4)      # a truncated, non-canonical state
    psi = po.to_dense(m)
    can, nrm = po.canonicalize(m)
    rng = np.random.default_rng(100 + seed)
    u = rng.random((200, n))
    got = po.sample(can, u)
    for i in range(len(u)):
        assert np.array_equal(got[i], _dense_conditional_sample(psi, n, u[i]))
    assert abs(nrm - np.linalg.norm(psi)) < 1e-12


def test_sampling_special_cases_and_frequencies():
    """Product and GHZ states, and empirical frequencies against |psi|^2 (N = 5)."""
    n = 5
    # |1 0 1 1 0>: deterministic bits
    m = po.product_state(n)
    x = np.array([[0, 1], [1, 0]], np.complex128)
    for q in (0, 2, 3):
        po.apply_layer(m, [q if q < n - 1 else q - 1],
                       [np.kron(x, np.eye(2)) if q < n - 1 else np.kron(np.eye(2), x)], chi_max=4)
    can, _ = po.canonicalize(m)
    rng = np.random.default_rng(5)
    assert np.all(po.sample(can, rng.random((50, n))) == np.array([1, 0, 1, 1, 0], np.uint8))
    # GHZ: all bits equal, each value with probability 1/2
    h = np.array([[1, 1], [1, -1]], np.complex128) / np.sqrt(2)
    cnot = np.eye(4, dtype=np.complex128)[[0, 1, 3, 2]]
    g = po.product_state(n)
    po.apply_layer(g, [0], [cnot @ np.kron(h, np.eye(2))], chi_max=8)
    for q in range(1, n - 1):
        po.apply_layer(g, [q], [cnot], chi_max=8)
    can, _ = po.canonicalize(g)
    bits = po.sample(can, rng.random((4000, n)))
    assert np.all(bits == bits[:, :1])
    assert abs(bits[:, 0].mean() - 0.5) < 0.03
    # a random 5-qubit state: outcome frequencies within 5 standard deviations of |psi|^2
    r = po.product_state(n)
    for bonds, gates in inputs.brickwork_circuit(n, 6, 9):
        po.apply_layer(r, bonds, gates, chi_max=8)
    psi = po.to_dense(r)
    prob = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    can, _ = po.canonicalize(r)
    s = 20000
    bits = po.sample(can, rng.random((s, n)))
    idx = bits.astype(np.int64) @ (1 << np.arange(n - 1, -1, -1))
    freq = np.bincount(idx, minlength=2 ** n) / s
    assert np.all(np.abs(freq - prob) <= 5 * np.sqrt(prob * (1 - prob) / s) + 1e-12)


def test_layer_with_a_parallel_map_equals_the_ordered_layer():
    """The gates of a layer act on disjoint sites (Sec. II.C): applying them all at once
    through a thread pool gives the ordered result (Lambda, Gamma and stats)."""
    from concurrent.futures import ThreadPoolExecutor

    n = 12
    layers = inputs.brickwork_circuit(n, 8, seed=6)
    a, b = po.product_state(n), po.product_state(n)
    with ThreadPoolExecutor(4) as ex:
        for bonds, gates in layers:
            sa, ta = po.apply_layer(a, bonds, gates, chi_max=6, eps_reading="complement")
            sb, tb = po.apply_layer(b, bonds, gates, chi_max=6, eps_reading="complement",
                                    map_fn=ex.map)
            assert ta == tb
            assert [x["k"] for x in sa] == [x["k"] for x in sb]
            assert np.allclose([x["nu"] for x in sa], [x["nu"] for x in sb], rtol=0, atol=1e-14)
    assert max(float(np.max(np.abs(x - y))) for x, y in zip(a.lam, b.lam)) < 1e-13
    assert abs(po.overlap(a, b) - po.norm(a) ** 2) < 1e-12 * po.norm(a) ** 2
