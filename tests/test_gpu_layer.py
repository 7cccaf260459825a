"""Layer-level parity on the GPU: apply_layer (theta, SVD, truncation, nu, regauge, PtSU)
against the oracle on the same seeded circuits, and the exact queries against the oracle."""

import numpy as np
import pytest

from oracle import ptebd_oracle as po
from oracle import statevector as sv
from paper_2312_02667_amd import inputs, ptebd
from tests.gpu_util import lambda_diff, oracle_cutoff, say, to_oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("seed", [0, 1])
def test_small_exact_circuit(precision, seed):
    """N=10, depth 8, chi_max=32 (nothing truncated), Haar U(4): GPU vs oracle vs brute force."""
    n, depth = 10, 8
    layers = inputs.brickwork_circuit(n, depth, seed, special=False)
    psi = sv.run_circuit(n, layers)
    ref = po.product_state(n)
    m = ptebd.MPS(n, 32, precision)
    lam_tol = 1e-12 if precision == "fp64" else 2e-6
    for li, (bonds, gates) in enumerate(layers):
        say(f"small circuit {precision} seed={seed} layer {li + 1}")
        st = m.apply_layer(bonds, gates, chi_max=32, cutoff=1e-12)
        po.apply_layer(ref, bonds, gates, chi_max=32, cutoff=oracle_cutoff(1e-12, precision))
        assert not st["triggered"]
        assert m.bond_dims() == ref.bond_dims()
        assert lambda_diff(to_oracle(m), ref) <= lam_tol
        # nothing is compressed, so no nu is applied (Algorithm 1's "else" branch)
        assert np.all(st["nu"] == 1.0)
    f_tol = 1e-12 if precision == "fp64" else 1e-10
    dense = po.to_dense(to_oracle(m))
    assert 1 - sv.fidelity(psi, dense) <= f_tol
    # FP32 Jacobi rotations keep column norms to ~u sqrt(rotations per column) per update,
    # so the norm and <Z> carry a few 1e-7 after 36 gates (3.6e-7 and 3.9e-7 measured)
    assert abs(m.norm() - 1.0) <= (1e-12 if precision == "fp64" else 2e-6)
    assert np.max(np.abs(m.expect_z() - sv.expect_z(psi, n))) <= (1e-12 if precision == "fp64" else 2e-6)
    # FP32 recovers the left vectors as theta Y / sigma (preconditioned SVD): their
    # orthogonality error is ~u sigma_1 / sigma_j for the smallest kept sigma_j (absolute,
    # LAPACK-like accuracy), which the canonical distance sees directly: 6.9e-6 measured
    # with the Jacobi converged to u sqrt(R)
    assert m.canon_distance() <= (1e-10 if precision == "fp64" else 2e-5)
    m.close()


def test_truncated_circuit_fp64_matches_oracle():
    """N=100, depth 20, chi_max=64, cutoff 1e-12, Haar SU(4), FP64: per-layer bond dims,
    Lambda, eps and nu against the oracle; final fidelity, norm and <Z>."""
    n, depth, chi = 100, 20, 64
    layers = inputs.brickwork_circuit(n, depth, seed=0)
    ref = po.product_state(n)
    m = ptebd.MPS(n, chi, "fp64")
    for li, (bonds, gates) in enumerate(layers):
        say(f"N=100 chi=64 fp64 layer {li + 1}")
        st = m.apply_layer(bonds, gates, chi_max=chi, cutoff=1e-12)
        stats, trig = po.apply_layer(ref, bonds, gates, chi_max=chi, cutoff=1e-12)
        assert st["triggered"] == trig
        assert list(st["k"]) == [s["k"] for s in stats]
        # eps = sum of discarded sigma^2 and nu = (1-eps)^(-1/2) inherit the trajectory's
        # Lambda drift (bounded below by 1e-9): |d eps| <= 2 sum sigma |d sigma| <~ 1e-10
        assert np.max(np.abs(st["eps"] - np.array([s["eps"] for s in stats]))) <= 1e-10
        assert np.max(np.abs(st["nu"] - np.array([s["nu"] for s in stats]))) <= 1e-10
        assert lambda_diff(to_oracle(m), ref) <= 1e-9
    other = ptebd.MPS(n, chi, "fp64")
    other.import_state(ref.gam, ref.lam)
    ov = m.overlap(other)
    err_f = 1 - abs(ov) ** 2 / (m.norm() ** 2 * other.norm() ** 2)
    say(f"err_F = {err_f:.3e}, |n-1| = {abs(m.norm() - 1):.3e}")
    assert err_f <= 1e-10
    # under the literal eps reading the norm grows in this heavily truncated regime (about
    # 22 after 20 layers, for the oracle as well), so norms are compared relatively
    assert abs(m.norm() - po.norm(ref)) <= 1e-9 * po.norm(ref)
    assert np.max(np.abs(m.expect_z() - po.expect_z(ref))) <= 1e-9
    assert abs(m.norm_estimate() - ref.prod_nu) <= 1e-9 * ref.prod_nu
    assert abs(m.fidelity_estimate() - ref.prod_one_minus_eps) <= 1e-10
    m.close()
    other.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ptsu_and_no_stabilize_match_oracle(precision):
    """chi_max=6 with g=2 PtSU steps (IPMC), the nu ablation flag and the three eps
    readings, on N=12."""
    n, depth, chi = 12, 8, 6
    layers = inputs.brickwork_circuit(n, depth, seed=4)
    for stabilize, rel in ((True, "literal"), (False, "literal"), (True, "relative"),
                           (True, "complement"), (False, "complement")):
        ref = po.product_state(n)
        m = ptebd.MPS(n, 16, precision)
        for li, (bonds, gates) in enumerate(layers):
            say(f"ptsu {precision} stabilize={stabilize} eps_reading={rel} layer {li + 1}")
            st = m.apply_layer(bonds, gates, chi_max=chi, cutoff=1e-12, ptsu_steps=2,
                               stabilize=stabilize, eps_reading=rel)
            _, trig = po.apply_layer(ref, bonds, gates, chi_max=chi,
                                     cutoff=oracle_cutoff(1e-12, precision), ptsu_steps=2,
                                     stabilize=stabilize, eps_reading=rel)
            assert st["triggered"] == trig
            assert st["ptsu_done"] == (2 if trig else 0)
            assert m.bond_dims() == ref.bond_dims()
            # complement reading: nu rescales Lambda by the FP32 kept weight at every update
            # (~u sqrt(chi) relative each), so Lambda drifts like the norm bound below
            # (measured: 1.6e-5 complement, at most 1.1e-6 otherwise)
            lam_tol = 1e-10 if precision == "fp64" else (3e-5 if rel == "complement" else 3e-6)
            assert lambda_diff(to_oracle(m), ref) <= lam_tol
        # under the complement reading nu_i rescales by the kept weight of the FP32 theta,
        # whose squared norm carries ~u sqrt(chi) relative rounding: a few 1e-7 per update,
        # ~1e-5 over the ~90 updates (gates and tSU) of this circuit (2.4e-5 measured; at
        # most 1.1e-6 on the other readings)
        norm_tol = 1e-10 if precision == "fp64" else (5e-5 if rel == "complement" else 3e-6)
        assert abs(m.norm() - po.norm(ref)) <= norm_tol
        # 9.2e-6 measured under the complement reading, at most 4.1e-7 otherwise
        assert abs(m.canon_distance() - po.canon_distance(ref)) <= (1e-9 if precision == "fp64" else 2e-5)
        m.close()


def test_theorem4_ptsu_on_gpu():
    """Sec. III.D protocol prepared by the oracle; N/2 PtSU steps on the GPU restore the
    canonical form (Theorem 4) while keeping the norm."""
    n, chi = 20, 16
    mt = inputs.random_mps_tensors(n, chi, seed=0)
    raw = po.VidalMPS(mt, [np.ones(1)] + [np.ones(t.shape[2]) for t in mt])
    can, _ = po.canonicalize(raw)
    po.parallel_compress(can, chi // 2)
    po.scale_norm(can, 1.0 / po.norm(can))
    m = ptebd.MPS(n, chi, "fp64")
    m.import_state(can.gam, can.lam)
    c0 = m.canon_distance()
    assert abs(c0 - po.canon_distance(can)) <= 1e-12
    say(f"C before PtSU {c0:.3e}")
    m.ptsu(n // 2, cutoff=1e-15)
    c1 = m.canon_distance()
    say(f"C after {n // 2} PtSU steps {c1:.3e}")
    assert c0 > 1e-3 and c1 <= 1e-10
    assert abs(m.norm() - 1.0) <= 1e-10
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_queries_match_oracle(precision):
    n = 12
    ga, la = inputs.random_vidal_state(n, 16, seed=11)
    gb, lb = inputs.random_vidal_state(n, 12, seed=12)
    a, b = po.VidalMPS(ga, la), po.VidalMPS(gb, lb)
    ma = ptebd.MPS(n, 16, precision)
    mb = ptebd.MPS(n, 16, "fp64")
    ma.import_state(ga, la)
    mb.import_state(gb, lb)
    # an imported state: FP32 storage rounding only (norm 8.9e-9 relative measured)
    tol = 1e-12 if precision == "fp64" else 1e-6
    say(f"queries {precision}")
    assert abs(ma.norm() - po.norm(a)) <= tol * po.norm(a)
    ov = ma.overlap(mb)
    ref = po.overlap(a, b)
    assert abs(ov - ref) <= tol * po.norm(a) * po.norm(b)
    assert np.max(np.abs(ma.expect_z() - po.expect_z(a))) <= tol * 10
    assert abs(ma.canon_distance() - po.canon_distance(a)) <= tol * 10 * po.canon_distance(a)
    ma.close()
    mb.close()


def test_layer_errors_leave_state_unchanged():
    n = 6
    m = ptebd.MPS(n, 8, "fp64")
    rng = np.random.default_rng(0)
    u = inputs.haar_unitary(rng)
    m.apply_layer([0, 2, 4], [u, u, u], chi_max=8)
    before = to_oracle(m)
    bad = [
        (dict(bonds=[0, 1], gates=[u, u], chi_max=8), ptebd.EOVERLAP),
        (dict(bonds=[5], gates=[u], chi_max=8), ptebd.EINVAL),
        (dict(bonds=[0], gates=[u * np.nan], chi_max=8), ptebd.EINVAL),
        (dict(bonds=[0], gates=[u], chi_max=9), ptebd.EINVAL),
        (dict(bonds=[0], gates=[u], chi_max=8, cutoff=-1.0), ptebd.EINVAL),
    ]
    for kwargs, code in bad:
        with pytest.raises(ptebd.PtebdError) as ei:
            m.apply_layer(**kwargs)
        assert ei.value.code == code
    after = to_oracle(m)
    assert lambda_diff(before, after) == 0.0
    for x, y in zip(before.gam, after.gam):
        assert np.array_equal(x, y)
    m.close()


@pytest.mark.parametrize("precision,n,scaled", [("fp32", 8, 4), ("fp64", 8, 4), ("fp32", 130, 100)])
def test_device_error_leaves_state_unchanged(precision, n, scaled):
    """An error found on the device commits nothing.  Lambda[scaled] is multiplied by 10, so
    the gate at q = scaled - 1 sees sum sigma^2 near 100 and, cut to chi = 2 under the literal
    reading, a discarded weight above 1 (EANNIHILATED: nu = (1 - eps)^(-1/2) does not exist,
    Eq. (lren)).  That is known only after theta, the SVD and the truncation have run for
    every gate of the layer; Gamma, Lambda, the bond dimensions and the estimates must still
    be bit-identical afterwards.  At n = 130 the odd layer has 64 gates and runs as two
    halves on two streams, and the failing gate sits in the second half.  The handle keeps
    working: the same layer without truncation then matches the oracle."""
    chi = 16 if n == 8 else 8
    layers = inputs.brickwork_circuit(n, 6, seed=5)
    m = ptebd.MPS(n, chi, precision)
    for bonds, gates in layers:
        m.apply_layer(bonds, gates, chi_max=chi)
    ref = to_oracle(m)
    lam = [x.copy() for x in ref.lam]
    lam[scaled] = lam[scaled] * 10.0
    m.import_state(ref.gam, lam)
    before, dims = to_oracle(m), m.bond_dims()
    est = (m.norm_estimate(), m.fidelity_estimate())
    bonds, gates = layers[1]
    assert scaled - 1 in list(bonds)
    with pytest.raises(ptebd.PtebdError) as ei:
        m.apply_layer(bonds, gates, chi_max=2)
    assert ei.value.code == ptebd.EANNIHILATED
    after = to_oracle(m)
    assert m.bond_dims() == dims
    assert (m.norm_estimate(), m.fidelity_estimate()) == est
    for x, y in zip(before.lam, after.lam):
        assert np.array_equal(x, y)
    for x, y in zip(before.gam, after.gam):
        assert np.array_equal(x, y)
    m.apply_layer(bonds, gates, chi_max=chi, stabilize=False)
    po.apply_layer(before, bonds, gates, chi_max=chi, cutoff=oracle_cutoff(1e-12, precision),
                   stabilize=False)
    scale = max(float(np.max(x)) for x in before.lam)
    assert lambda_diff(before, to_oracle(m)) <= (1e-4 if precision == "fp32" else 1e-10) * scale
    m.close()


def test_kernel_profiling_counts_launches():
    n = 16
    layers = inputs.brickwork_circuit(n, 6, seed=2)
    m = ptebd.MPS(n, 32, "fp32")
    m.set_profiling(True)
    for bonds, gates in layers:
        m.apply_layer(bonds, gates, chi_max=16)
    st = m.kernel_stats()
    say(str(st))
    for name in ("theta", "jacobi", "finalize", "writeback"):
        assert st[name]["launches"] > 0 and st[name]["total_ms"] > 0
    assert st["theta"]["launches"] == len(layers)
    assert st["jacobi"]["flops"] > 0 and st["theta"]["flops"] > 0
    m.set_profiling(False)
    m.close()


def test_svd_params_round_trip_and_validation():
    m = ptebd.MPS(6, 8, "fp32")
    p = m.svd_params()
    assert p == {"max_sweeps": 30, "tol_factor": 1.0, "inner_sweeps": 2, "inner_repeat": 1e-2,
                 "sort_pairs": 1, "precondition": 1, "streams": 2, "block_cols": 16,
                 "graphs": 1}
    m.set_svd_params(inner_sweeps=3, inner_repeat=0.0, precondition=False)
    q = m.svd_params()
    assert q["inner_sweeps"] == 3 and q["inner_repeat"] == 0.0 and q["precondition"] == 0
    for bad in (dict(max_sweeps=0), dict(tol_factor=-1.0), dict(inner_sweeps=65),
                dict(inner_repeat=-1.0), dict(inner_repeat=float("inf")), dict(sort_pairs=2),
                dict(precondition=3), dict(streams=0), dict(streams=3), dict(block_cols=24),
                dict(graphs=2)):
        with pytest.raises(ptebd.PtebdError):
            m.set_svd_params(**bad)
        assert m.svd_params() == q          # nothing changed
    with pytest.raises(TypeError):
        m.set_svd_params(unknown=1)
    m.close()
    d = ptebd.MPS(6, 8, "fp64")
    assert d.svd_params()["inner_sweeps"] == 1 and d.svd_params()["inner_repeat"] == 0.0
    assert d.svd_params()["tol_factor"] == 4.0
    with pytest.raises(ptebd.PtebdError):
        d.set_svd_params(block_cols=32)      # 32-column blocks: FP32 handles only
    d.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("reading", ["literal", "complement"])
def test_nu_only_on_compressed_layers_matches_oracle(precision, reading):
    """A canonical state with two bonds scaled (0.9, 1.3), gates at q = 3 and q = 0: with
    chi_max = 16 nothing is compressed and both bonds keep their singular values (nu = 1); with
    chi_max = 3 the layer is compressed and both bonds, the untruncated one too, are
    multiplied by their nu.  Lambda, eps and nu against the oracle."""
    n = 8
    g, l = inputs.random_vidal_state(n, 8, seed=5)
    raw = po.VidalMPS(g, l)
    can, _ = po.canonicalize(raw)
    po.scale_norm(can, 1.0 / po.norm(can))
    can.lam[1] = 0.9 * can.lam[1]
    can.lam[4] = 1.3 * can.lam[4]
    rng = np.random.default_rng(50)
    gates = [inputs.haar_unitary(rng), inputs.haar_unitary(rng)]
    tol = 1e-12 if precision == "fp64" else 2e-6
    for chi_max, want_trig in ((16, False), (3, True)):
        say(f"nu trigger {precision} {reading} chi_max={chi_max}")
        ref = can.copy()
        stats, trig = po.apply_layer(ref, [3, 0], gates, chi_max=chi_max,
                                     cutoff=oracle_cutoff(1e-12, precision), eps_reading=reading)
        assert trig == want_trig
        m = ptebd.MPS(n, 16, precision)
        m.import_state(can.gam, can.lam)
        st = m.apply_layer([3, 0], gates, chi_max=chi_max, cutoff=1e-12, eps_reading=reading)
        assert st["triggered"] == want_trig
        assert m.bond_dims() == ref.bond_dims()
        assert lambda_diff(to_oracle(m), ref) <= tol
        assert np.max(np.abs(st["nu"] - np.array([x["nu"] for x in stats]))) <= tol
        assert np.max(np.abs(st["eps"] - np.array([x["eps"] for x in stats]))) <= tol
        if not want_trig:
            assert np.all(st["nu"] == 1.0)
        m.close()


def test_overlap_of_handles_on_different_streams():
    """Two handles on two different HIP streams: the overlap query runs every kernel on the
    first handle's stream (the second's site tensors are staged in the first's scratch), so
    the result matches the oracle."""
    n = 12
    ga, la = inputs.random_vidal_state(n, 16, seed=31)
    gb, lb = inputs.random_vidal_state(n, 16, seed=32)
    sa, sb = ptebd.Stream(), ptebd.Stream()
    ma = ptebd.MPS(n, 16, "fp64", stream=sa)
    mb = ptebd.MPS(n, 16, "fp32", stream=sb)
    ma.import_state(ga, la)
    mb.import_state(gb, lb)
    a, b = po.VidalMPS(ga, la), to_oracle(mb)
    ref = po.overlap(a, b)
    for _ in range(3):
        ov = ma.overlap(mb)
        assert abs(ov - ref) <= 1e-12 * po.norm(a) * po.norm(b)
        ov2 = mb.overlap(ma)
        assert abs(ov2 - np.conj(ref)) <= 1e-12 * po.norm(a) * po.norm(b)
    ma.close()
    mb.close()
    sa.close()
    sb.close()
