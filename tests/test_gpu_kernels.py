"""Kernel-level parity on the GPU: the theta contraction against the oracle's two-site
wavefunction, and the batched Jacobi SVD against LAPACK on the spectra families of the
workload (Gaussian, graded to 1e-12, near-degenerate, rank-deficient, Haar-circuit theta)."""

import zlib

import numpy as np
import pytest

from oracle import ptebd_oracle as po
from paper_2312_02667_amd import inputs, ptebd
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

# FP64: products of O(1) numbers, K <= 64 terms -> relative error ~1e-15; FP32 inputs and
# accumulation are rounded to 2^-24 -> ~1e-7 relative, 20x margin.
THETA_TOL = {"fp64": 1e-13, "fp32": 2e-6}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_theta_matches_oracle(precision):
    n, chi = 14, 40  # bulk bonds 40 (one full 32-tile plus a ragged 8), edges 1..32
    g, l = inputs.random_vidal_state(n, chi, seed=3)
    ref = po.VidalMPS(g, l)
    m = ptebd.MPS(n, 64, precision)
    m.import_state(g, l)
    rng = np.random.default_rng(9)
    for q in [0, 1, 3, 6, 7, 11, 12]:
        for gate in [inputs.haar_unitary(rng), None]:
            say(f"theta {precision} q={q} gate={'haar' if gate is not None else 'identity'}")
            th = m.debug_theta(q, gate)
            th_ref = po.two_site_theta(ref, q, gate)
            assert th.shape == th_ref.shape
            err = np.max(np.abs(th - th_ref)) / np.max(np.abs(th_ref))
            assert err < THETA_TOL[precision], err
    m.close()


def _haar_theta(rng, chi):
    """theta of a Haar gate on a random (non-canonical) chi x 2 x chi pair."""
    n = 2 * max(1, int(np.ceil(np.log2(chi)))) + 4
    g, l = inputs.random_vidal_state(n, chi, seed=int(rng.integers(1 << 30)))
    mps = po.VidalMPS(g, l)
    q = n // 2 - 1
    assert len(mps.lam[q]) == len(mps.lam[q + 1]) == len(mps.lam[q + 2]) == chi
    return po.two_site_theta(mps, q, inputs.haar_unitary(rng))


def _matrices(kind, rng, m, n):
    k = min(m, n)
    if kind == "gauss":
        return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    uu, _ = np.linalg.qr(rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k)))
    vv, _ = np.linalg.qr(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
    if kind == "graded":
        s = 10.0 ** np.linspace(0, -12, k)
    elif kind == "degenerate":
        s = np.repeat(np.linspace(1.0, 0.1, (k + 1) // 2), 2)[:k]
        s[1::2] *= 1 + 1e-10
    elif kind == "rankdef":
        s = np.zeros(k)
        s[: max(1, k // 4)] = np.linspace(1.0, 0.2, max(1, k // 4))
    else:
        raise ValueError(kind)
    return (uu * s[None, :]) @ vv.conj().T


SVD_TOL = {"fp64": dict(s=5e-13, rec=5e-13, orth=1e-10),
           "fp32": dict(s=5e-6, rec=5e-6, orth=5e-4)}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,m,n", [
    ("gauss", 37, 50), ("gauss", 80, 80), ("gauss", 130, 96), ("graded", 64, 64),
    ("degenerate", 48, 48), ("rankdef", 64, 64), ("gauss", 1, 7), ("gauss", 9, 1),
    ("gauss", 2, 2), ("gauss", 16, 16), ("gauss", 5, 12), ("gauss", 17, 33),
])
def test_svd_matches_lapack(precision, kind, m, n):
    rng = np.random.default_rng(zlib.crc32(f"{kind}{m}x{n}".encode()))
    a = np.stack([_matrices(kind, rng, m, n) for _ in range(3)])
    say(f"svd {precision} {kind} {m}x{n}")
    s, u, vh, sw, code = ptebd.svd_batched(a, precision)
    assert code == 0
    tol = SVD_TOL[precision]
    for b in range(a.shape[0]):
        s_ref = np.linalg.svd(a[b], compute_uv=False)
        s1 = s_ref[0]
        assert np.max(np.abs(s[b] - s_ref)) <= tol["s"] * s1 * max(1, np.sqrt(max(m, n)) / 4)
        rec = (u[b] * s[b][None, :]) @ vh[b]
        assert np.linalg.norm(rec - a[b]) <= tol["rec"] * np.linalg.norm(a[b]) * max(1, np.sqrt(max(m, n)) / 4)
        keep = s[b] > 1e-6 * s1 if precision == "fp64" else s[b] > 1e-2 * s1
        uk, vk = u[b][:, keep], vh[b][keep, :]
        assert np.linalg.norm(uk.conj().T @ uk - np.eye(uk.shape[1])) <= tol["orth"]
        assert np.linalg.norm(vk @ vk.conj().T - np.eye(vk.shape[0])) <= tol["orth"]
    say(f"  sweeps {list(sw)}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_svd_haar_theta_full_size(precision):
    """512 x 512 theta of a saturated chi = 256 bond (the workload's largest SVD)."""
    rng = np.random.default_rng(17)
    a = np.stack([_haar_theta(rng, 256) for _ in range(2)])
    assert a.shape == (2, 512, 512)
    say(f"svd {precision} haar theta 512x512")
    s, u, vh, sw, code = ptebd.svd_batched(a, precision)
    assert code == 0
    tol = SVD_TOL[precision]
    for b in range(a.shape[0]):
        s_ref = np.linalg.svd(a[b], compute_uv=False)
        assert np.max(np.abs(s[b] - s_ref)) <= tol["s"] * s_ref[0] * 6
        rec = (u[b] * s[b][None, :]) @ vh[b]
        assert np.linalg.norm(rec - a[b]) <= tol["rec"] * np.linalg.norm(a[b]) * 6
    say(f"  sweeps {list(sw)}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_svd_exactly_parallel_equal_columns(precision):
    """Rank-one matrices whose nonzero columns are exactly parallel with exactly equal norms
    (the two-site wavefunction between two singlet dimers).  The rotation that merges them
    leaves a numerically zero column; the SVD must converge (no sweep cap) with finite
    values, sigma = (|a|, 0, ...), instead of rotating that rounding residue until the
    rotation angle overflows."""
    u = np.array([1.0, 0.0, 0.0, -1.0]) / np.sqrt(2)
    mats = [np.outer(u, np.array([1.0, 0.0, 0.0, 1.0]) / np.sqrt(2)),
            np.outer(u, np.array([1.0, 0.0, 0.0, 1.0j]) / np.sqrt(2)),
            np.outer(np.ones(8) / np.sqrt(8), np.ones(8) / np.sqrt(8)),
            np.kron(np.eye(2), np.outer(u, u))]
    for a in mats:
        s, uu, vh, sw, code = ptebd.svd_batched(a.astype(np.complex128), precision)
        say(f"parallel columns {a.shape} {precision}: sweeps {sw.tolist()}, sigma {np.round(s[0], 6).tolist()}")
        assert code == 0
        assert np.all(np.isfinite(s)) and np.all(np.isfinite(uu)) and np.all(np.isfinite(vh))
        s_ref = np.linalg.svd(a, compute_uv=False)
        assert np.max(np.abs(s[0] - s_ref)) <= (1e-14 if precision == "fp64" else 1e-6)
        assert sw[0] <= 12  # residues are still orthogonalized among themselves: 9 FP64 sweeps measured at 8 x 8
        r = int(np.sum(s_ref > 1e-8))
        rec = (uu[0][:, :r] * s[0][:r]) @ vh[0][:r]
        assert np.linalg.norm(rec - a) <= (1e-14 if precision == "fp64" else 1e-6)
