"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only draws random numbers and lays out index lists; it contains none of the
pTEBD arithmetic (no contraction, SVD, truncation or regauging).

* Circuits are layered brickworks of two-qubit gates on a 1D chain (the circuit
  decomposition into layers of non-overlapping local unitaries, Sec. IV, Eq. (circ_decomp)).
  Layer 1 acts on the pairs (0,1),(2,3),... and layer 2 on (1,2),(3,4),...; the first layer
  matches the first layer of the paper's 1D random circuit (App. A).
* Gates are Haar-random U(4) unitaries drawn with Mezzadri's method (QR of a complex
  Ginibre matrix with the phases of R's diagonal moved into Q), optionally projected to SU(4)
  by dividing by det(U)^(1/4) (principal branch).  Index convention of a gate matrix:
  ``U[(s' t'), (s t)]`` row-major 4x4 with the left site's bit as the high bit.
* Random MPS tensors for the canonical-form experiment of Sec. III.D: every entry is
  a + ib with a, b uniform in [-1, 1].

Random streams: ``numpy.random.default_rng(SeedSequence([seed, circuit_id]))`` (PCG64), gates
drawn in (layer, ascending bond) order.
"""

from __future__ import annotations

import numpy as np


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


def haar_unitary(rng: np.random.Generator, n: int = 4, special: bool = True) -> np.ndarray:
    """One Haar-random n x n unitary (Mezzadri's QR method); SU(n) if ``special``."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    q = q * (d / np.abs(d))[None, :]
    if special:
        q = q / np.linalg.det(q) ** (1.0 / n)
    return q.astype(np.complex128)


def brickwork_bonds(n_sites: int, layer: int) -> np.ndarray:
    """Left sites q of the gates of brickwork layer ``layer`` (1-based): odd layers start at 0."""
    start = 0 if layer % 2 == 1 else 1
    return np.arange(start, n_sites - 1, 2, dtype=np.int32)


def brickwork_circuit(n_sites: int, depth: int, seed: int, circuit_id: int = 0,
                      special: bool = True):
    """Haar brickwork circuit: list over layers of (bonds int32[n], gates complex128[n,4,4])."""
    rng = _rng(seed, circuit_id)
    layers = []
    for layer in range(1, depth + 1):
        bonds = brickwork_bonds(n_sites, layer)
        gates = np.stack([haar_unitary(rng, 4, special) for _ in bonds]) if len(bonds) else \
            np.zeros((0, 4, 4), np.complex128)
        layers.append((bonds, gates))
    return layers


def saturated_bond_dims(n_sites: int, chi: int) -> list[int]:
    """Bond dimensions chi_i = min(chi, 2^i, 2^(N-i)) for i = 0..N (chi_0 = chi_N = 1)."""
    out = []
    for i in range(n_sites + 1):
        e = min(i, n_sites - i)
        out.append(int(min(chi, 2 ** min(e, 62))))
    return out


def random_mps_tensors(n_sites: int, chi: int, seed: int, stream: int = 0):
    """Site tensors M[q] of shape (chi_q, 2, chi_{q+1}) with entries a+ib, a,b ~ U[-1,1]."""
    rng = _rng(seed, stream)
    dims = saturated_bond_dims(n_sites, chi)
    out = []
    for q in range(n_sites):
        shape = (dims[q], 2, dims[q + 1])
        out.append(rng.uniform(-1.0, 1.0, shape) + 1j * rng.uniform(-1.0, 1.0, shape))
    return out


def random_vidal_state(n_sites: int, chi: int, seed: int, stream: int = 0):
    """Synthetic Vidal-form data at a saturated bond dimension, for kernel-level workloads.

    Gamma[q] has shape (chi_q, 2, chi_{q+1}) with complex Gaussian entries of variance
    1/(2 chi_q); Lambda[i] (i = 1..N-1) is a descending positive spectrum with
    log-uniform spread over four decades, scaled to unit 2-norm; Lambda[0] = Lambda[N] = (1).
    The state is not canonical; it only has the shapes and value ranges of a saturated one.
    """
    rng = _rng(seed, stream)
    dims = saturated_bond_dims(n_sites, chi)
    gammas = []
    for q in range(n_sites):
        shape = (dims[q], 2, dims[q + 1])
        g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        gammas.append(g / np.sqrt(2.0 * dims[q]))
    lambdas = []
    for i in range(n_sites + 1):
        if i == 0 or i == n_sites:
            lambdas.append(np.ones(1))
            continue
        lam = np.sort(10.0 ** rng.uniform(-4.0, 0.0, dims[i]))[::-1]
        lambdas.append(lam / np.linalg.norm(lam))
    return gammas, lambdas


def random_state_vector(n_sites: int, seed: int, stream: int = 0) -> np.ndarray:
    """Normalized complex Gaussian state vector of 2^N amplitudes (site 0 = most significant bit)."""
    rng = _rng(seed, stream)
    v = rng.standard_normal(2 ** n_sites) + 1j * rng.standard_normal(2 ** n_sites)
    return v / np.linalg.norm(v)
