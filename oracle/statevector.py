"""Brute-force state-vector simulation (test infrastructure only; independent of the MPS code).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may use it.

Amplitude index of |sigma_0 ... sigma_{N-1}> is sum_q sigma_q 2^(N-1-q): site 0 is the most
significant bit, i.e. Psi_{sigma_1 ... sigma_N} in C order (Sec. II.A).  A two-qubit gate at q
acts on the middle index of psi reshaped to (2^q, 4, 2^(N-q-2)), whose value is
2*sigma_q + sigma_{q+1}; the gate matrix is U[(s' t'), (s t)].
"""

from __future__ import annotations

import numpy as np


def zero_state(n_sites: int) -> np.ndarray:
    psi = np.zeros(2 ** n_sites, np.complex128)
    psi[0] = 1.0
    return psi


def apply_gate(psi: np.ndarray, n_sites: int, q: int, gate: np.ndarray) -> np.ndarray:
    v = psi.reshape(2 ** q, 4, 2 ** (n_sites - q - 2))
    return np.einsum("ij,ajb->aib", np.asarray(gate, np.complex128), v).reshape(-1)


def run_circuit(n_sites: int, layers, psi: np.ndarray | None = None) -> np.ndarray:
    psi = zero_state(n_sites) if psi is None else psi.copy()
    for bonds, gates in layers:
        for q, u in zip(bonds, gates):
            psi = apply_gate(psi, n_sites, int(q), u)
    return psi


def expect_z(psi: np.ndarray, n_sites: int) -> np.ndarray:
    p = np.abs(psi) ** 2
    total = p.sum()
    out = np.zeros(n_sites)
    for q in range(n_sites):
        v = p.reshape(2 ** q, 2, 2 ** (n_sites - q - 1)).sum(axis=(0, 2))
        out[q] = (v[0] - v[1]) / total
    return out


def fidelity(psi_exact: np.ndarray, psi: np.ndarray) -> float:
    """F = |<psi_exact|psi>|^2 / (<psi_exact|psi_exact> <psi|psi>)  (Eq. (F), normalized)."""
    num = abs(np.vdot(psi_exact, psi)) ** 2
    return float(num / (np.vdot(psi_exact, psi_exact).real * np.vdot(psi, psi).real))


def schmidt_values(psi: np.ndarray, n_sites: int, bond: int) -> np.ndarray:
    """Singular values of Psi reshaped with sites [0, bond) as rows (Sec. II.B)."""
    m = psi.reshape(2 ** bond, 2 ** (n_sites - bond))
    return np.linalg.svd(m, compute_uv=False)


def apply_one(psi: np.ndarray, n_sites: int, q: int, u: np.ndarray) -> np.ndarray:
    """A single-qubit gate u[s', s] on qubit q."""
    v = psi.reshape(2 ** q, 2, 2 ** (n_sites - q - 1))
    return np.einsum("ij,ajb->aib", np.asarray(u, np.complex128), v).reshape(-1)


def apply_pair(psi: np.ndarray, n_sites: int, qa: int, qb: int, gate: np.ndarray) -> np.ndarray:
    """A two-qubit gate U[(s'_a s'_b), (s_a s_b)] on any two distinct qubits (qa the high bit),
    applied by moving the two qubit axes of the amplitude tensor to the front."""
    t = psi.reshape((2,) * n_sites)
    t = np.moveaxis(t, (qa, qb), (0, 1)).reshape(4, -1)
    t = (np.asarray(gate, np.complex128) @ t).reshape((2, 2) + (2,) * (n_sites - 2))
    return np.moveaxis(t, (0, 1), (qa, qb)).reshape(-1)
