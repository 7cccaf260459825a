"""Dense helpers for pinning the oracle (tests only; independent of oracle code).

* ``vidal_from_dense``: Vidal's successive-SVD construction of the canonical form of a state
  vector (Sec. II.B: each Lambda is the singular-value spectrum of Psi reshaped across the bond).
* ``dense_with_projectors``: contraction of a Vidal MPS with the projector P_i onto the first
  ``keep[i]`` basis states of every bond inserted explicitly as a diagonal 0/1 matrix
  (Sec. III.B), written as plain matrix products over the full bond spaces.
"""

import numpy as np


def vidal_from_dense(psi, n_sites, tol=1e-14):
    """Return (gammas, lambdas) lists with gammas[q] of shape (chi_q, 2, chi_{q+1})."""
    psi = np.asarray(psi, np.complex128)
    lams = [np.ones(1)]
    gams = []
    rest = psi.reshape(1, -1)  # (chi_left, remaining)
    lam_left = np.ones(1)
    for q in range(n_sites - 1):
        chi_l = rest.shape[0]
        m = rest.reshape(chi_l * 2, -1)
        u, s, vh = np.linalg.svd(m, full_matrices=False)
        keep = max(1, int(np.sum(s > tol * s[0])))
        u, s, vh = u[:, :keep], s[:keep], vh[:keep]
        gams.append(u.reshape(chi_l, 2, keep) / lam_left[:, None, None])
        lams.append(s)
        lam_left = s
        rest = (s[:, None] * vh)
    chi_l = rest.shape[0]
    last = rest.reshape(chi_l, 2, 1)
    gams.append(last / lam_left[:, None, None])
    lams.append(np.ones(1))
    return gams, lams


def dense_with_projectors(gams, lams, keep):
    """Contract Lambda[0] Gamma[0] P_1 Lambda[1] P_1 Gamma[1] ... with P_i = diag(1..1,0..0)."""
    n = len(gams)
    psi = np.ones((1, 1), np.complex128)
    for q in range(n):
        chi = len(lams[q])
        lam_mat = np.diag(lams[q]).astype(np.complex128)
        if 0 < q < n and keep is not None and q in keep:
            p = np.diag((np.arange(chi) < keep[q]).astype(float))
            lam_mat = p @ lam_mat @ p
        g = gams[q]
        cols = []
        for s in range(2):
            cols.append(psi @ lam_mat @ g[:, s, :])
        # physical index order: previous sites (rows of psi) then s
        psi = np.stack(cols, axis=1).reshape(-1, g.shape[2])
    return (psi * lams[n][None, :]).reshape(-1)
