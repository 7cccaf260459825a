"""CPU oracle for the pTEBD layer (test infrastructure only).

This module is test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library never calls it.  It is
plain NumPy in complex128 / float64 and shares no code with the HIP path.

Notation (0-based sites q = 0..N-1, bonds i = 0..N):
  * ``gam[q]`` has shape (chi_q, 2, chi_{q+1}); ``lam[i]`` is a float64 vector of length chi_i,
    descending, with lam[0] = lam[N] = (1).  This is the Vidal form of Sec. II.B, Eq.
    (mps_cano_decomp): Psi = Lambda^[0] Gamma^[1] Lambda^[1] ... Gamma^[N] Lambda^[N]; the
    paper's 1-based site i is our q = i-1 and its bond i is our bond i.
  * A gate "at q" acts on sites (q, q+1), rewrites lam[q+1], gam[q], gam[q+1] and reads
    lam[q], lam[q+2].  Gate matrices are U[(s' t'), (s t)] with the left site as high bit.

Functions and the passages they follow:
  * ``bond_update``  -- the TEBD procedure of Sec. II.C (two-site wavefunction, gate, SVD,
    Vidal regauge with Lambda^{-1}), with the truncation of Sec. III.B (keep the chi' largest
    Schmidt values; local error eps_i of Theorem 1) and the norm stabilization factor
    nu_i = (1 - eps_i)^(-1/2) of Sec. III.C.2, Eq. (lren).
  * ``apply_layer``  -- one step of Algorithm 1 (pTEBD): all gates of a layer, then IPMC's
    g PtSU steps when the layer had to be compressed (Sec. III.E).
  * ``tsu``, ``ptsu_step`` -- trivial simple update (Sec. II.C, U = identity) and one
    parallel tSU step: all odd bonds, then all even bonds (Sec. III.D).
  * ``parallel_compress`` -- projector truncation of every bond of a Vidal MPS (Sec. III.B)
    with optional norm stabilization (Sec. III.C.2); used by the Theorem 1-4 pins.
  * ``overlap``, ``norm``, ``expect_z`` -- exact transfer-matrix contractions of the Vidal
    form (the quantum-map recursion of Lemma 2's proof with P = I).
  * ``canon_distance`` -- the distance to the canonical form, Eq. (dist_to_cano).
  * ``canonicalize`` -- sequential SVD sweeps restoring the canonical form (the
    ``Canonicalize`` step of Algorithm 1), used by the canonical-form experiment of Sec. III.D.
  * ``sample`` -- perfect sampling of bit strings from a canonical MPS (the measurement step
    after ``Canonicalize`` in Algorithm 1; the method of Ferris and Vidal cited there).
  * ``to_dense`` -- full contraction to a 2^N state vector (site 0 = most significant bit).
"""

from __future__ import annotations

import numpy as np


class AnnihilatedError(ValueError):
    """The two-site wavefunction vanished (all singular values zero)."""


class VidalMPS:
    """Open MPS in the Vidal form {Gamma, Lambda} (Sec. II.B)."""

    def __init__(self, gam, lam):
        self.gam = [np.array(g, dtype=np.complex128) for g in gam]
        self.lam = [np.array(x, dtype=np.float64) for x in lam]
        assert len(self.lam) == len(self.gam) + 1
        for q, g in enumerate(self.gam):
            assert g.shape == (len(self.lam[q]), 2, len(self.lam[q + 1])), (q, g.shape)
        # bookkeeping of the stabilized-norm estimate n*_upper = prod(nu) (Theorem 3)
        # and of the fidelity estimate prod(1 - eps)
        self.prod_nu = 1.0
        self.prod_one_minus_eps = 1.0

    @property
    def n_sites(self) -> int:
        return len(self.gam)

    def bond_dims(self):
        return [len(x) for x in self.lam]

    def copy(self) -> "VidalMPS":
        out = VidalMPS(self.gam, self.lam)
        out.prod_nu = self.prod_nu
        out.prod_one_minus_eps = self.prod_one_minus_eps
        return out


def product_state(n_sites: int) -> VidalMPS:
    """|0...0> with chi_0 = 1 (Sec. IV.A): Gamma[q] = e_0 of shape (1,2,1), all Lambda = (1)."""
    g = np.zeros((1, 2, 1), np.complex128)
    g[0, 0, 0] = 1.0
    return VidalMPS([g.copy() for _ in range(n_sites)], [np.ones(1) for _ in range(n_sites + 1)])


def _svd(m: np.ndarray):
    try:
        return np.linalg.svd(m, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesvd")


def two_site_theta(mps: VidalMPS, q: int, gate) -> np.ndarray:
    """Two-site wavefunction Lambda[q] Gamma[q] Lambda[q+1] Gamma[q+1] Lambda[q+2] (Sec. II.C),
    with the gate applied when ``gate`` is not None.  Returned as a matrix with rows (a, s')
    and columns (t', c)."""
    ll, lm, lr = mps.lam[q], mps.lam[q + 1], mps.lam[q + 2]
    a_t = ll[:, None, None] * mps.gam[q] * lm[None, None, :]
    b_t = mps.gam[q + 1] * lr[None, None, :]
    theta = np.einsum("asm,mtc->astc", a_t, b_t)
    if gate is not None:
        u4 = np.asarray(gate, np.complex128).reshape(2, 2, 2, 2)  # [s', t', s, t]
        theta = np.einsum("xyst,astc->axyc", u4, theta)
    return theta.reshape(len(ll) * 2, 2 * len(lr))


EPS_READINGS = ("literal", "relative", "complement")


def bond_update(mps: VidalMPS, q: int, gate, chi_max: int | None, cutoff: float,
                stabilize: bool = True, eps_reading: str = "literal",
                apply_nu: bool = True) -> dict:
    """One TEBD procedure at bond q+1 with truncation and norm stabilization.

    Steps (Sec. II.C; Sec. III.B; Theorem 1; Eq. (lren)):
      1. theta = gate . (Lambda[q] Gamma[q] Lambda[q+1] Gamma[q+1] Lambda[q+2]);
      2. SVD theta = X S Y^dagger;
      3. r = #{sigma > cutoff * sigma_1}; k = min(chi_max, r) (k = r when chi_max is None);
         eps is Theorem 1's local error, which on a normalized canonical input is the
         discarded weight, sum_{a >= k} sigma_a^2 = 1 - sum_{a < k} sigma_a^2 (there the
         Schmidt values have unit norm).  Away from that input the two forms differ, and
         ``eps_reading`` picks one: "literal" the discarded sigma^2; "relative" the discarded
         sigma^2 divided by sum sigma^2; "complement" 1 - sum of the kept sigma^2, which
         makes nu rescale the kept values to unit norm;
      4. nu = (1 - eps)^(-1/2) when stabilizing, else 1;  Lambda[q+1] = nu * S[:k]
         (with ``apply_nu`` False, Lambda[q+1] = S[:k] and the caller decides on nu);
      5. Gamma[q] = X[:, :k] / Lambda[q],  Gamma[q+1] = Y^dagger[:k] / Lambda[q+2].
    """
    ll, lr = mps.lam[q], mps.lam[q + 2]
    m = two_site_theta(mps, q, gate)
    x, s, yh = _svd(m)
    if not (s[0] > 0.0):
        raise AnnihilatedError(f"two-site wavefunction at q={q} vanished")
    r = int(np.count_nonzero(s > cutoff * s[0]))
    k = r if chi_max is None else min(int(chi_max), r)
    if eps_reading == "literal":
        eps = float(np.sum(s[k:] ** 2))
    elif eps_reading == "relative":
        eps = float(np.sum(s[k:] ** 2)) / float(np.sum(s ** 2))
    elif eps_reading == "complement":
        eps = 1.0 - float(np.sum(s[:k] ** 2))
    else:
        raise ValueError(f"eps_reading must be one of {EPS_READINGS}")
    if stabilize:
        if eps >= 1.0:
            raise AnnihilatedError(f"discarded weight {eps} >= 1 at q={q}")
        nu = (1.0 - eps) ** -0.5
    else:
        nu = 1.0
    mps.lam[q + 1] = nu * s[:k] if apply_nu else s[:k].copy()
    mps.gam[q] = x[:, :k].reshape(len(ll), 2, k) / ll[:, None, None]
    mps.gam[q + 1] = yh[:k].reshape(k, 2, len(lr)) / lr[None, None, :]
    return {"q": q, "k": k, "r": r, "eps": eps, "nu": nu, "sigma": s}


def _check_disjoint(n_sites: int, bonds) -> None:
    used = set()
    for q in bonds:
        q = int(q)
        if q < 0 or q + 1 >= n_sites:
            raise ValueError(f"bond {q} out of range")
        if q in used or q + 1 in used:
            raise ValueError(f"gates overlap at site {q}")
        used.update((q, q + 1))


def tsu(mps: VidalMPS, q: int, cutoff: float) -> dict:
    """Trivial simple update at bond q+1: the TEBD procedure with U = I (gate skipped), no
    chi truncation (cutoff only) and no norm stabilization (Sec. II.C; Sec. III.D)."""
    return bond_update(mps, q, None, None, cutoff, stabilize=False)


def ptsu_step(mps: VidalMPS, cutoff: float) -> None:
    """One PtSU step: tSU on all odd bonds (pairs (0,1),(2,3),...), then all even bonds."""
    n = mps.n_sites
    for q in range(0, n - 1, 2):
        tsu(mps, q, cutoff)
    for q in range(1, n - 1, 2):
        tsu(mps, q, cutoff)


def _gate_on_its_bond(task):
    """One gate of a layer applied to its own two sites: (Gamma[q], Gamma[q+1], Lambda[q],
    Lambda[q+1], Lambda[q+2], gate, chi_max, cutoff, stabilize, eps_reading) -> (the two new
    Gammas, the new Lambda[q+1] without nu, stats).  A gate reads and writes nothing else
    (Sec. II.C), which is what lets the gates of a layer run in any order or at once."""
    gq, gq1, ll, lm, lr, gate, chi_max, cutoff, stabilize, eps_reading = task
    local = VidalMPS([gq, gq1], [ll, lm, lr])
    st = bond_update(local, 0, gate, chi_max, cutoff, stabilize, eps_reading, apply_nu=False)
    return local.gam[0], local.gam[1], local.lam[1], st


def apply_layer(mps: VidalMPS, bonds, gates, chi_max: int, cutoff: float = 1e-12,
                ptsu_steps: int = 0, stabilize: bool = True, eps_reading: str = "literal",
                map_fn=None):
    """One pTEBD step (Algorithm 1): the TEBD procedure on every gate of the layer, each bond
    cut to chi_max.  If some gate's rank exceeded chi_max ("if chi~ > chi") the layer is
    compressed by IPMC (Sec. III.E): the truncated bonds' Schmidt values are multiplied by
    their nu_i (norm stabilization, Sec. III.C.2) and ``ptsu_steps`` PtSU steps follow.
    Otherwise the bonds keep their singular values as they are and nu_i = 1 (the "else"
    branch of Algorithm 1; the cutoff still drops values below cutoff * sigma_1).

    Gates touch disjoint sites and read only Lambda[q], Lambda[q+2], which no gate of the same
    layer writes, so the order of the gates does not matter; they are processed in ascending q,
    or, with ``map_fn`` (a map over the per-gate tasks, e.g. a thread pool's), all at once.
    Returns (list of per-gate stats in ascending-q order, triggered flag); each gate's "nu"
    is the factor actually applied.
    """
    bonds = [int(q) for q in bonds]
    _check_disjoint(mps.n_sites, bonds)
    order = np.argsort(bonds, kind="stable")
    stats = [None] * len(bonds)
    if map_fn is None:
        for idx in order:
            stats[idx] = bond_update(mps, bonds[idx], gates[idx], chi_max, cutoff, stabilize,
                                     eps_reading, apply_nu=False)
    else:
        tasks = [(mps.gam[q], mps.gam[q + 1], mps.lam[q], mps.lam[q + 1], mps.lam[q + 2],
                  gates[idx], chi_max, cutoff, stabilize, eps_reading)
                 for idx, q in ((i, bonds[i]) for i in order)]
        for idx, (g0, g1, lm, st) in zip(order, map_fn(_gate_on_its_bond, tasks)):
            q = bonds[idx]
            mps.gam[q], mps.gam[q + 1], mps.lam[q + 1] = g0, g1, lm
            stats[idx] = st
    triggered = any(st["r"] > chi_max for st in stats)
    for idx, st in enumerate(stats):
        if triggered:
            q = bonds[idx]
            mps.lam[q + 1] = st["nu"] * mps.lam[q + 1]
        else:
            st["nu"] = 1.0
        mps.prod_nu *= st["nu"]
        mps.prod_one_minus_eps *= (1.0 - st["eps"])
    if triggered:
        for _ in range(int(ptsu_steps)):
            ptsu_step(mps, cutoff)
    return stats, triggered


def parallel_compress(mps: VidalMPS, chi_keep: int, stabilize: bool = False,
                      bonds=None) -> dict:
    """Parallel MPS compression by projectors (Sec. III.B): on every inner bond i (or on the
    listed bonds) keep the chi_keep largest Lambda entries and the matching slices of the
    neighbouring Gammas.  With ``stabilize`` every kept Lambda[i] is multiplied by
    nu_i = (1 - eps_i)^(-1/2) (Eq. (lren)).  Returns eps_i and nu_i per bond."""
    n = mps.n_sites
    bonds = range(1, n) if bonds is None else bonds
    eps, nus = {}, {}
    for i in bonds:
        lam = mps.lam[i]
        k = min(int(chi_keep), len(lam))
        e = float(np.sum(lam[k:] ** 2))
        nu = (1.0 - e) ** -0.5 if stabilize else 1.0
        mps.lam[i] = nu * lam[:k]
        mps.gam[i - 1] = mps.gam[i - 1][:, :, :k]
        mps.gam[i] = mps.gam[i][:k, :, :]
        eps[i], nus[i] = e, nu
    return {"eps": eps, "nu": nus}


# ----------------------------------------------------------------------------- queries

def _site_a(mps: VidalMPS, q: int) -> np.ndarray:
    """A-tensor Lambda[q] Gamma[q] of shape (chi_q, 2, chi_{q+1})."""
    return mps.lam[q][:, None, None] * mps.gam[q]


def overlap(bra: VidalMPS, ket: VidalMPS) -> complex:
    """<bra|ket> by a left-to-right transfer sweep E <- sum_s A_s^dagger E B_s."""
    assert bra.n_sites == ket.n_sites
    e = np.ones((1, 1), np.complex128)
    for q in range(ket.n_sites):
        a = _site_a(bra, q)
        b = _site_a(ket, q)
        e = sum(a[:, s, :].conj().T @ e @ b[:, s, :] for s in range(2))
    n = ket.n_sites
    return complex(bra.lam[n][0] * ket.lam[n][0] * e[0, 0])


def norm(mps: VidalMPS) -> float:
    """Exact wavefunction norm sqrt(<Psi|Psi>)."""
    return float(np.sqrt(max(overlap(mps, mps).real, 0.0)))


def fidelity_error(a: VidalMPS, b: VidalMPS) -> float:
    """1 - |<a|b>|^2 / (<a|a><b|b>)."""
    ab = overlap(a, b)
    return float(1.0 - abs(ab) ** 2 / (overlap(a, a).real * overlap(b, b).real))


def expect_z(mps: VidalMPS) -> np.ndarray:
    """<Z_q> / <Psi|Psi> for every site, from left and right environments."""
    n = mps.n_sites
    left = [np.ones((1, 1), np.complex128)]
    for q in range(n):
        a = _site_a(mps, q)
        left.append(sum(a[:, s, :].conj().T @ left[-1] @ a[:, s, :] for s in range(2)))
    right = [None] * (n + 1)
    right[n] = np.ones((1, 1), np.complex128) * (mps.lam[n][0] ** 2)
    for q in range(n - 1, -1, -1):
        a = _site_a(mps, q)
        right[q] = sum(a[:, s, :] @ right[q + 1] @ a[:, s, :].conj().T for s in range(2))
    nrm2 = float(np.real(np.trace(left[n] @ right[n])))
    z = np.zeros(n)
    for q in range(n):
        a = _site_a(mps, q)
        val = 0.0
        for s, zs in ((0, 1.0), (1, -1.0)):
            t = a[:, s, :].conj().T @ left[q] @ a[:, s, :]
            val += zs * np.real(np.trace(t @ right[q + 1]))
        z[q] = val / nrm2
    return z


def canon_distance(mps: VidalMPS) -> float:
    """Distance to the canonical form, Eq. (dist_to_cano), for the state scaled to norm 1.

    The scaling multiplies every inner Lambda[i] (i = 1..N-1) by n^(-1/(N-1)).  With
    A = Lambda[q] Gamma[q] and B = Gamma[q] Lambda[q+1]:
    C = 1/(2N) sum_q ||sum_s A_s^dagger A_s - I|| + ||sum_s B_s B_s^dagger - I|| (Frobenius).
    """
    n = mps.n_sites
    nrm = norm(mps)
    scale = nrm ** (-1.0 / (n - 1)) if n > 1 else 1.0 / nrm
    lam = [x.copy() for x in mps.lam]
    for i in range(1, n):
        lam[i] = lam[i] * scale
    if n == 1:
        lam[0] = lam[0] * scale
    total = 0.0
    for q in range(n):
        a = lam[q][:, None, None] * mps.gam[q]
        b = mps.gam[q] * lam[q + 1][None, None, :]
        ga = sum(a[:, s, :].conj().T @ a[:, s, :] for s in range(2))
        gb = sum(b[:, s, :] @ b[:, s, :].conj().T for s in range(2))
        total += np.linalg.norm(ga - np.eye(ga.shape[0])) + np.linalg.norm(gb - np.eye(gb.shape[0]))
    return float(total / (2 * n))


def canonicalize(mps: VidalMPS, cutoff: float = 0.0):
    """Sequential restoration of the canonical form (the ``Canonicalize`` step of Algorithm 1).

    A left-to-right sweep of QR decompositions makes every site left-isometric and carries
    the whole state into the last site, whose norm is the wavefunction norm n.  After
    dividing by n, a right-to-left sweep of SVDs produces each bond's Schmidt values
    Lambda[i] (sum of squares 1) and right-isometric B tensors; Gamma[q] = B[q] / Lambda[q+1].
    Returns (canonical normalized VidalMPS, n).  Singular values at or below cutoff * sigma_1
    are dropped.
    """
    n = mps.n_sites
    ms = [_site_a(mps, q) for q in range(n)]
    ms[-1] = ms[-1] * mps.lam[n][None, None, :]
    for q in range(n - 1):
        cl, _, cr = ms[q].shape
        qm, rm = np.linalg.qr(ms[q].reshape(cl * 2, cr))
        ms[q] = qm.reshape(cl, 2, qm.shape[1])
        ms[q + 1] = np.einsum("ij,jsk->isk", rm, ms[q + 1])
    nrm = float(np.linalg.norm(ms[n - 1]))
    carry = ms[n - 1] / nrm
    lam = [None] * (n + 1)
    lam[0] = np.ones(1)
    lam[n] = np.ones(1)
    rights = [None] * n
    for q in range(n - 1, 0, -1):
        cl, _, cr = carry.shape
        u, s, vh = _svd(carry.reshape(cl, 2 * cr))
        keep = max(1, int(np.count_nonzero(s > cutoff * s[0])))
        u, s, vh = u[:, :keep], s[:keep], vh[:keep]
        rights[q] = vh.reshape(keep, 2, cr)
        lam[q] = s
        carry = np.einsum("isk,kj->isj", ms[q - 1], u * s[None, :])
    rights[0] = carry
    gam = [rights[q] / lam[q + 1][None, None, :] for q in range(n)]
    return VidalMPS(gam, lam), nrm


def sample(mps: VidalMPS, uniforms: np.ndarray, return_margins: bool = False):
    """Perfect sampling from a state in canonical form, one bit string per row of
    ``uniforms`` (shape (S, N), values in [0, 1)); returns uint8 bits of shape (S, N), and
    with ``return_margins`` also each sample's smallest |u - p_0 / (p_0 + p_1)| along its
    path (how close a decision came to flipping).

    With the right-isometric tensors B[q] = Gamma[q] Lambda[q+1] of the canonical form, the
    probability of sigma_q given the bits already drawn is |v B[q]_sigma|^2 / |v|^2, where the
    row vector v is the contraction of the drawn prefix (v = (1) before site 0).  Site by
    site: w_s = v B[q]_s for s = 0, 1; p_s = |w_s|^2; sigma_q = 0 if u < p_0 / (p_0 + p_1),
    else 1; v = w_sigma / sqrt(p_sigma).  The decision is taken in float64.
    """
    n = mps.n_sites
    u = np.asarray(uniforms, np.float64)
    if u.ndim != 2 or u.shape[1] != n:
        raise ValueError("uniforms must have shape (n_samples, n_sites)")
    b = [mps.gam[q] * mps.lam[q + 1][None, None, :] for q in range(n)]
    bits = np.zeros(u.shape, np.uint8)
    margins = np.full(u.shape[0], np.inf)
    for i in range(u.shape[0]):
        v = np.ones(1, np.complex128)
        for q in range(n):
            w0 = v @ b[q][:, 0, :]
            w1 = v @ b[q][:, 1, :]
            p0 = float(np.vdot(w0, w0).real)
            p1 = float(np.vdot(w1, w1).real)
            margins[i] = min(margins[i], abs(u[i, q] - p0 / (p0 + p1)))
            if u[i, q] < p0 / (p0 + p1):
                v = w0 / np.sqrt(p0)
            else:
                bits[i, q] = 1
                v = w1 / np.sqrt(p1)
    return (bits, margins) if return_margins else bits


def scale_norm(mps: VidalMPS, factor: float) -> None:
    """Multiply the state by ``factor`` by scaling every inner Lambda[i] (i = 1..N-1) by
    factor^(1/(N-1)) (for N = 1, Lambda[0])."""
    n = mps.n_sites
    if n == 1:
        mps.lam[0] = mps.lam[0] * factor
        return
    f = factor ** (1.0 / (n - 1))
    for i in range(1, n):
        mps.lam[i] = mps.lam[i] * f


def to_dense(mps: VidalMPS) -> np.ndarray:
    """Contract the Vidal form to the 2^N amplitude vector, site 0 the most significant bit."""
    psi = np.ones((1, 1), np.complex128)  # (physical so far, bond)
    for q in range(mps.n_sites):
        a = _site_a(mps, q)
        psi = np.einsum("pa,asb->psb", psi, a).reshape(-1, a.shape[2])
    psi = psi * mps.lam[mps.n_sites][None, :]
    return psi.reshape(-1)
