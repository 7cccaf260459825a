"""The paper's benchmark circuit families as layers of nearest-neighbour two-qubit gates.

Host-side input preparation only (gate matrices and index lists; none of the pTEBD
arithmetic).  Every function returns a list of compiled layers ``(bonds int32[n],
gates complex128[n, 4, 4])`` for a 1D chain, gates acting on sites (q, q+1), matrix
convention U[(s' t'), (s t)] with the left site as the high bit.

* RQC-1D (App. A): per physical layer a random single-qubit gate
  exp[-i theta (sin a cos f X + sin a sin f Y + cos a Z)] on every qubit, then CZ on
  (0,1),(2,3),... for odd layers and (1,2),(3,4),... for even layers.  theta, a, f uniform.
* PQC-1D (App. A): singlet dimers on (0,1),(2,3),..., then eSWAP(theta) = exp(-i theta P/2)
  on (1,2),(3,4),... for odd layers and (0,1),(2,3),... for even layers, theta uniform.
* RQC-2D (App. A): an L_x x L_y lattice, layers in the order A, B, C, D, A, ...; A and B couple
  neighbours within a column, C and D neighbours in adjacent columns (C: columns 2k, 2k+1;
  D: columns 2k+1, 2k+2); single-qubit random gates on every qubit in every layer.  The 1D
  path visits the lattice column by column, so A and B act on path neighbours and C and D
  are routed with SWAP layers (``compile_2d``).
* PQC-2D (App. A): a first A layer of singlet dimers, then eSWAP layers B, C, D, A, ...

Each family is first generated as physical layers (``*_physical``: single-qubit gates and
two-qubit gates on lattice couplings, which the tests apply directly to a state vector) and
then compiled.  Single-qubit gates are folded exactly into the next two-qubit gate acting on
their qubit (App. A notes this is always possible); gates still pending at the end are applied
as one or two final layers of product gates.  The uniform ranges are [0, 2 pi) for theta and phi and [0, pi] for
the polar angle alpha (the paper states only that they are uniform).
"""

from __future__ import annotations

import numpy as np

from . import inputs

X = np.array([[0, 1], [1, 0]], np.complex128)
Y = np.array([[0, -1j], [1j, 0]], np.complex128)
Z = np.array([[1, 0], [0, -1]], np.complex128)
I2 = np.eye(2, dtype=np.complex128)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], np.complex128)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """exp[-i theta (n . sigma)] with n = (sin a cos f, sin a sin f, cos a)."""
    theta = rng.uniform(0.0, 2.0 * np.pi)
    a = rng.uniform(0.0, np.pi)
    f = rng.uniform(0.0, 2.0 * np.pi)
    ns = np.sin(a) * np.cos(f) * X + np.sin(a) * np.sin(f) * Y + np.cos(a) * Z
    return np.cos(theta) * I2 - 1j * np.sin(theta) * ns


def eswap(theta: float) -> np.ndarray:
    """exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P, P the SWAP."""
    return np.cos(theta / 2) * np.eye(4) - 1j * np.sin(theta / 2) * SWAP


def singlet_preparation() -> np.ndarray:
    """A two-qubit unitary mapping |00> to the singlet (|01> - |10>)/sqrt2."""
    s = 1 / np.sqrt(2.0)
    cols = np.array([[0, s, -s, 0], [1, 0, 0, 0], [0, 0, 0, 1], [0, s, s, 0]], np.complex128).T
    return cols


class _Folder:
    """Collects two-qubit gates on path pairs and folds pending single-qubit gates in."""

    def __init__(self, n_sites: int):
        self.n = n_sites
        self.pending = [I2.copy() for _ in range(n_sites)]
        self.layers = []

    def single(self, site: int, u: np.ndarray) -> None:
        self.pending[site] = u @ self.pending[site]

    def layer(self, pairs_gates) -> None:
        bonds, gates = [], []
        for q, g in sorted(pairs_gates, key=lambda x: x[0]):
            g = g @ np.kron(self.pending[q], self.pending[q + 1])
            self.pending[q] = I2.copy()
            self.pending[q + 1] = I2.copy()
            bonds.append(q)
            gates.append(g)
        if bonds:
            self.layers.append((np.asarray(bonds, np.int32), np.stack(gates)))

    def flush(self) -> list:
        todo = [q for q in range(self.n) if not np.allclose(self.pending[q], I2)]
        for parity in (0, 1):
            pg = []
            for q in range(parity, self.n - 1, 2):
                if q in todo or q + 1 in todo:
                    pg.append((q, np.kron(self.pending[q], self.pending[q + 1])))
            for q, _ in pg:
                self.pending[q] = I2.copy()
                self.pending[q + 1] = I2.copy()
                todo = [t for t in todo if t not in (q, q + 1)]
            if pg:
                self.layers.append((np.asarray([q for q, _ in pg], np.int32),
                                    np.stack([g for _, g in pg])))
        return self.layers


def compile_1d(n_sites: int, physical) -> list:
    """Compile a physical 1D circuit, a list of (singles {qubit: 2x2}, [(q, q+1, 4x4)]), to
    layers of two-qubit gates with the single-qubit gates folded in."""
    f = _Folder(n_sites)
    for singles, pairs in physical:
        for q, u in singles.items():
            f.single(q, u)
        pg = []
        for qa, qb, g in pairs:
            if qb != qa + 1:
                raise ValueError("1D circuits couple chain neighbours (q, q+1) only")
            pg.append((qa, g))
        f.layer(pg)
    return f.flush()


def rqc_1d_physical(n_sites: int, depth: int, seed: int, circuit_id: int = 0) -> list:
    """RQC-1D physical layers l = 1..depth: a random rotation on every qubit, then CZ on
    (0,1),(2,3),... (l odd) or (1,2),(3,4),... (l even).  The paper takes N odd and D even;
    any N >= 2 and D >= 1 are accepted here."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, circuit_id, 101]))
    out = []
    for layer in range(1, depth + 1):
        singles = {q: random_rotation(rng) for q in range(n_sites)}
        out.append((singles, [(int(q), int(q) + 1, CZ)
                              for q in inputs.brickwork_bonds(n_sites, layer)]))
    return out


def pqc_1d_physical(n_sites: int, depth: int, seed: int, circuit_id: int = 0) -> list:
    """PQC-1D (Heisenberg HVA): singlets on (0,1),(2,3),..., then ``depth`` eSWAP layers,
    l = 1..depth, on (1,2),(3,4),... (l odd) and (0,1),(2,3),... (l even)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, circuit_id, 202]))
    out = [({}, [(q, q + 1, singlet_preparation()) for q in range(0, n_sites - 1, 2)])]
    for layer in range(1, depth + 1):
        start = 1 if layer % 2 == 1 else 0
        out.append(({}, [(q, q + 1, eswap(rng.uniform(0.0, 2.0 * np.pi)))
                         for q in range(start, n_sites - 1, 2)]))
    return out


def rqc_1d(n_sites: int, depth: int, seed: int, circuit_id: int = 0) -> list:
    return compile_1d(n_sites, rqc_1d_physical(n_sites, depth, seed, circuit_id))


def pqc_1d(n_sites: int, depth: int, seed: int, circuit_id: int = 0) -> list:
    return compile_1d(n_sites, pqc_1d_physical(n_sites, depth, seed, circuit_id))


# ----------------------------------------------------------------------------- 2D routing

def _oets_layers(order, target_rank):
    """Odd-even transposition sort of ``order`` (qubit at each path position) into ascending
    ``target_rank[qubit]``: (list of SWAP layers, each a list of left positions; new order)."""
    order = list(order)
    layers = []
    phase = 0
    idle = 0
    while idle < 2:
        swaps = []
        for p in range(phase, len(order) - 1, 2):
            if target_rank[order[p]] > target_rank[order[p + 1]]:
                order[p], order[p + 1] = order[p + 1], order[p]
                swaps.append(p)
        if swaps:
            layers.append(swaps)
            idle = 0
        else:
            idle += 1
        phase ^= 1
    return layers, order


def _interleave_rank(lx: int, ly: int, left_cols):
    """Path rank of every qubit when each column pair (x, x+1), x in left_cols, is interleaved
    ((x,0),(x+1,0),(x,1),(x+1,1),...) and every other column keeps its order."""
    rank = {}
    pos = 0
    coupled = set(left_cols)
    x = 0
    while x < lx:
        if x in coupled and x + 1 < lx:
            for y in range(ly):
                rank[x * ly + y] = pos
                rank[(x + 1) * ly + y] = pos + 1
                pos += 2
            x += 2
        else:
            for y in range(ly):
                rank[x * ly + y] = pos
                pos += 1
            x += 1
    return rank


def lattice_couplings(lx: int, ly: int, kind: int):
    """Qubit pairs (qa, qb) of physical layer kind 0..3 = A, B, C, D; qubit (x, y) = x ly + y.
    A: (x, 2j)-(x, 2j+1); B: (x, 2j+1)-(x, 2j+2); C: (2k, y)-(2k+1, y); D: (2k+1, y)-(2k+2, y).
    With an odd extent the edge qubits of that direction stay idle, as in the paper."""
    pairs = []
    if kind in (0, 1):
        for x in range(lx):
            for y in range(kind, ly - 1, 2):
                pairs.append((x * ly + y, x * ly + y + 1))
    else:
        for x in range(kind - 2, lx - 1, 2):
            for y in range(ly):
                pairs.append((x * ly + y, (x + 1) * ly + y))
    return pairs


def _path_rank(lx: int, ly: int, kind: int):
    """Path arrangement a physical layer of ``kind`` needs: column by column for A and B, the
    C (D) column pairs interleaved for C (D)."""
    if kind in (0, 1):
        return {q: q for q in range(lx * ly)}
    return _interleave_rank(lx, ly, range(kind - 2, lx - 1, 2))


def compile_2d(lx: int, ly: int, physical) -> list:
    """Compile a physical 2D circuit to nearest-neighbour layers on the column-by-column path.

    ``physical`` is a list of (kind, singles, pairs): ``kind`` 0..3 (A..D), ``singles`` a dict
    {qubit: 2x2} applied first, ``pairs`` [(qa, qb, 4x4 with qa the high bit)].  Before each
    layer the path is sorted, by odd-even transposition SWAP layers, into the arrangement that
    layer needs; at the end it is sorted back to the natural order, so the compiled circuit
    maps the input state to the output state qubit by qubit."""
    n = lx * ly
    f = _Folder(n)
    order = list(range(n))

    def sort_to(rank):
        nonlocal order
        layers, order = _oets_layers(order, rank)
        for sw in layers:
            f.layer([(p, SWAP) for p in sw])

    for kind, singles, pairs in physical:
        sort_to(_path_rank(lx, ly, kind))
        for p, q in enumerate(order):
            if q in singles:
                f.single(p, singles[q])
        where = {q: p for p, q in enumerate(order)}
        pg = []
        for qa, qb, g in pairs:
            pa, pb = where[qa], where[qb]
            if abs(pa - pb) != 1:
                raise AssertionError("routing left a coupling non-adjacent")
            pg.append((pa, g) if pa < pb else (pb, SWAP @ g @ SWAP))
        f.layer(pg)
    sort_to({q: q for q in range(n)})
    return f.flush()


def rqc_2d_physical(lx: int, ly: int, depth: int, seed: int, circuit_id: int = 0) -> list:
    """RQC-2D as physical layers A, B, C, D, A, ...: a random rotation on every qubit, then
    CZ on the layer's couplings."""
    n = lx * ly
    rng = np.random.default_rng(np.random.SeedSequence([seed, circuit_id, 303]))
    out = []
    for layer in range(depth):
        kind = layer % 4
        singles = {q: random_rotation(rng) for q in range(n)}
        out.append((kind, singles, [(a, b, CZ) for a, b in lattice_couplings(lx, ly, kind)]))
    return out


def pqc_2d_physical(lx: int, ly: int, depth: int, seed: int, circuit_id: int = 0) -> list:
    """PQC-2D as physical layers: the first (an A layer) prepares singlets on the A couplings
    (L_y even), the remaining depth - 1 layers follow B, C, D, A, ... with eSWAP gates."""
    if ly % 2:
        raise ValueError("PQC-2D needs an even L_y")
    rng = np.random.default_rng(np.random.SeedSequence([seed, circuit_id, 404]))
    out = [(0, {}, [(a, b, singlet_preparation()) for a, b in lattice_couplings(lx, ly, 0)])]
    for layer in range(1, depth):
        kind = layer % 4
        out.append((kind, {}, [(a, b, eswap(rng.uniform(0.0, 2.0 * np.pi)))
                               for a, b in lattice_couplings(lx, ly, kind)]))
    return out


def rqc_2d(lx: int, ly: int, depth: int, seed: int, circuit_id: int = 0) -> list:
    """RQC-2D compiled to the column-by-column path (``compile_2d``)."""
    return compile_2d(lx, ly, rqc_2d_physical(lx, ly, depth, seed, circuit_id))


def pqc_2d(lx: int, ly: int, depth: int, seed: int, circuit_id: int = 0) -> list:
    """PQC-2D compiled to the column-by-column path (``compile_2d``)."""
    return compile_2d(lx, ly, pqc_2d_physical(lx, ly, depth, seed, circuit_id))


def cd_compiled_depth(lx: int, ly: int) -> int:
    """Compiled layers of one routed C + D pair of physical layers (SWAP layers and the two
    gate layers), starting and ending in the natural order."""
    n = lx * ly
    order = list(range(n))
    depth = 0
    for kind in (2, 3):
        layers, order = _oets_layers(order, _path_rank(lx, ly, kind))
        depth += len(layers) + 1
    layers, order = _oets_layers(order, {q: q for q in range(n)})
    return depth + len(layers)


def compiled_depth_2d(lx: int, ly: int, physical_depth: int) -> int:
    """Compiled depth of a 2D circuit of a physical depth that is a multiple of 4: each A and
    each B layer is one compiled layer, each C + D pair ``cd_compiled_depth`` layers."""
    if physical_depth % 4:
        raise ValueError("the 2D circuits have a physical depth that is a multiple of 4")
    return physical_depth // 2 + (physical_depth // 4) * cd_compiled_depth(lx, ly)
