"""Synthetic s-type Gaussian overlap matrices (stand-ins for the paper's
STO-3G water-cluster and Glu-Ala helix overlap matrices, Sec. 5).

Everything here is seeded and deterministic.  The recipe:

* geometry in Angstrom, converted to bohr with ``BOHR_PER_ANGSTROM``;
* water: 7 s-functions per molecule, O{130.7, 5.03, 0.38, 0.85, 0.17},
  H1{0.42}, H2{0.42} (bohr^-2), molecules on a jittered simple-cubic lattice
  at liquid density with uniformly random orientations;
* chain: a helical backbone (radius 2.3 A, 100 deg and 1.5 A rise per
  residue) with 20 centres per residue drawn uniformly in a 3 A ball around
  the backbone point, rejected when closer than ``min_dist`` to an earlier
  centre; one s-function per centre, exponents cycling through the 7 water
  exponents;
* S_ij = (2 sqrt(a_i a_j) / (a_i + a_j))^{3/2} exp(-a_i a_j r^2 / (a_i + a_j)),
  so diag(S) = 1;
* atoms sorted by a 63-bit Morton code (21 bits per axis over the bounding
  cube, stable sort), each atom keeping its functions in listed order;
* the matrix is cut into b x b blocks (row-major), the last block row/column
  zero-padded when b does not divide n; only blocks holding an element above
  ``elem_eps`` are listed, both (i, j) and (j, i) of the symmetric pattern.

No inverse-factorization arithmetic lives here: block truncation at tau is the
method's job and is done by its consumers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BOHR_PER_ANGSTROM = 1.8897261254578281
WATER_EXPONENTS = (130.7, 5.03, 0.38, 0.85, 0.17, 0.42, 0.42)
WATER_DENSITY = 0.03343  # molecules per cubic Angstrom (1 g/cm^3)
R_OH = 0.9572            # Angstrom
ANGLE_HOH = 104.52       # degrees


@dataclass
class BlockMatrix:
    """A block-sparse matrix as a sorted, unique block list.

    ``brow``/``bcol`` are int32 block coordinates sorted by (brow, bcol);
    ``vals`` is float64 of shape (nnzb, b, b), row-major blocks.  Entries of
    the padded tail (row or column index >= n) are zero.
    """
    n: int
    b: int
    brow: np.ndarray
    bcol: np.ndarray
    vals: np.ndarray

    @property
    def nb(self) -> int:
        return (self.n + self.b - 1) // self.b

    @property
    def nnzb(self) -> int:
        return int(self.brow.shape[0])

    def row_ptr(self) -> np.ndarray:
        rp = np.zeros(self.nb + 1, dtype=np.int64)
        np.add.at(rp, self.brow.astype(np.int64) + 1, 1)
        return np.cumsum(rp)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def _random_rotations(rng: np.random.Generator, count: int) -> np.ndarray:
    """Uniform random rotation matrices from uniform unit quaternions
    (Shoemake's subgroup algorithm)."""
    u = rng.random((count, 3))
    s1 = np.sqrt(1.0 - u[:, 0])
    s2 = np.sqrt(u[:, 0])
    t1 = 2.0 * np.pi * u[:, 1]
    t2 = 2.0 * np.pi * u[:, 2]
    w, x, y, z = s2 * np.cos(t2), s1 * np.sin(t1), s1 * np.cos(t1), s2 * np.sin(t2)
    rot = np.empty((count, 3, 3))
    rot[:, 0, 0] = 1 - 2 * (y * y + z * z)
    rot[:, 0, 1] = 2 * (x * y - z * w)
    rot[:, 0, 2] = 2 * (x * z + y * w)
    rot[:, 1, 0] = 2 * (x * y + z * w)
    rot[:, 1, 1] = 1 - 2 * (x * x + z * z)
    rot[:, 1, 2] = 2 * (y * z - x * w)
    rot[:, 2, 0] = 2 * (x * z - y * w)
    rot[:, 2, 1] = 2 * (y * z + x * w)
    rot[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return rot


def _morton_order(points: np.ndarray) -> np.ndarray:
    """Stable argsort of points by a 63-bit Morton code, 21 bits per axis over
    the bounding cube (one scale for all axes, so a long thin system is
    ordered along its length); ties keep generation order."""
    lo = points.min(axis=0)
    span = float(np.max(points.max(axis=0) - lo))
    span = span if span > 0 else 1.0
    q = np.floor((points - lo) / span * ((1 << 21) - 1)).astype(np.uint64)
    q = np.minimum(q, np.uint64((1 << 21) - 1))

    def spread(v: np.ndarray) -> np.ndarray:
        v = v & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v

    code = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1)) | (spread(q[:, 2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


def water_cluster(n_mol: int, seed: int):
    """Centres (bohr) and exponents of ``n_mol`` water molecules (7 functions
    per molecule), atoms in Morton order.

    Returns (centres[n,3], exponents[n]) with n = 7 * n_mol.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    box = (n_mol / WATER_DENSITY) ** (1.0 / 3.0)
    ns = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    while ns ** 3 < n_mol:
        ns += 1
    spacing = box / ns
    idx = np.arange(n_mol)
    sites = np.stack([idx // (ns * ns), (idx // ns) % ns, idx % ns], axis=1).astype(np.float64)
    sites = (sites + 0.5) * spacing
    jitter = rng.uniform(-0.15, 0.15, size=(n_mol, 3)) * spacing
    oxygen = sites + jitter
    rot = _random_rotations(rng, n_mol)
    half = math.radians(ANGLE_HOH) / 2.0
    h_local = np.array([[R_OH * math.sin(half), 0.0, R_OH * math.cos(half)],
                        [-R_OH * math.sin(half), 0.0, R_OH * math.cos(half)]])
    h1 = oxygen + np.einsum("mij,j->mi", rot, h_local[0])
    h2 = oxygen + np.einsum("mij,j->mi", rot, h_local[1])
    # atoms in generation order: O, H1, H2 per molecule
    atoms = np.stack([oxygen, h1, h2], axis=1).reshape(-1, 3)
    atom_kind = np.tile(np.array([0, 1, 1]), n_mol)
    order = _morton_order(atoms)
    centres, exps = [], []
    o_exp = np.array(WATER_EXPONENTS[:5])
    for a in order:
        if atom_kind[a] == 0:
            centres.append(np.repeat(atoms[a][None, :], 5, axis=0))
            exps.append(o_exp)
        else:
            centres.append(atoms[a][None, :])
            exps.append(np.array([WATER_EXPONENTS[5]]))
    centres = np.concatenate(centres) * BOHR_PER_ANGSTROM
    exps = np.concatenate(exps)
    return centres, exps


def helix_chain(n_res: int, seed: int, per_res: int = 20, min_dist: float = 1.0,
                radius: float = 2.3, twist_deg: float = 100.0, rise: float = 1.5,
                ball: float = 3.0):
    """Centres (bohr) and exponents of a quasi-linear helical chain with
    ``per_res`` s-type centres per residue.  Returns (centres[n,3], exponents[n])
    with n = per_res * n_res, Morton-ordered."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cell = min_dist
    grid: dict = {}
    pts = np.empty((n_res * per_res, 3))
    count = 0
    md2 = min_dist * min_dist
    for r in range(n_res):
        ang = math.radians(twist_deg) * r
        centre = np.array([radius * math.cos(ang), radius * math.sin(ang), rise * r])
        placed = 0
        while placed < per_res:
            cand = rng.uniform(-ball, ball, size=(64, 3))
            cand = cand[np.einsum("ij,ij->i", cand, cand) <= ball * ball]
            for c in cand:
                if placed == per_res:
                    break
                p = centre + c
                key = (int(math.floor(p[0] / cell)), int(math.floor(p[1] / cell)), int(math.floor(p[2] / cell)))
                ok = True
                for dx in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dz in (-1, 0, 1):
                            for q in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                                d = p - pts[q]
                                if d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < md2:
                                    ok = False
                                    break
                            if not ok:
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if ok:
                    pts[count] = p
                    grid.setdefault(key, []).append(count)
                    count += 1
                    placed += 1
    exps = np.array([WATER_EXPONENTS[i % 7] for i in range(count)])
    order = _morton_order(pts)
    return pts[order] * BOHR_PER_ANGSTROM, exps[order]


# ----------------------------------------------------------------------------
# overlap matrix
# ----------------------------------------------------------------------------

def _overlap_values(ci, cj, ai, aj):
    r2 = np.einsum("ij,ij->i", ci - cj, ci - cj)
    s = ai + aj
    pref = (2.0 * np.sqrt(ai * aj) / s) ** 1.5
    return pref * np.exp(-(ai * aj / s) * r2)


def overlap_dense(centres: np.ndarray, exps: np.ndarray) -> np.ndarray:
    """Dense overlap matrix (small n only)."""
    n = centres.shape[0]
    d = centres[:, None, :] - centres[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", d, d)
    ai = exps[:, None]
    aj = exps[None, :]
    s = ai + aj
    S = (2.0 * np.sqrt(ai * aj) / s) ** 1.5 * np.exp(-(ai * aj / s) * r2)
    S[np.arange(n), np.arange(n)] = 1.0
    return S


def overlap_blocks(centres: np.ndarray, exps: np.ndarray, b: int, elem_eps: float = 0.0) -> BlockMatrix:
    """Block list of the overlap matrix.  Elements below ``elem_eps`` are left
    out (``elem_eps = 0`` keeps every pair whose exponential does not
    underflow)."""
    n = centres.shape[0]
    mu_min = float(exps.min()) / 2.0  # smallest reduced exponent a*a/(a+a)
    if elem_eps > 0.0:
        rcut = math.sqrt(-math.log(elem_eps) / mu_min)
    else:
        rcut = math.sqrt(745.0 / mu_min)
    ext = centres.max(axis=0) - centres.min(axis=0)
    if n <= 16000 and float(np.linalg.norm(ext)) <= rcut:
        S = overlap_dense(centres, exps)
        if elem_eps > 0.0:
            S[S < elem_eps] = 0.0
        return dense_to_blocks(S, b)
    from scipy.spatial import cKDTree
    tree = cKDTree(centres)
    pairs = tree.query_pairs(rcut, output_type="ndarray")
    i = pairs[:, 0].astype(np.int64)
    j = pairs[:, 1].astype(np.int64)
    v = _overlap_values(centres[i], centres[j], exps[i], exps[j])
    keep = v >= elem_eps if elem_eps > 0.0 else v > 0.0
    i, j, v = i[keep], j[keep], v[keep]
    d = np.arange(n, dtype=np.int64)
    rows = np.concatenate([i, j, d])
    cols = np.concatenate([j, i, d])
    vals = np.concatenate([v, v, np.ones(n)])
    return _coo_to_blocks(n, b, rows, cols, vals)


def _coo_to_blocks(n: int, b: int, rows, cols, vals) -> BlockMatrix:
    nb = (n + b - 1) // b
    key = (rows // b) * nb + (cols // b)
    ukeys, inv = np.unique(key, return_inverse=True)
    out = np.zeros((ukeys.shape[0], b, b))
    out[inv, rows % b, cols % b] = vals
    brow = (ukeys // nb).astype(np.int32)
    bcol = (ukeys % nb).astype(np.int32)
    return BlockMatrix(n=n, b=b, brow=brow, bcol=bcol, vals=out)


def dense_to_blocks(A: np.ndarray, b: int, keep_zero_blocks: bool = False) -> BlockMatrix:
    """Cut a dense n x n matrix into its nonzero b x b blocks."""
    n = A.shape[0]
    nb = (n + b - 1) // b
    P = np.zeros((nb * b, nb * b))
    P[:n, :n] = A
    T = P.reshape(nb, b, nb, b).transpose(0, 2, 1, 3)
    nz = np.ones((nb, nb), bool) if keep_zero_blocks else np.any(T != 0.0, axis=(2, 3))
    br, bc = np.nonzero(nz)
    return BlockMatrix(n=n, b=b, brow=br.astype(np.int32), bcol=bc.astype(np.int32),
                       vals=np.ascontiguousarray(T[br, bc]))


def blocks_to_dense(B: BlockMatrix) -> np.ndarray:
    nb = B.nb
    P = np.zeros((nb, nb, B.b, B.b))
    P[B.brow, B.bcol] = B.vals
    return P.transpose(0, 2, 1, 3).reshape(nb * B.b, nb * B.b)[:B.n, :B.n].copy()


def random_on_pattern(pattern: BlockMatrix, seed: int) -> BlockMatrix:
    """N(0,1) values on ``pattern``'s blocks, in its block order, zero in the
    padded tail."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = rng.standard_normal(pattern.vals.shape)
    _zero_padding(pattern, vals)
    return BlockMatrix(pattern.n, pattern.b, pattern.brow.copy(), pattern.bcol.copy(), vals)


def random_symmetric_on_pattern(pattern: BlockMatrix, seed: int, unit_norm: bool = True) -> BlockMatrix:
    """A symmetric N(0,1) direction on a symmetric block pattern, optionally
    scaled to unit Frobenius norm."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = rng.standard_normal(pattern.vals.shape)
    pos = {(int(r), int(c)): k for k, (r, c) in enumerate(zip(pattern.brow, pattern.bcol))}
    out = np.zeros_like(vals)
    for k, (r, c) in enumerate(zip(pattern.brow, pattern.bcol)):
        t = pos[(int(c), int(r))]
        out[k] = 0.5 * (vals[k] + vals[t].T)
    _zero_padding(pattern, out)
    if unit_norm:
        out /= np.sqrt(np.sum(out * out))
    return BlockMatrix(pattern.n, pattern.b, pattern.brow.copy(), pattern.bcol.copy(), out)


def _zero_padding(pattern: BlockMatrix, vals: np.ndarray) -> None:
    b, n, nb = pattern.b, pattern.n, pattern.nb
    tail = n - (nb - 1) * b
    if tail == b:
        return
    last_r = pattern.brow == nb - 1
    last_c = pattern.bcol == nb - 1
    vals[last_r, tail:, :] = 0.0
    vals[last_c, :, tail:] = 0.0


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

CONFIGS = {
    0: dict(name="water-100", kind="water", count=100, b=32, tau=0.0, seed=0),
    1: dict(name="chain-5000", kind="chain", count=5000, b=64, tau=1e-10, seed=1),
    2: dict(name="water-20000", kind="water", count=20000, b=64, tau=1e-8, seed=2),
    3: dict(name="water-2000", kind="water", count=2000, b=64, tau=0.0, seed=3),
    4: dict(name="water-150000", kind="water", count=150000, b=64, tau=1e-8, seed=4),
}


def config_matrix(k: int, count: int | None = None, b: int | None = None, tau: float | None = None):
    """(BlockMatrix S, config dict) for workload ``k``; ``count`` (molecules or
    residues), ``b`` and ``tau`` override the workload's own values for
    reduced-size cases."""
    cfg = dict(CONFIGS[k])
    if count is not None:
        cfg["count"] = count
    if b is not None:
        cfg["b"] = b
    if tau is not None:
        cfg["tau"] = tau
    if cfg["kind"] == "water":
        centres, exps = water_cluster(cfg["count"], cfg["seed"])
    else:
        centres, exps = helix_chain(cfg["count"], cfg["seed"])
    eps = 1e-3 * cfg["tau"] / cfg["b"] if cfg["tau"] > 0 else 0.0
    S = overlap_blocks(centres, exps, cfg["b"], eps)
    cfg["n"] = S.n
    return S, cfg
