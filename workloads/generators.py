"""Seeded generators of sparse symmetric positive-definite test matrices.

Every generator returns a :class:`CSR` with int32 ``rowptr``/``colind`` (column
indices sorted and unique within each row, the diagonal always stored) and
float64 ``vals``. The pattern is structurally symmetric and the values are
exactly symmetric (each unordered pair is drawn once and mirrored).

The workloads stand in for the paper's inputs, which are not available:
random SPD matrices (Section 4.1), overlap matrices of 3D atomic systems
(Section 4.3) and the linear-density regime of Section 5.3. Recipes:

* ``banded_spd`` -- half-bandwidth ``hb``; off-diagonals ``0.3*U(-1,1)``,
  diagonal ``1 + sum |off-diagonal|`` (strictly diagonally dominant, so SPD).
* ``overlap_matrix`` -- atoms uniform in a periodic cube at a given number
  density, ``nbf`` basis functions per atom all centred on the atom,
  ``A_ij = exp(-alpha r^2) * c_ij`` with ``c_ij ~ U(0.5, 1)`` drawn once per
  unordered pair, kept for atom pairs closer than ``rcut`` (minimum image),
  then a diagonal shift ``sigma*I`` that sets the condition number to kappa.
* ``mixed_density_overlap`` -- the same with a smooth 4x density variation
  along x and two atom classes whose pair cutoff is the mean of their radii,
  which spreads the submatrix sizes over a wide range.

None of this module computes anything of the method itself.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

BASE_SEED = 1710_10899


@dataclass
class CSR:
    rowptr: np.ndarray  # int32 [n+1]
    colind: np.ndarray  # int32 [nnz]
    vals: np.ndarray    # float64 [nnz]
    n: int
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    def row_sizes(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _from_coo(rows, cols, vals, n, meta=None) -> CSR:
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    if m.indptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32 index range")
    return CSR(m.indptr.astype(np.int32), m.indices.astype(np.int32),
               m.data.astype(np.float64), n, dict(meta or {}))


def extreme_eigenvalues(csr: CSR) -> tuple[float, float]:
    """(lambda_min, lambda_max) of the symmetric matrix; dense for small n."""
    if csr.n <= 3000:
        w = np.linalg.eigvalsh(csr.dense())
        return float(w[0]), float(w[-1])
    from scipy.sparse.linalg import eigsh
    a = csr.to_scipy()
    # a seeded start vector: without one ARPACK draws its own, differently on
    # every call, and the extremes (hence the shift and every diagonal entry)
    # moved in their last bits from one generation of a workload to the next
    v0 = np.random.default_rng(BASE_SEED).standard_normal(csr.n)
    lmax = eigsh(a, k=1, which="LA", tol=1e-13, return_eigenvectors=False, ncv=48, v0=v0)[0]
    lmin = eigsh(a, k=1, which="SA", tol=1e-13, return_eigenvectors=False, ncv=64,
                 maxiter=100000, v0=v0)[0]
    return float(lmin), float(lmax)


def shift_to_kappa(csr: CSR, kappa: float, extremes: tuple[float, float] | None = None) -> CSR:
    """Add sigma*I so that lambda_max/lambda_min of the result equals kappa.
    `extremes` = (lambda_min, lambda_max) of csr when already known."""
    lmin, lmax = extremes if extremes is not None else extreme_eigenvalues(csr)
    sigma = (lmax - kappa * lmin) / (kappa - 1.0)
    diag_pos = _diag_positions(csr)
    vals = csr.vals.copy()
    vals[diag_pos] += sigma
    meta = dict(csr.meta)
    meta.update(kappa_target=float(kappa), sigma=float(sigma),
                lmin_unshifted=lmin, lmax_unshifted=lmax,
                lmin=lmin + sigma, lmax=lmax + sigma)
    return CSR(csr.rowptr, csr.colind, vals, csr.n, meta)


def _diag_positions(csr: CSR) -> np.ndarray:
    pos = np.empty(csr.n, dtype=np.int64)
    for i in range(csr.n):
        a, b = csr.rowptr[i], csr.rowptr[i + 1]
        k = np.searchsorted(csr.colind[a:b], i)
        if k >= b - a or csr.colind[a + k] != i:
            raise ValueError(f"row {i} has no stored diagonal")
        pos[i] = a + k
    return pos


# ---------------------------------------------------------------------------
# Plain structured matrices


def banded_spd(n: int = 1024, hb: int = 8, seed: int = BASE_SEED + 1, scale: float = 0.3) -> CSR:
    rng = _rng(seed)
    rows, cols, vals = [], [], []
    for d in range(1, hb + 1):
        i = np.arange(n - d)
        v = scale * rng.uniform(-1.0, 1.0, size=n - d)
        rows += [i, i + d]
        cols += [i + d, i]
        vals += [v, v]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    diag = 1.0 + np.bincount(r, weights=np.abs(v), minlength=n)
    r = np.concatenate([r, np.arange(n)])
    c = np.concatenate([c, np.arange(n)])
    v = np.concatenate([v, diag])
    return _from_coo(r, c, v, n, dict(kind="banded", hb=hb, seed=seed))


def diagonal_spd(n: int = 300, seed: int = BASE_SEED + 11, lo: float = 0.25, hi: float = 4.0) -> CSR:
    rng = _rng(seed)
    d = rng.uniform(lo, hi, size=n)
    i = np.arange(n)
    return _from_coo(i, i, d, n, dict(kind="diagonal", seed=seed))


def _random_spd_block(rng, m: int, kappa: float) -> np.ndarray:
    q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    lam = np.exp(rng.uniform(0.0, np.log(kappa), size=m)) if m > 1 else np.array([rng.uniform(1, kappa)])
    b = (q * lam) @ q.T
    return 0.5 * (b + b.T)


def block_diagonal_spd(sizes=(1, 7, 13, 64, 100), seed: int = BASE_SEED + 12,
                       kappa: float = 50.0, permute: bool = False) -> CSR:
    """Dense SPD diagonal blocks; optional symmetric random permutation."""
    rng = _rng(seed)
    n = int(sum(sizes))
    rows, cols, vals = [], [], []
    off = 0
    for m in sizes:
        b = _random_spd_block(rng, m, kappa)
        ii, jj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        rows.append((ii + off).ravel())
        cols.append((jj + off).ravel())
        vals.append(b.ravel())
        off += m
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    perm = np.arange(n)
    if permute:
        perm = rng.permutation(n)
        r, c = perm[r], perm[c]
    return _from_coo(r, c, v, n, dict(kind="block_diagonal", sizes=list(sizes), seed=seed,
                                      perm=perm.tolist() if permute else None))


def dense_spd(n: int = 48, seed: int = BASE_SEED + 13, kappa: float = 20.0) -> CSR:
    rng = _rng(seed)
    b = _random_spd_block(rng, n, kappa)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return _from_coo(ii.ravel(), jj.ravel(), b.ravel(), n, dict(kind="dense", seed=seed))


def dense_with_spectrum(eigs, seed: int = BASE_SEED + 17) -> CSR:
    """Dense symmetric matrix Q diag(eigs) Q^T with Q a seeded random
    orthogonal matrix (QR of a Gaussian matrix): prescribed, possibly
    repeated, eigenvalues."""
    rng = _rng(seed)
    eigs = np.asarray(eigs, dtype=np.float64)
    n = eigs.shape[0]
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    q = q * np.sign(np.diag(r))
    b = (q * eigs) @ q.T
    b = 0.5 * (b + b.T)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return _from_coo(ii.ravel(), jj.ravel(), b.ravel(), n, dict(kind="dense_spectrum", seed=seed))


def random_sparse_spd(n: int = 200, density: float = 0.05, seed: int = BASE_SEED + 14,
                      kappa: float = 10.0) -> CSR:
    """Random symmetric pattern (each i<j kept with probability density),
    N(0,1) values, diagonal shifted to the requested condition number."""
    rng = _rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.shape[0]) < density
    iu, ju = iu[keep], ju[keep]
    v = rng.standard_normal(iu.shape[0])
    r = np.concatenate([iu, ju, np.arange(n)])
    c = np.concatenate([ju, iu, np.arange(n)])
    vv = np.concatenate([v, v, np.zeros(n)])
    csr = _from_coo(r, c, vv, n, dict(kind="random_sparse", density=density, seed=seed))
    # explicit zeros on the diagonal must survive the COO->CSR conversion
    if csr.nnz != r.shape[0]:
        csr = _force_pattern(r, c, vv, n, csr.meta)
    return shift_to_kappa(csr, kappa)


def _force_pattern(r, c, v, n, meta) -> CSR:
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(rowptr.astype(np.int32), c.astype(np.int32), v.astype(np.float64), n, dict(meta))


def arrowhead_spd(n: int = 96, seed: int = BASE_SEED + 15) -> CSR:
    """First row/column full plus the diagonal: one submatrix of size n,
    n-1 submatrices of size 2."""
    rng = _rng(seed)
    v = 0.5 * rng.uniform(-1, 1, size=n - 1) / np.sqrt(n)
    i = np.arange(1, n)
    r = np.concatenate([np.zeros(n - 1, dtype=np.int64), i, np.arange(n)])
    c = np.concatenate([i, np.zeros(n - 1, dtype=np.int64), np.arange(n)])
    d = 1.0 + rng.uniform(0, 1, size=n)
    vv = np.concatenate([v, v, d])
    return _from_coo(r, c, vv, n, dict(kind="arrowhead", seed=seed))


def explicit_zero_pattern(seed: int = BASE_SEED + 16) -> CSR:
    """Banded SPD matrix with some stored entries set to an explicit 0.0,
    kept in the pattern (the stored pattern, not the numeric one, defines
    the submatrices)."""
    base = banded_spd(n=40, hb=3, seed=seed)
    rng = _rng(seed + 1)
    vals = base.vals.copy()
    rows = np.repeat(np.arange(base.n), base.row_sizes())
    off = np.nonzero(rows < base.colind)[0]
    pick = rng.choice(off, size=6, replace=False)
    for q in pick:
        i, j = rows[q], base.colind[q]
        vals[q] = 0.0
        a, b = base.rowptr[j], base.rowptr[j + 1]
        vals[a + np.searchsorted(base.colind[a:b], i)] = 0.0
    return CSR(base.rowptr, base.colind, vals, base.n, dict(kind="explicit_zeros", seed=seed))


# ---------------------------------------------------------------------------
# Overlap-type matrices of 3D atomic systems


def _atom_pairs(pos: np.ndarray, box: float, rcut_pair) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Unordered atom pairs (a<b) within the cutoff under periodic minimum
    image; ``rcut_pair`` is a float or a per-atom radius array (pair cutoff
    = mean of the two radii). Returns (a, b, r)."""
    from scipy.spatial import cKDTree
    tree = cKDTree(pos, boxsize=box)
    rmax = float(np.max(rcut_pair))
    pairs = tree.query_pairs(rmax, output_type="ndarray")
    a, b = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    d = pos[a] - pos[b]
    d -= box * np.round(d / box)
    r = np.sqrt(np.einsum("ij,ij->i", d, d))
    if np.ndim(rcut_pair) == 0:
        keep = r < rcut_pair
    else:
        keep = r < 0.5 * (rcut_pair[a] + rcut_pair[b])
    swap = a > b
    a2 = np.where(swap, b, a)
    b2 = np.where(swap, a, b)
    return a2[keep], b2[keep], r[keep]


def _overlap_from_pairs(n_atoms: int, nbf: int, a, b, r, alpha: float, rng, meta) -> CSR:
    n = n_atoms * nbf
    mu = np.arange(nbf)
    # off-diagonal atom blocks: nbf*nbf entries per unordered pair, mirrored
    npair = a.shape[0]
    c = rng.uniform(0.5, 1.0, size=(npair, nbf, nbf))
    val = np.exp(-alpha * r * r)[:, None, None] * c
    rows_ab = (a[:, None, None] * nbf + mu[None, :, None]) + 0 * mu[None, None, :]
    cols_ab = (b[:, None, None] * nbf + mu[None, None, :]) + 0 * mu[None, :, None]
    # same-atom blocks: c_{mu nu} drawn for mu <= nu and mirrored, exp(0) = 1
    iu, ju = np.triu_indices(nbf)
    cs = rng.uniform(0.5, 1.0, size=(n_atoms, iu.shape[0]))
    blk = np.zeros((n_atoms, nbf, nbf))
    blk[:, iu, ju] = cs
    blk[:, ju, iu] = cs
    at = np.arange(n_atoms)
    rows_aa = (at[:, None, None] * nbf + mu[None, :, None]) + 0 * mu[None, None, :]
    cols_aa = (at[:, None, None] * nbf + mu[None, None, :]) + 0 * mu[None, :, None]
    rows = np.concatenate([rows_ab.ravel(), cols_ab.ravel(), rows_aa.ravel()])
    cols = np.concatenate([cols_ab.ravel(), rows_ab.ravel(), cols_aa.ravel()])
    vals = np.concatenate([val.ravel(), val.ravel(), blk.ravel()])
    del rows_ab, cols_ab, val, c
    return _from_coo(rows.astype(np.int32), cols.astype(np.int32), vals, n, meta)


def overlap_matrix(n_atoms: int = 512, density: float = 0.1, nbf: int = 13, rcut: float = 4.14,
                   kappa: float = 1e2, alpha: float = 0.3, seed: int = BASE_SEED + 2) -> CSR:
    rng = _rng(seed)
    box = (n_atoms / density) ** (1.0 / 3.0)
    pos = rng.uniform(0.0, box, size=(n_atoms, 3))
    a, b, r = _atom_pairs(pos, box, rcut)
    meta = dict(kind="overlap", n_atoms=n_atoms, density=density, nbf=nbf, rcut=rcut,
                box=box, alpha=alpha, seed=seed)
    csr = _overlap_from_pairs(n_atoms, nbf, a, b, r, alpha, rng, meta)
    return shift_to_kappa(csr, kappa) if kappa else csr


def mixed_density_overlap(n_atoms: int = 4096, mean_density: float = 0.1, nbf: int = 13,
                          r_small: float = 2.8, r_large: float = 5.8, kappa: float = 1e2,
                          alpha: float = 0.3, seed: int = BASE_SEED + 3) -> CSR:
    """Number density varies smoothly by 4x along x (rho(x) proportional to
    1 + 1.5*(1 - cos(2 pi x / L))); half the atoms carry radius r_small, half
    r_large; a pair interacts when closer than the mean of their radii."""
    rng = _rng(seed)
    box = (n_atoms / mean_density) ** (1.0 / 3.0)
    # rejection sampling of x from the 4x density profile
    xs = []
    while sum(len(v) for v in xs) < n_atoms:
        x = rng.uniform(0.0, box, size=2 * n_atoms)
        w = (1.0 + 1.5 * (1.0 - np.cos(2.0 * np.pi * x / box))) / 4.0
        xs.append(x[rng.random(x.shape[0]) < w])
    x = np.concatenate(xs)[:n_atoms]
    pos = np.column_stack([x, rng.uniform(0.0, box, size=(n_atoms, 2))])
    radius = np.where(rng.random(n_atoms) < 0.5, r_small, r_large)
    a, b, r = _atom_pairs(pos, box, radius)
    meta = dict(kind="mixed_density_overlap", n_atoms=n_atoms, mean_density=mean_density,
                nbf=nbf, r_small=r_small, r_large=r_large, box=box, alpha=alpha, seed=seed)
    csr = _overlap_from_pairs(n_atoms, nbf, a, b, r, alpha, rng, meta)
    return shift_to_kappa(csr, kappa) if kappa else csr


def upstream_gradient(csr: CSR, seed: int) -> np.ndarray:
    """W ~ N(0,1) on X's pattern (X has exactly A's pattern)."""
    return _rng(seed).standard_normal(csr.nnz)


# ---------------------------------------------------------------------------
# Named workloads (index 1..5); index 0 is not used.

CONFIGS = {
    1: dict(name="banded_n1024_hb8", p=2, kappa=None),
    2: dict(name="overlap_512atoms_n6656", p=2, kappa=1e2),
    3: dict(name="mixed_overlap_4096atoms_n53248", p=2, kappa=1e2),
    4: dict(name="overlap_1024atoms_n13312", p=2, kappa=1e2),
    5: dict(name="overlap_16384atoms_n212992", p=2, kappa=1e6),
}


# Extreme eigenvalues (lambda_min, lambda_max) of the unshifted matrices of
# the two largest workloads, as printed by `python -m workloads.compute_extremes`
# (Lanczos, tolerance 1e-13): the shift is then placed without repeating it.
UNSHIFTED_EXTREMES = {
    3: (-2.3929758500221108, 86.66767021272706),
    5: (-2.1097858092000483, 62.6631285096728),
}


# condition number of each named workload when none is given (the banded
# workload is diagonally dominant and not shifted)
DEFAULT_KAPPA = {2: 1e2, 3: 1e2, 4: 1e2, 5: 1e6}


def make_config(idx: int, kappa: float | None = None, unshifted: bool = False) -> CSR:
    seed = BASE_SEED + idx
    if idx == 1:
        return banded_spd(1024, 8, seed=seed)
    if idx == 2:
        return overlap_matrix(512, 0.1, 13, 4.14, None if unshifted else (kappa or DEFAULT_KAPPA[2]), seed=seed)
    if idx == 4:
        return overlap_matrix(1024, 0.1, 13, 4.14, None if unshifted else (kappa or DEFAULT_KAPPA[4]), seed=seed)
    if idx == 3:
        csr = mixed_density_overlap(4096, kappa=None, seed=seed)
        k = kappa or DEFAULT_KAPPA[3]
    elif idx == 5:
        csr = overlap_matrix(16384, 0.1, 13, 4.47, None, seed=seed)
        k = kappa or DEFAULT_KAPPA[5]
    else:
        raise ValueError(f"unknown workload {idx}")
    return csr if unshifted else shift_to_kappa(csr, k, UNSHIFTED_EXTREMES.get(idx))
