"""Helpers for the GPU tests: move a CSR to the device, compare with the
oracle, print the case before each GPU step."""
import sys

import numpy as np


def banner(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(csr, dtype=None):
    import torch
    dt = dtype or torch.float64
    rp = torch.from_numpy(csr.rowptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(csr.colind.astype(np.int32)).cuda()
    va = torch.from_numpy(csr.vals).to(dt).cuda()
    return rp, ci, va


def rel_fro(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def segments(csr, vec, cols):
    return np.concatenate([vec[csr.rowptr[j]:csr.rowptr[j + 1]] for j in cols])


def check_launch_shapes(csr):
    """Host-side check that the arrays match what the kernels assume."""
    assert csr.rowptr.shape[0] == csr.n + 1
    assert csr.rowptr[0] == 0 and csr.rowptr[-1] == csr.colind.shape[0] == csr.vals.shape[0]
    assert np.all(np.diff(csr.rowptr) >= 1)
    assert csr.colind.min() >= 0 and csr.colind.max() < csr.n
    assert np.diff(csr.rowptr).max() <= 2048


def affected_columns(csr, q):
    """Columns j whose submatrix holds the stored entry q = (i, k): R_i and
    R_k both contain j (the pattern is symmetric)."""
    rows = np.searchsorted(csr.rowptr, q, side="right") - 1
    i, k = int(rows), int(csr.colind[q])
    ri = csr.colind[csr.rowptr[i]:csr.rowptr[i + 1]]
    rk = csr.colind[csr.rowptr[k]:csr.rowptr[k + 1]]
    return np.intersect1d(ri, rk)


_POOL = {}


def _pool_init(rowptr, colind, vals, n, p, w):
    _POOL.update(rowptr=rowptr, colind=colind, vals=vals, n=n, p=p, w=w)


def _oracle_adjoint_job(cols):
    import oracle
    g = oracle.adjoint(_POOL["rowptr"], _POOL["colind"], _POOL["vals"], _POOL["n"], _POOL["p"], _POOL["w"],
                       cols=cols, check=False)
    nz = np.nonzero(g)[0]
    return nz, g[nz]


def oracle_adjoint_parallel(csr, p, w, cols, workers=8, chunk=16):
    """The oracle's adjoint summed over the given columns, the columns split
    over worker processes with single-threaded BLAS (CPU only; the matrix is
    sent to each worker once; the sum order differs from one call over the
    whole set only by rounding)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    cols = np.asarray(sorted(set(int(c) for c in cols)))
    parts = [cols[i:i + chunk] for i in range(0, cols.size, chunk)]
    out = np.zeros(csr.nnz)
    # only the rows of the submatrices are read: the workers get a copy of
    # the matrix with every other row emptied (same row numbers), and the
    # result comes back at the original positions
    rows = np.unique(np.concatenate([csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]] for j in cols]))
    sizes = np.zeros(csr.n, dtype=np.int64)
    sizes[rows] = csr.row_sizes()[rows]
    rp = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([np.arange(csr.rowptr[r], csr.rowptr[r + 1]) for r in rows])
    sub = (rp, csr.colind[pos], csr.vals[pos], csr.n, p, np.asarray(w)[pos])
    workers = max(1, min(workers, len(parts), os.cpu_count() or 1))
    keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in keep:
        os.environ[k] = "1"
    try:
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=_pool_init,
                                    initargs=sub) as ex:
            for k, (nz, v) in enumerate(ex.map(_oracle_adjoint_job, parts)):
                out[pos[nz]] += v
                print(f"oracle: {min((k + 1) * chunk, cols.size)} of {cols.size} submatrices", flush=True)
    finally:
        for k, v in keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return out


def atom_block_entries(csr, nbf, pairs, per_pair, rng):
    """Stored entries (positions) of the nbf x nbf blocks of the given atom
    pairs, per_pair of each, seeded. All entries of one block share their
    set of affected columns."""
    picks = []
    for a, b in pairs:
        block = []
        for i in range(a * nbf, (a + 1) * nbf):
            seg = csr.colind[csr.rowptr[i]:csr.rowptr[i + 1]]
            lo, hi = np.searchsorted(seg, [b * nbf, (b + 1) * nbf])
            block.extend(range(csr.rowptr[i] + lo, csr.rowptr[i] + hi))
        block = np.asarray(block)
        assert block.size == nbf * nbf, (a, b, block.size)
        picks.extend(rng.choice(block, per_pair, replace=False).tolist())
    return np.asarray(picks)


def neighbour_atom(csr, nbf, a, rng):
    """A seeded atom other than a whose block with a is stored."""
    seg = csr.colind[csr.rowptr[a * nbf]:csr.rowptr[a * nbf + 1]] // nbf
    cand = np.unique(seg[seg != a])
    return int(rng.choice(cand))
