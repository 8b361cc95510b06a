"""Autotuner for the persistent large-order launches.

Picks, per range of submatrix order, the launch parameters of the
persistent kernels by timing the library's own phases on seeded
overlap-type workloads whose orders fall in each range: workgroups per
compute unit of the FP64 and FP32 dense stages and of the tridiagonal
eigensolver, and the panel width and workgroups per compute unit of the
tridiagonal reduction (FP64 and FP32), and the edge between the
one-wavefront Jacobi bucket and the reduction path (timed on a workload of
orders on both sides of it). The result is a table file with lines "kind
m_hi value" (kind 0 / 1 = FP32 / FP64 dense kernels, 2 = tridiagonal
eigensolver, 3 / 4 = FP64 / FP32 reduction panel width, 5 / 6 = FP64 / FP32
reduction workgroups per compute unit, 7 = largest order of the
one-wavefront bucket); point the
environment variable SUBMAT_TUNE_FILE at it (the library reads it at its
first call, or when submat_set_option(SUBMAT_OPT_TUNE_FILE, 1) is called).

  python -m paper_1710_10899_amd.autotune --out tune.txt [--quick]

Needs a GPU. Every step runs in the library's HIP kernels; this module only
chooses launch parameters.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import tempfile
import time

# built-in table of the library (kind, m_hi, blocks per CU); a row with
# m_hi = 2**30 covers every larger order
DEFAULTS = [(1, 128, 8), (1, 256, 4), (1, 1024, 2), (1, 1 << 30, 1),
            (0, 128, 8), (0, 256, 4), (0, 1024, 2), (0, 1 << 30, 1),
            (2, 256, 8), (2, 512, 6), (2, 1024, 4), (2, 1 << 30, 1),
            (3, 1 << 30, 16), (4, 1 << 30, 16), (5, 1 << 30, 2), (6, 1 << 30, 3),
            (7, 1 << 30, 32)]
# one-wavefront bucket edges tried (orders above go to the reduction path)
EDGE_CANDIDATES = (32, 40, 48, 56, 64)
EDGE_WORKLOAD_MAX_ORDER = 96
# reduction candidates: (panel width, workgroups per compute unit)
REDUCTION_CANDIDATES = ((8, 2), (16, 2), (24, 2), (32, 2), (16, 1), (32, 1), (16, 3), (24, 3), (16, 4))
BUCKETS = (128, 256, 512, 1024)
DENSE_PHASES = ("gather", "tridiagonalise", "back-transform", "apply-column", "adjoint")
EIG_PHASES = ("tridiagonal-eig", "reorthogonalise")


def write_table(path, table):
    with open(path, "w") as fh:
        for kind, m_hi, bpc in table:
            fh.write(f"{kind} {m_hi} {bpc}\n")


def table_with(table, kind, m_hi, bpc):
    out = [(k, h, b) for (k, h, b) in table if not (k == kind and h == m_hi)]
    out.append((kind, m_hi, bpc))
    return sorted(out)


def workload_for(bucket, n_atoms, seed):
    """Overlap-type workload (13 basis functions per atom, density 0.1/A^3)
    whose largest submatrix order does not exceed `bucket`: the pair cutoff
    is shrunk until it fits."""
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import generators as G
    target = 0.7 * bucket
    rc = ((target / 13.0 - 1.0) / (0.1 * 4.0 / 3.0 * math.pi)) ** (1.0 / 3.0)
    while True:
        csr = G.overlap_matrix(n_atoms=n_atoms, nbf=13, rcut=rc, kappa=100.0, seed=seed)
        if csr.row_sizes().max() <= bucket or rc < 1.0:
            return csr
        rc *= 0.95


def time_phases(csr, precision, phases, reps):
    import numpy as np
    import torch

    from . import api
    rp = torch.from_numpy(csr.rowptr).cuda()
    ci = torch.from_numpy(csr.colind).cuda()
    va = torch.from_numpy(csr.vals).cuda()
    gx = torch.from_numpy(np.ones(csr.nnz)).cuda()
    best = math.inf
    for _ in range(reps):
        ph = api.time_phases(rp, ci, va, 2, precision, grad_x=gx, fn="inv_root")
        best = min(best, sum(ph[k][0] for k in (phases if phases is not None else ph) if k in ph))
    return best


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default="tune.txt")
    ap.add_argument("--candidates", default="1,2,3,4,6,8")
    ap.add_argument("--atoms", type=int, default=160, help="atoms per workload (13 columns each)")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--quick", action="store_true", help="two buckets, three candidates")
    args = ap.parse_args(argv)

    import torch

    from . import _lib
    _lib.load()
    torch.cuda.set_device(0)
    cands = [int(c) for c in args.candidates.split(",")]
    buckets = BUCKETS
    if args.quick:
        cands, buckets = [1, 2, 4], (256, 1024)
    table = list(DEFAULTS)
    fd, tmp = tempfile.mkstemp(suffix=".txt")
    os.close(fd)
    old_env = os.environ.get("SUBMAT_TUNE_FILE")
    os.environ["SUBMAT_TUNE_FILE"] = tmp
    try:
        for bi, bucket in enumerate(buckets):
            t0 = time.perf_counter()
            csr = workload_for(bucket, args.atoms, seed=171010899 + 500 + bi)
            m = csr.row_sizes()
            print(f"[autotune] bucket m<={bucket}: n={csr.n} m {m.min()}..{m.max()} "
                  f"(generated in {time.perf_counter() - t0:.1f}s)", flush=True)
            for kind, precision, phases in ((1, "f64", DENSE_PHASES), (0, "f32_mixed", DENSE_PHASES),
                                            (2, "f64", EIG_PHASES)):
                res = {}
                for c in cands:
                    write_table(tmp, table_with(table, kind, bucket, c))
                    _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1)
                    res[c] = time_phases(csr, precision, phases, args.reps)
                bpc = min(res, key=res.get)
                table = table_with(table, kind, bucket, bpc)
                print(f"[autotune]   kind {kind}: " + ", ".join(f"{c}:{v:.2f}ms" for c, v in res.items())
                      + f" -> {bpc}", flush=True)
            for kn, kc, precision in ((3, 5, "f64"), (4, 6, "f32_mixed")):
                res = {}
                for nb, pc in (REDUCTION_CANDIDATES if not args.quick else ((16, 2), (16, 3), (24, 2))):
                    write_table(tmp, table_with(table_with(table, kn, bucket, nb), kc, bucket, pc))
                    _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1)
                    res[(nb, pc)] = time_phases(csr, precision, ("tridiagonalise",), args.reps)
                nb, pc = min(res, key=res.get)
                table = table_with(table_with(table, kn, bucket, nb), kc, bucket, pc)
                print(f"[autotune]   reduction {precision}: " + ", ".join(f"nb={a} x{b}:{v:.2f}ms"
                                                                     for (a, b), v in res.items())
                      + f" -> nb={nb} x{pc}", flush=True)
        # the bucket edge: forward + adjoint over every phase of a workload
        # whose orders straddle the candidates
        csr = workload_for(EDGE_WORKLOAD_MAX_ORDER, args.atoms, seed=171010899 + 590)
        m = csr.row_sizes()
        print(f"[autotune] bucket edge: n={csr.n} m {m.min()}..{m.max()}", flush=True)
        res = {}
        for e in (EDGE_CANDIDATES if not args.quick else (48, 64)):
            write_table(tmp, table_with(table, 7, 1 << 30, e))
            _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1)
            res[e] = time_phases(csr, "f64", None, args.reps)
        edge = min(res, key=res.get)
        table = table_with(table, 7, 1 << 30, edge)
        print("[autotune]   edge: " + ", ".join(f"{e}:{v:.2f}ms" for e, v in res.items()) + f" -> {edge}",
              flush=True)
    finally:
        if old_env is None:
            os.environ.pop("SUBMAT_TUNE_FILE", None)
        else:
            os.environ["SUBMAT_TUNE_FILE"] = old_env
        _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1 if old_env else 0)
        os.unlink(tmp)
    write_table(args.out, table)
    print(f"[autotune] wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
