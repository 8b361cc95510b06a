"""Parity at the full sizes of the two largest named workloads, in the
launch configuration of the benchmark (batched, persistent kernels, graph
replay), on sampled outputs the FP64 oracle computes column by column:

  * mixed-density overlap matrix, 4096 atoms (n = 53,248, orders 52-1534,
    both the one-wavefront and the large-order path), kappa 1e2 and 1e4,
    FP64 and FP32 with FP64 fallback;
  * ill-conditioned overlap matrix, 16,384 atoms (n = 212,992, orders
    ~500, kappa 1e6, workspace in several chunks), FP64 for p = 1 and 3,
    FP32 with fallback for p = 2, and the FP64 adjoint on a sampled entry.

Tolerances: FP64 1e-10 (kappa <= 1e4) and 1e-9 at kappa = 1e6 (the
eigendecomposition's backward error eps * ||S|| moves lambda_min by a
relative eps * kappa ~ 1e-10); FP32 1e-4 at kappa <= 1e3, and 5e-3 where
the FP32 pass keeps submatrices up to kappa_max = 1e5 (error ~ kappa u32,
u32 = 6e-8, capped by the 1e5 threshold at ~6e-3)."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, check_launch_shapes, rel_fro, segments, to_dev
from workloads import generators as G

pytestmark = pytest.mark.gpu

_CACHE = {}


def workload(idx, kappa=None):
    key = (idx, kappa)
    if key not in _CACHE:
        _CACHE.clear()
        _CACHE[key] = G.make_config(idx, kappa=kappa)
    return _CACHE[key]


def sample_columns(csr, count, seed):
    """Columns spread over the order distribution: the smallest and largest
    submatrix plus seeded picks between."""
    m = csr.row_sizes()
    order = np.argsort(m, kind="stable")
    rng = np.random.default_rng(seed)
    picks = [order[0], order[-1]] + list(rng.choice(csr.n, count - 2, replace=False))
    return sorted(set(int(c) for c in picks))


def forward(csr, p, precision):
    import torch
    import paper_1710_10899_amd as sm
    check_launch_shapes(csr)
    rp, ci, va = to_dev(csr)
    x = torch.full_like(va, float("nan"))
    sm.invroot_fwd(rp, ci, va, p, precision, out=x)
    st = sm.query_status()
    out = x.cpu().numpy()
    del rp, ci, va, x
    torch.cuda.empty_cache()
    return out, st


def oracle_segments(csr, p, cols):
    segs, bad = oracle.forward_columns(csr.rowptr, csr.colind, csr.vals, p, cols)
    assert not bad
    return np.concatenate([segs[j] for j in cols])


@pytest.mark.parametrize("kappa", [1e2, 1e4])
def test_mixed_density_workload_full_size(kappa, gpu_lib):
    csr = workload(3, kappa)
    cols = sample_columns(csr, 10, G.BASE_SEED + 300)
    ref = oracle_segments(csr, 2, cols)
    for precision, tol in (("f64", 1e-10), ("f32_mixed", 1e-4 if kappa <= 1e3 else 5e-3)):
        banner(f"mixed-density n={csr.n} kappa={kappa:g} {precision}")
        x, st = forward(csr, 2, precision)
        assert np.all(np.isfinite(x)) and st["nonpositive"] == 0 and st["unconverged"] == 0
        err = rel_fro(segments(csr, x, cols), ref)
        print(f"kappa={kappa:g} {precision} rel_err={err:.3e} status={st}", flush=True)
        assert err <= tol


def test_ill_conditioned_workload_full_size(gpu_lib):
    csr = workload(5)
    cols = sample_columns(csr, 8, G.BASE_SEED + 301)
    for p, precision, tol in ((2, "f32_mixed", 5e-3), (1, "f64", 1e-9), (3, "f64", 1e-9)):
        banner(f"kappa=1e6 n={csr.n} p={p} {precision}")
        x, st = forward(csr, p, precision)
        assert np.all(np.isfinite(x)) and st["nonpositive"] == 0 and st["unconverged"] == 0
        err = rel_fro(segments(csr, x, cols), oracle_segments(csr, p, cols))
        print(f"p={p} {precision} rel_err={err:.3e} status={st}", flush=True)
        assert err <= tol


def test_ill_conditioned_workload_adjoint_sampled_entry(gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    csr = workload(5)
    w = G.upstream_gradient(csr, G.BASE_SEED + 105)
    banner(f"adjoint f64 kappa=1e6 n={csr.n} (recompute)")
    rp, ci, va = to_dev(csr)
    ga = sm.invroot_bwd(rp, ci, va, torch.from_numpy(w).cuda(), 2).cpu().numpy()
    st = sm.query_status()
    print(f"gpu adjoint done, status {st}", flush=True)
    assert np.all(np.isfinite(ga)) and st["unconverged"] == 0
    rows = np.repeat(np.arange(csr.n), csr.row_sizes())
    q = int(np.random.default_rng(G.BASE_SEED + 206).choice(csr.nnz))
    i, k = rows[q], csr.colind[q]
    ri = csr.colind[csr.rowptr[i]:csr.rowptr[i + 1]]
    rk = csr.colind[csr.rowptr[k]:csr.rowptr[k + 1]]
    cols = np.intersect1d(ri, rk)
    ref = np.zeros(csr.nnz)
    for c0 in range(0, cols.size, 64):  # the oracle in chunks, printing its progress
        ref += oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w, cols=cols[c0:c0 + 64], check=False)
        print(f"oracle: {min(c0 + 64, cols.size)} of {cols.size} submatrices", flush=True)
    print(f"entry {q} ({i},{k}) over {cols.size} submatrices: gpu {ga[q]:.15e} oracle {ref[q]:.15e}", flush=True)
    assert abs(ga[q] - ref[q]) <= 1e-9 * max(1.0, np.abs(ref).max())
