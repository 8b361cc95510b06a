"""Full-size parity of the differentiation workload (overlap-type matrix of
1024 atoms x 13 basis functions, n = 13,312, kappa = 1e2), in the launch
configuration of the benchmark (batched, persistent kernels, graph replay):

  * forward, p = 1 and 2, FP64 and FP32 with FP64 fallback, on 40 sampled
    columns against the oracle computed column by column;
  * adjoint, p = 1 and 2, FP64 and FP32 with fallback (eigenvectors kept
    from the forward), on 32 sampled stored entries against the oracle's
    sum over every submatrix that holds the entry;
  * central finite differences (h = 1e-6) of L = <W, X.vals> through the
    GPU forward on 8 stored entries per p, L summed over the affected
    columns only (the others do not move).

Tolerances: FP64 1e-10 (relative Frobenius over the sample), FP32 1e-4
(kappa <= 1e3); finite differences 1e-6 relative + 1e-7 absolute."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import (affected_columns, atom_block_entries, banner, check_launch_shapes,
                            neighbour_atom, oracle_adjoint_parallel, rel_fro, segments, to_dev)
from workloads import generators as G

pytestmark = pytest.mark.gpu

NBF = 13
_CACHE = {}


def workload():
    if "csr" not in _CACHE:
        _CACHE["csr"] = G.make_config(4)
    return _CACHE["csr"]


def sample_columns(csr, count, seed):
    m = csr.row_sizes()
    order = np.argsort(m, kind="stable")
    rng = np.random.default_rng(seed)
    picks = [order[0], order[-1]] + list(rng.choice(csr.n, count - 2, replace=False))
    return sorted(set(int(c) for c in picks))


@pytest.mark.parametrize("p", [1, 2])
def test_config4_forward_sampled_columns(p, gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    csr = workload()
    check_launch_shapes(csr)
    cols = sample_columns(csr, 40, G.BASE_SEED + 400 + p)
    segs, bad = oracle.forward_columns(csr.rowptr, csr.colind, csr.vals, p, cols)
    assert not bad
    ref = np.concatenate([segs[j] for j in cols])
    rp, ci, va = to_dev(csr)
    for precision, tol in (("f64", 1e-10), ("f32_mixed", 1e-4)):
        banner(f"config4 forward p={p} {precision} n={csr.n}")
        x = torch.full_like(va, float("nan"))
        sm.invroot_fwd(rp, ci, va, p, precision, out=x)
        st = sm.query_status()
        xh = x.cpu().numpy()
        assert np.all(np.isfinite(xh)) and st["nonpositive"] == 0 and st["unconverged"] == 0
        err = rel_fro(segments(csr, xh, cols), ref)
        print(f"p={p} {precision} forward rel_err={err:.3e} over {len(cols)} columns, status {st}", flush=True)
        assert err <= tol


def _entries(csr, seed):
    rng = np.random.default_rng(seed)
    a = int(rng.integers(csr.n // NBF))
    b = neighbour_atom(csr, NBF, a, rng)
    c = int(rng.integers(csr.n // NBF))
    return atom_block_entries(csr, NBF, [(a, b), (c, c)], 16, rng)


@pytest.mark.parametrize("p", [1, 2])
def test_config4_adjoint_sampled_entries(p, gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    csr = workload()
    check_launch_shapes(csr)
    w = G.upstream_gradient(csr, G.BASE_SEED + 104)
    picks = _entries(csr, G.BASE_SEED + 410 + p)
    cols = np.unique(np.concatenate([affected_columns(csr, q) for q in picks]))
    banner(f"config4 adjoint oracle p={p}: {picks.size} entries over {cols.size} submatrices")
    ref = oracle_adjoint_parallel(csr, p, w, cols)[picks]
    rp, ci, va = to_dev(csr)
    gx = torch.from_numpy(w).cuda()
    for precision, tol in (("f64", 1e-10), ("f32_mixed", 1e-4)):
        banner(f"config4 adjoint p={p} {precision} (eigenvectors kept)")
        nb = sm.saved_bytes(rp, ci, torch.float64, precision)
        saved = torch.empty(nb, dtype=torch.uint8, device="cuda")
        sm.invroot_fwd(rp, ci, va, p, precision, saved)
        ga = sm.invroot_bwd(rp, ci, va, gx, p, precision, saved).cpu().numpy()
        st = sm.query_status()
        del saved
        torch.cuda.empty_cache()
        assert np.all(np.isfinite(ga)) and st["unconverged"] == 0
        err = rel_fro(ga[picks], ref)
        print(f"p={p} {precision} adjoint rel_err={err:.3e} over {picks.size} entries", flush=True)
        assert err <= tol


@pytest.mark.parametrize("p", [1, 2])
def test_config4_adjoint_central_differences(p, gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    csr = workload()
    w = G.upstream_gradient(csr, G.BASE_SEED + 104)
    rp, ci, va = to_dev(csr)
    gx = torch.from_numpy(w).cuda()
    banner(f"config4 central differences p={p}: adjoint")
    ga = sm.invroot_bwd(rp, ci, va, gx, p).cpu().numpy()
    rng = np.random.default_rng(G.BASE_SEED + 420 + p)
    picks = np.concatenate([_entries(csr, G.BASE_SEED + 430 + p)[:4], rng.choice(csr.nnz, 4, replace=False)])
    h = 1e-6
    vp, vm = va.clone(), va.clone()
    xp, xm = torch.empty_like(va), torch.empty_like(va)
    for q in picks:
        cols = affected_columns(csr, q)
        idx = np.concatenate([np.arange(csr.rowptr[j], csr.rowptr[j + 1]) for j in cols])
        vp.copy_(va)
        vm.copy_(va)
        vp[int(q)] += h
        vm[int(q)] -= h
        sm.invroot_fwd(rp, ci, vp, p, out=xp)
        sm.invroot_fwd(rp, ci, vm, p, out=xm)
        lp = float(np.dot(w[idx], xp.cpu().numpy()[idx]))
        lm = float(np.dot(w[idx], xm.cpu().numpy()[idx]))
        fd = (lp - lm) / (2 * h)
        print(f"p={p} entry {q}: fd {fd:.10e} adjoint {ga[q]:.10e} ({cols.size} columns)", flush=True)
        assert abs(fd - ga[q]) <= 1e-6 * max(1.0, abs(ga[q])) + 1e-7, (q, fd, ga[q])
