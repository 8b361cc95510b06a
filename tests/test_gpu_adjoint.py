"""Adjoint parity (Daleckii-Krein) of the HIP library against the FP64 CPU
oracle's gradient and against central finite differences of the GPU
forward."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, check_launch_shapes, rel_fro, to_dev
from workloads import generators as G

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


def gpu_backward(csr, p, w, precision="f64", dtype=None, keep=False):
    import torch
    import paper_1710_10899_amd as sm
    check_launch_shapes(csr)
    rp, ci, va = to_dev(csr, dtype)
    gx = torch.from_numpy(w).to(va.dtype).cuda()
    saved = None
    if keep:
        nb = sm.saved_bytes(rp, ci, va.dtype, precision)
        saved = torch.empty(max(nb, 8), dtype=torch.uint8, device="cuda")
        sm.invroot_fwd(rp, ci, va, p, precision, saved)
    ga = torch.full_like(va, float("nan"))
    sm.invroot_bwd(rp, ci, va, gx, p, precision, saved, out=ga)
    st = sm.query_status()
    return ga.double().cpu().numpy(), st


CASES = {
    "banded-n200-hb4": lambda: G.banded_spd(200, 4),
    "blockdiag-3-20-64-100": lambda: G.block_diagonal_spd((3, 20, 64, 100), kappa=30.0),
    "random-sparse-n150": lambda: G.random_sparse_spd(150, 0.08, kappa=20.0),
    "overlap-40atoms": lambda: G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=81),
}


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_fp64_matches_oracle(name, p, gpu_lib):
    csr = CASES[name]()
    w = G.upstream_gradient(csr, G.BASE_SEED + 100)
    banner(f"adjoint f64 {name} p={p} n={csr.n} mmax={csr.row_sizes().max()}")
    ga, st = gpu_backward(csr, p, w)
    ref = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, p, w)
    assert np.all(np.isfinite(ga))
    assert rel_fro(ga, ref) <= TOL64


@pytest.mark.parametrize("name", ["blockdiag-3-20-64-100", "overlap-40atoms"])
def test_saved_eigvecs_equal_recompute(name, gpu_lib):
    csr = CASES[name]()
    w = G.upstream_gradient(csr, G.BASE_SEED + 101)
    banner(f"adjoint saved vs recompute {name}")
    g1, _ = gpu_backward(csr, 2, w, keep=False)
    g2, _ = gpu_backward(csr, 2, w, keep=True)
    assert rel_fro(g2, g1) <= 1e-14


def test_adjoint_mixed_precision(gpu_lib):
    import torch
    csr = CASES["overlap-40atoms"]()
    w = G.upstream_gradient(csr, G.BASE_SEED + 102)
    ref = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w)
    for dtype in (torch.float64, torch.float32):
        for keep in (False, True):
            banner(f"adjoint f32_mixed dtype={dtype} keep={keep}")
            ga, _ = gpu_backward(csr, 2, w, "f32_mixed", dtype, keep)
            err = rel_fro(ga, ref)
            print(f"dtype={dtype} keep={keep} rel_err={err:.3e}", flush=True)
            assert err <= TOL32


def test_adjoint_central_finite_differences(gpu_lib):
    """dL/dA.vals[q] against (L(A + h e_q) - L(A - h e_q)) / 2h with the GPU
    forward, h = 1e-6, on sampled stored entries."""
    import torch
    import paper_1710_10899_amd as sm
    csr = G.overlap_matrix(n_atoms=24, nbf=13, rcut=4.14, kappa=50.0, seed=82)
    w = G.upstream_gradient(csr, G.BASE_SEED + 103)
    banner("adjoint vs central FD (GPU forward)")
    ga, _ = gpu_backward(csr, 2, w)
    rp, ci, va = to_dev(csr)
    wt = torch.from_numpy(w).cuda()
    rng = np.random.default_rng(G.BASE_SEED + 200)
    h = 1e-6
    diag = np.concatenate([csr.rowptr[j] + np.nonzero(csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]] == j)[0]
                           for j in range(0, csr.n, 37)])
    picks = np.concatenate([rng.choice(csr.nnz, 24, replace=False), diag[:8]])
    for q in picks:
        vp = va.clone()
        vp[q] += h
        vm = va.clone()
        vm[q] -= h
        lp = float((wt * sm.invroot_fwd(rp, ci, vp, 2)).sum())
        lm = float((wt * sm.invroot_fwd(rp, ci, vm, 2)).sum())
        fd = (lp - lm) / (2 * h)
        assert abs(fd - ga[q]) <= 1e-6 * max(1.0, abs(ga[q])) + 1e-7, (q, fd, ga[q])


def test_autograd_function(gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    csr = G.banded_spd(120, 5)
    w = G.upstream_gradient(csr, G.BASE_SEED + 104)
    rp, ci, va = to_dev(csr)
    banner("autograd Function")
    v = va.clone().requires_grad_(True)
    x = sm.invroot(rp, ci, v, 2, keep_eigvecs=True)
    loss = (torch.from_numpy(w).cuda() * x).sum()
    (g,) = torch.autograd.grad(loss, v)
    ref = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w)
    assert rel_fro(g.cpu().numpy(), ref) <= TOL64
