"""Parity of the other spectral functions (positive p-th roots, real powers;
Section 4, "Applicability to other matrix operations") between the HIP
library, called through the C ABI, and the FP64 oracle: forward and adjoint,
both order paths (one wavefront per submatrix up to m = 64, the blocked
large-order pipeline above), FP64 and FP32 with FP64 fallback.

Tolerances: FP64 1e-10 relative Frobenius, as for the inverse root (the
eigendecomposition is shared; f and its divided differences are evaluated
in FP64 with relative error of a few ulps); FP32 mixed 1e-4 at kappa <= 1e2
(u32 * kappa ~ 6e-6, with margin for the f32 eigenvectors)."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, check_launch_shapes, rel_fro, segments, to_dev
from workloads import generators as G

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4

FUNCS = [("root", 2), ("root", 3), ("power", 0.5), ("power", -1.5), ("power", 2.0), ("power", 1.0 / 3.0)]

CASES = {
    "blockdiag-1-7-13-64-100-perm": lambda: G.block_diagonal_spd((1, 7, 13, 64, 100), permute=True),
    "dense-n130": lambda: G.dense_spd(130, kappa=30.0),
    "random-sparse-n300": lambda: G.random_sparse_spd(300, 0.05, kappa=50.0),
    "overlap-40atoms": lambda: G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=81),
}


def gpu_forward(csr, fn, param, precision="f64", dtype=None, saved=None):
    import torch
    import paper_1710_10899_amd as sm
    check_launch_shapes(csr)
    rp, ci, va = to_dev(csr, dtype)
    x = torch.full_like(va, float("nan"))
    sm.matfun_fwd(rp, ci, va, fn, param, precision, saved, out=x)
    st = sm.query_status()
    return x.double().cpu().numpy(), st


def gpu_backward(csr, fn, param, w, precision="f64", dtype=None, keep=False):
    import torch
    import paper_1710_10899_amd as sm
    check_launch_shapes(csr)
    rp, ci, va = to_dev(csr, dtype)
    gx = torch.from_numpy(w).to(va.dtype).cuda()
    saved = None
    if keep:
        nb = sm.saved_bytes(rp, ci, va.dtype, precision)
        saved = torch.empty(max(nb, 8), dtype=torch.uint8, device="cuda")
        sm.matfun_fwd(rp, ci, va, fn, param, precision, saved)
    ga = torch.full_like(va, float("nan"))
    sm.matfun_bwd(rp, ci, va, gx, fn, param, precision, saved, out=ga)
    st = sm.query_status()
    return ga.double().cpu().numpy(), st


@pytest.mark.parametrize("fn,param", FUNCS)
@pytest.mark.parametrize("name", list(CASES))
def test_matfun_forward_fp64_matches_oracle(name, fn, param, gpu_lib):
    csr = CASES[name]()
    banner(f"matfun forward f64 {name} {fn}({param:g}) n={csr.n} mmax={csr.row_sizes().max()}")
    x, st = gpu_forward(csr, fn, param)
    ref, bad = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, param, fn=fn)
    assert bad == 0 and st["nonpositive"] == 0 and st["unconverged"] == 0
    assert np.all(np.isfinite(x))
    err = rel_fro(x, ref)
    print(f"{name} {fn}({param:g}) rel_err={err:.3e}", flush=True)
    assert err <= TOL64


def test_matfun_power_one_returns_A_and_power_two_returns_A_squared(gpu_lib):
    """Structural identities of the method, checked on the GPU result
    directly: alpha = 1 gives A, alpha = 2 gives A^2 sampled on A's
    pattern (column-based)."""
    csr = CASES["overlap-40atoms"]()
    banner("matfun power 1 and 2 identities")
    x1, _ = gpu_forward(csr, "power", 1.0)
    assert rel_fro(x1, csr.vals) <= 1e-12
    A = csr.to_scipy()
    A2 = (A @ A).tocsr()
    rows = np.repeat(np.arange(csr.n), csr.row_sizes())
    x2, _ = gpu_forward(csr, "power", 2.0)
    assert rel_fro(x2, np.asarray(A2[csr.colind, rows]).ravel()) <= 1e-12


def test_matfun_mixed_precision(gpu_lib):
    import torch
    csr = G.overlap_matrix(n_atoms=64, nbf=13, rcut=4.14, kappa=100.0, seed=77)
    for fn, param in (("root", 2), ("power", 0.7)):
        ref, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, param, fn=fn)
        for dtype in (torch.float64, torch.float32):
            banner(f"matfun f32_mixed {fn}({param:g}) dtype={dtype}")
            x, st = gpu_forward(csr, fn, param, "f32_mixed", dtype)
            err = rel_fro(x, ref)
            print(f"{fn}({param:g}) dtype={dtype} rel_err={err:.3e} fallback={st['fallback']}", flush=True)
            assert err <= TOL32


def test_matfun_plain_path_equals_batched(gpu_lib):
    csr = CASES["blockdiag-1-7-13-64-100-perm"]()
    banner("matfun plain vs batched root(2)")
    xb, _ = gpu_forward(csr, "root", 2)
    xp, _ = gpu_forward(csr, "root", 2, "f64_plain")
    assert rel_fro(xp, xb) <= 1e-13


@pytest.mark.parametrize("fn,param", [("root", 2), ("root", 3), ("power", 0.7), ("power", -1.3)])
@pytest.mark.parametrize("name", ["blockdiag-1-7-13-64-100-perm", "overlap-40atoms"])
def test_matfun_adjoint_fp64_matches_oracle(name, fn, param, gpu_lib):
    csr = CASES[name]()
    w = G.upstream_gradient(csr, G.BASE_SEED + 110)
    banner(f"matfun adjoint f64 {name} {fn}({param:g})")
    ga, st = gpu_backward(csr, fn, param, w)
    ref = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, param, w, fn=fn)
    assert np.all(np.isfinite(ga)) and st["unconverged"] == 0
    err = rel_fro(ga, ref)
    print(f"{name} {fn}({param:g}) adjoint rel_err={err:.3e}", flush=True)
    assert err <= TOL64


def test_matfun_adjoint_power_one_is_symmetrised_upstream(gpu_lib):
    """alpha = 1: the gradient of sum(W * X) with X = A (a function of the
    symmetric part of each submatrix) is (W + W^T)/2 on the pattern."""
    csr = CASES["overlap-40atoms"]()
    w = G.upstream_gradient(csr, G.BASE_SEED + 111)
    banner("matfun adjoint power 1 closed form")
    ga, _ = gpu_backward(csr, "power", 1.0, w)
    W = csr.to_scipy().copy()
    W.data = w.copy()
    Wt = W.T.tocsr()
    Wt.sort_indices()
    assert rel_fro(ga, 0.5 * (w + Wt.data)) <= 1e-12


def test_matfun_saved_eigvecs_serve_every_function(gpu_lib):
    """The saved eigendecompositions do not depend on f: a buffer filled by
    an inverse-root forward gives the same root adjoint as a recompute."""
    import torch
    import paper_1710_10899_amd as sm
    csr = CASES["overlap-40atoms"]()
    w = G.upstream_gradient(csr, G.BASE_SEED + 112)
    banner("matfun saved buffer across functions")
    rp, ci, va = to_dev(csr)
    nb = sm.saved_bytes(rp, ci, va.dtype, "f64")
    saved = torch.empty(max(nb, 8), dtype=torch.uint8, device="cuda")
    sm.invroot_fwd(rp, ci, va, 2, "f64", saved)
    gx = torch.from_numpy(w).cuda()
    g_saved = sm.matfun_bwd(rp, ci, va, gx, "root", 2, "f64", saved).cpu().numpy()
    g_fresh = sm.matfun_bwd(rp, ci, va, gx, "root", 2, "f64").cpu().numpy()
    assert rel_fro(g_saved, g_fresh) <= 1e-14


def test_matfun_autograd(gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    csr = G.banded_spd(120, 5)
    w = G.upstream_gradient(csr, G.BASE_SEED + 113)
    rp, ci, va = to_dev(csr)
    banner("matfun autograd power(-0.25)")
    v = va.clone().requires_grad_(True)
    x = sm.matfun(rp, ci, v, "power", -0.25, keep_eigvecs=True)
    (g,) = torch.autograd.grad((torch.from_numpy(w).cuda() * x).sum(), v)
    ref = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, -0.25, w, fn="power")
    assert rel_fro(g.cpu().numpy(), ref) <= TOL64


def test_matfun_full_size_sampled_columns(gpu_lib):
    """The 6656-column overlap workload (orders ~160-700, the batched
    launch configuration of the benchmark), square root and a real power,
    on sampled columns the oracle computes one by one."""
    csr = G.make_config(2)
    m = csr.row_sizes()
    order = np.argsort(m, kind="stable")
    rng = np.random.default_rng(G.BASE_SEED + 302)
    cols = sorted(set([int(order[0]), int(order[-1])] + [int(c) for c in rng.choice(csr.n, 6, replace=False)]))
    for fn, param in (("root", 2), ("power", 0.7)):
        banner(f"matfun full size n={csr.n} {fn}({param:g})")
        x, st = gpu_forward(csr, fn, param)
        assert np.all(np.isfinite(x)) and st["nonpositive"] == 0 and st["unconverged"] == 0
        segs, bad = oracle.forward_columns(csr.rowptr, csr.colind, csr.vals, param, cols, fn)
        assert bad == 0
        err = rel_fro(segments(csr, x, cols), np.concatenate([segs[j] for j in cols]))
        print(f"{fn}({param:g}) sampled rel_err={err:.3e}", flush=True)
        assert err <= TOL64
