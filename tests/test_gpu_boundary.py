"""The C ABI's contract beyond the arithmetic: per-stream workspaces (calls on
two streams in flight at once), the deterministic adjoint option, saved-
buffer validation, and plan-cache safety when index arrays are freed and
their addresses reused by another pattern of the same n and nnz."""
import gc

import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, check_launch_shapes, rel_fro, to_dev
from workloads import generators as G

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


def permuted(csr, seed):
    """P A P^T for a seeded permutation P: same n and nnz, another pattern."""
    perm = np.random.default_rng(seed).permutation(csr.n)
    a = csr.to_scipy()[perm][:, perm].tocsr()
    a.sort_indices()
    return G.CSR(a.indptr.astype(np.int32), a.indices.astype(np.int32), a.data.astype(np.float64), csr.n,
                 dict(csr.meta, permuted=seed))


def test_two_streams_in_flight(gpu_lib):
    """Forward and adjoint of two matrices, and of one matrix twice, issued on
    two streams without waiting in between: every result equals the
    oracle's (each stream works in its own workspace and status block)."""
    import torch
    import paper_1710_10899_amd as sm
    mats = [G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=81), G.banded_spd(200, 6)]
    for csr in mats:
        check_launch_shapes(csr)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    dev = [to_dev(c) for c in mats]
    ws = [torch.from_numpy(G.upstream_gradient(c, G.BASE_SEED + 150 + i)).cuda() for i, c in enumerate(mats)]
    torch.cuda.synchronize()
    # same pattern on both streams, then different patterns on each
    jobs = [(0, s1), (0, s2), (1, s1), (1, s2)]
    outs = []
    banner("two streams: forward + adjoint in flight together")
    for k, s in jobs:
        rp, ci, va = dev[k]
        with torch.cuda.stream(s):
            x = sm.invroot_fwd(rp, ci, va, 2)
            g = sm.invroot_bwd(rp, ci, va, ws[k], 2)
        outs.append((k, s, x, g))
    torch.cuda.synchronize()
    for k, s, x, g in outs:
        csr = mats[k]
        xr, bad = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 2)
        gr = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, G.upstream_gradient(csr, G.BASE_SEED + 150 + k))
        ex, eg = rel_fro(x.cpu().numpy(), xr), rel_fro(g.cpu().numpy(), gr)
        print(f"matrix {k}: forward {ex:.2e} adjoint {eg:.2e}", flush=True)
        assert ex <= TOL64 and eg <= TOL64
    for s in (s1, s2):
        with torch.cuda.stream(s):
            st = sm.query_status()
        assert st == {"nonpositive": 0, "fallback": 0, "unconverged": 0}


def _det_case(name):
    return {
        "overlap-40atoms": lambda: G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=81),
        "blockdiag-3-20-64-100": lambda: G.block_diagonal_spd((3, 20, 64, 100), kappa=30.0),
        "banded-n200-hb4": lambda: G.banded_spd(200, 4),
        "random-sparse-n150": lambda: G.random_sparse_spd(150, 0.08, kappa=20.0),
    }[name]()


@pytest.mark.parametrize("name", ["overlap-40atoms", "blockdiag-3-20-64-100", "banded-n200-hb4",
                                  "random-sparse-n150"])
@pytest.mark.parametrize("precision", ["f64", "f32_mixed"])
def test_deterministic_adjoint(name, precision, gpu_lib):
    """SUBMAT_OPT_DETERMINISTIC: two runs are bit-identical, grad_a is exactly
    symmetric (entry (r, c) equals entry (c, r)), and it matches the oracle
    like the atomic path; also with the large-order work split over several
    chunks (small workspace budget)."""
    import torch
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    csr = _det_case(name)
    w = G.upstream_gradient(csr, G.BASE_SEED + 160)
    ref = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w)
    tpos = np.empty(csr.nnz, dtype=np.int64)
    rows = np.repeat(np.arange(csr.n), csr.row_sizes())
    key = rows.astype(np.int64) * csr.n + csr.colind
    tkey = csr.colind.astype(np.int64) * csr.n + rows
    tpos[:] = np.searchsorted(key, tkey)
    assert np.array_equal(key[tpos], tkey)
    tol = TOL64 if precision == "f64" else TOL32
    try:
        for budget in (0.0, 2.5e6):
            _lib.submat_set_option(_lib.SUBMAT_OPT_WS_BYTES, budget)
            rp, ci, va = to_dev(csr)
            gx = torch.from_numpy(w).cuda()
            _lib.submat_set_option(_lib.SUBMAT_OPT_DETERMINISTIC, 1)
            banner(f"deterministic adjoint {name} {precision} budget={budget:g}")
            g1 = sm.invroot_bwd(rp, ci, va, gx, 2, precision).cpu().numpy()
            g2 = sm.invroot_bwd(rp, ci, va, gx, 2, precision).cpu().numpy()
            _lib.submat_set_option(_lib.SUBMAT_OPT_DETERMINISTIC, 0)
            ga = sm.invroot_bwd(rp, ci, va, gx, 2, precision).cpu().numpy()
            err, erra = rel_fro(g1, ref), rel_fro(ga, ref)
            print(f"{name} {precision} budget={budget:g}: deterministic {err:.2e}, atomic {erra:.2e}", flush=True)
            assert np.array_equal(g1.view(np.int64), g2.view(np.int64))
            assert np.array_equal(g1, g1[tpos])
            assert err <= tol and rel_fro(g1, ga) <= tol
            del rp, ci, va, gx
            _lib.submat_release()
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_DETERMINISTIC, 0)
        _lib.submat_set_option(_lib.SUBMAT_OPT_WS_BYTES, 0.0)


def test_saved_buffer_mismatch_rejected(gpu_lib):
    """A saved buffer is accepted only by a backward call with the pattern,
    value type and precision of the forward that filled it."""
    import torch
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    csr = G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=81)
    rp, ci, va = to_dev(csr)
    gx = torch.from_numpy(G.upstream_gradient(csr, G.BASE_SEED + 170)).cuda()
    nb = sm.saved_bytes(rp, ci, torch.float64, "f64")
    saved = torch.empty(nb, dtype=torch.uint8, device="cuda")
    other = torch.empty(nb, dtype=torch.uint8, device="cuda")
    banner("saved buffer validation")
    with pytest.raises(_lib.SubmatError) as e:
        sm.invroot_bwd(rp, ci, va, gx, 2, "f64", other)   # never filled
    assert e.value.code == _lib.SUBMAT_ESAVED
    sm.invroot_fwd(rp, ci, va, 2, "f64", saved)
    with pytest.raises(_lib.SubmatError) as e:
        sm.invroot_bwd(rp, ci, va, gx, 2, "f32_mixed", saved)   # FP64 forward, mixed backward
    assert e.value.code == _lib.SUBMAT_ESAVED
    with pytest.raises(_lib.SubmatError) as e:
        sm.invroot_bwd(rp, ci, va.float(), gx.float(), 2, "f64", saved)   # other value type
    assert e.value.code == _lib.SUBMAT_ESAVED
    g = sm.invroot_bwd(rp, ci, va, gx, 2, "f64", saved).cpu().numpy()
    ref = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, G.upstream_gradient(csr, G.BASE_SEED + 170))
    assert rel_fro(g, ref) <= TOL64


def test_int64_csr_patterns_with_equal_n_and_nnz(gpu_lib):
    """invroot_csr on int64-index sparse tensors: two different patterns of
    the same n and nnz, one after the other (the first freed in between, so
    its int32 index copies' addresses can be handed to the second), each
    equal to the oracle's."""
    import torch
    import paper_1710_10899_amd as sm
    base = G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=81)
    for k, csr in enumerate((base, permuted(base, 7), permuted(base, 8))):
        a = torch.sparse_csr_tensor(torch.from_numpy(csr.rowptr.astype(np.int64)),
                                    torch.from_numpy(csr.colind.astype(np.int64)),
                                    torch.from_numpy(csr.vals), (csr.n, csr.n)).cuda()
        assert a.crow_indices().dtype == torch.int64
        banner(f"invroot_csr int64 pattern {k}")
        x = sm.invroot_csr(a, 2)
        ref, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 2)
        err = rel_fro(x.values().cpu().numpy(), ref)
        print(f"pattern {k}: {err:.2e}", flush=True)
        assert err <= TOL64
        assert torch.equal(x.crow_indices(), a.crow_indices()) and torch.equal(x.col_indices(), a.col_indices())
        del a, x
        gc.collect()


@pytest.mark.parametrize("small_max", [16, 40, 64])
def test_every_column_processed_exactly_once(small_max, gpu_lib):
    """Status slot 6 counts the columns whose output a call wrote: it equals
    n for the forward and the adjoint whatever the split between the
    one-wavefront and the large-order buckets (bucket edge small_max), the
    number of workspace chunks, the precision passes (FP32 with forced FP64
    redos) or the per-column path."""
    import torch
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    csr = G.block_diagonal_spd((1, 7, 13, 30, 50, 64, 100, 140), kappa=40.0, permute=True)
    w = G.upstream_gradient(csr, G.BASE_SEED + 180)
    s = torch.cuda.current_stream().cuda_stream
    try:
        _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, small_max)
        for budget in (0.0, 3e6):
            _lib.submat_set_option(_lib.SUBMAT_OPT_WS_BYTES, budget)
            rp, ci, va = to_dev(csr)
            gx = torch.from_numpy(w).cuda()
            for precision, kmax in (("f64", 1e5), ("f32_mixed", 1e5), ("f32_mixed", 2.0), ("f64_plain", 1e5)):
                _lib.submat_set_option(_lib.SUBMAT_OPT_KAPPA_MAX, kmax)
                banner(f"columns once: small_max={small_max} budget={budget:g} {precision} kappa_max={kmax:g}")
                sm.invroot_fwd(rp, ci, va, 2, precision)
                nf = _lib.submat_query_counters(s, 7)[6]
                sm.invroot_bwd(rp, ci, va, gx, 2, precision)
                nb = _lib.submat_query_counters(s, 7)[6]
                assert nf == csr.n and nb == csr.n, (nf, nb, csr.n)
            _lib.submat_release()
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_KAPPA_MAX, 1e5)
        _lib.submat_set_option(_lib.SUBMAT_OPT_WS_BYTES, 0.0)
        _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, 0)


@pytest.mark.parametrize("precision", ["f64", "f32_mixed"])
def test_xcd_queues_bit_identical(precision, gpu_lib):
    """SUBMAT_OPT_XCD_QUEUES only changes which workgroup takes which
    (submatrix, column block) unit of the back-transformation and of the
    adjoint's products: the saved eigenvectors, the forward and the
    (deterministic) adjoint are bit-identical with one queue per XCD and with
    a single queue, and both equal the oracle."""
    import torch
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    csr = G.overlap_matrix(n_atoms=48, nbf=13, rcut=4.14, kappa=100.0, seed=85)
    check_launch_shapes(csr)
    w = G.upstream_gradient(csr, G.BASE_SEED + 190)
    rp, ci, va = to_dev(csr)
    gx = torch.from_numpy(w).cuda()
    nb = sm.saved_bytes(rp, ci, torch.float64, precision)
    outs = []
    try:
        _lib.submat_set_option(_lib.SUBMAT_OPT_DETERMINISTIC, 1)
        for queues in (1, 0):
            _lib.submat_set_option(_lib.SUBMAT_OPT_XCD_QUEUES, queues)
            banner(f"xcd queues={queues} {precision}")
            saved = torch.zeros(nb, dtype=torch.uint8, device="cuda")
            x = sm.invroot_fwd(rp, ci, va, 2, precision, saved).cpu().numpy()
            g1 = sm.invroot_bwd(rp, ci, va, gx, 2, precision, saved).cpu().numpy()
            g2 = sm.invroot_bwd(rp, ci, va, gx, 2, precision).cpu().numpy()
            outs.append((x, g1, g2, saved.cpu().numpy()))
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_XCD_QUEUES, 1)
        _lib.submat_set_option(_lib.SUBMAT_OPT_DETERMINISTIC, 0)
    (x1, g11, g21, s1), (x0, g10, g20, s0) = outs
    assert np.array_equal(s1, s0)
    assert np.array_equal(x1.view(np.int64), x0.view(np.int64))
    assert np.array_equal(g11.view(np.int64), g10.view(np.int64))
    assert np.array_equal(g21.view(np.int64), g20.view(np.int64))
    tol = TOL64 if precision == "f64" else TOL32
    xr, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, 2)
    gr = oracle.adjoint(csr.rowptr, csr.colind, csr.vals, csr.n, 2, w)
    ex, e1, e2 = rel_fro(x1, xr), rel_fro(g11, gr), rel_fro(g21, gr)
    print(f"{precision}: forward {ex:.2e}, adjoint saved {e1:.2e}, recomputed {e2:.2e}", flush=True)
    assert ex <= tol and e1 <= tol and e2 <= tol


def test_library_loaded_before_torch_uses_torch_runtime(gpu_lib):
    """A process that loads the library and sets an option before torch
    touches the GPU still computes correctly (the binding brings torch's HIP
    runtime in first). Runs in a child process with a fresh interpreter."""
    import subprocess
    import sys
    code = (
        "from paper_1710_10899_amd import _lib\n"
        "_lib.submat_set_option(_lib.SUBMAT_OPT_CLUSTER_TOL, 1e-5)\n"
        "import numpy as np, torch\n"
        "import oracle\n"
        "from workloads import generators as G\n"
        "import paper_1710_10899_amd as sm\n"
        "c = G.banded_spd(200, 6)\n"
        "rp, ci, va = (torch.from_numpy(v).cuda() for v in (c.rowptr, c.colind, c.vals))\n"
        "x = sm.invroot_fwd(rp, ci, va, 2).cpu().numpy()\n"
        "r, _ = oracle.forward(c.rowptr, c.colind, c.vals, c.n, 2)\n"
        "print('rel', float(np.linalg.norm(x - r) / np.linalg.norm(r)))\n")
    banner("library loaded before torch, in a child process")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240,
                         cwd=str(__import__("pathlib").Path(__file__).resolve().parents[1]))
    print(out.stdout[-500:], out.stderr[-2000:], flush=True)
    assert out.returncode == 0
    rel = float(out.stdout.split("rel")[-1])
    assert rel <= TOL64
