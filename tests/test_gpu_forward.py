"""Forward parity of the HIP library against the FP64 CPU oracle, through
the C ABI (ctypes binding). FP64 bar: relative Frobenius error <= 1e-10;
FP32 mixed bar: <= 1e-4 at condition numbers <= 1e3; pattern bit-exact."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, check_launch_shapes, rel_fro, segments, to_dev
from workloads import generators as G

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


def gpu_forward(csr, p, precision="f64", dtype=None, poison=True):
    import torch
    import paper_1710_10899_amd as sm
    check_launch_shapes(csr)
    rp, ci, va = to_dev(csr, dtype)
    x = torch.full_like(va, float("nan")) if poison else torch.zeros_like(va)
    sm.invroot_fwd(rp, ci, va, p, precision, out=x)
    st = sm.query_status()
    assert np.array_equal(rp.cpu().numpy(), csr.rowptr) and np.array_equal(ci.cpu().numpy(), csr.colind)
    return x.double().cpu().numpy(), st


def oracle_forward(csr, p, cols=None):
    if cols is None:
        x, bad = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, p)
        return x, bad
    segs, bad = oracle.forward_columns(csr.rowptr, csr.colind, csr.vals, p, cols)
    return np.concatenate([segs[j] for j in cols]), bad


CASES = {
    "banded-n1024-hb8": lambda: G.make_config(1),
    "diagonal-n300": lambda: G.diagonal_spd(300),
    "blockdiag-1-7-13-64-100-perm": lambda: G.block_diagonal_spd((1, 7, 13, 64, 100), permute=True),
    "dense-n48": lambda: G.dense_spd(48),
    "dense-n130": lambda: G.dense_spd(130, kappa=30.0),
    "arrowhead-n96": lambda: G.arrowhead_spd(96),
    "explicit-zeros": lambda: G.explicit_zero_pattern(),
    "random-sparse-n300": lambda: G.random_sparse_spd(300, 0.05, kappa=50.0),
    "overlap-64atoms": lambda: G.overlap_matrix(n_atoms=64, nbf=13, rcut=4.14, kappa=100.0, seed=77),
}


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("name", list(CASES))
def test_forward_fp64_matches_oracle(name, p, gpu_lib):
    csr = CASES[name]()
    banner(f"forward f64 {name} p={p} n={csr.n} nnz={csr.nnz} mmax={csr.row_sizes().max()}")
    x, st = gpu_forward(csr, p)
    ref, bad = oracle_forward(csr, p)
    assert bad == 0 and st["nonpositive"] == 0 and st["unconverged"] == 0
    assert np.all(np.isfinite(x))
    assert rel_fro(x, ref) <= TOL64
    # per column too
    worst = max(rel_fro(x[csr.rowptr[j]:csr.rowptr[j + 1]], ref[csr.rowptr[j]:csr.rowptr[j + 1]])
                for j in range(0, csr.n, max(1, csr.n // 97)))
    assert worst <= 10 * TOL64


def test_diagonal_is_elementwise(gpu_lib):
    csr = G.diagonal_spd(300)
    for p in (1, 2, 3, 4):
        banner(f"diagonal elementwise p={p}")
        x, _ = gpu_forward(csr, p)
        ref = csr.vals ** (-1.0 / p)
        assert np.max(np.abs(x - ref) / ref) <= 4e-16


def test_overlap_workload_full_size_sampled(gpu_lib):
    csr = G.make_config(2)
    banner(f"forward f64 overlap n={csr.n} nnz={csr.nnz} (oracle on sampled columns)")
    x, st = gpu_forward(csr, 2)
    assert np.all(np.isfinite(x)) and st["unconverged"] == 0 and st["nonpositive"] == 0
    rng = np.random.default_rng(G.BASE_SEED + 300)
    m = csr.row_sizes()
    cols = sorted(set(rng.choice(csr.n, 40, replace=False).tolist()) | {int(np.argmax(m)), int(np.argmin(m))})
    ref, _ = oracle_forward(csr, 2, cols)
    assert rel_fro(segments(csr, x, cols), ref) <= TOL64


@pytest.mark.parametrize("kappa", [1e2, 1e3])
def test_mixed_precision_accuracy(kappa, gpu_lib):
    import torch
    csr = G.overlap_matrix(n_atoms=64, nbf=13, rcut=4.14, kappa=kappa, seed=78)
    banner(f"forward f32_mixed overlap kappa={kappa}")
    ref, _ = oracle_forward(csr, 2)
    for dtype in (torch.float64, torch.float32):
        x, st = gpu_forward(csr, 2, "f32_mixed", dtype)
        err = rel_fro(x, ref)
        print(f"kappa={kappa} dtype={dtype} rel_err={err:.3e} fallback={st['fallback']}", flush=True)
        assert err <= TOL32


def test_mixed_precision_small_path(gpu_lib):
    csr = G.make_config(1)
    banner("forward f32_mixed banded")
    ref, _ = oracle_forward(csr, 2)
    x, st = gpu_forward(csr, 2, "f32_mixed")
    assert rel_fro(x, ref) <= TOL32 and st["fallback"] == 0


def test_mixed_precision_fallback_equals_fp64(gpu_lib):
    """A kappa threshold below every submatrix's condition number sends all
    of them to FP64: the result is then the FP64 path's, bit for bit."""
    from paper_1710_10899_amd import _lib
    csr = G.block_diagonal_spd((5, 30, 80, 120), kappa=40.0)
    banner("forward f32_mixed forced fallback")
    x64, _ = gpu_forward(csr, 2, "f64")
    old = _lib.submat_get_option(_lib.SUBMAT_OPT_KAPPA_MAX)
    try:
        _lib.submat_set_option(_lib.SUBMAT_OPT_KAPPA_MAX, 1.0000001)
        xm, st = gpu_forward(csr, 2, "f32_mixed")
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_KAPPA_MAX, old)
    assert st["fallback"] == csr.n
    assert np.array_equal(x64, xm)


def test_ill_conditioned_falls_back(gpu_lib):
    """Submatrices whose own condition number exceeds the threshold (here:
    dense blocks with kappa ~ 1e7, so S_j is the block) are redone in FP64;
    a global kappa alone does not force this, since a principal submatrix
    is never worse conditioned than A but may be much better."""
    csr = G.block_diagonal_spd((12, 40, 90), kappa=1e7)
    kap = [np.linalg.cond(csr.dense()[a:b, a:b]) for a, b in ((0, 12), (12, 52), (52, 142))]
    banner(f"forward f32_mixed blocks kappa={[f'{k:.1e}' for k in kap]}")
    ref, _ = oracle_forward(csr, 2)
    x, st = gpu_forward(csr, 2, "f32_mixed")
    print(f"fallback={st['fallback']} of {csr.n}; rel_err={rel_fro(x, ref):.3e}", flush=True)
    expect = sum(b - a for (a, b), k in zip(((0, 12), (12, 52), (52, 142)), kap) if k > 1e5)
    assert st["fallback"] == expect > 0
    assert rel_fro(x, ref) <= 1e-8


def test_plain_path_equals_batched(gpu_lib):
    csr = G.block_diagonal_spd((3, 20, 64, 90), kappa=20.0)
    banner("forward f64_plain vs batched")
    xb, _ = gpu_forward(csr, 2, "f64")
    xp, _ = gpu_forward(csr, 2, "f64_plain")
    assert np.array_equal(xb, xp)


def test_graph_replay_is_bit_identical(gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    csr = G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=80)
    banner("graph replay vs direct launches")
    rp, ci, va = to_dev(csr)
    _lib.submat_set_option(_lib.SUBMAT_OPT_USE_GRAPH, 0)
    try:
        direct = sm.invroot_fwd(rp, ci, va, 2).cpu().numpy()
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_USE_GRAPH, 1)
    x = torch.empty_like(va)
    for k in range(4):
        x.fill_(float("nan"))
        sm.invroot_fwd(rp, ci, va, 2, out=x)
        torch.cuda.synchronize()
        _ = (va * 2).sum().item()  # unrelated eager work between replays
        assert np.array_equal(x.cpu().numpy(), direct), k


def test_float32_values_fp64_compute(gpu_lib):
    import torch
    csr = G.make_config(1)
    banner("forward f64 compute on float32 values")
    x, _ = gpu_forward(csr, 2, "f64", torch.float32)
    c32 = G.CSR(csr.rowptr, csr.colind, csr.vals.astype(np.float32).astype(np.float64), csr.n)
    ref, _ = oracle_forward(c32, 2)
    assert rel_fro(x, ref) <= 1e-6


@pytest.mark.parametrize("which", ["small", "large"])
def test_non_spd_segment_is_nan_and_counted(which, gpu_lib):
    csr = G.banded_spd(60, 2) if which == "small" else G.block_diagonal_spd((70, 10), kappa=10.0)
    vals = csr.vals.copy()
    j = 5
    d = csr.rowptr[j] + np.searchsorted(csr.colind[csr.rowptr[j]:csr.rowptr[j + 1]], j)
    vals[d] = -50.0
    bad_csr = G.CSR(csr.rowptr, csr.colind, vals, csr.n)
    banner(f"non-SPD input on the {which} path")
    x, st = gpu_forward(bad_csr, 2)
    ref, nbad = oracle_forward(bad_csr, 2)
    assert st["nonpositive"] == nbad >= 1
    assert np.array_equal(np.isnan(x), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert rel_fro(x[ok], ref[ok]) <= TOL64


def test_pattern_errors(gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib

    def run(rowptr, colind):
        rp = torch.tensor(rowptr, dtype=torch.int32, device="cuda")
        ci = torch.tensor(colind, dtype=torch.int32, device="cuda")
        va = torch.ones(len(colind), dtype=torch.float64, device="cuda")
        sm.invroot_fwd(rp, ci, va, 2)

    banner("pattern errors")
    with pytest.raises(_lib.SubmatError) as e:
        run([0, 2, 3], [0, 1, 1])          # (0,1) stored, (1,0) not
    assert e.value.code == _lib.SUBMAT_EPATTERN
    with pytest.raises(_lib.SubmatError) as e:
        run([0, 2, 4], [1, 0, 0, 1])       # row 0 unsorted
    assert e.value.code == _lib.SUBMAT_EPATTERN
    with pytest.raises(_lib.SubmatError) as e:
        run([0, 1, 2, 3], [0, 2, 1])       # rows 1, 2 miss their diagonal; asymmetric too
    assert e.value.code in (_lib.SUBMAT_ENODIAG, _lib.SUBMAT_EPATTERN)
    with pytest.raises(_lib.SubmatError) as e:
        run([0, 2, 4], [0, 1, 0, 1 + 5])   # out of range
    assert e.value.code == _lib.SUBMAT_EPATTERN
    with pytest.raises(_lib.SubmatError) as e:
        run([0, 1, 2], [1, 0])             # symmetric but no diagonal
    assert e.value.code == _lib.SUBMAT_ENODIAG


def test_sparse_csr_wrapper_reuses_pattern(gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    csr = G.banded_spd(50, 3)
    rp, ci, va = to_dev(csr)
    a = torch.sparse_csr_tensor(rp, ci, va, (csr.n, csr.n))
    banner("sparse csr wrapper")
    xcsr = sm.invroot_csr(a, 2)
    assert torch.equal(xcsr.crow_indices(), a.crow_indices())
    assert torch.equal(xcsr.col_indices(), a.col_indices())
    ref, _ = oracle_forward(csr, 2)
    assert rel_fro(xcsr.values().cpu().numpy(), ref) <= TOL64


def test_repeated_eigenvalues(gpu_lib):
    """Exactly repeated eigenvalues (multiplicities 40, 40, 30) in one dense
    submatrix of order 150: the tridiagonal eigensolver sees split blocks
    and near-coincident eigenvalues."""
    eigs = np.concatenate([np.full(40, 1.0), np.full(40, 2.0), np.full(30, 3.5), np.linspace(4.0, 9.0, 40)])
    csr = G.dense_with_spectrum(eigs)
    banner("repeated eigenvalues, dense n=150")
    for p in (1, 2):
        x, st = gpu_forward(csr, p)
        ref, _ = oracle_forward(csr, p)
        err = rel_fro(x, ref)
        print(f"p={p} rel_err={err:.3e} status={st}", flush=True)
        assert err <= TOL64 and st["unconverged"] == 0


def test_near_degenerate_eigenvalues_unsplit(gpu_lib):
    """Distinct eigenvalues in groups of four at relative gaps 1e-4, 1e-8 and
    1e-12 in one dense submatrix of order 160: T does not split, so every
    eigenvalue is found by the count-safeguarded search, which has to isolate
    members of a group before its Newton steps apply."""
    base = np.linspace(1.0, 9.0, 40)
    eigs = np.concatenate([base, base * (1 + 1e-4), base * (1 + 1e-8), base * (1 + 1e-12)])
    csr = G.dense_with_spectrum(eigs, seed=G.BASE_SEED + 19)
    banner("near-degenerate eigenvalues, dense n=160")
    for p in (1, 2):
        x, st = gpu_forward(csr, p)
        ref, _ = oracle_forward(csr, p)
        err = rel_fro(x, ref)
        print(f"p={p} rel_err={err:.3e} status={st}", flush=True)
        assert err <= TOL64 and st["unconverged"] == 0


@pytest.mark.parametrize("ctol", [0.0, 1e-5, 1e-2, 0.5])
def test_cluster_tolerance_paths(ctol, gpu_lib):
    """Twisted factorisation only (0), the earlier default (1e-5), many
    clusters (1e-2), every eigenvalue of a block in one cluster (0.5, inverse
    iteration throughout): all meet the FP64 bar."""
    from paper_1710_10899_amd import _lib
    csr = G.overlap_matrix(n_atoms=24, nbf=13, rcut=4.14, kappa=100.0, seed=83)
    banner(f"cluster tolerance {ctol}")
    default = _lib.submat_get_option(_lib.SUBMAT_OPT_CLUSTER_TOL)
    _lib.submat_set_option(_lib.SUBMAT_OPT_CLUSTER_TOL, ctol)
    try:
        x, st = gpu_forward(csr, 2)
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_CLUSTER_TOL, default)
    ref, _ = oracle_forward(csr, 2)
    err = rel_fro(x, ref)
    print(f"ctol={ctol} rel_err={err:.3e} status={st}", flush=True)
    assert err <= TOL64 and st["unconverged"] == 0


def test_results_independent_of_launch_grid(gpu_lib, tmp_path, monkeypatch):
    """The per-submatrix arithmetic does not depend on how many workgroups
    the persistent kernels run: bit-identical outputs for other tables."""
    from paper_1710_10899_amd import _lib
    from paper_1710_10899_amd import autotune
    csr = G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=84)
    banner("launch-grid independence")
    ref, _ = gpu_forward(csr, 2)
    table = autotune.DEFAULTS
    for kind, bpc in ((1, 1), (1, 3), (2, 1)):
        table = autotune.table_with(table, kind, 1024, bpc)
    path = tmp_path / "tune.txt"
    autotune.write_table(path, table)
    monkeypatch.setenv("SUBMAT_TUNE_FILE", str(path))
    _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1)
    try:
        x, _ = gpu_forward(csr, 2)
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 0)
    assert np.array_equal(x, ref)


def test_bucket_edge_from_tuning_table(gpu_lib, tmp_path, monkeypatch):
    """The one-wavefront bucket edge comes from the tuning table (kind 7):
    with edge 40 the orders 50 and 64 run on the reduction path (its phases
    launch), with the built-in 64 they do not; both equal the oracle."""
    import torch
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    from paper_1710_10899_amd import autotune
    csr = G.block_diagonal_spd((1, 7, 30, 50, 64), kappa=40.0, permute=True)
    ref, _ = oracle_forward(csr, 2)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("SUBMAT_TUNE_FILE", str(path))
    rp, ci, va = to_dev(csr)
    try:
        _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, 0)  # the table's edge
        for edge in (40, 64):
            autotune.write_table(path, autotune.table_with(autotune.DEFAULTS, 7, 1 << 30, edge))
            _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 1)
            assert _lib.submat_get_option(_lib.SUBMAT_OPT_SMALL_MAX) == edge
            banner(f"bucket edge {edge} from the tuning table")
            x = torch.empty_like(va)
            ph = sm.time_phases(rp, ci, va, 2, "f64")
            sm.invroot_fwd(rp, ci, va, 2, "f64", out=x)
            err = rel_fro(x.cpu().numpy(), ref)
            large = ph.get("tridiagonalise", (0.0, 0))[1]
            print(f"edge {edge}: reduction launches {large}, rel_err {err:.2e}", flush=True)
            assert err <= TOL64
            assert (large > 0) == (edge == 40)
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_TUNE_FILE, 0)
        _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, 0)
