"""The forward entry point that allocates nothing
(submat_invroot_fwd_noalloc), through the C ABI: its output equals that of
submat_invroot_fwd on the same inputs bit for bit (and the oracle's within
1e-10 for FP64, 1e-4 for FP32 with fallback), on two calls in a row, the
second on a smaller input; columns above order 64 and invalid patterns are reported on
the device, and sizes beyond the scratch are rejected synchronously."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, check_launch_shapes, rel_fro, to_dev
from workloads import generators as G

pytestmark = pytest.mark.gpu


def _noalloc(csr, p, precision, dtype=None):
    import torch
    from paper_1710_10899_amd import _lib
    check_launch_shapes(csr)
    rp, ci, va = to_dev(csr, dtype)
    x = torch.full_like(va, float("nan"))
    code = _lib.SUBMAT_F64 if va.dtype == torch.float64 else _lib.SUBMAT_F32
    prec = {"f64": _lib.SUBMAT_PREC_F64, "f32_mixed": _lib.SUBMAT_PREC_F32_MIXED}[precision]
    s = torch.cuda.current_stream().cuda_stream
    _lib.submat_invroot_fwd_noalloc(rp.data_ptr(), ci.data_ptr(), va.data_ptr(), csr.n, csr.nnz, p, code, prec,
                                    x.data_ptr(), s)
    counters = _lib.submat_query_counters(s, 6)
    return x.double().cpu().numpy(), counters


def _planned(csr, p, precision, dtype=None):
    """The planned entry point with every order up to 64 on the one-wavefront
    kernel, the one the entry point that allocates nothing runs."""
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    rp, ci, va = to_dev(csr, dtype)
    _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, 64)
    try:
        return sm.invroot_fwd(rp, ci, va, p, precision).double().cpu().numpy()
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_SMALL_MAX, 0)


@pytest.mark.parametrize("precision", ["f64", "f32_mixed"])
def test_noalloc_matches_planned_entry_point(precision, gpu_lib):
    big = G.make_config(1)                      # n = 1024, orders 9..17
    small = G.banded_spd(300, 5, seed=G.BASE_SEED + 91)
    mixed = G.block_diagonal_spd((1, 7, 13, 40, 64, 33), kappa=30.0, permute=True)
    for csr in (big, small, mixed):
        for p in (1, 2, 3):
            banner(f"noalloc {precision} n={csr.n} mmax={csr.row_sizes().max()} p={p}")
            x, ctr = _noalloc(csr, p, precision)
            ref = _planned(csr, p, precision)
            assert ctr[4] == 0 and ctr[5] == 0 and ctr[0] == 0 and ctr[2] == 0
            assert np.all(np.isfinite(x))
            err = rel_fro(x, ref)
            xo, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, csr.n, p)
            print(f"n={csr.n} p={p} {precision}: vs planned {err:.2e}, vs oracle {rel_fro(x, xo):.2e}", flush=True)
            # the same kernel with the same per-submatrix arithmetic: equal bits
            assert np.array_equal(x, ref), err
            assert rel_fro(x, xo) <= (1e-10 if precision == "f64" else 1e-4)


def test_noalloc_float32_values(gpu_lib):
    import torch
    csr = G.make_config(1)
    banner("noalloc float32 values")
    x, _ = _noalloc(csr, 2, "f64", torch.float32)
    ref = _planned(csr, 2, "f64", torch.float32)
    assert rel_fro(x, ref) <= 1e-6


def test_noalloc_limits(gpu_lib):
    from paper_1710_10899_amd import _lib
    # a column of order 65 or more: its segment is NaN and counted, the rest computed
    csr = G.block_diagonal_spd((5, 70, 12), kappa=30.0)
    banner("noalloc order above 64")
    x, ctr = _noalloc(csr, 2, "f64")
    m = csr.row_sizes()
    long_cols = np.nonzero(m > 64)[0]
    assert ctr[4] == long_cols.size
    for j in range(csr.n):
        seg = x[csr.rowptr[j]:csr.rowptr[j + 1]]
        assert (np.isnan(seg).all() if m[j] > 64 else np.isfinite(seg).all())
    # an invalid pattern (a diagonal entry missing) writes nothing and is counted
    bad = G.explicit_zero_pattern()
    import torch
    rp, ci, va = to_dev(bad)
    keep = torch.ones(bad.nnz, dtype=torch.bool)
    rows = np.repeat(np.arange(bad.n), bad.row_sizes())
    drop = int(np.nonzero(bad.colind == rows)[0][0])
    keep[drop] = False
    ci2 = ci[keep.cuda()].contiguous()
    va2 = va[keep.cuda()].contiguous()
    rp2 = torch.from_numpy(np.concatenate([[0], np.cumsum(bad.row_sizes() - (np.arange(bad.n) == rows[drop]))])
                           .astype(np.int32)).cuda()
    x2 = torch.full_like(va2, 7.0)
    s = torch.cuda.current_stream().cuda_stream
    banner("noalloc invalid pattern")
    _lib.submat_invroot_fwd_noalloc(rp2.data_ptr(), ci2.data_ptr(), va2.data_ptr(), bad.n, int(va2.numel()), 2, 0, 0,
                                    x2.data_ptr(), s)
    ctr = _lib.submat_query_counters(s, 6)
    assert ctr[5] == 1 and torch.all(x2 == 7.0)
    # sizes beyond the scratch are rejected before any device work
    with pytest.raises(_lib.SubmatError) as e:
        _lib.submat_invroot_fwd_noalloc(rp.data_ptr(), ci.data_ptr(), va.data_ptr(), (1 << 20) + 1, 1 << 21, 2, 0, 0,
                                        x2.data_ptr(), s)
    assert e.value.code == _lib.SUBMAT_ETOOBIG
    with pytest.raises(_lib.SubmatError) as e:
        _lib.submat_invroot_fwd_noalloc(rp.data_ptr(), ci.data_ptr(), va.data_ptr(), bad.n, bad.nnz, 2, 0,
                                        _lib.SUBMAT_PREC_F64_PLAIN, x2.data_ptr(), s)
    assert e.value.code == _lib.SUBMAT_EINVAL
