"""Guard against a pattern changed under a cached plan (a broken caller
contract): the index arrays keep their addresses, n and nnz, but hold
another valid pattern. Columns whose order no longer fits the slot planned
for them are not computed (NaN segment, counted in status slot 4); nothing
outside the plan's memory is touched; after submat_release_pattern the new
pattern is planned afresh and equals the oracle."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import banner, check_launch_shapes, rel_fro, to_dev
from tests.test_gpu_boundary import permuted
from workloads import generators as G

pytestmark = pytest.mark.gpu


def test_pattern_changed_under_cached_plan(gpu_lib):
    import torch
    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    a = G.overlap_matrix(n_atoms=40, nbf=13, rcut=4.14, kappa=100.0, seed=81)
    b = permuted(a, 7)
    check_launch_shapes(a)
    check_launch_shapes(b)
    ma, mb = a.row_sizes(), b.row_sizes()
    assert ma.min() > 64, "every column on the large-order path"
    # the plan's slot of column j: order rounded up to 16, and the chunk's
    # largest order (one chunk here)
    slot = np.minimum((ma + 15) // 16 * 16, ma.max())
    expect_stale = mb > slot
    assert expect_stale.any() and not expect_stale.all()
    rp, ci, va = to_dev(a)
    banner("stale plan: plan built for pattern A")
    x = sm.invroot_fwd(rp, ci, va, 2)
    torch.cuda.synchronize()
    # pattern B written into A's index arrays: same addresses, n, nnz
    rp.copy_(torch.from_numpy(b.rowptr).cuda())
    ci.copy_(torch.from_numpy(b.colind).cuda())
    va.copy_(torch.from_numpy(b.vals).cuda())
    torch.cuda.synchronize()
    banner("stale plan: pattern B under A's plan")
    x = sm.invroot_fwd(rp, ci, va, 2).cpu().numpy()
    stale = _lib.submat_query_counters(torch.cuda.current_stream().cuda_stream, 5)[4]
    seg_nan = np.array([np.isnan(x[b.rowptr[j]:b.rowptr[j + 1]]).all() for j in range(b.n)])
    print(f"stale columns counted {stale}, expected {int(expect_stale.sum())}", flush=True)
    assert stale == int(expect_stale.sum())
    assert seg_nan[expect_stale].all()
    banner("stale plan: released and replanned")
    sm.release_pattern(rp, ci)
    x = sm.invroot_fwd(rp, ci, va, 2).cpu().numpy()
    ref, _ = oracle.forward(b.rowptr, b.colind, b.vals, b.n, 2)
    assert rel_fro(x, ref) <= 1e-10
