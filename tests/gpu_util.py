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
