"""Prints the extreme eigenvalues of the unshifted large named workloads
(configs 3 and 5), which `generators.make_config` uses to place their
diagonal shift without repeating the Lanczos runs (minutes for n = 212,992).

  python -m workloads.compute_extremes
"""
from __future__ import annotations

import time

from workloads import generators as G


def main():
    for idx in (3, 5):
        t0 = time.perf_counter()
        csr = G.make_config(idx, unshifted=True)
        lmin, lmax = G.extreme_eigenvalues(csr)
        print(f"    {idx}: ({lmin!r}, {lmax!r}),  # {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
