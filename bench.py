"""Benchmark: one step = submatrix-method forward + Daleckii-Krein adjoint over
the whole overlap-type workload (512 atoms, 13 basis functions per atom,
n = 6656, ~400 stored entries per column, kappa = 1e2, p = 2), inputs resident
in HBM. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision f64|f32_mixed]
                  [--workload 1..5] [--fn inv_root|root|power] [--p P] [--alpha A]

The default is the inverse square root; --fn selects the other spectral
functions (positive p-th root, real power), which run the same kernels.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (vector = matrix)
FP32_PEAK_TFLOPS = 157.3    # MI355X dense FP32 (matrix / packed vector)
FP64_VALU_PEAK = 78.6       # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_VALU_PEAK = 78.6       # unpacked FP32 VALU: same lane rate as FP64
HBM_PEAK_GBS = 8000.0

WORKLOAD_NAMES = {
    1: "banded SPD matrix, n=1024, half-bandwidth 8, p={p}; forward + adjoint",
    2: "overlap-type SPD matrix, 512 atoms x 13 basis functions (n=6656), ~400 stored entries per column, "
       "kappa={kappa:g}, p={p}; forward + adjoint",
    3: "mixed-density overlap-type SPD matrix, 4096 atoms x 13 (n=53248), orders 52-1534, kappa={kappa:g}, "
       "p={p}; forward + adjoint",
    4: "overlap-type SPD matrix, 1024 atoms x 13 (n=13312), kappa={kappa:g}, p={p}; forward + adjoint",
    5: "overlap-type SPD matrix, 16384 atoms x 13 (n=212992), ~500 stored entries per column, kappa={kappa:g}, "
       "p={p}; forward + adjoint",
}

# library kernel (substring of its symbol) -> phase of submat_time_phases
KERNEL_PHASE = {"k_small": "small-jacobi", "k_gather_large": "gather", "k_tridiagonalise": "tridiagonalise",
                "k_tridiag_eig": "tridiagonal-eig", "k_eig_orth": "reorthogonalise",
                "k_back_prep": "back-transform", "k_back_apply": "back-transform",
                "k_apply_column": "apply-column", "k_column_factored": "apply-column",
                "k_adj_": "adjoint", "k_adjoint": "adjoint", "k_plan_pattern": "plan-reset"}
CSRC = os.path.join(ROOT, "paper_1710_10899_amd", "csrc")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def flops_model(m):
    """Algorithmic flops per column: forward (10/3)m^3 + 3m^2 (tridiagonal
    reduction 4/3, applying the reflectors to the eigenvectors of T 2, then
    f and the column), adjoint 3m^3 + 5m^2 (Q M and the symmetric product
    with Q^T)."""
    m = m.astype("float64")
    return float(((10.0 / 3.0) * m ** 3 + 3 * m ** 2).sum()), float((3.0 * m ** 3 + 5 * m ** 2).sum())


def phase_work(m, phase, elt=8, small_max=32):
    """Algorithmic work of a phase summed over one step's launches of it
    (all columns of its bucket): (amount, unit, bound). Flop counts are those
    of the benchmark model above; the reduction, the back-transformation and
    the adjoint are rated against the FP64 (or FP32) peak, which on this
    chip is the same for vector and matrix instructions. `elt` is the byte
    width of the pass (8 FP64, 4 FP32)."""
    big = m[m > small_max].astype("float64")
    small = m[m <= small_max].astype("float64")
    if phase == "tridiagonalise":
        return float((4.0 / 3.0) * (big ** 3).sum()), "flop", "mfma"
    if phase == "back-transform":
        return float(2.0 * (big ** 3).sum()), "flop", "mfma"
    if phase == "adjoint":
        return float(3.0 * (big ** 3).sum() + 5.0 * (big ** 2).sum()), "flop", "mfma"
    if phase == "gather":
        return float((4.0 + elt) * (big ** 2).sum()), "byte", "hbm"
    if phase == "apply-column":
        return float(3.0 * (big ** 2).sum()), "flop", "alu"
    if phase == "small-jacobi":
        return float(((10.0 / 3.0) * small ** 3 + 3 * small ** 2 + 3 * small ** 3 + 5 * small ** 2).sum()), \
            "flop", "alu"
    return None, None, None


def reduction_bytes(m, elt=8, small_max=32):
    """The reduction's compulsory stream: the lower triangle of the trailing
    matrix once per column, sum_k elt (m-k)^2 / 2 ~ (elt/6) m^3 bytes."""
    big = m[m > small_max].astype("float64")
    return float(elt / 6.0 * (big ** 3).sum())


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_source_hash() -> str:
    """sha256 over the HIP library's sources with comments and blank space
    removed: the counters in profiles/traffic_*.json stay valid across edits
    that cannot change a kernel."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1710_10899_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            text = open(os.path.join(csrc, f), encoding="utf-8").read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            text = " ".join(text.split())
            h.update(f.encode())
            h.update(text.encode())
    return h.hexdigest()


WORKLOAD_TAGS = {1: "banded_n1024", 2: "overlap_n6656", 3: "mixed_overlap_n53248", 4: "overlap_n13312",
                 5: "overlap_n212992"}


def traffic_file(workload: int, precision: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{WORKLOAD_TAGS[workload]}_{precision}.json")


def measured_counters(phase: str, workload: int, precision: str):
    """Per-launch figures of a phase's kernel from the committed counter
    summary of this workload: HBM bytes (FETCH + WRITE, calibrated) and
    executed flops (VALU FMA/ADD/MUL + MFMA ops), or None when absent or
    recorded for other kernel sources."""
    try:
        with open(traffic_file(workload, precision)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("phases", {}).get(phase)


def _phase_of(name: str):
    for k, ph in KERNEL_PHASE.items():
        if k in name:
            return ph + ("/f32" if ("<float" in name or "IfE" in name) else "")
    return None


def _read_counters(path, names, reduce="mean"):
    """{kernel: {counter: mean (or max) over dispatches of the per-dispatch
    sum}} from a rocprofv3 counter_collection.csv."""
    import csv
    import collections
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] in names:
                per[(r["Kernel_Name"], r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
    byk = collections.defaultdict(lambda: collections.defaultdict(list))
    for (k, _), d in per.items():
        for c, v in d.items():
            byk[k][c].append(v)
    if reduce == "max":
        return {k: {c: max(v) for c, v in d.items()} for k, d in byk.items()}
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in byk.items()}


def summarise_profile(d: str, command: str, workload: int, precision: str) -> None:
    """Turns one rocprofv3 kernel-trace run (kt_*) and the counter runs of
    this benchmark (fetch_*: FETCH_SIZE, write_*: WRITE_SIZE, dram_*:
    TCC_EA0_RDREQ_DRAM_sum + TCC_EA0_RDREQ_sum, flops_*: the FP64 or FP32
    VALU FMA/ADD/MUL and MFMA op counters; all --output-format csv), made
    with --copy-probe, into profiles/<workload>_fwd_adjoint_<precision>.md
    and the matching traffic_*.json. The 1 GiB probe copy calibrates the
    byte counters: scale = bytes moved / bytes the counter reports for it."""
    import csv

    from workloads import generators as G
    stats = {}
    with open(os.path.join(d, "kt_kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            stats[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]) / 1e6, float(r["Percentage"]))
    ctr, scale = {}, {}
    for tag, cname in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        path = os.path.join(d, f"{tag}_counter_collection.csv")
        byk = {k: v[cname] * 1024.0 for k, v in _read_counters(path, {cname}).items()}
        # the probe is the largest single dispatch outside the library (the
        # 1 GiB copy; other copies of the same kernel are the small inputs)
        peak = {k: v[cname] * 1024.0 for k, v in _read_counters(path, {cname}, "max").items()}
        probe = max((v for k, v in peak.items() if _phase_of(k) is None), default=0.0)
        scale[tag] = (1 << 30) / probe if probe > 0 else float("nan")
        ctr[tag] = {k: scale[tag] * v for k, v in byk.items()}
    dram, flops = {}, {}
    fp = "F64" if precision == "f64" else "F32"
    fnames = {f"SQ_INSTS_VALU_FMA_{fp}", f"SQ_INSTS_VALU_ADD_{fp}", f"SQ_INSTS_VALU_MUL_{fp}",
              f"SQ_INSTS_VALU_MFMA_MOPS_{fp}"}
    if os.path.exists(os.path.join(d, "dram_counter_collection.csv")):
        dram = _read_counters(os.path.join(d, "dram_counter_collection.csv"),
                              {"TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_RDREQ_sum"})
    if os.path.exists(os.path.join(d, "flops_counter_collection.csv")):
        for k, v in _read_counters(os.path.join(d, "flops_counter_collection.csv"), fnames).items():
            # VALU counts are wave instructions (64 lanes, an FMA is 2 flops);
            # MFMA ops are counted in units of 512
            flops[k] = 64.0 * (2.0 * v.get(f"SQ_INSTS_VALU_FMA_{fp}", 0.0) + v.get(f"SQ_INSTS_VALU_ADD_{fp}", 0.0)
                               + v.get(f"SQ_INSTS_VALU_MUL_{fp}", 0.0)) + 512.0 * v.get(f"SQ_INSTS_VALU_MFMA_MOPS_{fp}", 0.0)
    sha = kernel_source_hash()
    tag = WORKLOAD_TAGS[workload]
    phases = {}
    # the profiled commands take the workload's default condition number and p = 2
    name = WORKLOAD_NAMES[workload].format(kappa=G.DEFAULT_KAPPA.get(workload, 0.0), p=2).split(";")[0]
    lines = [f"# rocprofv3 summary: submatrix-method kernels, {tag} ({name}), "
             f"forward + adjoint, {precision}", "", "Commands (from the repository root, `cd /tmp && export "
             "TMPDIR=/tmp` first; the output directory is then passed to `python bench.py --summarise-profile DIR "
             f"--workload {workload} --precision {precision}`):", "", "```", command, "```", "",
             f"Counter calibration (1 GiB device copy): FETCH_SIZE x{scale['fetch']:.3f}, "
             f"WRITE_SIZE x{scale['write']:.3f}. Executed flops = 64 (2 FMA + ADD + MUL) + 512 MFMA_MOPS "
             f"({fp} counters, per dispatch). DRAM share = TCC_EA0_RDREQ_DRAM_sum / TCC_EA0_RDREQ_sum.",
             f"Kernel sources sha256 (comments and blank space removed): `{sha}`", "",
             "| kernel | phase | calls | avg ms | % time | HBM read GB/launch | HBM write GB/launch | GB/s | "
             "executed TFLOP/launch | executed TFLOP/s | DRAM share of L2 read misses |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, (calls, ms, pct) in sorted(stats.items(), key=lambda kv: -kv[1][2]):
        ph = _phase_of(name)
        fb, wb = ctr["fetch"].get(name), ctr["write"].get(name)
        fl = flops.get(name)
        dr = dram.get(name)
        share = (dr["TCC_EA0_RDREQ_DRAM_sum"] / dr["TCC_EA0_RDREQ_sum"]) if dr and dr.get("TCC_EA0_RDREQ_sum") else None
        short = name.split("(")[0].replace("void ", "")[:60]
        cells = [f"`{short}`", ph or "-", str(calls), f"{ms:.3f}", f"{pct:.2f}"]
        if fb is not None and wb is not None:
            cells += [f"{fb / 1e9:.2f}", f"{wb / 1e9:.2f}", f"{(fb + wb) / (ms / 1e3) / 1e9:.0f}"]
        else:
            cells += ["-", "-", "-"]
        cells += [f"{fl / 1e12:.4f}" if fl else "-", f"{fl / (ms / 1e3) / 1e12:.2f}" if fl else "-",
                  f"{share:.3f}" if share is not None else "-"]
        lines.append("| " + " | ".join(cells) + " |")
        want = "/f32" in (ph or "") if precision != "f64" else "/f32" not in (ph or "")
        if ph is not None and want and fb is not None and wb is not None:
            # a phase of several kernels (one launch each per pass) sums them
            key = ph.replace("/f32", "")
            if key in phases:
                e = phases[key]
                e["kernel"] += " + " + short
                e["avg_ms"] += ms
                e["fetch_bytes"] += fb
                e["write_bytes"] += wb
                e["executed_flop"] = (e["executed_flop"] or 0.0) + (fl or 0.0) if (e["executed_flop"] or fl) else None
                e["dram_share"] = None
            else:
                phases[key] = {"kernel": short, "avg_ms": ms, "fetch_bytes": fb, "write_bytes": wb,
                               "executed_flop": fl, "dram_share": share}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{tag}_fwd_adjoint_{precision}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(traffic_file(workload, precision), "w") as fh:
        json.dump({"source_sha256": sha, "command": command, "fetch_scale": scale["fetch"],
                   "write_scale": scale["write"], "phases": phases}, fh, indent=1)
    print("\n".join(lines))


# ------------------------------------------------------------- cpu baseline

_W = {}


def _pool_init(rowptr, colind, vals, wvals, p, fn):
    _W.update(rowptr=rowptr, colind=colind, vals=vals, wvals=wvals, p=p, fn=fn)


def _pool_work(cols):
    import oracle
    segs, _ = oracle.forward_columns(_W["rowptr"], _W["colind"], _W["vals"], _W["p"], cols, _W["fn"])
    oracle.adjoint(_W["rowptr"], _W["colind"], _W["vals"], len(_W["rowptr"]) - 1, _W["p"], _W["wvals"],
                   cols=cols, check=False, fn=_W["fn"])
    return segs


def cpu_baseline(csr, w, p, n_sample=None, fn="inv_root"):
    """The FP64 oracle (forward + adjoint per column) on a seeded sample of
    columns, one single-threaded-BLAS worker process per available host core
    (at most 16). Returns
    the line's cpu_baseline object and the oracle's forward segments of the
    sampled columns (for the accuracy check of the GPU output)."""
    import multiprocessing as mp

    import numpy as np
    # one worker per host core the process may run on, at most 16: a GPU's
    # share of the host on the machines this runs on
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(avail, 16))
    if n_sample is None:
        # about 10 s of wall time (~160 core-seconds): ~4900 columns at the
        # 6656-column workload's mean m^3 on 16 cores (about 32 ms per column
        # and core, measured), scaled by this workload's and the core count
        m3 = float((csr.row_sizes().astype(np.float64) ** 3).mean())
        n_sample = int(max(32, min(csr.n, 300 * cores * 6.9e7 / m3)))
    rng = np.random.default_rng(171010899 + 400)
    cols = np.sort(rng.choice(csr.n, min(n_sample, csr.n), replace=False))
    chunks = [cols[i::cores * 4].tolist() for i in range(cores * 4)]
    chunks = [c for c in chunks if c]
    saved_env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved_env:
        os.environ[k] = "1"
    segs = {}
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(cores, initializer=_pool_init, initargs=(csr.rowptr, csr.colind, csr.vals, w, p, fn)) as pool:
            pool.map(_pool_work, [[int(cols[0])]] * cores)  # workers up and warm
            t0 = time.perf_counter()
            for part in pool.map(_pool_work, chunks):
                segs.update(part)
            dt = time.perf_counter() - t0
    finally:
        for k, v in saved_env.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    done = len(segs)
    return {"value": done / dt, "unit": "submatrices/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "affinity_cpus": avail,
            "sample": f"{done} seeded columns of the same workload, forward + adjoint per column, "
                      f"{cores} processes with single-threaded BLAS, {dt:.2f} s wall"}, segs


def plain_path(sm, _lib, rp, ci, va, gx, fn, param, m, n_sample=96):
    """The per-column comparison path (FP64, one launch per kernel per
    column, no batching, no graph) on an order-stratified sample of the
    benchmark's own columns: every k-th column of each size bucket (buckets
    ordered by decreasing order). Both directions are warmed once, then
    timed; the rate is extrapolated to all columns by the flop model."""
    import numpy as np
    import torch
    n = m.size
    stride = max(1, n // n_sample)
    order = np.argsort(-m, kind="stable")
    edge = int(_lib.submat_get_option(_lib.SUBMAT_OPT_SMALL_MAX))  # the library's bucket edge
    small = order[m[order] <= edge]
    large = order[m[order] > edge]
    picked = np.concatenate([small[::stride], large[::stride]])
    _lib.submat_set_option(_lib.SUBMAT_OPT_PLAIN_STRIDE, stride)
    try:
        x = torch.empty_like(va)
        ga = torch.empty_like(va)
        sm.matfun_fwd(rp, ci, va, fn, param, "f64_plain", out=x)
        sm.matfun_bwd(rp, ci, va, gx, fn, param, "f64_plain", out=ga)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sm.matfun_fwd(rp, ci, va, fn, param, "f64_plain", out=x)
        sm.matfun_bwd(rp, ci, va, gx, fn, param, "f64_plain", out=ga)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        _lib.submat_set_option(_lib.SUBMAT_OPT_PLAIN_STRIDE, 1)
    f_all = sum(flops_model(m))
    f_smp = sum(flops_model(m[picked]))
    t_all = dt * f_all / f_smp
    return {"value": n / t_all, "unit": "submatrices/s", "sampled_columns": int(picked.size),
            "sample_seconds": dt, "extrapolated_seconds_per_step": t_all,
            "gflops_algorithmic": f_all / t_all / 1e9,
            "workload": f"every {stride}-th column of each size bucket of the same workload (m mean "
                        f"{m[picked].mean():.0f}), forward + adjoint, extrapolated to all {n} columns by the "
                        f"flop model"}, x, picked


# ----------------------------------------------------- consumer workloads


def spmv_roofline(rp, ci, vals, n, nnz, reps=200):
    """Average duration of the library's SpMV kernel (one launch per call,
    on torch's current stream, timed with HIP events around `reps`
    back-to-back calls) against HBM: algorithmic bytes per launch = values
    and column indices (12 nnz), row pointers (4 (n + 1)), x read once and
    y written (16 n)."""
    import torch

    import paper_1710_10899_amd as sm
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        sm.spmv(rp, ci, vals, x, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sm.spmv(rp, ci, vals, x, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 12.0 * nnz + 4.0 * (n + 1) + 16.0 * n
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"kernel": "k_spmv", "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": None, "launch_ms": ms,
            "bytes_per_launch": nbytes}


def run_residual(args):
    """||X^p A - I||_2 of the submatrix-method result on the named workload:
    one evaluation = the Lanczos iteration on R^T R in the library."""
    import torch

    import paper_1710_10899_amd as sm
    from workloads import generators as G
    csr = G.make_config(args.workload, kappa=args.kappa)
    rp = torch.from_numpy(csr.rowptr).cuda()
    ci = torch.from_numpy(csr.colind).cuda()
    va = torch.from_numpy(csr.vals).cuda()
    x = sm.invroot_fwd(rp, ci, va, args.p)
    for _ in range(args.warmup):
        norm, steps = sm.residual_norm(rp, ci, va, x, args.p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        norm, steps = sm.residual_norm(rp, ci, va, x, args.p)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    log(f"residual norm {norm:.6e} after {steps} Lanczos steps, {ms:.2f} ms")
    out = {"metric": "residual-norm evaluations/s (||X^p A - I||_2, Lanczos on R^T R)", "value": 1e3 / ms,
           "unit": "evaluations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": WORKLOAD_NAMES[args.workload].format(kappa=csr.meta.get("kappa_target", 0.0),
                                                                       p=args.p).replace("forward + adjoint",
                                                                                         "residual metric"),
                      "n": csr.n, "nnz": csr.nnz, "p": args.p, "lanczos_steps": steps, "residual_norm": norm},
           "roofline": spmv_roofline(rp, ci, va, csr.n, csr.nnz)}
    if not args.no_cpu_baseline:
        from oracle import krylov_oracle as ko
        xh = x.cpu().numpy()
        t0 = time.perf_counter()
        ref = ko.residual_norm_sparse(xh, csr.rowptr, csr.colind, csr.vals, csr.n, args.p)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "evaluations/s", "cores": 1, "kind": "oracle",
                               "sample": f"one evaluation on the same workload and X (ARPACK on the sparse "
                                         f"operator, scipy, {dt:.2f} s; value {ref:.6e})"}
    print(json.dumps(out), flush=True)


def run_pcg(args):
    """A x = b, b = ones, on an ill-conditioned overlap-type matrix of the
    paper's preconditioning range (384 atoms x 13 = 4992 unknowns, kappa
    1e5): plain CG and CG on K^T A K y = K^T b with K the submatrix-method
    A^(-1/2); tolerance 1e-6, at most 2 n iterations. One step = forming K
    and the preconditioned solve."""
    import numpy as np
    import torch

    import paper_1710_10899_amd as sm
    from workloads import generators as G
    csr = G.overlap_matrix(n_atoms=384, nbf=13, rcut=4.14, kappa=args.kappa or 1e5, seed=G.BASE_SEED + 60)
    rp = torch.from_numpy(csr.rowptr).cuda()
    ci = torch.from_numpy(csr.colind).cuda()
    va = torch.from_numpy(csr.vals).cuda()
    b = torch.ones(csr.n, dtype=torch.float64, device="cuda")
    k = torch.empty_like(va)

    def precond_solve():
        sm.invroot_fwd(rp, ci, va, 2, out=k)
        return sm.pcg(rp, ci, va, b, k, tol=1e-6)

    for _ in range(args.warmup):
        _, info = precond_solve()
        _, plain = sm.pcg(rp, ci, va, b, None, tol=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = precond_solve()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    _, plain = sm.pcg(rp, ci, va, b, None, tol=1e-6)
    torch.cuda.synchronize()
    ms_plain = 1e3 * (time.perf_counter() - t0)
    log(f"preconditioned: {info['iters']} iterations, {ms:.2f} ms incl. K; plain: {plain['iters']} iterations, "
        f"{ms_plain:.2f} ms")
    out = {"metric": "preconditioned CG solves/s (K = submatrix-method A^(-1/2) formed in every solve)",
           "value": 1e3 / ms, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"overlap-type SPD matrix, 384 atoms x 13 (n={csr.n}), kappa="
                                  f"{csr.meta.get('kappa_target', 0.0):g}, b = ones, tol 1e-6, max 2n iterations",
                      "n": csr.n, "nnz": csr.nnz,
                      "iterations_preconditioned": info["iters"], "iterations_plain": plain["iters"],
                      "relres_preconditioned": info["relres"], "true_relres_preconditioned": info["true_relres"],
                      "relres_plain": plain["relres"], "ms_plain_solve": ms_plain},
           "roofline": spmv_roofline(rp, ci, va, csr.n, csr.nnz)}
    if not args.no_cpu_baseline:
        from oracle import krylov_oracle as ko
        kh = k.cpu().numpy()
        t0 = time.perf_counter()
        _, it_o, _ = ko.cg(csr.rowptr, csr.colind, csr.vals, np.ones(csr.n), tol=1e-6, kvals=kh)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "sample": f"the preconditioned CG solve on the same system with the same K "
                                         f"(K formation excluded), scipy sparse products, {it_o} iterations, "
                                         f"{dt:.2f} s"}
    print(json.dumps(out), flush=True)


def run_error_study(args):
    """The error study of Section 4.1 on synthetic inputs: random sparse SPD
    matrices of density 0.05 (random symmetric pattern, N(0,1) values,
    diagonal shift to an exact condition number kappa), n = 256..4096, kappa = 2..1e3 for p = 1, and
    p = 2, 3 at kappa = 2; two seeds per point. For each matrix the library
    forms X and evaluates ||X^p A - I||_2. The oracle (dense residual of its
    own X) is run beside it on one seed of every point with n <= 1024."""
    import numpy as np
    import torch

    import oracle
    import paper_1710_10899_amd as sm
    from workloads import generators as G
    sizes = (256, 512, 1024, 2048, 4096)
    kappas = (2.0, 10.0, 100.0, 1000.0)
    seeds = (0, 1)
    rows, parity, t_gpu, t_cpu, cpu_n = [], [], 0.0, 0.0, 0
    for n in sizes:
        for kappa in kappas:
            for sd in seeds:
                csr = G.random_sparse_spd(n, 0.05, seed=G.BASE_SEED + 700 + 10 * sd + n + int(kappa), kappa=kappa)
                rp = torch.from_numpy(csr.rowptr).cuda()
                ci = torch.from_numpy(csr.colind).cuda()
                va = torch.from_numpy(csr.vals).cuda()
                for p in ((1, 2, 3) if kappa == 2.0 else (1,)):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    x = sm.invroot_fwd(rp, ci, va, p)
                    norm, steps = sm.residual_norm(rp, ci, va, x, p)
                    torch.cuda.synchronize()
                    t_gpu += time.perf_counter() - t0
                    rows.append({"n": n, "kappa": kappa, "p": p, "seed": sd, "density": csr.nnz / n / n,
                                 "m_max": int(csr.row_sizes().max()), "residual": norm, "lanczos_steps": steps})
                    if sd == 0 and n <= 1024:
                        t0 = time.perf_counter()
                        xo, _ = oracle.forward(csr.rowptr, csr.colind, csr.vals, n, p, check=False)
                        ref = oracle.residual_norm(xo, csr.rowptr, csr.colind, csr.vals, n, p)
                        t_cpu += time.perf_counter() - t0
                        cpu_n += 1
                        parity.append(abs(norm - ref) / ref)
                log(f"n={n} kappa={kappa:g} seed={sd}: " + ", ".join(
                    f"p={r['p']} {r['residual']:.3e}" for r in rows if r["n"] == n and r["kappa"] == kappa
                    and r["seed"] == sd))
    table = {}
    for r in rows:
        table.setdefault(f"p={r['p']} kappa={r['kappa']:g}", {}).setdefault(str(r["n"]), []).append(r["residual"])
    summary = {k: {n_: float(np.mean(v)) for n_, v in d.items()} for k, d in table.items()}
    out = {"metric": "matrices/s through X and ||X^p A - I||_2 (error study, Section 4.1)",
           "value": len(rows) / t_gpu, "unit": "matrices/s", "n_gpus": 1, "steps": len(rows), "warmup": 0,
           "ms_per_step": 1e3 * t_gpu / len(rows), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "random sparse SPD, density 0.05, N(0,1) values shifted to an exact kappa, "
                                  "n 256-4096, kappa 2-1e3, p 1 (and 2, 3 at kappa 2), 2 seeds",
                      "mean_residual": summary,
                      "max_rel_diff_vs_oracle": float(max(parity)) if parity else None,
                      "oracle_cases": len(parity)},
           "rows": rows}
    out["cpu_baseline"] = {"value": cpu_n / t_cpu if t_cpu else None, "unit": "matrices/s", "cores": 1,
                           "kind": "oracle", "sample": f"{cpu_n} matrices with n <= 1024 (oracle X and dense "
                                                      f"residual), {t_cpu:.1f} s"}
    print(json.dumps(out), flush=True)


def run_refine(args):
    """Refinement of the submatrix-method inverse (p = 1) on the named
    workload by Newton-Schulz to ||I - A X||_F / sqrt(n) <= 1e-14; one step
    = the seed's densification plus all refinement steps. The dominant
    kernel is the FP64 DGEMM (2 n^3 flops per product, two per step)."""
    import numpy as np
    import torch

    import paper_1710_10899_amd as sm
    from workloads import generators as G
    csr = G.make_config(args.workload, kappa=args.kappa)
    n = csr.n
    rp = torch.from_numpy(csr.rowptr).cuda()
    ci = torch.from_numpy(csr.colind).cuda()
    va = torch.from_numpy(csr.vals).cuda()
    x = sm.invroot_fwd(rp, ci, va, 1)
    X = torch.empty((n, n), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        _, info = sm.refine_inverse(rp, ci, va, x, tol=1e-14, out=X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = sm.refine_inverse(rp, ci, va, x, tol=1e-14, out=X)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    # one Newton-Schulz step (two DGEMMs, a copy, the residual) as the
    # difference of 5 fixed steps and none, timed with HIP events on the
    # library's stream (torch's current stream)
    def timed(k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sm.refine_inverse(rp, ci, va, x, max_iter=k, tol=0.0, out=X)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)
    timed(1)
    step_ms = (timed(5) - timed(0)) / 5
    gemm_ms = step_ms / 2
    tf = 4.0 * n ** 3 / (step_ms / 1e3) / 1e12
    log(f"refinement: {info['iters']} steps to {info['residual']:.2e} in {ms:.1f} ms; one step {step_ms:.2f} ms "
        f"({tf:.1f} TFLOP/s)")
    out = {"metric": "refinements/s (Newton-Schulz on the p = 1 result to ||I - A X||_F / sqrt(n) <= 1e-14)",
           "value": 1e3 / ms, "unit": "refinements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": WORKLOAD_NAMES[args.workload].format(kappa=csr.meta.get("kappa_target", 0.0),
                                                                       p=1).replace("forward + adjoint",
                                                                                    "dense refinement"),
                      "n": n, "newton_schulz_steps": info["iters"], "final_residual": info["residual"],
                      "flops_per_step": 4.0 * n ** 3},
           "roofline": {"kernel": "Newton-Schulz step (two rocBLAS DGEMMs, n x n x n)", "bound": "mfma",
                        "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS,
                        "traffic": None, "launch_ms": gemm_ms}}
    if not args.no_cpu_baseline:
        import threadpoolctl  # noqa: F401  (reports the BLAS thread count)
        from oracle import krylov_oracle as ko
        xh = x.cpu().numpy()
        t0 = time.perf_counter()
        ko.refine_inverse(csr.rowptr, csr.colind, csr.vals, xh, tol=0.0, maxit=1)
        dt = time.perf_counter() - t0
        info_t = threadpoolctl.threadpool_info()
        cores = max((d.get("num_threads", 1) for d in info_t), default=1)
        out["cpu_baseline"] = {"value": 1.0 / (dt * max(info["iters"], 1)), "unit": "refinements/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"one Newton-Schulz step of the oracle (numpy, two dense products) on the "
                                         f"same workload, {dt:.1f} s, scaled to the GPU's {info['iters']} steps"}
    print(json.dumps(out), flush=True)


# --------------------------------------------------------------------- main


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32_mixed"])
    ap.add_argument("--p", type=int, default=2, help="root order of the inverse root / root functions")
    ap.add_argument("--fn", default="inv_root", choices=["inv_root", "root", "power"],
                    help="spectral function: lambda^(-1/p), lambda^(1/p) or lambda^alpha")
    ap.add_argument("--alpha", type=float, default=0.7, help="exponent of --fn power")
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 5],
                    help="named synthetic workload (2 = the 6656-column overlap matrix the metric is quoted on)")
    ap.add_argument("--kappa", type=float, default=None, help="condition number of the workload (its default if unset)")
    ap.add_argument("--mode", default="step", choices=["step", "residual", "pcg", "error-study", "refine"],
                    help="step: forward + adjoint (the headline); residual: the residual metric ||X^p A - I||_2; "
                         "pcg: CG on A x = b with and without the submatrix-method preconditioner; "
                         "error-study: the residual against n and kappa on random sparse SPD matrices; "
                         "refine: Newton-Schulz refinement of the p = 1 result")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-phases", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device-to-device copy first (calibrates HBM byte counters)")
    ap.add_argument("--summarise-profile", metavar="DIR",
                    help="summarise rocprofv3 csv output of this benchmark into profiles/ and exit")
    ap.add_argument("--profile-command", default="", help="command line recorded with --summarise-profile")
    args = ap.parse_args()
    if args.summarise_profile:
        summarise_profile(args.summarise_profile, args.profile_command, args.workload, args.precision)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                          "(sharding the columns over several GPUs is not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1710_10899_amd as sm
    from paper_1710_10899_amd import _lib
    from workloads import generators as G

    _lib.load()
    torch.cuda.set_device(0)
    if args.mode == "residual":
        run_residual(args)
        return
    if args.mode == "pcg":
        run_pcg(args)
        return
    if args.mode == "error-study":
        run_error_study(args)
        return
    if args.mode == "refine":
        run_refine(args)
        return
    run_step(args, np, torch, sm, _lib, G)


def run_step(args, np, torch, sm, _lib, G):
    """The headline: one step = forward + adjoint over every column of the
    workload, inputs resident in HBM, eigenvectors kept between the two
    calls when they fit a saved buffer (else the adjoint recomputes them)."""
    t0 = time.perf_counter()
    csr = G.make_config(args.workload, kappa=args.kappa)
    w = G.upstream_gradient(csr, G.BASE_SEED + args.workload + 100)
    log(f"workload n={csr.n} nnz={csr.nnz} m={csr.row_sizes().min()}..{csr.row_sizes().max()} "
        f"generated in {time.perf_counter() - t0:.1f}s")
    m = csr.row_sizes()
    rp = torch.from_numpy(csr.rowptr).cuda()
    ci = torch.from_numpy(csr.colind).cuda()
    dt = torch.float64
    va = torch.from_numpy(csr.vals).to(dt).cuda()
    gx = torch.from_numpy(w).to(dt).cuda()
    x = torch.empty_like(va)
    ga = torch.empty_like(va)
    prec = args.precision
    nb = sm.saved_bytes(rp, ci, dt, prec)
    free_b, _ = torch.cuda.mem_get_info()
    if nb <= 0.4 * free_b:
        saved = torch.empty(max(nb, 8), dtype=torch.uint8, device="cuda")
        log(f"saved eigenvector buffer {nb / 2**30:.2f} GiB")
    else:
        saved = None
        log(f"saved eigenvectors would need {nb / 2**30:.1f} GiB: the adjoint recomputes them")
    fn = args.fn
    param = args.alpha if fn == "power" else args.p
    fn_name = {"inv_root": f"p={args.p}", "root": f"f=lambda^(1/{args.p})",
               "power": f"f=lambda^{args.alpha:g}"}[fn]

    def step():
        sm.matfun_fwd(rp, ci, va, fn, param, prec, saved, out=x)
        sm.matfun_bwd(rp, ci, va, gx, fn, param, prec, saved, out=ga)

    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 1 GiB read + 1 GiB written")

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i} done")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    st = sm.query_status()
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step; status {st}")
    value = csr.n / (ms_per_step / 1e3)
    f_fwd, f_bwd = flops_model(m)
    gflops = (f_fwd + f_bwd) / (ms_per_step / 1e3) / 1e9
    peak_tf = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    elt = 8 if prec == "f64" else 4

    out = {
        "metric": "submatrices/s + GFLOP/s (% FP64/FP32 peak), fwd+adjoint vs plain FP64 path",
        "value": value,
        "unit": "submatrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "f64" else "f32+f64-fallback",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[args.workload].format(kappa=csr.meta.get("kappa_target", 0.0),
                                                                    p=args.p).replace(f"p={args.p}", fn_name),
                   "n": csr.n, "nnz": csr.nnz, "function": fn, "param": param, "precision": prec,
                   "eigenvectors": "kept between forward and adjoint" if saved is not None else "recomputed",
                   "m_min": int(m.min()), "m_mean": float(m.mean()), "m_max": int(m.max()),
                   "parallelism": "single GPU"},
        "gflops_algorithmic": gflops,
        "frac_of_peak": gflops / (peak_tf * 1e3),
        "status": st,
    }

    edge = int(_lib.submat_get_option(_lib.SUBMAT_OPT_SMALL_MAX))  # one-wavefront bucket edge
    if not args.no_phases:
        # per-phase device time of one forward + adjoint (direct launches,
        # HIP events on the library's stream = torch's current stream)
        ph_f = sm.time_phases(rp, ci, va, param, prec, fn=fn)
        ph = sm.time_phases(rp, ci, va, param, prec, grad_x=gx, fn=fn)
        counters = _lib.submat_query_counters(torch.cuda.current_stream().cuda_stream, 4)
        table = {}
        for k, (ms, nl) in ph.items():
            if not nl:
                continue
            amount, unit, bound = phase_work(m, k, elt, edge)
            row = {"ms_per_launch": round(ms / nl, 3), "launches": nl, "ms_total": round(ms, 3)}
            if amount is not None:
                # passes over the columns: the forward's, plus the adjoint's
                # when it recomputes the eigendecomposition (launches beyond
                # those of the forward alone)
                nf = ph_f[k][1]
                reps = (1 if nf else 0) + (1 if nl > nf else 0)
                rate = reps * amount / (ms / 1e3)
                row["achieved"] = rate / (1e9 if unit == "byte" else 1e12)
                row["unit"] = "GB/s" if unit == "byte" else "TFLOP/s"
                row["bound"] = bound
            table[k] = row
        out["phases"] = table
        dom = max((k for k in table if k != "plan-reset"), key=lambda k: table[k]["ms_total"])
        d = table[dom]
        meas = measured_counters(dom, args.workload, prec)
        if d.get("unit") == "TFLOP/s":
            peak = peak_tf if d["bound"] == "mfma" else (FP64_VALU_PEAK if prec == "f64" else FP32_VALU_PEAK)
            out["roofline"] = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": peak,
                               "unit": "TFLOP/s", "frac": d["achieved"] / peak,
                               "traffic": meas["fetch_bytes"] + meas["write_bytes"] if meas else None,
                               "launch_ms": d["ms_per_launch"],
                               "executed_tflop_per_launch": (meas["executed_flop"] / 1e12
                                                             if meas and meas.get("executed_flop") else None)}
            if dom == "tridiagonalise":
                gb = d["achieved"] * 1e12 * reduction_bytes(m, elt, edge) / phase_work(m, dom, elt, edge)[0] / 1e9
                out["roofline"]["bytes_view"] = {"achieved": gb, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                                 "frac": gb / HBM_PEAK_GBS,
                                                 "note": "lower triangle of the trailing matrix streamed once "
                                                         "per column"}
        else:
            out["roofline"] = {"kernel": dom, "bound": d.get("bound", "latency"), "achieved": d.get("achieved"),
                               "peak": HBM_PEAK_GBS if d.get("unit") == "GB/s" else None, "unit": d.get("unit"),
                               "frac": d["achieved"] / HBM_PEAK_GBS if d.get("unit") == "GB/s" else None,
                               "traffic": meas["fetch_bytes"] + meas["write_bytes"] if meas else None,
                               "launch_ms": d["ms_per_launch"]}
        out["inverse_iteration_vectors"] = counters[3]
        log(f"phases {table}")

    if not args.no_plain:
        pl, xp, picked = plain_path(sm, _lib, rp, ci, va, gx, fn, param, m)
        pl["speedup_batched_vs_plain"] = value / pl["value"]
        xs = x.cpu().numpy()
        xps = xp.cpu().numpy()
        idx = np.concatenate([np.arange(csr.rowptr[j], csr.rowptr[j + 1]) for j in picked])
        pl["rel_fro_vs_batched"] = float(np.linalg.norm(xps[idx] - xs[idx]) / np.linalg.norm(xs[idx]))
        out["plain_f64_path"] = pl
        log(f"plain path {pl['value']:.1f} submatrices/s (extrapolated from {pl['sampled_columns']} columns)")

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb, segs = cpu_baseline(csr, w, param, fn=fn)
        out["cpu_baseline"] = cb
        xs = x.double().cpu().numpy()
        cols = sorted(segs)
        got = np.concatenate([xs[csr.rowptr[j]:csr.rowptr[j + 1]] for j in cols])
        ref = np.concatenate([segs[j] for j in cols])
        out["accuracy"] = {"rel_fro_forward_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                           "max_column_rel_err": float(max(
                               np.linalg.norm(xs[csr.rowptr[j]:csr.rowptr[j + 1]] - segs[j]) / np.linalg.norm(segs[j])
                               for j in cols)),
                           "columns": len(cols),
                           "note": "the GPU forward of the last timed step against the oracle on the "
                                   "cpu_baseline sample"}
        log(f"cpu baseline {cb['value']:.1f} submatrices/s; forward rel err vs oracle "
            f"{out['accuracy']['rel_fro_forward_vs_oracle']:.2e}")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
