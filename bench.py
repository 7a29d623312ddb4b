"""Throughput of the p-multigrid solve phase on one MI355X.

A step is one FP64 V-cycle of the p-multigrid method with the ILUT smoother
(residual SpMVs, forward and backward ILUT substitutions, lumped L2
restriction, two h-multigrid V-cycles at p = 1, lumped L2 prolongation, and
the residual-norm stopping test read back to the host), on the default
workload: 2-D Poisson on the unit square, B-splines of degree p = 5 on a
uniform mesh h = 1/1024 (1,054,729 interior unknowns), ILUT(1e-12, 1).
Inputs are synthetic (manufactured solution sin(pi x) sin(pi y)) and are
resident in HBM when the timed region starts; host setup (assembly, ILUT,
upload) is timed separately and excluded.

Prints one JSON line: value = unknowns x V-cycles / second (whole job), a
roofline entry for the dominant kernel measured with HIP events during the
timed steps, and the FP64 CPU oracle timed on a bounded sample of the same
workload on this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "V-cycle DOF·iter/s + HBM GB/s frac; served solves/s, p50/p99 latency vs plain"

# kernel class -> (kernel name in the rocprofv3 trace, info field of its bytes per launch)
KERNELS = {
    "residual": ("csr_kernel<double, 32, 0>", "bytes_spmv"),
    "lower": ("trisolve_lower<double>", "bytes_trisolve_l"),
    "upper": ("trisolve_upper<double>", "bytes_trisolve_u"),
    "restrict": ("csr_kernel<double, 32, 2>", "bytes_restrict"),
    "prolong": ("csr_kernel<double, 32, 3>", "bytes_prolong"),
}


def _kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "pmg_device.hip"):
        h.update(open(os.path.join(ROOT, "paper_1901_01685_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel_class, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != _kernel_source_hash() or d.get("workload") != workload:
        return None
    k = d.get("kernels", {}).get(kernel_class)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(p, nel_full, n_full, budget_s=20.0):
    """The FP64 oracle as it stands, single-threaded, on a bounded sample of
    the workload: the same problem family (2-D unit square, same p) at
    h = 1/nel_s, V-cycles repeated for about budget_s seconds; reported in
    unknowns x V-cycles / second."""
    import numpy as np
    import oracle
    nel_s = 128
    t0 = time.perf_counter()
    o = oracle.Oracle(2, p, nel_s)
    t_setup = time.perf_counter() - t0
    b = o.f()
    x = np.zeros(o.n)
    r = o.residual(b, x)
    cycles = 0
    t0 = time.perf_counter()
    while True:
        x, r = o.vcycle(b, x, r)
        cycles += 1
        el = time.perf_counter() - t0
        if el >= budget_s or cycles >= 5000:
            break
    o.close()
    return {
        "value": o.n * cycles / el,
        "unit": "DOF*iter/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle V-cycles on the same 2-D unit-square p={p} problem at h=1/{nel_s} "
                   f"(n={o.n}; the timed workload is h=1/{nel_full}, n={n_full}): {cycles} cycles in "
                   f"{el:.1f} s, setup {t_setup:.1f} s excluded; single-threaded C, FP64"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--degree", type=int, default=5)
    ap.add_argument("--nel", type=int, default=1024)
    ap.add_argument("--dim", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 512 MiB (3 times), the reference for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solve phase here runs on a single MI355X; "
              "multi-GPU sharding is a design note only (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1901_01685_amd as pmg

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 26, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                          "launches": 3}))
        return
    t0 = time.perf_counter()
    s = pmg.Solver(dim=args.dim, degree=args.degree, n_elem=args.nel, device=0)
    t_setup = time.perf_counter() - t0
    info = s.info
    n = s.n
    print(f"# setup {t_setup:.1f} s (assembly {info.t_assembly:.1f}, ILUT {info.t_ilut:.1f}, "
          f"upload {info.t_upload:.1f}); n={n} nnz(A)={info.nnz_a} nnz(L)={info.nnz_l} nnz(U)={info.nnz_u}",
          file=sys.stderr, flush=True)
    b = torch.empty(n, dtype=torch.float64, device=dev)
    s.rhs(b)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    r = torch.empty(n, dtype=torch.float64, device=dev)
    r0 = s.residual(b, x, r, norm=True)
    for _ in range(args.warmup):
        s.vcycle(b, x, r, norm=True)
    torch.cuda.synchronize()
    print(f"# warmup done, relres {s.residual(b, x, r, norm=True) / r0:.3e}", file=sys.stderr, flush=True)

    # timed region: K V-cycles, each ending with the stopping-test norm on the host
    x.zero_()
    s.residual(b, x, r, norm=True)
    s.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rel = 1.0
    for _ in range(args.steps):
        rel = s.vcycle(b, x, r, norm=True) / r0
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile_enable(False)
    ms_step = 1e3 * el / args.steps
    value = n * args.steps / el

    # dominant kernel by total time per V-cycle
    per_class = {c: (ms, cnt) for c, (ms, cnt) in prof.items() if cnt > 0}
    dom = max((c for c in per_class if c in KERNELS), key=lambda c: per_class[c][0])
    ms_tot, cnt = per_class[dom]
    avg_s = ms_tot / cnt / 1e3
    nbytes = getattr(info, KERNELS[dom][1])
    achieved = nbytes / avg_s / 1e9
    workload = f"2d-unit-square-p{args.degree}-h1/{args.nel}" if args.dim == 2 else \
        f"3d-unit-cube-p{args.degree}-h1/{args.nel}"
    roofline = {
        "bound": "hbm",
        "kernel": KERNELS[dom][0],
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": _traffic(dom, workload),
        "avg_launch_ms": round(1e3 * avg_s, 4),
        "bytes_per_launch": int(nbytes),
        "per_step_ms": {c: round(v[0] / args.steps, 4) for c, v in per_class.items()},
        "vcycle_bytes": int(info.bytes_vcycle),
        "vcycle_GBps": round(info.bytes_vcycle / (ms_step / 1e3) / 1e9, 1),
        "dag_levels": [int(info.dag_levels_l), int(info.dag_levels_u)],
    }
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "dim": args.dim, "degree": args.degree, "n_elem": args.nel,
                   "unknowns": n, "precision": "fp64", "ilut": [1e-12, 1.0], "final_relres": rel,
                   "setup_s": round(t_setup, 1), "parallelism": "1 GPU"},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.degree, args.nel, n, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
