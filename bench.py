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

Prints one JSON line: value = unknowns x V-cycles / second (whole job; each
V-cycle replayed from its cached HIP graph), a roofline entry for the dominant
kernel whose launch durations are measured with HIP events on the launch
stream over a second timed run of the same V-cycles (kernel by kernel, as
event profiling requires), and the FP64 CPU oracle timed on a bounded sample
of the same workload on this host's cores.
"""
import argparse
import subprocess
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
def kernel_map(info, dim, degree):
    """Each kernel follows the layout the library reports for its operator:
    Kronecker factors on the box, the stencil layout, or CSR."""
    kron_a = info.residual_layout == 2
    stencil_a = info.residual_layout == 1
    rb = info.resid_rows  # rows per thread, the residual kernels' last template argument

    def transfer(add, cls):
        if info.transfer_layout == 2:
            # the 1-D factor has W = p + 2 entries per row; held in registers up to 8
            return f"kron_xgrid<double, {dim}, {add}, {8 if degree + 2 <= 8 else 0}>"
        if info.transfer_layout == 1:
            return f"xgrid_spmv<double, {dim}, {add}>"
        return f"csr_kernel<double, G, {cls}>"
    return {
        # the stencil kernel is instantiated per stencil width up to 11 (degree 5)
        "residual": (f"kron_resid<double, {dim}, false, {2 * degree + 1}, {rb}>" if kron_a
                     else (f"stencil_resid<double, {dim}, false, {2 * degree + 1}, {rb}>" if degree <= 5
                           else f"stencil_resid<double, {dim}, false, 0, {rb}>") if stencil_a
                     else "csr_kernel<double, G, 0>", "bytes_spmv"),
        "lower": ("trisolve_lower<double>", "bytes_trisolve_l"),
        "upper": ("trisolve_upper<double>", "bytes_trisolve_u"),
        "restrict": (transfer("false", 2), "bytes_restrict"),
        "prolong": (transfer("true", 3), "bytes_prolong"),
    }


def _kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "tri_layout.hpp", "grid_layout.hpp", "pmg_device.hip"):
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
    if d.get("kernel_source_hash") != _kernel_source_hash():
        return None
    k = d.get("workloads", {}).get(workload, {}).get("kernels", {}).get(kernel_class)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(p, nel_full, n_full, budget_s=20.0, pde=0, nel_s=256, dim=2):
    """The FP64 oracle as it stands, single-threaded, on a bounded sample of
    the workload: the same problem family (unit square or cube, same p) at
    h = 1/nel_s, V-cycles repeated for about budget_s seconds; reported in
    unknowns x V-cycles / second."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    o = oracle.Oracle(dim, p, nel_s, pde=pde)
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
    model, ncpu = host_cpu()
    return {
        "value": o.n * cycles / el,
        "unit": "DOF*iter/s",
        "cores": 1,
        "kind": "oracle",
        "host": {"cpu_model": model, "nproc": ncpu},
        "sample": (f"oracle V-cycles on the same {'2-D unit-square' if dim == 2 else '3-D unit-cube'} "
                   f"{'CDR ' if pde else ''}p={p} problem at h=1/{nel_s} "
                   f"(n={o.n}; the timed workload is h=1/{nel_full}, n={n_full}): {cycles} cycles in "
                   f"{el:.1f} s, setup {t_setup:.1f} s excluded; single-threaded C, FP64, in a process of its "
                   f"own beside the GPU legs"),
    }


def host_cpu():
    """CPU model and logical cores of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy of nbytes (read + write counted), timed with
    events on the copy's stream: the attainable HBM bandwidth beside the
    8 TB/s peak."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    gbs = 2 * nbytes / t / 1e9
    return {"GBps": round(gbs, 1), "bytes_per_copy": 2 * nbytes, "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def mixed_config4(pmg, torch, dev, reps=3):
    """Benchmark 1 (quarter annulus, radii 1 and 2) at p = 5, h = 1/512:
    FP32 V-cycles inside FP64 defect correction against plain FP64 V-cycles,
    both from x = 0 to a 1e-10 relative FP64 residual, on the same operators
    (one handle holding both precisions).  Reports ms per solve (median of
    reps after one untimed solve), solves/s, outer steps, the final FP64
    relative residual, and the mixed solution's relative difference from the
    FP64 one."""
    import numpy as np
    t0 = time.perf_counter()
    s = pmg.Solver(2, 5, 512, geometry=pmg.GEOM_QUARTER_ANNULUS, rhs_kind=pmg.RHS_ANNULUS,
                   precision=pmg.FP32_IN_FP64, device=0)
    t_setup = time.perf_counter() - t0
    b = torch.empty(s.n, dtype=torch.float64, device=dev)
    s.rhs(b)
    res, xs = {}, {}
    for name, prec in (("mixed", pmg.FP32_IN_FP64), ("fp64", pmg.FP64)):
        s.set_precision(prec)
        x = torch.zeros(s.n, dtype=torch.float64, device=dev)
        s.solve(b, x, tol=1e-10)
        times = []
        for _ in range(reps):
            x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, it, rel, *_ = s.solve(b, x, tol=1e-10)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
        ms = 1e3 * float(np.median(times))
        res[name] = {"status": int(st), "outer_steps": int(it), "relres_fp64": float(rel), "ms": round(ms, 3),
                     "solves_per_s": round(1e3 / ms, 2)}
        xs[name] = x.clone()
    diff = float(torch.linalg.vector_norm(xs["mixed"] - xs["fp64"]) / torch.linalg.vector_norm(xs["fp64"]))
    out = {"workload": "2d-quarter-annulus-p5-h1/512", "unknowns": s.n, "tol": 1e-10,
           "setup_s": round(t_setup, 1), **res, "mixed_vs_fp64_rel_diff": diff,
           "speedup_mixed_over_fp64": round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)}
    s.close()
    return out


def class_setup_cost(dim, p, nel):
    """Work of a class's ILUT, n * M^2 (M the rule-2 limit), which dominates
    its setup: 3.2e10 for the cube at p = 3, h = 1/64 (51 s with the device
    ILUT), 3.3e10 for the cube at p = 2, h = 1/128 (187 s)."""
    n1d = nel + p - 2
    return n1d ** dim * ((2 * p + 1) ** dim) ** 2


def serve_leg(args, sample_cost=None):
    """Continuous-batching server on the serving workload: a seeded stream of
    2-D/3-D unit-square/cube Poisson solves, p uniform in {2..5}, h uniform in
    {1/32, 1/64, 1/128, 1/256}, manufactured right-hand sides with integer
    frequencies 1..4 per axis, Poisson arrivals (mean 200 requests/s), FP32
    V-cycles inside FP64 defect correction to a 1e-10 relative residual.  The
    server's budget is 70 % of the device memory with its default class limit
    (a quarter of it), which rejects exactly the classes that cannot fit
    (3-D n_el = 256, and n_el = 128 at p >= 4).  Classes are set up before the
    stream (setup time reported, not in the latencies).  With sample_cost,
    only requests of classes whose host setup work (class_setup_cost) is at
    most that are submitted, so the setup stays bounded; the others are
    counted as outside the sample.  Compared with plain FP64 single solves (one
    at a time, FP64 V-cycles) and mixed-precision single solves on the same
    requests."""
    import numpy as np
    import paper_1901_01685_amd as pmg

    rng = np.random.default_rng(args.seed)
    n_warm, n_timed = args.serve_warmup, args.serve_requests
    total = n_warm + n_timed
    dims = rng.choice([2, 3], size=total)
    degs = rng.integers(2, 6, size=total)
    nels = rng.choice([32, 64, 128, 256], size=total)
    freqs = rng.integers(1, 5, size=(total, 3))
    gaps = rng.exponential(1.0 / args.rate, size=total)
    arrivals = np.cumsum(gaps)
    srv = pmg.Server(max_slots=args.slots, precision=pmg.FP32_IN_FP64, tol=1e-10,
                     tri_waves_per_cu=args.serve_tri_waves)
    opts = srv.effective_options()
    all_classes = sorted(set(zip(dims.tolist(), degs.tolist(), nels.tolist())))
    in_sample = {c for c in all_classes if sample_cost is None or class_setup_cost(*c) <= sample_cost}
    t0 = time.perf_counter()
    admitted, rejected_classes = set(), []
    for c in all_classes:
        if c not in in_sample:
            continue
        print(f"# class {c}: setting up", file=sys.stderr, flush=True)
        st = srv.prepare(*c)
        if st == pmg.OK:
            admitted.add(c)
        else:
            rejected_classes.append(c)
        print(f"# class {c}: {'ready' if st == pmg.OK else 'rejected (%d)' % st}", file=sys.stderr, flush=True)
    t_setup = time.perf_counter() - t0

    # open loop at the arrival rate
    clock0 = srv.clock()
    tickets = []
    rejected = outside = 0
    for i in range(total):
        c = (int(dims[i]), int(degs[i]), int(nels[i]))
        if c not in in_sample:
            outside += i >= n_warm
            continue
        target = clock0 + arrivals[i]
        while srv.clock() < target:
            time.sleep(max(0.0, min(0.001, target - srv.clock())))
        st, t = srv.submit(*c, freq=tuple(int(v) for v in freqs[i]))
        if st != pmg.OK:
            rejected += i >= n_warm
            continue
        tickets.append((i, t))
    lat, outer, fails, fin, sub = [], [], 0, [], []
    for i, t in tickets:
        st, info, _ = srv.wait(t, want_x=False)
        if i < n_warm:
            continue
        if st != pmg.OK:
            fails += 1
            continue
        lat.append(info["t_finish"] - info["t_submit"])
        outer.append(info["iterations"])
        fin.append(info["t_finish"])
        sub.append(info["t_submit"])
    lat = np.array(lat)
    open_loop = {
        "rate_req_s": args.rate, "requests": n_timed, "submitted": n_timed - outside, "outside_sample": outside,
        "completed": len(lat), "rejected_budget": rejected, "failed": fails,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3), "solves_per_s": len(lat) / (max(fin) - min(sub)),
        "mean_outer_steps": float(np.mean(outer)),
    }

    # the same admitted requests, all submitted at once (saturating load)
    idx = [i for i in range(n_warm, total) if (int(dims[i]), int(degs[i]), int(nels[i])) in admitted]
    idx = idx[: args.closed_requests]

    def run_batch(slots, precision, sequential):
        srv.configure(slots, precision)
        t0 = time.perf_counter()
        if sequential:
            for i in idx:
                st, t = srv.submit(int(dims[i]), int(degs[i]), int(nels[i]), freq=tuple(int(v) for v in freqs[i]))
                st, info, _ = srv.wait(t, want_x=False)
                assert st == pmg.OK and info["relres"] <= 1e-10
        else:
            ts = []
            for i in idx:
                st, t = srv.submit(int(dims[i]), int(degs[i]), int(nels[i]), freq=tuple(int(v) for v in freqs[i]))
                ts.append(t)
            for t in ts:
                st, info, _ = srv.wait(t, want_x=False)
                assert st == pmg.OK and info["relres"] <= 1e-10
        return len(idx) / (time.perf_counter() - t0)

    served = run_batch(args.slots, pmg.FP32_IN_FP64, False)
    plain64 = run_batch(1, pmg.FP64, True)
    mixed1 = run_batch(1, pmg.FP32_IN_FP64, True)
    stats = srv.stats()
    srv.close()
    return {
        "workload": "serving: 2-D/3-D unit square/cube, p in 2..5, h in 1/32..1/256, freq 1..4, Poisson arrivals",
        "seed": args.seed, "slots": args.slots, "tol": 1e-10, "tri_waves_per_cu": args.serve_tri_waves,
        "budget_GB": round(opts.budget_bytes / 1e9, 1), "class_limit_GB": round(opts.max_class_bytes / 1e9, 1),
        "sample": (None if sample_cost is None else
                   f"classes whose ILUT work n*M^2 <= {sample_cost:.3g} (setup bounded for this run): "
                   f"{len(in_sample)} of {len(all_classes)}"),
        "classes_admitted": len(admitted), "classes_rejected": [list(c) for c in rejected_classes],
        "setup_s": round(t_setup, 1),
        "open_loop": open_loop,
        "closed_loop_requests": len(idx),
        "served_solves_per_s": served,
        "plain_fp64_single_solves_per_s": plain64,
        "mixed_single_solves_per_s": mixed1,
        "served_over_plain": round(served / plain64, 3),
        "server_stats": stats,
    }


def serve_bench(args):
    """--serve: the whole serving workload (every class the budget admits)."""
    out = {"metric": METRIC, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
           "dtype": "f32-in-f64", "data": "synthetic"}
    leg = serve_leg(args, sample_cost=args.serve_sample_cost)
    out["value"] = leg["served_solves_per_s"]
    out["config"] = {"workload": leg["workload"]}
    out.update(leg)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--degree", type=int, default=5)
    ap.add_argument("--nel", type=int, default=1024)
    ap.add_argument("--dim", type=int, default=2)
    ap.add_argument("--pde", choices=("poisson", "cdr"), default="poisson",
                    help="cdr: benchmark 2's convection-diffusion-reaction operator on the unit square")
    ap.add_argument("--projection", choices=("direct", "indirect"), default="direct",
                    help="indirect: p -> p-1 -> ... -> 1 (Appendix A variant)")
    ap.add_argument("--mass", choices=("lumped", "consistent"), default="lumped",
                    help="consistent: consistent mass matrices in the transfers (Appendix B variant)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the benchmark-1 mixed-precision leg")
    ap.add_argument("--no-copy", action="store_true", help="skip the device-copy bandwidth leg")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--serve", action="store_true", help="continuous-batching serving benchmark")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--closed-requests", type=int, default=600)
    ap.add_argument("--serve-sample-cost", type=float, default=None,
                    help="serve only classes whose ILUT work n*M^2 is at most this (default run: 3.25e10; --serve: all)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg of the default run")
    ap.add_argument("--serve-tri-waves", type=int, default=1,
                    help="waves per CU of each slot's triangular-solve grid (0: as many as fit)")
    ap.add_argument("--cpu-nel", type=int, default=256, help="elements per direction of the CPU oracle's sample")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 512 MiB (3 times), the reference for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solve phase here runs on a single MI355X; "
              "multi-GPU sharding is a design note only (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.cpu_baseline_only:
        n_full = (args.nel + args.degree - 2) ** args.dim
        print(json.dumps(cpu_baseline(args.degree, args.nel, n_full, args.cpu_budget, pde=int(args.pde == "cdr"),
                                      nel_s=args.cpu_nel, dim=args.dim)), flush=True)
        return
    # the CPU oracle baseline runs in a process of its own, beside the GPU legs
    cpu_proc = None
    if not (args.no_cpu_baseline or args.serve or args.calibrate_copy):
        cpu_proc = subprocess.Popen(
            [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--dim", str(args.dim),
             "--degree", str(args.degree), "--nel", str(args.nel), "--pde", args.pde,
             "--cpu-budget", str(args.cpu_budget), "--cpu-nel", str(args.cpu_nel if args.dim == 2 else 16)],
            stdout=subprocess.PIPE, text=True)

    try:
        gpu_legs(args, cpu_proc)
    finally:
        if cpu_proc is not None and cpu_proc.poll() is None:
            cpu_proc.kill()
            cpu_proc.communicate()


def gpu_legs(args, cpu_proc):
    import torch
    import paper_1901_01685_amd as pmg

    dev = torch.device("cuda:0")
    if args.serve:
        serve_bench(args)
        return
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
    pde = pmg.PDE_CDR if args.pde == "cdr" else pmg.PDE_POISSON
    print(f"# setting up dim={args.dim} p={args.degree} h=1/{args.nel}", file=sys.stderr, flush=True)
    s = pmg.Solver(dim=args.dim, degree=args.degree, n_elem=args.nel, pde=pde, device=0,
                   projection=pmg.PROJ_INDIRECT if args.projection == "indirect" else pmg.PROJ_DIRECT,
                   mass_transfer=pmg.MASS_CONSISTENT if args.mass == "consistent" else pmg.MASS_LUMPED)
    t_setup = time.perf_counter() - t0
    info = s.info
    n = s.n
    print(f"# setup {t_setup:.1f} s (assembly {info.t_assembly:.1f}, ILUT {info.t_ilut:.1f} "
          f"{'device' if info.ilut_on_device else 'host'}, schedules {info.t_schedule:.1f}, "
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

    # timed region: K V-cycles, each ending with the stopping-test norm on the
    # host; each V-cycle is one replay of the cached HIP graph of its kernels
    x.zero_()
    s.residual(b, x, r, norm=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rel = 1.0
    for _ in range(args.steps):
        rel = s.vcycle(b, x, r, norm=True) / r0
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = 1e3 * el / args.steps
    value = n * args.steps / el

    # kernel timing: the same K V-cycles with HIP events recorded around every
    # step on the launch stream (event profiling launches the kernels one by
    # one instead of from the graph; the kernels and their inputs are the same)
    x.zero_()
    s.residual(b, x, r, norm=True)
    s.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.vcycle(b, x, r, norm=True)
    torch.cuda.synchronize()
    el_eager = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile_enable(False)

    # whole solves to a relative residual of 1e-8 on the same problem: V-cycles
    # alone (stationary p-multigrid) and BiCGSTAB with one V-cycle per
    # preconditioning; each is run once untimed so its graphs are captured
    solves = {}
    for name, fn in (("vcycles", s.solve), ("bicgstab", s.bicgstab)):
        x.zero_()
        fn(b, x, tol=1e-8)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, relr, _, _, _ = fn(b, x, tol=1e-8)
        torch.cuda.synchronize()
        el_s = time.perf_counter() - t0
        solves[name] = {"status": int(st), "iterations": int(it), "relres": float(relr),
                        "ms": round(1e3 * el_s, 3), "ms_per_iteration": round(1e3 * el_s / max(it, 1), 4)}

    # dominant kernel by total time per V-cycle
    KERNELS = kernel_map(info, args.dim, args.degree)
    per_class = {c: (ms, cnt) for c, (ms, cnt) in prof.items() if cnt > 0}
    dom = max((c for c in per_class if c in KERNELS), key=lambda c: per_class[c][0])
    ms_tot, cnt = per_class[dom]
    avg_s = ms_tot / cnt / 1e3
    nbytes = getattr(info, KERNELS[dom][1])
    achieved = nbytes / avg_s / 1e9
    workload = f"2d-unit-square-p{args.degree}-h1/{args.nel}" if args.dim == 2 else \
        f"3d-unit-cube-p{args.degree}-h1/{args.nel}"
    if pde == pmg.PDE_CDR:
        workload = f"2d-unit-square-cdr-p{args.degree}-h1/{args.nel}"
    if args.projection != "direct" or args.mass != "lumped":
        workload += f"-{args.projection}-{args.mass}"
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
        "bytes_per_launch_by_class": {c: int(getattr(info, KERNELS[c][1])) for c in KERNELS},
        "per_step_ms": {c: round(v[0] / args.steps, 4) for c, v in per_class.items()},
        "ms_per_step_kernel_by_kernel": round(1e3 * el_eager / args.steps, 4),
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
        "config": {"workload": workload, "pde": args.pde, "projection": args.projection, "mass": args.mass,
                   "dim": args.dim, "degree": args.degree, "n_elem": args.nel,
                   "unknowns": n, "precision": "fp64", "ilut": [1e-12, 1.0], "final_relres": rel,
                   "setup_s": round(t_setup, 1), "parallelism": "1 GPU",
                   "setup_breakdown_s": {"assembly": round(info.t_assembly, 2), "ilut": round(info.t_ilut, 2),
                                         "ilut_on_device": int(info.ilut_on_device),
                                         "schedules": round(info.t_schedule, 2), "upload": round(info.t_upload, 2)},
                   "chunk_levels": [int(info.chunk_levels_l), int(info.chunk_levels_u)]},
        "roofline": roofline,
        "solves": solves,
    }
    s.close()
    del b, x, r
    torch.cuda.empty_cache()
    if not args.no_copy:
        out["copy_bandwidth"] = copy_bandwidth(torch, dev)
        print(f"# device copy {out['copy_bandwidth']['GBps']} GB/s", file=sys.stderr, flush=True)
    if not args.no_mixed and args.dim == 2 and pde == pmg.PDE_POISSON:
        print("# benchmark 1 at p=5, h=1/512: mixed vs FP64 to 1e-10", file=sys.stderr, flush=True)
        out["mixed_config4"] = mixed_config4(pmg, torch, dev)
    if not args.no_serving and args.dim == 2 and pde == pmg.PDE_POISSON:
        print("# serving leg", file=sys.stderr, flush=True)
        sargs = argparse.Namespace(**vars(args))
        sargs.serve_requests, sargs.serve_warmup, sargs.closed_requests = 400, 50, 200
        out["serving"] = serve_leg(sargs, sample_cost=args.serve_sample_cost or 3.25e10)
    if cpu_proc is not None:
        print("# waiting for the CPU oracle baseline", file=sys.stderr, flush=True)
        try:
            so, _ = cpu_proc.communicate(timeout=600)
            out["cpu_baseline"] = json.loads(so.strip().splitlines()[-1]) if cpu_proc.returncode == 0 else None
        except (subprocess.TimeoutExpired, ValueError, IndexError):
            cpu_proc.kill()
            cpu_proc.communicate()
            out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
