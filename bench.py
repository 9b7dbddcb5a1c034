#!/usr/bin/env python3
"""Benchmark: solves/s of the two-stage preconditioned FGMRES on one MI355X.

One step = the whole hot path for one Jacobian: the recurring setup of the flow
stage (fixed-stress and quasi-IMPES operators, pressure AMG, BILU(0) factors,
precision mirrors -- rebuilt every step as after a Newton update) followed by the
FGMRES(100) solve to rtol 1e-8 with Algorithm 1 applied every iteration.  The
mechanics AMG is set up once before the timed region, as in the paper (the
elasticity operator does not change).  Inputs are synthetic and already resident
in HBM when timing starts.

Prints ONE JSON line.  Extra fields: the FP64-preconditioner rate on the same
workload, per-phase times, iterations, the roofline of the dominant instrumented
kernel (timed with HIP events on its launch stream inside the timed steps; the
per-kernel table comes from one untimed step with every instrumented kernel
bracketed, since each bracket costs two event records) and the CPU oracle baseline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(s):
    """Algorithmic bytes of y = A x with the FP64 block matrix (values + column
    indices + row pointers, x read once, y written once)."""
    b = 0
    for blk in (s.Auu, s.Auf, s.Afu, s.Aff):
        nb, br, bc = blk.vals.shape
        b += nb * (br * bc * 8 + 4) + 4 * (blk.rowptr.shape[0])
    return b + 2 * 8 * s.N


def kernel_fingerprint(names):
    """SHA-256 of the source text in kernels.h of a kernel, or of several (a kernel and
    the device functions it runs; each from its template line, if any, to its closing
    brace): recorded with HBM counters so that they are reported only while the kernel
    is unchanged."""
    import hashlib
    import re
    text = open(os.path.join(ROOT, "paper_1812_05540_amd", "csrc", "kernels.h")).read()
    h = hashlib.sha256()
    for name in ([names] if isinstance(names, str) else names):
        m = re.search(r"\n(?:template <[^\n]*>\n)?__(?:global|device)__[^\n]*\bvoid %s\(" % name, text)
        if not m:
            return None
        end = text.find("\n}\n", m.end())
        h.update(text[m.start():end + 3].encode())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, profile):
    """HBM bytes per launch recorded in a profile summary, if its fingerprint matches."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_fingerprint"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("kernel_fingerprint") != kernel_fingerprint(kernel):
        return None
    return int(rec["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in rec else None


# instrumented kernel -> (kernel template in kernels.h, HBM-counter summary under profiles/)
KERNEL_SOURCES = {
    "system_spmv": (("spmv2_row", "spmv_sys"), "system_spmv_grf64_traffic.md"),
    "cgs2_project": ("mdot", "cgs2_project_grf64_traffic.md"),
    "cgs2_subtract_project": ("gemv_sub_mdot", "cgs2_fused_grf64_traffic.md"),
    "cgs2_subtract_norm": ("gemv_sub", "cgs2_subtract_grf64_traffic.md"),
    "bilu_subdomain": ("bilu_sub", "bilu_subdomain_grf64_traffic.md"),
    "dcgs2_project": ("mdot2", "dcgs2_project_grf64_traffic.md"),
    "dcgs2_subtract": ("gemv_sub2", "dcgs2_subtract_grf64_traffic.md"),
}


def dominant_kernel(kernels):
    """The instrumented kernel with the most event time."""
    return max(((n, v) for n, v in kernels.items() if v["launches"]), key=lambda kv: kv[1]["seconds"])[0]


def roofline_line(name, k, kernels_all, workload):
    """Roofline line of kernel `name` from its timed-region totals k: algorithmic bytes per
    launch / mean launch duration, against HBM peak."""
    per_launch_s = k["seconds"] / k["launches"]
    per_launch_b = k["bytes"] / k["launches"]
    achieved = per_launch_b / per_launch_s / 1e9
    src, prof = KERNEL_SOURCES.get(name, (None, None))
    traffic = recorded_traffic(src, prof) if src and workload == "grf64" else None
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=name,
                launches=k["launches"], us_per_launch=round(per_launch_s * 1e6, 2),
                algorithmic_bytes_per_launch=int(per_launch_b),
                share_of_instrumented_time=round(kernels_all[name]["seconds"] /
                                                 sum(v["seconds"] for v in kernels_all.values()), 3))


def run_gpu(args, s, b):
    import torch
    from paper_1812_05540_amd import ps

    ps.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ctx = ps.ps_ctx_create(0, 0)
    bd = torch.as_tensor(b, dtype=torch.float64, device=dev)
    out = {}
    precs = [("fp32", ps.PS_FP32_PREC)]
    if args.precision in ("both", "fp64"):
        precs = ([("fp32", ps.PS_FP32_PREC)] if args.precision == "both" else []) + [("fp64", ps.PS_FP64)]
    xs = {}
    for name, prec in precs:
        opts = dict(precision=prec, ml_sweeps=args.ml_sweeps, smoother=args.smoother_code,
                    ml_kind=args.ml_kind_code, orth=args.orth_code)
        sv = ps.Solver(ctx, s, mech_key=1, **opts)
        t0 = time.perf_counter()
        sv.setup()                                # mechanics AMG (once) + flow stage
        first_setup = time.perf_counter() - t0
        x = torch.zeros(s.N, dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            sv.setup()
            r = sv.solve(bd, x, args.rtol)
        torch.cuda.synchronize()
        if name == precs[0][0]:
            # one untimed step with every instrumented kernel bracketed by HIP events (on
            # the streams they run on): the per-kernel table and the dominant kernel
            ps.ps_kernel_timing(True)
            sv.setup()
            sv.solve(bd, x, args.rtol)
            out["kernels"] = ps.ps_kernel_stats()
            dom = dominant_kernel(out["kernels"])
            # the timed steps bracket only that kernel (each bracket adds two event records)
            ps.ps_kernel_timing(1 << ps.kernel_index(dom))
        t_setup = t_solve = 0.0
        its = []
        res = None
        t_all = time.perf_counter()
        for _ in range(args.steps):
            t0 = time.perf_counter()
            sv.setup()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            res = sv.solve(bd, x, args.rtol)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            t_setup += t1 - t0
            t_solve += t2 - t1
            its.append(res["iterations"])
        torch.cuda.synchronize()
        total = time.perf_counter() - t_all
        if name == precs[0][0]:
            out["roofline"] = roofline_line(dom, ps.ps_kernel_stats()[dom], out["kernels"], args.workload)
            ps.ps_kernel_timing(False)
        xs[name] = x.clone()
        out[name] = dict(status=res["status"], iterations=its[-1], rel_residual=res["rel_residual"],
                         restarts=res["restarts"], ms_per_step=1e3 * total / args.steps,
                         solves_per_s=args.steps / total, setup_ms=1e3 * t_setup / args.steps,
                         solve_ms=1e3 * t_solve / args.steps, first_setup_s=first_setup,
                         footprint_gb=sv.footprint() / 1e9)
        log(name, json.dumps(out[name]))
        if name == precs[-1][0]:
            # roofline of the FP64 system SpMV: HIP events on the launch stream
            y = torch.empty_like(x)
            for _ in range(3):
                sv.spmv(x, y, stream)
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record(stream)
            for _ in range(args.kernel_reps):
                sv.spmv(x, y, stream)
            end.record(stream)
            end.synchronize()
            t_ms = start.elapsed_time(end) / args.kernel_reps
            nbytes = spmv_bytes(s)
            achieved = nbytes / (t_ms * 1e-3) / 1e9
            out["spmv"] = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=round(achieved / HBM_PEAK_GBS, 4),
                               kernel="system SpMV y = A x (FP64 SELL-64, node rows + cell rows)",
                               ms=round(t_ms, 4), algorithmic_bytes=nbytes)
            # plain copy of known size (1 GiB read + 1 GiB written): the box's attainable
            # stream bandwidth, and the calibration kernel for the HBM traffic counters
            src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            torch.mul(src, 1.0, out=dst)
            start.record(stream)
            for _ in range(5):
                torch.mul(src, 1.0, out=dst)
            end.record(stream)
            end.synchronize()
            t_copy = start.elapsed_time(end) / 5
            out["spmv"]["copy_GBs"] = round(2 * src.numel() * 8 / (t_copy * 1e-3) / 1e9, 1)
            del src, dst
        sv.close()
    if "fp32" in xs and "fp64" in xs:
        d = (xs["fp32"] - xs["fp64"]).norm() / xs["fp64"].norm()
        out["fp32_vs_fp64_solution_rel_diff"] = float(d)
    ps.ps_ctx_destroy(ctx)
    return out


def cpu_baseline(s, b, its_gpu, budget_s, args):
    """The oracle (FP64, NumPy/SciPy, one thread) on a bounded sample of the same
    workload: its flow-stage setup plus up to two FGMRES iterations (mechanics AMG
    built once beforehand, as on the GPU); solves/s extrapolated with the GPU's
    iteration count."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import precond as P, amg, Options
    from oracle.fgmres import fgmres
    o = Options(smoother=args.smoother, ml_kind=args.ml_kind, ml_sweeps=args.ml_sweeps, orth=args.orth)
    t0 = time.perf_counter()
    sdc = amg.build(P.sdc_matrix(s), smoother=args.smoother)
    t_mech = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = P.setup(s, o, mechanics=sdc)
    t_setup = time.perf_counter() - t0
    A = st.mats["A"]
    n_it = 2 if t_setup < budget_s else 1
    t0 = time.perf_counter()
    fgmres(lambda v: A @ v, lambda v: P.apply_precond(st, v), b, 1e-30, 100, n_it, orth=args.orth)
    t_it = (time.perf_counter() - t0) / n_it
    per_solve = t_setup + its_gpu * t_it
    return dict(value=round(1.0 / per_solve, 6), unit="solves/s", cores=1, kind="oracle",
                nproc=os.cpu_count(),
                sample="oracle on the same workload: flow-stage setup (%.1f s) + %d FGMRES "
                       "iteration(s) (%.2f s each), extrapolated to %d iterations; mechanics AMG "
                       "(%.1f s, once) excluded as on the GPU" % (t_setup, n_it, t_it, its_gpu, t_mech))


SERVING_SIZES = (16, 24, 32, 48, 64)


def per_grid_cases():
    """The small configuration (8^3, i.i.d. fields) and the first request of each smaller
    grid size of the serving stream (its own field, its subdomain partition), for the
    per-grid GPU and oracle timings."""
    from synth import workload
    from synth.configs import serving_request, serving_request_spec
    from synth.jacobian import box_partition
    s, b = workload(grid=(8, 8, 8), kind="iid", seed=1, rhs_seed=101)
    cases = [("8^3 i.i.d. (two-phase)", s, b)]
    for n in SERVING_SIZES[:-1]:
        i = next(i for i in range(10000) if serving_request_spec(i)[0] == n)
        s, b = serving_request(i)
        s.ml_part = box_partition(n, n, n, min(n, 32), min(n, 32), min(n, 16))
        cases.append(("%d^3 serving request %d" % (n, i), s, b))
    return cases


def run_per_grid(args, cases):
    """FP32-path solves/s of each case alone (flow setup + solve, best of three, after a
    device-path setup and one warm-up solve), with the benchmark's options."""
    import torch
    from paper_1812_05540_amd import ps
    ctx = ps.ps_ctx_create(0, 0)
    out = []
    try:
        for label, s, b in cases:
            sv = ps.Solver(ctx, s, precision=ps.PS_FP32_PREC, ml_sweeps=args.ml_sweeps,
                           smoother=args.smoother_code, ml_kind=args.ml_kind_code, orth=args.orth_code)
            sv.setup()
            bd = torch.as_tensor(b, dtype=torch.float64, device="cuda")
            x = torch.zeros(s.N, dtype=torch.float64, device="cuda")
            sv.setup()
            sv.solve(bd, x, args.rtol)
            best, res = 1e30, None
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sv.setup()
                res = sv.solve(bd, x, args.rtol)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            sv.close()
            out.append(dict(grid=label, unknowns=int(s.N), iterations=res["iterations"], status=res["status"],
                            gpu_solves_per_s=round(1.0 / best, 2)))
    finally:
        ps.ps_ctx_destroy(ctx)
    return out


def per_grid_oracle(cases, rows, budget_s, args):
    """The oracle (one thread) on each case: flow setup + up to two FGMRES iterations,
    extrapolated to the GPU's iteration count (mechanics AMG excluded); cases stop once
    the budget is spent."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import precond as P, amg, Options
    from oracle.fgmres import fgmres
    o = Options(smoother=args.smoother, ml_kind=args.ml_kind, ml_sweeps=args.ml_sweeps, orth=args.orth)
    t_start = time.perf_counter()
    for (label, s, b), row in zip(cases, rows):
        if time.perf_counter() - t_start > budget_s:
            row["oracle"] = "skipped (budget)"
            continue
        sdc = amg.build(P.sdc_matrix(s), smoother=args.smoother)
        t0 = time.perf_counter()
        st = P.setup(s, o, mechanics=sdc)
        t_setup = time.perf_counter() - t0
        A = st.mats["A"]
        t0 = time.perf_counter()
        fgmres(lambda v: A @ v, lambda v: P.apply_precond(st, v), b, 1e-30, 100, 2, orth=args.orth)
        t_it = (time.perf_counter() - t0) / 2
        v = 1.0 / (t_setup + row["iterations"] * t_it)
        row["oracle_solves_per_s"] = round(v, 4)
        row["gpu_over_oracle"] = round(row["gpu_solves_per_s"] / v, 1)
    return rows


def _serving_request(job):
    """Request i of the serving mix (synth.configs.serving_request: grid n^3 drawn from
    16..64, its own seeded random field with sigma ~ U(1, 3), its own rhs; E fixed per grid
    size so that requests of one size share A_uu).  Runs in a worker process; A_uu is
    returned only for the first request of each size (the others take that copy), to keep
    the stream in host memory."""
    i, keep_auu = job
    import numpy as np
    from synth.configs import serving_request
    from synth.jacobian import box_partition
    s, b = serving_request(i)
    n = s.meta["grid"][0]
    s.ml_part = box_partition(n, n, n, min(n, 32), min(n, 32), min(n, 16))
    if not keep_auu:
        s.Auu = None
    return i, n, s, np.asarray(b)


def make_serving_stream(nreq, workers):
    """The request stream's systems, generated in fresh processes before the GPU is used."""
    import multiprocessing as mp
    from synth.configs import serving_request_spec
    first = {}
    for i in range(nreq):
        first.setdefault(serving_request_spec(i)[0], i)
    jobs = [(i, first[serving_request_spec(i)[0]] == i) for i in range(nreq)]
    # one BLAS thread per worker process (the workers already fill the cores)
    saved = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for v in saved:
        os.environ[v] = "1"
    try:
        with mp.get_context("spawn").Pool(max(1, min(workers, nreq))) as pool:
            out = pool.map(_serving_request, jobs, chunksize=1)
    finally:
        for v, old in saved.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old
    auu = {n: s.Auu for i, n, s, _ in out if first[n] == i}
    for _, n, s, _ in out:
        s.Auu = auu[n]
    return out


def run_serving(args, stream):
    """Mixed-size request stream against one context (continuous batching): each
    request is created, set up (flow stage), submitted and awaited by one of W client
    threads; latency runs from the request's arrival to its completion and includes
    queueing, ps_create, ps_setup and the solve.  The stream is replayed closed-loop
    first (capacity) and then with Poisson arrivals at 0.25, 0.5 and 0.9 of it."""
    import threading
    import numpy as np
    import torch
    from paper_1812_05540_amd import ps

    ps.load()
    dev = torch.device("cuda:0")
    ctx = ps.ps_ctx_create(0, int(args.serving_budget_gb * 1e9))
    opts = dict(precision=ps.PS_FP32_PREC, smoother=args.smoother_code, ml_kind=args.ml_kind_code,
                ml_sweeps=args.ml_sweeps, orth=args.orth_code)
    # resident state per grid size: the mechanics hierarchy and set-up handles that the
    # context keeps for the requests (released handles are reused by ps_create)
    first = {}
    for i, n, s, b in stream:
        first.setdefault(n, s)
    for n in SERVING_SIZES:
        if n not in first:
            continue
        warm = [ps.Solver(ctx, first[n], mech_key=n, **opts) for _ in range(min(args.serving_clients, 4))]
        for sv in warm:
            sv.setup()
        for sv in warm:
            sv.close()
    rng = np.random.Generator(np.random.PCG64(77))

    def serve(reqs, arrivals):
        lat, status, iters = [None] * len(reqs), [None] * len(reqs), [0] * len(reqs)
        nxt = [0]
        lock = threading.Lock()
        t0 = time.perf_counter()

        def worker():
            stream_ = torch.cuda.Stream()
            while True:
                with lock:
                    q = nxt[0]
                    nxt[0] += 1
                if q >= len(reqs):
                    return
                wait = t0 + arrivals[q] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
                i, n, s, b = reqs[q]
                try:
                    sv = ps.Solver(ctx, s, mech_key=n, **opts)
                    sv.setup()
                    with torch.cuda.stream(stream_):
                        bd = torch.as_tensor(b, device=dev)
                        x = torch.zeros(s.N, dtype=torch.float64, device=dev)
                    r = ps.ps_wait(ctx, sv.submit(bd, x, args.rtol, stream_))
                    sv.close()
                    status[q], iters[q] = r["status"], r["iterations"]
                    if r["status"] != ps.PS_OK:
                        log("serving request %d (%d^3): status %d after %d iterations, residual %.3g" %
                            (i, n, r["status"], r["iterations"], r["rel_residual"]))
                except ps.PsError as e:
                    log("serving request %d (%d^3) failed: %s" % (i, n, e))
                    status[q] = e.code
                except Exception as e:            # recorded as a failed request
                    log("serving request %d failed: %r" % (i, e))
                    status[q] = -100
                lat[q] = time.perf_counter() - (t0 + arrivals[q])

        th = [threading.Thread(target=worker) for _ in range(args.serving_clients)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        wall = time.perf_counter() - t0
        return np.array(lat), status, iters, wall

    nreq = len(stream)
    _, st, _, wall = serve(stream, [0.0] * nreq)
    mu = nreq / wall
    out = dict(capacity_rps=round(mu, 3), clients=args.serving_clients, requests_per_rate=nreq,
               stream="%d requests, each its own seeded field (sigma U(1,3)) and rhs, grids drawn from %s^3; "
                      "the same stream replayed closed-loop and at each arrival rate"
                      % (nreq, "/".join(str(n) for n in SERVING_SIZES)),
               rates=[])
    for frac in (0.25, 0.5, 0.9):
        gaps = rng.exponential(1.0 / (frac * mu), nreq)
        arrivals = np.cumsum(gaps) - gaps[0]
        lat, st, its, wall = serve(stream, list(arrivals))
        ok = [l for l, c in zip(lat, st) if c == ps.PS_OK]
        out["rates"].append(dict(load=frac, rate_rps=round(frac * mu, 3), p50_s=round(float(np.percentile(lat, 50)), 4),
                                 p99_s=round(float(np.percentile(lat, 99)), 4), max_s=round(float(lat.max()), 4),
                                 solves_per_s=round(len(ok) / wall, 3), failed=len(lat) - len(ok),
                                 mean_iterations=round(float(np.mean(its)), 1)))
        log("serving", json.dumps(out["rates"][-1]))
    launches, covered = ps.ps_ctx_batches(ctx)
    out["batched_step1"] = dict(launch_sequences=launches, requests=covered)
    ps.ps_ctx_destroy(ctx)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grf64")
    ap.add_argument("--precision", default="both", choices=["fp32", "fp64", "both"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--ml-sweeps", type=int, default=2,
                    help="local-stage sweeps (2: measured fastest to rtol 1e-8 on grf64)")
    ap.add_argument("--smoother", default="l1jac", choices=["cheb2", "l1jac"])
    ap.add_argument("--ml-kind", default="bilu0", choices=["bilu0", "bjacobi", "mcgs"])
    ap.add_argument("--ml-part", default="16,16,16",
                    help="processor-local local stage: subdomain box size in cells ('global': one domain)")
    ap.add_argument("--orth", default="dcgs2", choices=["cgs2", "dcgs2"],
                    help="FGMRES Arnoldi step: classical Gram-Schmidt twice, or with delayed re-orthogonalisation")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=64,
                    help="requests of the serving stream, each with its own field (0: skip; 512: the full "
                         "stream of the serving configuration)")
    ap.add_argument("--serving-workers", type=int, default=16, help="processes generating the stream")
    ap.add_argument("--serving-clients", type=int, default=6)
    ap.add_argument("--serving-budget-gb", type=float, default=200.0)
    ap.add_argument("--cpu-budget-s", type=float, default=30.0)
    ap.add_argument("--per-grid", type=int, default=1,
                    help="1: also time the 8^3 case and one request of each smaller serving grid alone, "
                         "GPU and oracle")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    args.smoother_code = 0 if args.smoother == "cheb2" else 1
    args.ml_kind_code = {"bilu0": 0, "bjacobi": 1, "mcgs": 2}[args.ml_kind]
    args.orth_code = {"cgs2": 0, "dcgs2": 1}[args.orth]

    from synth import workload
    from synth.configs import LOG10K_MAX
    t0 = time.perf_counter()
    s, b = workload(args.workload)
    if args.ml_part and args.ml_part != "global":
        from synth.jacobian import box_partition
        bx, by, bz = (int(v) for v in args.ml_part.split(","))
        s.ml_part = box_partition(*s.meta["grid"], bx, by, bz)
    log("workload %s: N=%d generated in %.1fs" % (args.workload, s.N, time.perf_counter() - t0))
    stream = None
    if args.serving_requests > 0:
        t0 = time.perf_counter()
        stream = make_serving_stream(args.serving_requests, args.serving_workers)
        log("serving stream: %d requests generated in %.1fs" % (len(stream), time.perf_counter() - t0))
    cases = per_grid_cases() if args.per_grid else None
    g = run_gpu(args, s, b)
    per_grid = run_per_grid(args, cases) if cases else None
    serving = run_serving(args, stream) if stream else None
    head = g.get("fp32") or g.get("fp64")
    line = {
        "metric": "solves/s to rtol 1e-8 (FP64 vs FP32 precond), SpMV HBM GB/s, p50/p99 latency",
        "value": round(head["solves_per_s"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner, f64 Krylov" if "fp32" in g else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%dx%d-cell %s-phase poromechanics Jacobian, N=%d, FGMRES(100) (%s) + "
                               "two-stage preconditioner, rtol %g; step = flow-stage setup + solve; "
                               "log10 permeability clipped above at %.1f (about 20 D); state: line-drive "
                               "pressure solved through the permeability field"
                               % (args.workload, *s.meta["grid"], "two" if s.nf == 2 else "three", s.N,
                                  "CGS2" if args.orth == "cgs2" else "delayed re-orthogonalisation",
                                  args.rtol, LOG10K_MAX),
                   "precision": "fp32-preconditioner" if "fp32" in g else "fp64",
                   "ml_sweeps": args.ml_sweeps, "smoother": args.smoother, "ml_kind": args.ml_kind,
                   "orth": args.orth,
                   "ml_part": args.ml_part if args.ml_part else "global"},
        "paths": {k: v for k, v in g.items() if k in ("fp32", "fp64")},
        "roofline": g["roofline"],
        "kernels_note": "one untimed FP32-path step with every instrumented kernel bracketed; the timed "
                        "steps bracket only the roofline kernel",
        "kernels": {n: dict(launches=v["launches"], us_per_launch=round(1e6 * v["seconds"] / v["launches"], 2),
                            GBs=round(v["bytes"] / v["seconds"] / 1e9, 1))
                    for n, v in g["kernels"].items() if v["launches"]},
        "spmv": g["spmv"],
    }
    if "fp64" in g and "fp32" in g:
        line["fp32_over_fp64_speedup"] = round(g["fp32"]["solves_per_s"] / g["fp64"]["solves_per_s"], 3)
        line["fp32_vs_fp64_solution_rel_diff"] = g.get("fp32_vs_fp64_solution_rel_diff")
    if serving:
        line["serving"] = serving
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s, b, head["iterations"], args.cpu_budget_s, args)
        if per_grid:
            per_grid = per_grid_oracle(cases, per_grid, args.cpu_budget_s, args)
    if per_grid:
        line["per_grid"] = per_grid
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
