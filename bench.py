#!/usr/bin/env python
"""Benchmark of the PHS-RBF hot path on one MI355X.

Workload: the 2D Taylor-Green decaying vortex (nu = 0.01) on [0, 2 pi]^2 with
about 250,000 Poisson-disk points (seed 2), PHS r^3 with degree-4 polynomials
on 30-point clouds, Courant number 10, velocity and pressure prescribed on the
boundary from the exact solution. One benchmark step is one pass of the whole
hot path over this input: neighbour search + weights (rbffd_build_stencils),
assembly (rbffd_assemble) and one BDF2 time step (simple_step: momentum
BiCGSTAB, pressure-correction BiCGSTAB, corrections, convergence tests) with
Krylov tolerance 1e-10 and at most --max-outer outer iterations.

The headline value is M point-iters/s: Krylov rows processed per second (a
momentum iteration on d right-hand sides counts d rows per point) over the
whole step, build included. Also reported: the roofline of the dominant kernel
(the sliced-ELL SpMV of the pressure-correction matrix) timed with HIP events on
the stream it runs on, and the FP64 oracle on the host CPU as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "M point-iters/s & converged solves/s vs plain FP64; p50/p99 latency at 1e-6"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(n, q, narrow=0.0):
    """Algorithmic bytes of one SpMV: q values (8 B) and q column indices per row,
    x read once and y written once (8 B each). Indices are 2 B on the fraction
    `narrow` of 64-row slices that the library stores as 16-bit offsets, else 4 B."""
    return int(round(n * (8 * q + q * (2 * narrow + 4 * (1 - narrow)) + 16)))


def narrow_fraction(col, n, q):
    """Fraction of rows in 64-row slices whose columns span fewer than 65536
    indices (the slices the library stores with 16-bit column offsets)."""
    c = col.reshape(n, q)
    npad = (n + 63) // 64 * 64
    lo = np.full(npad, np.iinfo(np.int64).max)
    hi = np.full(npad, -1)
    lo[:n] = c.min(1)
    hi[:n] = c.max(1)
    lo = lo.reshape(-1, 64).min(1)
    hi = hi.reshape(-1, 64).max(1)
    narrow = np.repeat((hi - lo) < 65536, 64)[:n]
    return float(narrow.mean())


def kt_bytes(n, q):
    """Algorithmic bytes of the dominant kernel KT (t = A s-hat with the partial
    dots t.s, t.t, r-hat.t): one SpMV at 12q + 16 B per row (q FP64 values, q
    4-byte column indices, s-hat read, t written) plus the two dot operands s
    and r-hat (16 B): 12q + 32 B per row."""
    return n * (12 * q + 32)


def kv_bytes(n, q):
    """KV (v = A p-hat with the partial r-hat.v): 12q + 16 + 8 B per row."""
    return n * (12 * q + 24)


def iteration_bytes(n, q):
    """One FP64 BiCGSTAB iteration: two SpMVs (12q + 16 B per row each) and
    about 20 vector sweeps of 8 B: 24q + 192 B per row."""
    return n * (24 * q + 192)


def bicgstab_iter_bytes(n, q, narrow=0.0):
    """Algorithmic bytes of one FP64 BiCGSTAB iteration: two SpMVs (their operand
    read and result write included) and the vectors the four kernels move
    besides: k_v reads r-hat (1); k_s reads r, v, r-hat, D^-1 and writes s,
    s-hat (6); k_t reads s, r-hat (2); k_x reads x, p-hat, s, t, v, D^-1 and
    writes x, r, p-hat (9)."""
    return 2 * spmv_bytes(n, q, narrow) + n * 8 * (1 + 6 + 2 + 9)


# the benchmark step's workload: the 2D Taylor-Green vortex on ~250k Poisson-disk
# points (default), or the 3D Ethier-Steinman flow on a 100^3 jittered lattice
# plus face points (~1.06M points)
WORKLOADS = {
    "taylor_green": {
        "k": 4, "make": lambda W: W.taylor_green_disk(),
        "sample": lambda W, a: W.taylor_green_disk(r=a.cpu_sample_r),
        "sample1": lambda W, a: W.taylor_green_disk(r=2 * a.cpu_sample_r),
        "text": "Taylor-Green vortex nu=0.01 on [0,2pi]^2, {n} Poisson-disk points (seed 2), PHS r^3 + degree-4 "
                "polynomials, q={q}, Co 10 (dt={dt:.5f})",
    },
    "beltrami": {
        "k": 3, "make": lambda W: W.beltrami_cube(n=100),
        "sample": lambda W, a: W.beltrami_cube(n=a.cpu_sample_cube),
        "sample1": lambda W, a: W.beltrami_cube(n=a.cpu_sample_cube * 2 // 3),
        "text": "Ethier-Steinman Beltrami flow nu=0.01 on [0,1]^3, {n} points (100^3 jittered lattice + faces, "
                "seed 4), PHS r^3 + degree-3 polynomials, q={q}, Co 10 (dt={dt:.5f})",
    },
}

COUNTER_SUMMARY = {"taylor_green": os.path.join(ROOT, "profiles", "k_t_pressure_tg250k_counters.txt"),
                   "beltrami": os.path.join(ROOT, "profiles", "k_t_pressure_beltrami1m_counters.txt")}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2106_07616_amd", "csrc", f) for f in ("krylov.hip", "internal.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(workload):
    """HBM bytes per KT launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by the copy-kernel calibration), or None when the summary is
    missing or was taken from different kernel sources."""
    try:
        with open(COUNTER_SUMMARY[workload]) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """Model name (lscpu) and the number of cores this process may use."""
    model = "unknown"
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable


def _omp_threads(nthreads):
    """Set the OpenMP thread count of the oracle's runtime (libgomp)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(nthreads))
    except OSError:
        pass


def cpu_baseline(args):
    """The FP64 oracle running the same benchmark step (operator build + one BDF2
    step at Co 10, same tolerances) on a smaller cloud from the same generator,
    in the same unit: with the OpenMP threads of the host (kNN, weights and the
    row loop of the sparse products in parallel, dot products sequential), and
    with one thread on a quarter-size cloud, which keeps the leg near 15 s."""
    import oracle
    import workloads as W
    oracle.build()
    c = WORKLOADS[args.workload]["sample"](W, args)
    c1 = WORKLOADS[args.workload]["sample1"](W, args)
    kdeg = WORKLOADS[args.workload]["k"]
    model, usable = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", usable))

    def leg(nthreads, c):
        _omp_threads(nthreads)
        t0 = time.perf_counter()
        ops = oracle.build_operators(c, kdeg)
        vel0, p0 = W.flow_fields(c, 0.0)
        dt = oracle.dt_from_courant(ops, vel0, 10.0, 1.0, 0.01)
        t_build = time.perf_counter() - t0
        velm, _ = W.flow_fields(c, -dt)
        ubc, pbc = W.flow_fields(c, dt)
        t1 = time.perf_counter()
        _, _, _, st = oracle.simple_step(ops, vel0, velm, p0, ubc, 1.0, 0.01, dt, tol_outer=1e-4,
                                         tol_krylov=args.tol_krylov,
                                         max_outer=args.max_outer, max_krylov=20000, p_bc=pbc)
        t_end = time.perf_counter()
        pi = c.n * (st["krylov_mom"] + st["krylov_p"]) + int((c.kind == W.DIRICHLET).sum()) * st["krylov_b"]
        return dict(value=round(pi / (t_end - t0) / 1e6, 3), t_build=t_build, t_step=t_end - t1, st=st, pi=pi,
                    t=t_end - t0, dt=dt, q=ops.q, n=c.n)

    full = leg(threads, c)
    one = leg(1, c1)
    _omp_threads(threads)
    st = full["st"]
    return {"value": full["value"], "unit": "M point-iters/s", "cores": threads, "kind": "oracle",
            "host": {"lscpu_model": model, "usable_cores": usable},
            "one_thread": {"value": one["value"], "cores": 1, "n_points": one["n"],
                           "build_s": round(one["t_build"], 2), "step_s": round(one["t_step"], 2)},
            "sample": f"FP64 oracle, one benchmark step on a {c.n}-point {c.name} cloud from the same generator "
                      f"(k={kdeg}, q={full['q']}, Co 10, dt={full['dt']:.5f}): operator build {full['t_build']:.2f} s "
                      f"({threads} OpenMP threads), step {full['t_step']:.2f} s "
                      f"(sequential dot products), {st['outer_iters']} outer / {st['krylov_mom']} momentum / {st['krylov_p']} pressure "
                      f"iterations, {full['pi']} point-iters in {full['t']:.2f} s; one thread on a {one['n']}-point cloud: "
                      f"{one['value']} M point-iters/s (build {one['t_build']:.2f} s, step {one['t_step']:.2f} s)"}


FP64_PEAK_TFLOPS = 78.6


def post_bench(args):
    """Post-processing on a 252k-point square with one circular hole, k = 4
    (q = 30): rbffd_interpolate of u, v, p at 1M scattered points, and
    rbffd_cylinder_forces at 360 surface points (Sec. 4)."""
    import torch

    import paper_2106_07616_amd as R
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    R.lib()
    k, nq, reps = 4, 1_000_000, 5
    cloud = W.holed_square(250_000, seed=5, n_holes=1)
    cx, cy, rad = cloud.meta["holes"][0]
    ctx = R.Context(0)
    solver = R.Solver(ctx, cloud, k)
    q, m, _ = R.rbffd_stencil_sizes(2, k)
    u, v, p = W.kovasznay(cloud.xyz[:, 0], cloud.xyz[:, 1], cloud.meta["Re"])
    vel = torch.tensor(np.stack([u, v]), device="cuda")
    pt = torch.tensor(p, device="cuda")
    fields = torch.tensor(np.stack([u, v, p]), device="cuda")
    # query points in the fluid: a point deep inside the hole would see only
    # the hole's circle, on which the degree-k polynomials are not unisolvent
    cand = np.random.default_rng(6).uniform(0.0, 1.0, size=(2 * nq, 2))
    cand = cand[np.hypot(cand[:, 0] - cx, cand[:, 1] - cy) > rad]
    qx = torch.tensor(cand[:nq], device="cuda")
    log(f"[post] cloud n={cloud.n} q={q} m={m}; {nq} query points")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return float(np.median(t))

    t_int = timed(lambda: R.rbffd_interpolate(ctx, solver.dcloud, k, qx, fields))
    mu = 1.0 / cloud.meta["Re"]
    t_f = timed(lambda: solver.cylinder_forces(vel, pt, (cx, cy), 2 * rad, mu, 360, rho=1.0, u_ref=1.0))
    F, cf = solver.cylinder_forces(vel, pt, (cx, cy), 2 * rad, mu, 360, rho=1.0, u_ref=1.0)
    ns = q + m
    flops = 2.0 / 3.0 * ns ** 3 + 2.0 * ns * ns   # LU of the saddle system + one solve, per query
    tflops = nq * flops / t_int / 1e12
    log(f"[post] interpolate: {t_int * 1e3:.1f} ms for {nq} points; forces: {t_f * 1e3:.2f} ms, F={F} C={cf}")
    print(json.dumps({
        "metric": "interpolated query points/s (3 fields) and cylinder force evaluations/s",
        "value": round(nq / t_int, 1), "unit": "query points/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": round(t_int * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"unit square with one circular hole (centre ({cx:.4f}, {cy:.4f}), radius {rad:.4f}), "
                               f"{cloud.n} points, PHS r^3 + degree-{k} polynomials, q={q}; Kovasznay fields; "
                               f"{nq} uniform random query points in the fluid; forces on the hole at 360 surface points",
                   "n_points": cloud.n, "q": q, "poly_degree": k},
        "cylinder_forces": {"ms_per_eval": round(t_f * 1e3, 3), "evals_per_s": round(1.0 / t_f, 1), "nsurf": 360,
                            "force": F, "coef": cf},
        "roofline": {"bound": "alu", "kernel": "whole rbffd_interpolate call (kNN + weights + sampling)",
                     "achieved": round(tflops, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP64_PEAK_TFLOPS, 4), "traffic": None,
                     "flops_per_query": flops},
    }))
    ctx.close()


def batch_flow_bench(args):
    """The batched configuration as flow instances: the 256 holed-square
    clouds of the batch (0-4 holes, 500-50k points log-uniform, degree 2-5,
    q = 2m) each carry the Kovasznay flow (no-slip on the holes, prescribed
    pressure on the edges and the holes) and take three BDF time steps at
    Co 1, with the outer tolerance of Sec. 3.2 (at most 5 outer iterations)
    and Krylov solves to 1e-8: every instance's step together
    (simple_step_batched: one batched solve per Krylov stage over all
    instances) against the same steps instance by instance (simple_step)."""
    import torch

    import paper_2106_07616_amd as R
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    R.lib()
    cfg = W.config_c3_sizes(args.batch_count)
    t0 = time.perf_counter()
    pp = W.PRESCRIBED_PRESSURE
    clouds = [(W.holed_square(nt, seed=sd, edge_kind=pp, hole_kind=pp), k) for nt, sd, k in cfg]
    npts = sum(c.n for c, _ in clouds)
    log(f"[batch-flow] {len(clouds)} clouds, {npts} points, generated in {time.perf_counter() - t0:.1f}s")
    ctx = R.Context(0)
    rho, mu, co, nsteps = 1.0, 1.0 / 40.0, 1.0, 3
    dcs = [R.DeviceCloud.from_numpy(c) for c, _ in clouds]
    ks = [k for _, k in clouds]
    R.rbffd_build_stencils_batched(ctx, dcs, ks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nbrs, ws, _ = R.rbffd_build_stencils_batched(ctx, dcs, ks)
    torch.cuda.synchronize()
    t_st = time.perf_counter() - t0
    ops = [R.rbffd_assemble(ctx, dc, nb, w, k) for dc, nb, w, k in zip(dcs, nbrs, ws, ks)]
    torch.cuda.synchronize()
    t_as = time.perf_counter() - t0 - t_st
    del nbrs, ws
    log(f"[batch-flow] batched stencil build {1e3 * t_st:.0f} ms, assembly {1e3 * t_as:.0f} ms")
    from types import SimpleNamespace
    solvers = [SimpleNamespace(ops=o) for o in ops]
    dts, fields = [], []
    for (c, _), o in zip(clouds, ops):
        vel, p = W.flow_fields(c)
        dts.append(2.0 * co / R.rbffd_convdiff_lambda(ctx, o, torch.tensor(vel, device="cuda"), rho, mu))
        fields.append((vel, p))
    kw = dict(tol_krylov=1e-8, max_outer=5, max_krylov=20000)

    def state():
        return ([torch.tensor(v, device="cuda") for v, _ in fields], [torch.tensor(v, device="cuda") for v, _ in fields],
                [torch.tensor(p, device="cuda") for _, p in fields])

    bcs = [(torch.tensor(v, device="cuda"), torch.tensor(p, device="cuda")) for v, p in fields]

    def run(batched):
        u, up, p = state()
        eps = [None] * len(clouds)
        stats = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for step in range(nsteps):
            alpha = R.BDF1 if step == 0 else R.BDF2
            tols = [R.outer_tolerance(dt, e, first=step == 0) for dt, e in zip(dts, eps)]
            if batched:
                st = R.simple_step_batched(ctx, [sv.ops for sv in solvers], u, up, p, [b[0] for b in bcs], rho, mu,
                                           dts, alpha=alpha, tol_outer=tols, p_bc=[b[1] for b in bcs], **kw)
            else:
                st = [R.simple_step(ctx, sv.ops, u[j], up[j], p[j], bcs[j][0], rho, mu, dts[j], alpha,
                                    tol_outer=tols[j], p_bc=bcs[j][1], **kw) for j, sv in enumerate(solvers)]
            eps = [s_["eps_steady"] for s_ in st]
            stats.append(st)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, [x.cpu().numpy() for x in u], stats

    run(True)
    t_b, u_b, st_b = run(True)
    t_s, u_s, st_s = run(False)
    diff = max(float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)) for a, b in zip(u_b, u_s))
    pi_b = sum(c.n * (s_["krylov_mom"] + s_["krylov_p"]) for st in st_b for (c, _), s_ in zip(clouds, st))
    ok_b = sum(1 for st in st_b for s_ in st if s_["status"] == 0)
    ok_s = sum(1 for st in st_s for s_ in st if s_["status"] == 0)
    out = {
        "metric": METRIC, "value": round(len(clouds) * nsteps / t_b, 2), "unit": "instance time steps/s",
        "n_gpus": 1, "steps": nsteps, "warmup": nsteps, "ms_per_step": round(t_b / nsteps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(clouds)} holed-square Kovasznay instances (0-4 holes, 500-50k points "
                               "log-uniform, k=2-5, q=2m; no-slip holes with prescribed pressure on edges and "
                               f"holes), {nsteps} BDF steps each at Co {co}, outer tolerance of Sec. 3.2 "
                               "(<= 5 outer iterations), Krylov to 1e-8", "instances": len(clouds), "points": npts},
        "batched": {"instance_steps_per_s": round(len(clouds) * nsteps / t_b, 2), "wall_ms": round(t_b * 1e3, 1),
                    "M_point_iters_per_s": round(pi_b / t_b / 1e6, 1), "steps_converged": f"{ok_b}/{len(clouds) * nsteps}"},
        "one_at_a_time": {"instance_steps_per_s": round(len(clouds) * nsteps / t_s, 2), "wall_ms": round(t_s * 1e3, 1),
                          "steps_converged": f"{ok_s}/{len(clouds) * nsteps}"},
        "speedup_batched_vs_one_at_a_time": round(t_s / t_b, 2),
        "stencils_batched_ms": round(t_st * 1e3, 1), "assembly_ms": round(t_as * 1e3, 1),
        "max_rel_diff_u_batched_vs_one_at_a_time": diff,
    }
    log(f"[batch-flow] batched {out['batched']}, one at a time {out['one_at_a_time']}, diff {diff:.1e}")
    print(json.dumps(out), flush=True)
    for sv in solvers:
        sv.ops.free()
    ctx.close()


def batch_bench(args):
    """The batched configuration: independent holed-square clouds (0-4 holes,
    prescribed pressure on the outer edges and the holes) with sizes
    log-uniform over 500-50k points and degrees 2-5 (q = 2m), one converged
    pressure-correction solve each at 1e-6 relative residual: one batched launch
    sequence against the same solves one at a time (plain FP64 path)."""
    import torch

    import paper_2106_07616_amd as R
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    R.lib()
    cfg = W.config_c3_sizes(args.batch_count)
    t0 = time.perf_counter()
    # p' = 0 on every boundary point (prescribed pressure): the homogeneous
    # Neumann closure on the holes leaves many of these systems beyond plain
    # Jacobi-BiCGSTAB
    clouds = [(W.holed_square(nt, seed=sd, edge_kind=W.PRESCRIBED_PRESSURE, hole_kind=W.PRESCRIBED_PRESSURE), k)
              for nt, sd, k in cfg]
    log(f"[batch] {len(clouds)} clouds, {sum(c.n for c, _ in clouds)} points, generated in {time.perf_counter() - t0:.1f}s")
    ctx = R.Context(0)
    dcs = [R.DeviceCloud.from_numpy(c) for c, _ in clouds]
    ks = [k for _, k in clouds]
    # stencils and operators cloud by cloud, then with the batched build (one
    # weight launch per register width), then assembly; FP64 operators plus FP32 copies
    for rep_ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one = [R.Solver(ctx, dc, k, precision=R.RBFFD_FP32_MATRIX) for dc, k in zip(dcs, ks)]
        torch.cuda.synchronize()
        t_build_one = time.perf_counter() - t0
        for sv in one:
            sv.ops.free()
        del one
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nbrs, ws, _ = R.rbffd_build_stencils_batched(ctx, dcs, ks)
        t_stencils_b = time.perf_counter() - t0
        ops_b = [R.rbffd_assemble(ctx, dc, nb, w, k, precision=R.RBFFD_FP32_MATRIX)
                 for dc, nb, w, k in zip(dcs, nbrs, ws, ks)]
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        if rep_ == 0:
            for o in ops_b:
                o.free()
    del nbrs, ws
    log(f"[batch] stencils + operators: cloud by cloud {t_build_one * 1e3:.1f} ms, batched build "
        f"{t_build * 1e3:.1f} ms (stencils {t_stencils_b * 1e3:.1f} ms)")
    from types import SimpleNamespace
    solvers = [SimpleNamespace(ops=o) for o in ops_b]
    npts = sum(c.n for c, _ in clouds)
    rhs = [torch.tensor(np.random.default_rng(5000 + j).standard_normal(c.n), device="cuda")
           for j, (c, _) in enumerate(clouds)]
    tol = 1e-6

    seq_status = []

    def sequential():
        lat, its = [], []
        xs = []
        seq_status.clear()
        for sv, b in zip(solvers, rhs):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            st = R.poisson_solve(ctx, sv.ops, b, x, tol=tol, max_iter=20000, allow_noconv=True)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ta)
            its.append(st["iters"])
            seq_status.append(st["status"])
            xs.append(x)
        return lat, its, xs

    def batched(pc=R.RBFFD_PREC_JACOBI, precision=R.RBFFD_FP64):
        xs = [torch.zeros_like(b) for b in rhs]
        torch.cuda.synchronize()
        ta = time.perf_counter()
        st = R.poisson_solve_batched(ctx, [sv.ops for sv in solvers], rhs, xs, tol=tol, max_iter=20000,
                                     allow_noconv=True, preconditioner=pc, precision=precision)
        torch.cuda.synchronize()
        return time.perf_counter() - ta, st, xs

    sequential()
    lat, its, xseq = sequential()
    batched()
    t_batch, stb, xb = batched()
    batched(R.RBFFD_PREC_BLOCK64)
    t_bj, stbj, xbj = batched(R.RBFFD_PREC_BLOCK64)
    ok_bj = [j for j, s_ in enumerate(stbj) if s_["status"] == 0 and seq_status[j] == 0]
    diff_bj = max((float((xbj[j] - xseq[j]).abs().max() / xseq[j].abs().max()) for j in ok_bj), default=None)
    batched(R.RBFFD_PREC_BLOCK64, R.RBFFD_FP32_MATRIX)
    t_mx, stmx, xmx = batched(R.RBFFD_PREC_BLOCK64, R.RBFFD_FP32_MATRIX)
    ok_mx = [j for j, s_ in enumerate(stmx) if s_["status"] == 0 and seq_status[j] == 0]
    diff_mx = max((float((xmx[j] - xseq[j]).abs().max() / xseq[j].abs().max()) for j in ok_mx), default=None)
    t_seq = sum(lat)
    ok = [j for j, s_ in enumerate(stb) if s_["status"] == 0 and seq_status[j] == 0]
    diff = max((float((xb[j] - xseq[j]).abs().max() / xseq[j].abs().max()) for j in ok), default=None)
    bad = [(clouds[j][0].name, clouds[j][1], stb[j]["status"], stb[j]["relres"]) for j in range(len(stb))
           if stb[j]["status"] != 0]
    if bad:
        log(f"[batch] systems that did not converge: {bad[:10]}")
    point_iters = sum(c.n * s_["iters"] for (c, _), s_ in zip(clouds, stb))
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC, "value": round(len(solvers) / t_batch, 3), "unit": "converged solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(solvers)} holed-square clouds (seeds 1000+i), {npts} points in total, "
                               f"500-50k points each, k=2..5, q=2m; one pressure-correction solve each at "
                               f"relative residual {tol:g}, batched", "instances": len(solvers), "points": npts},
        "batched": {"solves_per_s": round(len(solvers) / t_batch, 3), "wall_ms": round(t_batch * 1e3, 3),
                    "M_point_iters_per_s": round(point_iters / t_batch / 1e6, 1),
                    "iters_median": int(np.median([s_["iters"] for s_ in stb])),
                    "converged": int(sum(s_["status"] == 0 for s_ in stb)),
                    "max_true_relres": float(max(s_["relres"] for s_ in stb))},
        "sequential_fp64": {"solves_per_s": round(len(solvers) / t_seq, 3), "wall_ms": round(t_seq * 1e3, 3),
                            "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                            "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                            "iters_median": int(np.median(its)),
                            "converged": int(sum(st_ == 0 for st_ in seq_status))},
        "batched_block_jacobi": {"solves_per_s": round(len(solvers) / t_bj, 3), "wall_ms": round(t_bj * 1e3, 3),
                                 "M_point_iters_per_s": round(sum(c.n * s_["iters"] for (c, _), s_ in
                                                                  zip(clouds, stbj)) / t_bj / 1e6, 1),
                                 "iters_median": int(np.median([s_["iters"] for s_ in stbj])),
                                 "converged": int(sum(s_["status"] == 0 for s_ in stbj)),
                                 "max_true_relres": float(max(s_["relres"] for s_ in stbj)),
                                 "max_rel_diff_vs_sequential": diff_bj},
        "batched_fp32_matrix_block_jacobi": {
            "solves_per_s": round(len(solvers) / t_mx, 3), "wall_ms": round(t_mx * 1e3, 3),
            "iters_median": int(np.median([s_["iters"] for s_ in stmx])),
            "converged": int(sum(s_["status"] == 0 for s_ in stmx)),
            "max_true_relres": float(max(s_["relres"] for s_ in stmx)),
            "max_rel_diff_vs_sequential": diff_mx,
            "note": "FP32 matrix values in the Krylov SpMVs, FP64 vectors, FP64 residual refinement"},
        "speedup_batched_vs_sequential": round(t_seq / t_batch, 3),
        "speedup_batched_block_jacobi_vs_sequential": round(t_seq / t_bj, 3),
        "speedup_batched_fp32_matrix_block_jacobi_vs_sequential": round(t_seq / t_mx, 3),
        "max_rel_diff_batched_vs_sequential": diff,
        "stencils_and_assembly_ms": {"batched_build": round(t_build * 1e3, 1),
                                     "batched_stencils_alone": round(t_stencils_b * 1e3, 1),
                                     "cloud_by_cloud": round(t_build_one * 1e3, 1)},
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """The serving configuration with flow requests: a Poisson-arrival stream,
    70% 2D (half Kovasznay squares, half holed squares, 2k-200k points) and
    30% 3D Beltrami cubes (50k-500k points), degree 2-4, q = 2m, prescribed
    pressure on every boundary. A request is its stencils and operators and
    three BDF time steps at Co 5 (the outer tolerance of Sec. 3.2, at most 5
    outer iterations, Krylov solves to 1e-6). The arrival rate is 0.7 x the
    closed-loop rate of one request at a time; the same arrival sequence is
    served one at a time and by concurrent slots (paper_2106_07616_amd.serve),
    in FP64 and with FP32 matrix values and the block-Jacobi pressure solve."""
    import torch

    import paper_2106_07616_amd as R
    import workloads as W
    from paper_2106_07616_amd import serve as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    R.lib()
    rng = np.random.default_rng(5)
    t0 = time.perf_counter()
    reqs = []
    pp = W.PRESCRIBED_PRESSURE
    for i in range(args.serve_requests):
        u = rng.random()
        k = int(rng.integers(2, 5))
        if u < 0.7:
            npts = int(round(np.exp(rng.uniform(np.log(2e3), np.log(2e5)))))
            if rng.random() < 0.5:
                c = W.kovasznay_square(nx=max(8, int(round(np.sqrt(npts)))), seed=5000 + i, boundary_kind=pp)
            else:
                c = W.holed_square(npts, seed=5000 + i, edge_kind=pp, hole_kind=pp)
        else:
            npts = int(round(np.exp(rng.uniform(np.log(5e4), np.log(5e5)))))
            c = W.beltrami_cube(n=max(8, int(round(npts ** (1 / 3)))), seed=5000 + i)
        reqs.append((c, k))
    npts_all = sum(c.n for c, _ in reqs)
    log(f"[serve] {len(reqs)} flow requests, {npts_all} points, generated in {time.perf_counter() - t0:.1f}s")
    budget = 32 << 30
    warm = min(args.serve_warmup, len(reqs))

    def make(j, precision=R.RBFFD_FP64, pc=R.RBFFD_PREC_JACOBI):
        c, k = reqs[j]
        return S.FlowRequest(c, k, steps=3, courant=5.0, tol_krylov=1e-6, max_outer=5, tag=j, precision=precision,
                             preconditioner=pc, flow_fields=W.flow_fields)

    # closed-loop rate of one request at a time on the warm-up requests
    ctx = R.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(warm):
        S.run_request(ctx, make(j))
    torch.cuda.synchronize()
    closed = warm / (time.perf_counter() - t0)
    ctx.close()
    lam = 0.7 * closed
    arrivals = np.cumsum(np.random.default_rng(6).exponential(1.0 / lam, len(reqs)))
    log(f"[serve] closed-loop one-at-a-time rate {closed:.2f}/s, offered load {lam:.2f}/s")

    def run(slots, precision=R.RBFFD_FP64, pc=R.RBFFD_PREC_JACOBI):
        res, peak = S.serve_stream([make(j, precision, pc) for j in range(len(reqs))], arrivals, slots=slots,
                                   hbm_budget=budget)
        lat = np.array([r.latency for r in res[warm:]]) * 1e3
        fin = max(arrivals[j] + res[j].latency for j in range(warm, len(reqs)))
        span = fin - arrivals[warm]
        steps_ok = sum(1 for r in res[warm:] for st_ in r.stats if st_["status"] == 0)
        pi = sum(r_c.n * (st_["krylov_mom"] + st_["krylov_p"]) for (r_c, _), r in zip(reqs[warm:], res[warm:])
                 for st_ in r.stats)
        out = {"solves_per_s": round((len(reqs) - warm) / span, 3), "p50_ms": round(float(np.percentile(lat, 50)), 1),
               "p99_ms": round(float(np.percentile(lat, 99)), 1), "mean_ms": round(float(lat.mean()), 1),
               "M_point_iters_per_s": round(pi / span / 1e6, 1), "peak_concurrent": int(peak),
               "steps_converged": f"{steps_ok}/{3 * (len(reqs) - warm)}",
               "finite_results": int(sum(1 for r in res[warm:] if np.isfinite(r.u).all()))}
        return out, res

    seq, res_seq = run(1)
    log(f"[serve] one at a time: {seq}")
    cb, res_cb = run(4)
    log(f"[serve] 4 concurrent slots: {cb}")
    same = all(np.array_equal(a.u, b.u) and np.array_equal(a.p, b.p) for a, b in zip(res_seq, res_cb))
    cbm, _ = run(4, R.RBFFD_FP32_MATRIX, R.RBFFD_PREC_BLOCK64)
    log(f"[serve] 4 concurrent slots, FP32 matrix + block-Jacobi: {cbm}")
    out = {
        "metric": METRIC, "value": cb["solves_per_s"], "unit": "converged solves/s", "n_gpus": 1,
        "steps": len(reqs) - warm, "warmup": warm, "ms_per_step": cb["mean_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Poisson-arrival stream of {len(reqs)} flow requests (first {warm} excluded): 70% 2D "
                               "Kovasznay/holed squares 2k-200k points, 30% 3D Beltrami cubes 50k-500k points, "
                               "k=2-4, q=2m, prescribed pressure on the boundary; per request stencils, operators "
                               "and 3 BDF steps at Co 5 (outer tolerance min(1e-4, dt eps_s), <= 5 outer "
                               "iterations, Krylov to 1e-6); offered load "
                               f"{lam:.2f}/s = 0.7 x one-at-a-time closed-loop rate; HBM budget 32 GiB",
                   "requests": len(reqs), "points": npts_all},
        "one_at_a_time_fp64": seq, "concurrent_slots_fp64": cb, "concurrent_slots_fp32_matrix_block_jacobi": cbm,
        "results_equal_one_at_a_time_and_concurrent": bool(same),
        "p99_ratio_one_at_a_time_over_concurrent": round(seq["p99_ms"] / cb["p99_ms"], 3),
    }
    print(json.dumps(out), flush=True)


def serve_poisson_bench(args):
    """The serving configuration: a Poisson-arrival stream of solve requests,
    70% 2D (half Kovasznay squares, half holed squares, 2k-200k points) and 30%
    3D Beltrami cubes (50k-500k points), degree 2-4, q = 2m,
    prescribed pressure on every boundary. A request is served when its
    stencils and operators are built on the device and its pressure-correction
    solve (random right-hand side) reaches 1e-6. The arrival rate is 0.7 x the
    closed-loop rate of the one-at-a-time FP64 path; the same arrival sequence
    is served with continuous batching (rbffd_server) and one at a time."""
    import torch

    import paper_2106_07616_amd as R
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    R.lib()
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(args.serve_requests):
        u = rng.random()
        if u < 0.7:
            npts = int(round(np.exp(rng.uniform(np.log(2e3), np.log(2e5)))))
            k = int(rng.integers(2, 5))
            if rng.random() < 0.5:
                c = W.kovasznay_square(nx=max(8, int(round(np.sqrt(npts)))), seed=5000 + i,
                                       boundary_kind=W.PRESCRIBED_PRESSURE)
            else:
                c = W.holed_square(npts, seed=5000 + i, edge_kind=W.PRESCRIBED_PRESSURE,
                                   hole_kind=W.PRESCRIBED_PRESSURE)
        else:
            npts = int(round(np.exp(rng.uniform(np.log(5e4), np.log(5e5)))))
            k = int(rng.integers(2, 5))
            c = W.beltrami_cube(n=max(8, int(round(npts ** (1 / 3)))), seed=5000 + i)
        reqs.append((c, k, np.random.default_rng(9000 + i).standard_normal(c.n)))
    log(f"[serve] {len(reqs)} requests, {sum(r[0].n for r in reqs)} points")
    budget = 32 << 30
    ctx = R.Context(0, budget)
    tol = 1e-6

    def build_in(cx):
        def build(j):
            c, k, b = reqs[j]
            sv = R.Solver(cx, c, k, precision=R.RBFFD_FP32_MATRIX)   # FP64 operators plus FP32 copies
            return sv, torch.tensor(b, device="cuda")
        return build

    build = build_in(ctx)

    # closed-loop rate of the one-at-a-time path on the first requests
    warm = min(args.serve_warmup, len(reqs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(warm):
        sv, b = build(j)
        x = torch.zeros_like(b)
        R.poisson_solve(ctx, sv.ops, b, x, tol=tol, max_iter=20000, allow_noconv=True)
        sv.ops.free()
    torch.cuda.synchronize()
    closed_rate = warm / (time.perf_counter() - t0)
    lam = 0.7 * closed_rate
    arrivals = np.cumsum(np.random.default_rng(6).exponential(1.0 / lam, len(reqs)))
    log(f"[serve] closed-loop one-at-a-time rate {closed_rate:.2f}/s, offered load {lam:.2f}/s")

    def report(lat, fin, iters):
        lat = np.array(lat[warm:]) * 1e3
        span = max(fin[warm:]) - arrivals[warm]
        return {"solves_per_s": round((len(reqs) - warm) / span, 3), "p50_ms": round(float(np.percentile(lat, 50)), 1),
                "p99_ms": round(float(np.percentile(lat, 99)), 1), "mean_ms": round(float(lat.mean()), 1),
                "M_point_iters_per_s": round(sum(reqs[j][0].n * iters[j] for j in range(warm, len(reqs))) /
                                             span / 1e6, 1)}

    # one at a time, FIFO
    lat, fin, iters, conv = [0.0] * len(reqs), [0.0] * len(reqs), [0] * len(reqs), 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(len(reqs)):
        now = time.perf_counter() - t0
        if now < arrivals[j]:
            time.sleep(arrivals[j] - now)
        sv, b = build(j)
        x = torch.zeros_like(b)
        st = R.poisson_solve(ctx, sv.ops, b, x, tol=tol, max_iter=20000, allow_noconv=True)
        torch.cuda.synchronize()
        fin[j] = time.perf_counter() - t0
        lat[j] = fin[j] - arrivals[j]
        iters[j] = st["iters"]
        conv += st["status"] == 0
        sv.ops.free()
    seq = report(lat, fin, iters)
    seq["converged"] = int(conv)
    log(f"[serve] one at a time: {seq}")

    def continuous(pc, precision=R.RBFFD_FP64, builder=None):
        return serve_continuous(args, R, ctx, reqs, arrivals, build, report, tol, pc, precision, builder)

    cb = continuous(R.RBFFD_PREC_JACOBI)
    log(f"[serve] continuous batching: {cb}")
    cbj = continuous(R.RBFFD_PREC_BLOCK64)
    log(f"[serve] continuous batching, block-Jacobi: {cbj}")
    cbm = continuous(R.RBFFD_PREC_BLOCK64, R.RBFFD_FP32_MATRIX)
    log(f"[serve] continuous batching, FP32 matrix + block-Jacobi: {cbm}")
    ctx_b = R.Context(0, budget)
    builder = AsyncBuilder(torch, build_in(ctx_b))
    cba = continuous(R.RBFFD_PREC_BLOCK64, builder=builder)
    builder.close()
    ctx_b.close()
    log(f"[serve] continuous batching, block-Jacobi, operators built on a second stream: {cba}")
    out = {
        "metric": METRIC, "value": cb["solves_per_s"], "unit": "converged solves/s", "n_gpus": 1,
        "steps": len(reqs) - warm, "warmup": warm, "ms_per_step": cb["mean_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Poisson-arrival stream of {len(reqs)} solve requests (first {warm} excluded): 70% 2D "
                               "Kovasznay/holed squares 2k-200k points, 30% 3D Beltrami cubes 50k-500k points, "
                               "k=2-4, q=2m; stencils + operators + pressure-correction solve to 1e-6 per "
                               f"request; offered load {lam:.2f}/s = 0.7 x one-at-a-time closed-loop rate; "
                               f"HBM budget 32 GiB; at most {args.serve_large_limit} solve(s) above "
                               f"{args.serve_large_points} points in the batch at once", "requests": len(reqs)},
        "continuous_batching": cb, "continuous_batching_block_jacobi": cbj,
        "continuous_batching_fp32_matrix_block_jacobi": cbm,
        "continuous_batching_block_jacobi_async_build": cba, "one_at_a_time_fp64": seq,
        "p99_latency_ratio_one_at_a_time_over_batched": round(seq["p99_ms"] / cb["p99_ms"], 3),
        "p99_latency_ratio_one_at_a_time_over_batched_block_jacobi": round(seq["p99_ms"] / cbj["p99_ms"], 3),
        "p99_latency_ratio_one_at_a_time_over_batched_fp32_matrix_block_jacobi": round(seq["p99_ms"] / cbm["p99_ms"],
                                                                                       3),
    }
    ctx.close()
    print(json.dumps(out), flush=True)


class AsyncBuilder:
    """Builds the stencils and operators of arriving requests on a thread of
    its own, under a second library context and on a second stream (default
    priority), while the serving loop keeps the batch iterating. Each request
    is handed over once its stream has finished. Finished requests come back
    through release() and are freed on the same thread: every library call on
    the builder's context stays on one thread (calls on one context must not
    overlap), and the device synchronisation of a free happens off the
    serving loop."""

    def __init__(self, torch, build):
        import queue
        import threading
        self.torch, self.build = torch, build
        self.todo, self.ready = queue.Queue(), queue.Queue()
        self.stream = torch.cuda.Stream()
        self.err = None
        self.pending = 0
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def _run(self):
        try:
            with self.torch.cuda.stream(self.stream):
                while True:
                    j = self.todo.get()
                    if j is None:
                        return
                    if isinstance(j, tuple):   # ("free", solver): release its operators here
                        j[1].ops.free()
                        continue
                    sv, b = self.build(j)
                    self.stream.synchronize()
                    self.ready.put((j, sv, b))
        except BaseException as e:   # handed to the serving loop
            self.err = e
            self.ready.put(None)

    def submit(self, j):
        self.pending += 1
        self.todo.put(j)

    def release(self, sv):
        """Free a finished request's operators on the builder's thread."""
        self.todo.put(("free", sv))

    def take(self, timeout=None):
        """Finished builds: all that are ready, or (with a timeout) the next one."""
        import queue
        out = []
        try:
            item = self.ready.get(timeout=timeout) if timeout else self.ready.get_nowait()
            while True:
                if item is None:
                    raise RuntimeError("operator build failed") from self.err
                out.append(item)
                item = self.ready.get_nowait()
        except queue.Empty:
            pass
        self.pending -= len(out)
        return out

    def close(self):
        self.todo.put(None)
        self.thread.join()


def serve_continuous(args, R, ctx, reqs, arrivals, build, report, tol, pc, precision, builder=None):
    """Serve the arrival sequence with continuous batching (rbffd_server). With
    a builder, requests' operators are built by it while the batch runs."""
    import torch

    warm = min(args.serve_warmup, len(reqs))
    server = R.Server(ctx)
    lat, fin, iters, conv = [0.0] * len(reqs), [0.0] * len(reqs), [0] * len(reqs), 0
    live = {}
    nxt = 0
    peak = 0
    large = args.serve_large_points
    held = []   # arrived requests waiting for a large-system slot
    prebuilt = {}   # request -> (solver, right-hand side) finished by the builder
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < len(reqs):
        now = time.perf_counter() - t0
        # admit every request that has arrived, while the HBM budget allows; at
        # most serve_large_limit systems above serve_large_points run at once, so
        # large solves do not share the device with each other
        while nxt < len(reqs) and arrivals[nxt] <= now:
            if builder is None:
                held.append(nxt)
            else:
                builder.submit(nxt)
            nxt += 1
        if builder is not None:
            for j, sv, b in builder.take():
                prebuilt[j] = (sv, b)
                held.append(j)
        n_large = sum(1 for j, _ in live.values() if reqs[j][0].n > large)
        for j in list(held):
            if reqs[j][0].n > large and n_large >= args.serve_large_limit:
                continue
            try:
                sv, b = prebuilt.pop(j) if builder is not None else build(j)
                x = torch.zeros_like(b)
                t = server.submit(sv.ops, b, x, tol=tol, max_iter=20000, preconditioner=pc, precision=precision)
            except R.RbffdError as e:
                if e.code != -2:
                    raise
                if builder is not None:
                    prebuilt[j] = (sv, b)
                break   # over budget: admit after some solves finish
            live[t] = (j, sv)
            held.remove(j)
            n_large += reqs[j][0].n > large
        active = server.run(args.serve_chunk)
        peak = max(peak, active)
        for t, st in server.poll():
            j, sv = live.pop(t)
            fin[j] = time.perf_counter() - t0
            lat[j] = fin[j] - arrivals[j]
            iters[j] = st["iters"]
            conv += st["status"] == 0
            if builder is not None:
                builder.release(sv)   # its context belongs to the builder's thread
            else:
                sv.ops.free()
            done += 1
        if active == 0 and not held and builder is not None and builder.pending > 0:
            for j, sv, b in builder.take(timeout=0.001):   # nothing to iterate: wait for a build
                prebuilt[j] = (sv, b)
                held.append(j)
        elif active == 0 and not held and nxt < len(reqs):
            wait = arrivals[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
    server.close()
    cb = report(lat, fin, iters)
    cb["converged"] = int(conv)
    cb["peak_concurrent_solves"] = int(peak)
    return cb


def hbm_resident_section(args, R, W, torch, ctx):
    """The 1.06M-point Ethier-Steinman cube (3D, k = 3, q = 40): its working set
    exceeds the 256 MB Infinity Cache, so the BiCGSTAB kernels run from HBM.
    Measured here: the FP64 iteration's kernel times against the HBM roofline,
    converged pressure-correction solves at 1e-6 in FP64 and in both mixed
    modes (each preconditioner), and one time step (three outer iterations,
    Krylov to 1e-10) per precision with the per-field error against the
    closed-form flow and against the FP64 step."""
    dev = "cuda"
    k, co, rho, nu = 3, 10.0, 1.0, 0.01
    t0 = time.perf_counter()
    cloud = W.beltrami_cube(n=100)
    log(f"[bench] hbm section: cloud {cloud.name} n={cloud.n} generated in {time.perf_counter() - t0:.1f}s")
    n = cloud.n
    dcloud = R.DeviceCloud.from_numpy(cloud, dev)
    q, _, _ = R.rbffd_stencil_sizes(3, k)
    nbr, w, _ = R.rbffd_build_stencils(ctx, dcloud, k)   # first build: workspace set-up
    del nbr, w
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nbr, w, _ = R.rbffd_build_stencils(ctx, dcloud, k)
    torch.cuda.synchronize()
    t_st = time.perf_counter() - t0
    ops = R.rbffd_assemble(ctx, dcloud, nbr, w, k, precision=R.RBFFD_FP32_IR)
    torch.cuda.synchronize()
    t_as = time.perf_counter() - t0 - t_st
    del nbr, w
    rhs = torch.tensor(np.random.default_rng(1).standard_normal(n), device=dev)
    xk = torch.zeros(n, dtype=torch.float64, device=dev)
    kt = R.rbffd_krylov_kernel_times(ctx, ops, rhs, xk, reps=args.kernel_reps)

    def frac(b, us):
        return round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)

    solves = {}
    for name, prec, pc in (("fp64", R.RBFFD_FP64, R.RBFFD_PREC_JACOBI),
                           ("fp32_matrix_fp64_vectors", R.RBFFD_FP32_MATRIX, R.RBFFD_PREC_JACOBI),
                           ("fp32_vectors_and_matrix", R.RBFFD_FP32_IR, R.RBFFD_PREC_JACOBI),
                           ("fp64_block_jacobi", R.RBFFD_FP64, R.RBFFD_PREC_BLOCK64),
                           ("fp32_matrix_fp64_vectors_block_jacobi", R.RBFFD_FP32_MATRIX, R.RBFFD_PREC_BLOCK64),
                           ("fp32_vectors_and_matrix_block_jacobi", R.RBFFD_FP32_IR, R.RBFFD_PREC_BLOCK64)):
        lat, its, rel = [], [], []
        for rep in range(1 + args.hbm_solve_reps):
            xk.zero_()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            st = R.poisson_solve(ctx, ops, rhs, xk, tol=1e-6, max_iter=20000, precision=prec, allow_noconv=True,
                                 preconditioner=pc)
            torch.cuda.synchronize()
            if rep:
                lat.append(time.perf_counter() - ta)
                its.append(st["iters"])
                rel.append(st["relres"])
        solves[name] = {"solves_per_s": round(len(lat) / sum(lat), 2), "iters": int(np.median(its)),
                        "max_true_relres": float(max(rel)), "ms": round(float(np.median(lat)) * 1e3, 2)}
    for name in list(solves):
        base = "fp64_block_jacobi" if name.endswith("block_jacobi") else "fp64"
        solves[name]["speedup_vs_fp64_same_preconditioner"] = round(
            solves[name]["solves_per_s"] / solves[base]["solves_per_s"], 3)
    log(f"[bench] hbm section solves at 1e-6: {solves}")

    # one time step per precision, three outer iterations, Krylov to 1e-10
    vel0, p0 = W.flow_fields(cloud, 0.0)
    u0 = torch.tensor(vel0, device=dev)
    dt = 2.0 * co / R.binding.rbffd_convdiff_lambda(ctx, ops, u0, rho, nu, 200)
    velm, _ = W.flow_fields(cloud, -dt)
    ub_np, pb_np = W.flow_fields(cloud, dt)
    ubc, pbc = torch.tensor(ub_np, device=dev), torch.tensor(pb_np, device=dev)
    steps = {}
    fields = {}
    for name, prec, pc in (("fp64", R.RBFFD_FP64, R.RBFFD_PREC_JACOBI),
                           ("fp64_block_jacobi", R.RBFFD_FP64, R.RBFFD_PREC_BLOCK64),
                           ("fp32_matrix_fp64_vectors_block_jacobi", R.RBFFD_FP32_MATRIX, R.RBFFD_PREC_BLOCK64),
                           ("fp32_vectors_and_matrix_block_jacobi", R.RBFFD_FP32_IR, R.RBFFD_PREC_BLOCK64)):
        u, up, p = u0.clone(), torch.tensor(velm, device=dev), torch.tensor(p0, device=dev)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        st = R.simple_step(ctx, ops, u, up, p, ubc, rho, nu, dt, R.BDF2, tol_outer=0.0, tol_krylov=1e-10,
                           max_outer=3, max_krylov=20000, precision=prec, p_bc=pbc, preconditioner=pc)
        torch.cuda.synchronize()
        tm = time.perf_counter() - ta
        fields[name] = (u, p)
        ue = np.abs(u.cpu().numpy() - ub_np)
        steps[name] = {"ms": round(tm * 1e3, 1), "status": st["status"],
                       "krylov_iters": st["krylov_mom"] + st["krylov_p"],
                       "max_abs_error_vs_exact": dict(zip("uvw", [float(x) for x in ue.max(axis=1)]),
                                                      p=float(np.abs(p.cpu().numpy() - pb_np).max()))}
    u64, p64 = fields["fp64"]
    for name in steps:
        if name == "fp64":
            continue
        u, p = fields[name]
        steps[name]["rel_diff_vs_fp64"] = dict(
            zip("uvw", [float((u[e] - u64[e]).abs().max() / u64[e].abs().max()) for e in range(3)]),
            p=float((p - p64).abs().max() / p64.abs().max()))
        base = "fp64_block_jacobi" if name.endswith("block_jacobi") else "fp64"
        steps[name]["speedup_vs_fp64_same_preconditioner"] = round(steps[base]["ms"] / steps[name]["ms"], 3)
    log(f"[bench] hbm section steps: {steps}")
    ops.free()
    return {
        "workload": f"Ethier-Steinman Beltrami flow nu=0.01 on [0,1]^3, {n} points (100^3 jittered lattice + faces, "
                    f"seed 4), PHS r^3 + degree-3 polynomials, q={q}, Co 10 (dt={dt:.5f})",
        "stencils_ms": round(t_st * 1e3, 2), "assemble_ms": round(t_as * 1e3, 2),
        "roofline_fp64_iteration": {
            "k_t": {"us": round(kt["kt"], 2), "bytes": kt_bytes(n, q), "frac": frac(kt_bytes(n, q), kt["kt"])},
            "k_v": {"us": round(kt["kv"], 2), "bytes": kv_bytes(n, q), "frac": frac(kv_bytes(n, q), kt["kv"])},
            "k_s_us": round(kt["ks"], 2), "k_x_us": round(kt["kx"], 2),
            "iteration": {"us": round(kt["iteration"], 2), "bytes": iteration_bytes(n, q),
                          "frac": frac(iteration_bytes(n, q), kt["iteration"])},
            "peak_gbs": HBM_PEAK_GBS,
            "note": "working set ~%.0f MB, beyond the 256 MB Infinity Cache: HBM-resident" %
                    (iteration_bytes(n, q) / 1e6)},
        "converged_solves_1e-6": solves,
        "time_step_3_outer_iterations": steps,
    }


def weights_only(args):
    """Stencil builds of one cloud (kNN and weights), three times after one
    untimed build, with the mean time and the weights' points per second."""
    import torch

    import paper_2106_07616_amd as R
    import workloads as W
    cloud, k = {"tg250k_k4": (lambda: W.taylor_green_disk(), 4),
                "cube40_k4": (lambda: W.beltrami_cube(n=40), 4),
                "tg60k_k6": (lambda: W.taylor_green_disk(r=0.021), 6),
                "beltrami100_k3": (lambda: W.beltrami_cube(n=100), 3)}[args.weights_only]
    cloud = cloud()
    ctx = R.Context(0)
    dc = R.DeviceCloud.from_numpy(cloud)
    R.rbffd_build_stencils(ctx, dc, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        R.rbffd_build_stencils(ctx, dc, k)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    q, m, _ = R.rbffd_stencil_sizes(cloud.dim, k)
    print(json.dumps({"cloud": args.weights_only, "n": cloud.n, "unknowns": q + m, "build_ms": round(dt * 1e3, 3),
                      "points_per_s": round(cloud.n / dt, 0)}), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--max-outer", type=int, default=20)
    ap.add_argument("--tol-outer", type=float, default=None,
                    help="fixed outer tolerance of every step (default: the rule of Sec. 3.2, 1e-4 for the first "
                         "step of the run, then min(1e-4, dt eps_s))")
    ap.add_argument("--tol-krylov", type=float, default=1e-8,
                    help="relative tolerance of the momentum and pressure-correction Krylov solves")
    ap.add_argument("--precision", choices=["fp64", "fp32ir", "fp32matrix"], default="fp64")
    ap.add_argument("--spmv-reps", type=int, default=200)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--solve-reps", type=int, default=5)
    ap.add_argument("--mixed-step", action="store_true",
                    help="also run the step with both mixed-precision modes and with the block-Jacobi "
                         "pressure preconditioner, and report per-field differences")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm-section", action="store_true",
                    help="skip the 1.06M-point HBM-resident measurements added to the default line")
    ap.add_argument("--hbm-solve-reps", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["batch", "batch-flow", "serve", "serve-poisson", "post"],
                    default="taylor_green")
    ap.add_argument("--serve-requests", type=int, default=550)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-chunk", type=int, default=16)
    ap.add_argument("--serve-large-points", type=int, default=200_000)
    ap.add_argument("--serve-large-limit", type=int, default=1)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--cpu-sample-r", type=float, default=0.02)
    ap.add_argument("--cpu-sample-cube", type=int, default=30)
    ap.add_argument("--counters-only", action="store_true",
                    help="run only the SpMV timing, the timed BiCGSTAB kernels and a copy of known size "
                         "(for hardware counter runs)")
    ap.add_argument("--weights-only", choices=["tg250k_k4", "cube40_k4", "tg60k_k6", "beltrami100_k3"], default=None,
                    help="only build the stencils of one cloud a few times (for weight-kernel profiles): the "
                         "250k Taylor-Green disk at degree 4 (45 unknowns), a 40^3 cube at degree 4 (105) or a "
                         "60k Taylor-Green disk at degree 6 (84)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; runs on several GPUs are not supported (pass --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        batch_bench(args)
        return
    if args.workload == "batch-flow":
        batch_flow_bench(args)
        return
    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload == "serve-poisson":
        serve_poisson_bench(args)
        return
    if args.workload == "post":
        post_bench(args)
        return
    if args.weights_only:
        weights_only(args)
        return

    import torch

    import paper_2106_07616_amd as R
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    R.lib()
    dev = "cuda"
    precision = {"fp64": R.RBFFD_FP64, "fp32ir": R.RBFFD_FP32_IR, "fp32matrix": R.RBFFD_FP32_MATRIX}[args.precision]
    k, co, rho, nu = WORKLOADS[args.workload]["k"], 10.0, 1.0, 0.01
    t0 = time.perf_counter()
    cloud = WORKLOADS[args.workload]["make"](W)
    log(f"[bench] cloud {cloud.name}: n={cloud.n} generated in {time.perf_counter() - t0:.1f}s")
    ctx = R.Context(0)
    dcloud = R.DeviceCloud.from_numpy(cloud, dev)
    q, m, _ = R.rbffd_stencil_sizes(cloud.dim, k)
    n = cloud.n

    # time step from the Courant number (computed once, outside the timed region)
    solver = R.Solver(ctx, dcloud, k, precision=precision)
    vel0, p0 = W.flow_fields(cloud, 0.0)
    u0 = torch.tensor(vel0, device=dev)
    dt = solver.dt_from_courant(u0, co, rho, nu)
    velm, _ = W.flow_fields(cloud, -dt)
    ubc_np, pbc_np = W.flow_fields(cloud, dt)
    ubc = torch.tensor(ubc_np, device=dev)
    pbc = torch.tensor(pbc_np, device=dev)
    um1 = torch.tensor(velm, device=dev)
    pt0 = torch.tensor(p0, device=dev)
    log(f"[bench] dt={dt:.5f} (Co {co}) q={q} m={m}")

    # ---- dominant kernel: SpMV of the pressure-correction matrix -------------
    col_exp, _ = solver.ops.export_csr()
    narrow = narrow_fraction(col_exp.cpu().numpy(), n, q)
    del col_exp
    x = torch.tensor(np.sin(cloud.xyz[:, 0]) * np.cos(cloud.xyz[:, 1]), device=dev)
    for _ in range(10):
        solver.ops.apply(cloud.dim + 1, x)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    y = torch.empty_like(x)
    L = R.lib()
    stream = R.binding._stream()
    ev0.record()
    for _ in range(args.spmv_reps):
        L.rbffd_apply(ctx.handle, solver.ops.handle, cloud.dim + 1, R.binding._ptr(x), R.binding._ptr(y), stream)
    ev1.record()
    torch.cuda.synchronize()
    spmv_ms = ev0.elapsed_time(ev1) / args.spmv_reps
    spmv_gbs = spmv_bytes(n, q, narrow) / (spmv_ms * 1e-3) / 1e9
    log(f"[bench] spmv: {spmv_ms * 1e3:.1f} us/launch, {spmv_gbs:.0f} GB/s algorithmic")
    if args.counters_only:
        # the BiCGSTAB kernels as the roofline times them, then the calibration
        # for hardware byte counters: a plain copy of a known size (64 Mi
        # doubles = 512 MiB read + 512 MiB written per launch)
        rhs = torch.tensor(np.random.default_rng(1).standard_normal(n), device=dev)
        xk = torch.zeros(n, dtype=torch.float64, device=dev)
        ktimes = R.rbffd_krylov_kernel_times(ctx, solver.ops, rhs, xk, reps=args.kernel_reps)
        torch.cuda.synchronize()
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"spmv_us": spmv_ms * 1e3, "spmv_gbs": spmv_gbs, "n": n, "q": q,
                          "bytes_per_launch": spmv_bytes(n, q, narrow), "kernel_us": ktimes,
                          "kt_bytes_per_launch": kt_bytes(n, q), "copy_bytes_each_way": src.numel() * 8,
                          "source_sha256": kernel_source_hash()}))
        return

    # ---- pressure-correction BiCGSTAB alone: time per iteration --------------
    rhs = torch.tensor(np.random.default_rng(1).standard_normal(n), device=dev)
    xs = torch.zeros(n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pst = R.poisson_solve(ctx, solver.ops, rhs, xs, tol=1e-10, max_iter=20000, allow_noconv=True)
    torch.cuda.synchronize()
    t_ps = time.perf_counter() - t0
    it_us = t_ps / max(pst["iters"], 1) * 1e6
    log(f"[bench] poisson_solve: {pst['iters']} iterations, {it_us:.1f} us/iteration, relres {pst['relres']:.1e}")

    # ---- kernel times of the BiCGSTAB iteration (HIP events on the stream) ----
    xk = torch.zeros(n, dtype=torch.float64, device=dev)
    ktimes = R.rbffd_krylov_kernel_times(ctx, solver.ops, rhs, xk, reps=args.kernel_reps)
    kt_gbs = kt_bytes(n, q) / (ktimes["kt"] * 1e-6) / 1e9
    log(f"[bench] kernel times (us): {ktimes}; k_t {kt_gbs:.0f} GB/s for {kt_bytes(n, q) / 1e6:.1f} MB")
    del xk

    # ---- converged solves at 1e-6: plain FP64 against FP32 sweeps with FP64
    # refinement, on the same pressure-correction system ----------------------
    ops_mixed = R.rbffd_assemble(ctx, dcloud, solver.nbr, solver.w, k, precision=R.RBFFD_FP32_IR)

    def timed_solves(prec, reps, pc=R.RBFFD_PREC_JACOBI):
        lat, its, rel, fb = [], [], [], []
        for _ in range(reps):
            xs.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = R.poisson_solve(ctx, ops_mixed, rhs, xs, tol=1e-6, max_iter=20000, precision=prec, allow_noconv=True,
                                 preconditioner=pc)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            its.append(st["iters"])
            rel.append(st["relres"])
            fb.append(st["fp64_fallback"])
        lat_ms = np.array(lat) * 1e3
        return {"solves_per_s": round(len(lat) / sum(lat), 2), "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                "p99_ms": round(float(np.percentile(lat_ms, 99)), 3), "iters": int(np.median(its)),
                "max_true_relres": float(max(rel)), "fp64_fallback": int(max(fb))}

    timed_solves(R.RBFFD_FP64, 1)
    solves64 = timed_solves(R.RBFFD_FP64, args.solve_reps)
    timed_solves(R.RBFFD_FP32_IR, 1)
    solves32 = timed_solves(R.RBFFD_FP32_IR, args.solve_reps)
    timed_solves(R.RBFFD_FP32_MATRIX, 1)
    solves32m = timed_solves(R.RBFFD_FP32_MATRIX, args.solve_reps)
    timed_solves(R.RBFFD_FP64, 1, R.RBFFD_PREC_BLOCK64)
    solves64b = timed_solves(R.RBFFD_FP64, args.solve_reps, R.RBFFD_PREC_BLOCK64)
    timed_solves(R.RBFFD_FP32_IR, 1, R.RBFFD_PREC_BLOCK64)
    solves32b = timed_solves(R.RBFFD_FP32_IR, args.solve_reps, R.RBFFD_PREC_BLOCK64)
    timed_solves(R.RBFFD_FP32_MATRIX, 1, R.RBFFD_PREC_BLOCK64)
    solves32mb = timed_solves(R.RBFFD_FP32_MATRIX, args.solve_reps, R.RBFFD_PREC_BLOCK64)
    ops_mixed.free()
    log(f"[bench] solves at 1e-6: fp64 {solves64}  fp32 {solves32}  fp32 matrix {solves32m}  "
        f"fp64 block-Jacobi {solves64b}  fp32 block-Jacobi {solves32b}  fp32 matrix block-Jacobi {solves32mb}")

    # ---- the benchmark step: consecutive time steps of the run ----------------
    # Every step is one pass of the whole hot path: stencils and weights
    # (rbffd_build_stencils), assembly (rbffd_assemble) and one BDF2 time step
    # (simple_step) that advances the flow from t^n to t^{n+1}. The Dirichlet
    # data of every step are computed and copied to the device before the timed
    # region starts.
    nsteps = args.warmup + args.steps
    bc_dev = []
    for i in range(nsteps):
        ub, pb = W.flow_fields(cloud, (i + 1) * dt)
        bc_dev.append((torch.tensor(ub, device=dev), torch.tensor(pb, device=dev)))
    torch.cuda.synchronize()
    state = {"u": u0.clone(), "up": um1.clone(), "p": pt0.clone(), "i": 0, "eps": None}

    def outer_tol():
        # Sec. 3.2: 1e-4 at the first step, then min(1e-4, dt eps_s of the last step)
        if args.tol_outer is not None:
            return args.tol_outer
        return R.outer_tolerance(dt, state["eps"], first=state["i"] == 0)
    phase_s = {"stencils": 0.0, "assemble": 0.0, "time_step": 0.0}

    def one_step():
        ta = time.perf_counter()
        nbr, w, _ = R.rbffd_build_stencils(ctx, dcloud, k)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ops = R.rbffd_assemble(ctx, dcloud, nbr, w, k, precision=precision)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        phase_s["stencils"] += tb - ta
        phase_s["assemble"] += tc - tb
        ub, pb = bc_dev[state["i"]]
        st = R.simple_step(ctx, ops, state["u"], state["up"], state["p"], ub, rho, nu, dt, R.BDF2,
                           tol_outer=outer_tol(), tol_krylov=args.tol_krylov, max_outer=args.max_outer,
                           max_krylov=20000, precision=precision, p_bc=pb)
        state["eps"] = st["eps_steady"]
        torch.cuda.synchronize()
        phase_s["time_step"] += time.perf_counter() - tc
        state["i"] += 1
        pi = n * (st["krylov_mom"] + st["krylov_p"]) + ops.n_boundary * st["krylov_b"]
        ops.free()
        return st, pi

    for i in range(args.warmup):
        st, _ = one_step()
        log(f"[bench] warmup {i}: {st}")
    torch.cuda.synchronize()
    for key in phase_s:
        phase_s[key] = 0.0
    t0 = time.perf_counter()
    tot_pi = 0
    stats = []
    for i in range(args.steps):
        st, pi = one_step()
        tot_pi += pi
        stats.append(st)
        log(f"[bench] step {i}: {st} point-iters {pi}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    value = tot_pi / elapsed / 1e6
    last = stats[-1]
    unconverged = sum(1 for st_ in stats if st_["status"] != 0)
    # error against the closed-form flow at the last time level
    t_end = nsteps * dt
    ue_np, pe_np = W.flow_fields(cloud, t_end)
    u_fin = state["u"].cpu().numpy()
    p_fin = state["p"].cpu().numpy()
    err_u = float(np.abs(u_fin - ue_np).max())
    err_u_l1 = float(np.abs(u_fin - ue_np).mean())
    err_p = float(np.abs(p_fin - pe_np).max() / np.abs(pe_np).max())
    log(f"[bench] t={t_end:.4f} after {nsteps} steps: |u - exact| max {err_u:.3e} mean {err_u_l1:.3e}, "
        f"|p - exact| / |p| {err_p:.3e}; unconverged timed steps {unconverged}")

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "M point-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32ir": "f32 (f64 accumulation and refinement)",
                  "fp32matrix": "f32 matrix, f64 vectors"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload]["text"].format(n=n, q=q, dt=dt) +
                        f"; step = stencil build + assembly + one BDF2 time step advancing the flow (momentum and pressure-"
                        f"correction Krylov solves to {args.tol_krylov:g}, outer tolerance "
                        f"{'the rule min(1e-4, dt eps_s)' if args.tol_outer is None else args.tol_outer}, "
                        f"<= {args.max_outer} outer iterations); {nsteps} consecutive steps from t=0 "
                        f"({args.warmup} untimed)",
            "n_points": n, "q": q, "poly_degree": k, "max_outer": args.max_outer, "time_steps": nsteps,
        },
        "roofline": {
            "bound": "hbm",
            # the dominant kernel of the step: KT of the pressure-correction BiCGSTAB
            # (the library unrolls the row loop by 3 for widths divisible by 3 and not by 4)
            "kernel": f"k_t<double, double, 1, {3 if q % 3 == 0 and q % 4 else 4}> (t = A s-hat with dots t.s, t.t, "
                      "r-hat.t; pressure-correction BiCGSTAB)",
            "achieved": round(kt_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(kt_gbs / HBM_PEAK_GBS, 4),
            "traffic": counter_traffic(args.workload),
            "bytes_per_launch": kt_bytes(n, q),
            "bytes_per_row": f"12q + 32 = {12 * q + 32}",
            "us_per_launch": round(ktimes["kt"], 2),
            "k_v": {"us_per_launch": round(ktimes["kv"], 2), "bytes_per_launch": kv_bytes(n, q),
                    "frac": round(kv_bytes(n, q) / (ktimes["kv"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
            "k_s_us": round(ktimes["ks"], 2), "k_x_us": round(ktimes["kx"], 2),
            "iteration": {"us": round(ktimes["iteration"], 2), "bytes": iteration_bytes(n, q),
                          "bytes_per_row": f"24q + 192 = {24 * q + 192}",
                          "frac": round(iteration_bytes(n, q) / (ktimes["iteration"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
            "spmv_alone": {"us_per_launch": round(spmv_ms * 1e3, 2), "gbs_algorithmic": round(spmv_gbs, 1),
                           "index_bytes": f"{narrow:.4f} of rows with 2-byte column offsets, the rest 4-byte indices"},
            "note": ("working set ~%.0f MB fits the 256 MB Infinity Cache: effective bandwidth, not HBM"
                     if iteration_bytes(n, q) < 256e6 else
                     "working set ~%.0f MB exceeds the 256 MB Infinity Cache: HBM-resident") %
                    (iteration_bytes(n, q) / 1e6),
        },
        "phase_ms_per_step": {key: round(v / args.steps * 1e3, 3) for key, v in phase_s.items()},
        "stencil_points_per_s": round(n * args.steps / max(phase_s["stencils"], 1e-12), 0),
        "outer_iters": last["outer_iters"],
        "outer_delta": last["delta"],
        "krylov_iters": {"momentum": last["krylov_mom"], "pressure": last["krylov_p"], "boundary": last["krylov_b"]},
        "step_status": last["status"],
        "all_timed_steps_converged": unconverged == 0,
        "unconverged_timed_steps": unconverged,
        "error_vs_exact": {"t": round(t_end, 6), "u_max_abs": err_u, "u_mean_abs": err_u_l1, "p_max_rel": err_p},
        "bicgstab_us_per_iter": round(it_us, 2),
        "bicgstab_gbs": round(bicgstab_iter_bytes(n, q, narrow) / (it_us * 1e-6) / 1e9, 1),
        "converged_solves_1e-6": {
            "system": f"pressure-correction matrix of the same cloud, random right-hand side (seed 1), {args.solve_reps} solves each",
            "fp64": solves64,
            "fp32_vectors_and_matrix": solves32,
            "fp32_matrix_fp64_vectors": solves32m,
            "fp64_block_jacobi": solves64b,
            "fp32_vectors_and_matrix_block_jacobi": solves32b,
            "fp32_matrix_fp64_vectors_block_jacobi": solves32mb,
            "speedup_vs_fp64": {k_: round(v_["solves_per_s"] / solves64["solves_per_s"], 3) for k_, v_ in (
                ("fp32_vectors_and_matrix", solves32), ("fp32_matrix_fp64_vectors", solves32m),
                ("fp64_block_jacobi", solves64b), ("fp32_vectors_and_matrix_block_jacobi", solves32b),
                ("fp32_matrix_fp64_vectors_block_jacobi", solves32mb))},
            "note": "both mixed modes: FP64 row and dot accumulation, FP64 reliable residual updates; "
                    "entries without a suffix use the Jacobi preconditioner, *_block_jacobi the FP16 inverses "
                    "of the 64x64 diagonal blocks; speedups against fp64 with Jacobi",
        },
    }
    if args.mixed_step:
        # the same step with mixed-precision Krylov sweeps against the FP64 step:
        # per-field relative difference (max over points / max of the FP64 field)
        nbr, w, _ = R.rbffd_build_stencils(ctx, dcloud, k)
        ops_m = R.rbffd_assemble(ctx, dcloud, nbr, w, k, precision=R.RBFFD_FP32_IR)
        res = {}
        for name, prec, pc in (("fp64", R.RBFFD_FP64, R.RBFFD_PREC_JACOBI),
                               ("fp32", R.RBFFD_FP32_IR, R.RBFFD_PREC_JACOBI),
                               ("fp32matrix", R.RBFFD_FP32_MATRIX, R.RBFFD_PREC_JACOBI),
                               ("fp64_block_jacobi", R.RBFFD_FP64, R.RBFFD_PREC_BLOCK64),
                               ("fp32matrix_block_jacobi", R.RBFFD_FP32_MATRIX, R.RBFFD_PREC_BLOCK64)):
            u, up, p = u0.clone(), um1.clone(), pt0.clone()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            # three outer iterations each at Krylov tolerance 1e-10: the fields differ by the precision of the
            # Krylov sweeps alone
            st = R.simple_step(ctx, ops_m, u, up, p, ubc, rho, nu, dt, R.BDF2, tol_outer=0.0, tol_krylov=1e-10,
                               max_outer=3, max_krylov=20000, precision=prec, p_bc=pbc,
                               preconditioner=pc)
            torch.cuda.synchronize()
            res[name] = (u, p, st, time.perf_counter() - ta)
        u64, p64 = res["fp64"][0], res["fp64"][1]
        fields = {}
        for name in ("fp32", "fp32matrix", "fp64_block_jacobi", "fp32matrix_block_jacobi"):
            u, p, st, tm = res[name]
            du = [float((u[e] - u64[e]).abs().max() / u64[e].abs().max()) for e in range(cloud.dim)]
            dp = float((p - p64).abs().max() / p64.abs().max())
            fields[name] = {"ms": round(tm * 1e3, 1), "outer_iters": st["outer_iters"],
                            "krylov_iters": st["krylov_mom"] + st["krylov_p"],
                            "rel_diff_vs_fp64": dict(zip("uvw"[:cloud.dim], du), p=dp)}
        fields["fp64_ms"] = round(res["fp64"][3] * 1e3, 1)
        out["mixed_precision_step"] = fields
        ops_m.free()
    if args.workload == "taylor_green" and not args.no_hbm_section:
        out["hbm_resident_1m"] = hbm_resident_section(args, R, W, torch, ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
