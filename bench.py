#!/usr/bin/env python3
"""Benchmark: SIE matvecs/s and served solves/s of the GIBC/AIM solver on one
MI355X.

One step is one complete solve request on the copper-bar workload (100 x 10 x 5
um bar, sigma = 5.8e7 S/m, 20,088 triangles / 30,132 RWG functions, 10 GHz,
64^3 grid, near region 11 points across): mesh topology, grid and stencils,
near lists, FP64 near-field integrals with precorrection, Green's spectra,
plane-wave excitation, the nested GIBC solve (FP32 interior stages inside
FP64 refinement to the relative FP64 block residual given by --tol, default
1e-7; the nested solves preconditioned by the near-region operator in
restricted additive Schwarz form and run, inside each FP32 correction, to a
tolerance relaxed with the outer residual (--inner-relax 0.1); outer restart
1000) and the far field.
The FP32 currents are compared with an FP64 solve of the same request during
warmup (relative error gate 1e-3).  The synthetic
mesh is generated on the host before the timed region.

value = SIE matvecs / s over the timed steps, one SIE matvec being one AIM
operator product (L or K) of one medium for one right-hand side; solves/s and
p50/p99 step latency are reported beside it.  The roofline object covers the
dominant kernel (the near-field CSR product k_spmv_far in the path's
precision), timed with HIP events recorded by the library on the stream the
kernel runs on.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=64, help="rows of the oracle's dense matvec sample")
    ap.add_argument("--workload", choices=["bar", "fft", "batch", "serve", "counters"], default="bar",
                    help="bar: solve requests (default); fft: 4-field 256^3 convolution microbenchmark; "
                         "batch: 64 plane waves solved together on a 4,824-triangle copper bar; "
                         "serve: a Poisson stream of solve requests on the library's server; "
                         "counters: launches for HBM counter runs (1 GiB copy + copper-bar near-field products)")
    ap.add_argument("--nrhs", type=int, default=64, help="batch workload: plane waves")
    ap.add_argument("--requests", type=int, default=8, help="serve workload: requests of the trace")
    ap.add_argument("--max-tri", type=int, default=8000, help="serve workload: triangle cap per request")
    ap.add_argument("--max-iter", type=int, default=400, help="serve workload: outer iteration cap per solve")
    ap.add_argument("--inner-max-iter", type=int, default=300, help="serve workload: nested iteration cap")
    ap.add_argument("--slots", type=int, default=4, help="serve workload: concurrent requests")
    ap.add_argument("--tol", type=float, default=None,
                    help="relative FP64 block residual of every solve; default 1e-7 for the bar (its EFIE "
                         "conditioning turns a 1e-6 residual into ~1e-3 in the currents; 1e-7 keeps FP32 "
                         "within 1e-3 of FP64), 1e-6 for the batch and serve workloads")
    ap.add_argument("--restart", type=int, default=None,
                    help="outer GMRES restart length; default 1000 for the bar (its low-frequency EFIE "
                         "converges in a staircase that restarts would lengthen), 200 for the batch workload")
    ap.add_argument("--inner-relax", type=float, default=0.1,
                    help="relaxed nested tolerance inside the FP32 correction solves: nested solve j runs to "
                         "this x (correction target) / (outer residual estimate); 0: fixed tolerance")
    ap.add_argument("--precond", type=int, default=4,
                    help="preconditioner bit mask: 1 nested block-Jacobi, 2 outer block-Jacobi, 4 nested "
                         "near-region preconditioner in Schwarz form (conductive media)")
    a = ap.parse_args()
    if a.tol is None:
        a.tol = 1e-7 if a.workload == "bar" else 1e-6
    if a.restart is None:
        a.restart = 1000 if a.workload == "bar" else 200
    return a


SOLVE_OPTS = {}


def step(mesh, cfg, prec, tol, timing=False):
    """One solve request; returns (problem, report, setup_s, total_s)."""
    import torch
    from paper_2003_11679_amd import Problem
    xyz, tri = mesh
    o = cfg.objects[0]
    t0 = time.perf_counter()
    p = Problem(cfg.freq)
    p.add_object(xyz, tri, eps_r=o.eps_r, mu_r=o.mu_r, sigma=o.sigma)
    p.set_grid(-1, n=cfg.ext_grid_n, near_radius=cfg.near_radius)
    p.setup()
    t1 = time.perf_counter()
    if timing:
        p.set_timing(2)   # the near-field CSR product alone: two events per product
    w = cfg.waves[0]
    p.set_planewaves(w.khat, w.e0)
    rep = p.solve(prec, tol=tol, **SOLVE_OPTS)
    th = np.linspace(0.0, np.pi, 91)
    rhat = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)
    F = p.far_field(rhat)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    rep["far_field_max"] = float(np.abs(F).max())
    return p, rep, t1 - t0, t2 - t0


def spmv_bytes(p, prec):
    """Algorithmic HBM bytes of one k_spmv_far launch: CSR values and column
    indices in the stored form (16-bit offsets from each row's first column
    plus that base when every row spans fewer than 65536 columns, else 32-bit
    indices), row pointers, x read once, y written once, far-part operands
    (two triangles per row: coefficient and interpolation partials)."""
    rp, cols = p.near_pattern(-1)
    nnz = len(cols)
    E = p.num_rwg
    T = p.num_tri
    nrow = len(rp) - 1
    s = 8 if prec == 1 else 16          # complex element
    r = 4 if prec == 1 else 8           # real element
    full = rp[1:] > rp[:-1]
    span = cols[rp[1:][full] - 1] - cols[rp[:-1][full]] if full.any() else np.zeros(1)
    idx = nnz * 2 + nrow * 4 if span.max() < 65536 else nnz * 4
    return nnz * s + idx + (E + 1) * 8 + 2 * E * s + E * 8 + T * (12 * r + 5 * s), nnz


def cpu_baseline(cfg, mesh, rows):
    """The oracle's dense Galerkin matvec (plain definition, Sec. III-A) on a
    seeded sample of rows: every row integrates its two triangles against all
    triangles at both wavenumbers; extrapolated to matvecs/s."""
    from oracle.rwg import RWGMesh
    from oracle import mom, physics as ph
    m = RWGMesh([mesh])
    rng = np.random.default_rng(11683)
    sample = rng.choice(m.nrwg, size=rows, replace=False)
    T = len(m.tri)
    x = rng.standard_normal(m.nrwg) + 1j * rng.standard_normal(m.nrwg)
    k = ph.wavenumber(cfg.freq, cfg.objects[0].eps_r, 1.0, cfg.objects[0].sigma)
    t0 = time.perf_counter()
    for n in sample:
        tl = np.repeat([m.tp[n], m.tm[n]], T)
        sl = np.tile(np.arange(T), 2)
        A, P, K = mom.pair_blocks(m, k, tl, sl)
        L = A - P / k ** 2
        e = np.repeat([m.ep[n], m.em[n]], T)
        cols = m.tri_rwg[sl]                         # [2T,3]
        vals = L[np.arange(2 * T), e]                # [2T,3]
        _ = np.sum(vals * x[cols])
    dt = time.perf_counter() - t0
    rate = rows / dt / m.nrwg                        # matvecs/s
    return {"value": rate, "unit": "SIE matvecs/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": f"dense L-operator rows of the copper bar: {rows} seeded rows of {m.nrwg} "
                      f"(each row: its 2 triangles x all {T} triangles, oracle integration policy, "
                      f"C pair integrals with OpenMP), {dt:.1f} s, extrapolated to whole matvecs"}


def fft_bytes(nl, m, s, nf):
    """Algorithmic bytes of the pruned five-pass convolution: per field
    s [2 nx ny nz + 4 mx ny nz + 4 mx my nz] plus the spectrum octant."""
    nx, ny, nz = nl
    mx, my, mz = m
    per = s * (2 * nx * ny * nz + 4 * mx * ny * nz + 4 * mx * my * nz)
    octant = (mx // 2 + 1) * (my // 2 + 1) * (mz // 2 + 1) * s
    return nf * per + octant


def fft_micro(args):
    """4 fields of a full-occupancy 256^3 live box (complex64), FFT 512^3,
    times the Green's spectrum of k0 at 1 GHz with h = 3 lambda0 / 253."""
    import torch
    from workloads import geodesic_sphere, C0_NOMINAL
    from paper_2003_11679_amd import Problem
    lam0 = C0_NOMINAL / 1e9
    xyz, tri = geodesic_sphere(24, radius=1.5 * lam0)
    p = Problem(1e9)
    p.add_object(xyz, tri, eps_r=2.0, sigma=1.0)
    p.set_grid(-1, n=256, near_radius=1)
    p.set_quadrature(touch_out=3, touch_in=3, close_out=3, close_in=3, far_out=2, far_in=2)
    p.setup()
    g = p.grid(-1)
    nl = [int(v) for v in g["nl"]]
    m = [int(v) for v in g["m"]]
    dt = torch.complex64 if args.precision == "fp32" else torch.complex128
    s = 8 if dt == torch.complex64 else 16
    gen = torch.Generator(device="cuda").manual_seed(11685)
    src = torch.randn((4, nl[2], nl[1], nl[0]), dtype=dt, device="cuda", generator=gen)
    out = torch.empty_like(src)
    for _ in range(args.warmup + 1):
        p.convolve(-1, src, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        p.convolve(-1, src, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nb = fft_bytes(nl, m, s, 4)
    ach = nb / (ms * 1e-3) / 1e9
    print(json.dumps({"metric": "4-field zero-padded FFT convolution time", "value": ms, "unit": "ms",
                      "higher_is_better": False, "steps": args.steps, "warmup": args.warmup,
                      "dtype": "c64" if s == 8 else "c128", "data": "synthetic",
                      "config": {"workload": f"4 fields, live box {nl}, FFT {m}, G spectrum of k0 at 1 GHz"},
                      "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": ach / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": nb}}))


def batch_workload(args):
    """64 plane waves (8 x 8 incidence grid, alternating polarisation) on the
    4,824-triangle copper bar of the batching meshes (100 x 10 x 5 um, 90 x 9
    x 4 divisions, sigma 5.8e7 S/m, 10 GHz, 32^3 grid, near radius 5): one
    step is one solve of all waves together (lock-step GMRES over the
    right-hand sides, batched products: the near-field values are streamed
    once per batch)."""
    import torch
    from workloads import box_mesh
    from workloads.configs import multi_rhs_waves
    from paper_2003_11679_amd import Problem
    xyz, tri = box_mesh((100e-6, 10e-6, 5e-6), (90, 9, 4))
    waves = multi_rhs_waves()[:args.nrhs]
    prec = 1 if args.precision == "fp32" else 0
    opts = dict(tol=args.tol, restart=args.restart, precond=args.precond, inner_relax=args.inner_relax)

    def one(timing=False):
        p = Problem(10e9)
        p.add_object(xyz, tri, eps_r=1.0, sigma=5.8e7)
        p.set_grid(-1, n=32, near_radius=5)
        t0 = time.perf_counter()
        p.setup()
        if timing:
            p.set_timing(True)
        p.set_planewaves([w.khat for w in waves], [w.e0 for w in waves])
        rep = p.solve(prec, **opts)
        torch.cuda.synchronize()
        return p, rep, time.perf_counter() - t0

    for i in range(args.warmup):
        _, rep, dt = one()
        print(f"[bench] batch warmup {i}: {dt:.2f}s {rep}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    matvecs, reps = 0, []
    for i in range(args.steps):
        p, rep, dt = one(timing=True)
        matvecs += rep["matvecs"]
        reps.append(rep)
        print(f"[bench] batch step {i}: {dt:.2f}s {rep}", file=sys.stderr, flush=True)
    T = time.perf_counter() - t0
    st = p.stage_times()
    print(json.dumps({"metric": "RHS-matvecs/s of a batched multi-RHS solve", "value": matvecs / T,
                      "unit": "RHS-matvecs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": T / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "c64+f64" if prec == 1 else "c128", "data": "synthetic",
                      "config": {"workload": f"{len(waves)} plane waves (8x8 incidence grid, alternating "
                                             "polarisation), copper bar 100x10x5 um, 4824 triangles, 10 GHz, "
                                             f"32^3 grid, near radius 5, solve to {args.tol:g}"},
                      "solves_per_s": args.steps / T, "rhs_solves_per_s": args.steps * len(waves) / T,
                      "converged": all(r["converged"] for r in reps), "residual_fp64_max":
                      max(r["residual"] for r in reps), "outer_iters": reps[-1]["outer_iters"],
                      "batched_product_ms": {k: v[1] / max(v[0], 1) for k, v in st.items()}}))


def serve_workload(args):
    """The seeded Poisson request stream (50 req/s): each request a sphere,
    box or ellipsoid with its own material and frequency, submitted at its
    arrival time to the library's server (FP32 + FP64 refinement); latency =
    completion - arrival, queueing, setup and solve included."""
    import torch
    from workloads.configs import serving_trace, serving_mesh
    from paper_2003_11679_amd import Problem, Server
    trace = serving_trace()[:args.requests]
    reqs = []
    for r in trace:
        r = dict(r)
        r["nt"] = min(r["nt"], args.max_tri)
        xyz, tri = serving_mesh(r)
        ext = float(np.max(xyz.max(0) - xyz.min(0)))
        edge = float(np.mean(np.linalg.norm(xyz[tri[:, 1]] - xyz[tri[:, 0]], axis=1)))
        n = 8
        while ext / (n - 3) > edge and n < 256:
            n *= 2
        reqs.append((r, xyz, tri, n))
    prec = 1 if args.precision == "fp32" else 0
    srv = Server(max_slots=args.slots)
    t0 = time.perf_counter()
    tickets = []
    for r, xyz, tri, n in reqs:
        dt = r["t"] - trace[0]["t"] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        p = Problem(r["freq"], ctx=srv.ctx)
        p.add_object(xyz, tri, eps_r=r["eps_r"], sigma=r["sigma"])
        p.set_grid(-1, n=n, near_radius=3)
        tickets.append(srv.submit(p, (0.0, 0.0, -1.0), (1.0, 0.0, 0.0), prec, tol=args.tol, restart=100,
                                  precond=args.precond, max_iter=args.max_iter,
                                  inner_max_iter=args.inner_max_iter, inner_relax=args.inner_relax))
    # requests are reported as they start and as they finish (completion order)
    infos = [None] * len(tickets)
    started = [False] * len(tickets)
    left = set(range(len(tickets)))
    while left:
        for q in sorted(left):
            i = srv.poll(tickets[q])
            if i["running"] and not started[q]:
                started[q] = True
                print(f"[bench] request {q + 1}: started", file=sys.stderr, flush=True)
            if i["done"]:
                infos[q] = i
                left.discard(q)
                print(f"[bench] request {q + 1}: status {i['status']} latency "
                      f"{i['t_end_s'] - i['t_submit_s']:.2f}s run {i['t_end_s'] - i['t_start_s']:.2f}s "
                      f"{i['report']}", file=sys.stderr, flush=True)
                srv.take(tickets[q])
        time.sleep(0.005)
    T = time.perf_counter() - t0
    srv.close()
    lat = [i["t_end_s"] - i["t_submit_s"] for i in infos]
    conv = sum(1 for i in infos if i["status"] == 0)
    span = max(i["t_end_s"] for i in infos) - min(i["t_submit_s"] for i in infos)
    print(json.dumps({"metric": "served solves/s, p50/p99 latency", "value": len(infos) / span,
                      "unit": "solves/s", "n_gpus": 1, "steps": len(infos), "warmup": 0,
                      "ms_per_step": span / len(infos) * 1e3, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "c64+f64" if prec == 1 else "c128", "data": "synthetic",
                      "config": {"workload": f"first {len(infos)} requests of the seeded 50 req/s trace, "
                                             f"triangles capped at {args.max_tri}, {args.slots} slots, near "
                                             f"radius 3, solve to {args.tol:g} (caps {args.max_iter} outer / "
                                             f"{args.inner_max_iter} nested iterations)"},
                      "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
                      "converged": conv, "requests": len(infos), "wall_s": T,
                      "offered_rate": 50.0}))


def counters_workload(args):
    """Launches for `rocprofv3 --pmc FETCH_SIZE` / `WRITE_SIZE` runs: a plain
    1 GiB device copy (calibration of the counters) and five FP32 L products
    of the copper bar (k_spmv_far, the dominant kernel)."""
    import torch
    from workloads import bar_cfg
    from paper_2003_11679_amd import Problem
    a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    cfg = bar_cfg()
    ob = cfg.objects[0]
    p = Problem(cfg.freq)
    p.add_object(ob.xyz, ob.tri, eps_r=ob.eps_r, sigma=ob.sigma)
    p.set_grid(-1, n=cfg.ext_grid_n, near_radius=cfg.near_radius)
    p.setup()
    X = torch.randn(p.num_rwg, dtype=torch.complex64, device="cuda")
    Y = torch.empty_like(X)
    for _ in range(5):
        p.matvec(-1, 0, X, Y)
    torch.cuda.synchronize()
    nb, _ = spmv_bytes(p, 1)
    print(json.dumps({"copy_bytes": 2 ** 30, "k_spmv_far_algorithmic_bytes": nb}))


def spmv_traffic():
    """Measured HBM bytes per k_spmv_far<float> launch on the copper bar from
    the committed counter summary, if the kernel source is the one measured
    (else None)."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "k_spmv_far__copper_bar_traffic.md")
    src = os.path.join(ROOT, "paper_2003_11679_amd", "csrc", "k_grid.hip")
    if not os.path.exists(prof):
        return None
    import re
    m = re.search(r"bench-traffic: bytes_per_launch=(\d+) k_grid_sha256=([0-9a-f]+)", open(prof).read())
    if not m:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m.group(2):
        return None
    return int(m.group(1))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.workload == "fft":
        fft_micro(args)
        return
    if args.workload == "batch":
        batch_workload(args)
        return
    if args.workload == "serve":
        serve_workload(args)
        return
    if args.workload == "counters":
        counters_workload(args)
        return
    from workloads import bar_cfg
    cfg = bar_cfg()
    mesh = (cfg.objects[0].xyz, cfg.objects[0].tri)
    prec = 1 if args.precision == "fp32" else 0
    SOLVE_OPTS.update(restart=args.restart, precond=args.precond, inner_relax=args.inner_relax)
    print(f"[bench] workload bar {len(mesh[1])} triangles, precision {args.precision}, "
          f"warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    ref = None
    for i in range(args.warmup):
        p, rep, su, tot = step(mesh, cfg, prec, args.tol)
        print(f"[bench] warmup {i}: setup {su:.2f}s total {tot:.2f}s {rep}", file=sys.stderr, flush=True)
        if i == 0 and prec == 1:
            # FP64 reference of the same request (accuracy of the FP32 path)
            u32, v32 = p.currents()
            th = np.linspace(0.0, np.pi, 91)
            rhat = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)
            F32 = p.far_field(rhat)
            r64 = p.solve(0, tol=args.tol, **SOLVE_OPTS)
            u64, v64 = p.currents()
            F64 = p.far_field(rhat)
            ref = {"rel_err_u": float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64)),
                   "rel_err_v": float(np.linalg.norm(v32 - v64) / np.linalg.norm(v64)),
                   "rel_err_far_field": float(np.abs(F32 - F64).max() / np.abs(F64).max()),
                   "fp64_solve": r64}
            print(f"[bench] fp64 reference: {ref}", file=sys.stderr, flush=True)
        del p
    torch.cuda.synchronize()
    lat, matvecs, setups, reps = [], 0, [], []
    spmv_ms, spmv_n, s64_ms, s64_n = 0.0, 0, 0.0, 0
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        p, rep, su, tot = step(mesh, cfg, prec, args.tol, timing=True)
        st = p.stage_times()
        spmv_n += st["spmv"][0]; spmv_ms += st["spmv"][1]
        s64_n += st["spmv64"][0]; s64_ms += st["spmv64"][1]
        lat.append(tot); setups.append(su); reps.append(rep)
        matvecs += rep["matvecs"]
        print(f"[bench] step {i}: setup {su:.2f}s total {tot:.2f}s {rep}", file=sys.stderr, flush=True)
        if last is not None:
            del last
        last = p
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    nbytes, nnz = spmv_bytes(last, prec)
    # the solve runs near-field products in both precisions: the roofline
    # takes the launches of the path's own precision (FP32: all minus FP64)
    k_n, k_ms = (spmv_n - s64_n, spmv_ms - s64_ms) if prec == 1 else (s64_n, s64_ms)
    avg_ms = k_ms / max(k_n, 1)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    nb64, _ = spmv_bytes(last, 0)
    avg64 = s64_ms / max(s64_n, 1)
    conv = all(r["converged"] for r in reps)
    out = {
        "metric": "SIE matvecs/s + served solves/s, p50/p99 latency at rel err <=1e-3 vs FP64",
        "value": matvecs / T,
        "unit": "SIE matvecs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64" if prec == 1 else "c128",
        "data": "synthetic",
        "config": {"workload": "copper bar 100x10x5 um, sigma 5.8e7 S/m, 20088 triangles (30132 RWG), "
                               "10 GHz, 64^3 grid, near radius 5, plane wave -z x-polarised, 1 RHS, "
                               f"GIBC solve to a relative FP64 residual of {args.tol:g}",
                   "precision": args.precision, "nnz_near": int(nnz)},
        "solves_per_s": args.steps / T,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "setup_s_mean": float(np.mean(setups)),
        "converged": conv,
        "tol": args.tol,
        "fp32_vs_fp64": ref,
        "residual_fp64_max": max(r["residual"] for r in reps),
        "outer_iters": reps[-1]["outer_iters"], "inner_iters": reps[-1]["inner_iters"],
        "refine_sweeps": reps[-1]["refine_sweeps"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": spmv_traffic() if prec == 1 else None,
                     "kernel": "k_spmv_far<float>" if prec == 1 else "k_spmv_far<double>",
                     "avg_launch_ms": avg_ms, "launches": k_n, "bytes_per_launch": nbytes},
        "spmv_fp64": {"avg_launch_ms": avg64, "launches": s64_n, "bytes_per_launch": nb64,
                      "achieved_gbs": nb64 / (avg64 * 1e-3) / 1e9 if s64_n else None},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle dense row sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, mesh, args.cpu_rows)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
