#!/usr/bin/env python3
"""Benchmark: SIE matvecs/s and served solves/s of the GIBC/AIM solver on one
MI355X.

Default workload: the 8 x 8 array of lossy dielectric cubes (196,608
triangles, 294,912 RWG functions; eps_r ~ U[2, 10], sigma ~ U[0, 10] S/m,
1 GHz, cube edge 0.2 lambda0, pitch 0.4 lambda0; exterior grid 256^3 with FFT
512 x 512 x 64 on its live box, one 16^3 grid per cube, near region 11
points across).  One step is one complete solve request: mesh topology,
grids and stencils, near lists, FP64 near-field integrals with
precorrection, Green's spectra, the plane wave, the nested GIBC solve (FP32
interior stages, the 64 cubes batched into one launch per stage and solved
as 64 nested systems side by side, inside FP64 refinement to the relative
FP64 block residual --tol) and the far field.  The FP32 currents of the
first warmup request are compared with an FP64 solve of the same request
(relative error gate 1e-3).  --workload bar and sphere run the copper bar
and the dielectric sphere the same way.  The synthetic meshes are generated
on the host before the timed region; one request's problem is released
before the next one starts.

value = SIE matvecs / s over the timed steps: one SIE matvec is one L-type
AIM product (eq. AIM_Lin) of one medium for one right-hand side; K-type
products are counted beside it.  Solves/s and p50/p99 request latency are
reported too.  The roofline object covers the dominant kernel, the
near-field CSR product of the interior media (the nested operator) in FP32,
timed with HIP events the library records on the stream the kernel runs on.
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
    ap.add_argument("--workload", choices=["cubes", "bar", "sphere", "fft", "batch", "serve", "counters"],
                    default="cubes",
                    help="cubes (default), bar, sphere: solve requests on the cube array, copper bar or "
                         "dielectric sphere; fft: 4-field 256^3 convolution microbenchmark; "
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
                         "within 1e-3 of FP64), 1e-6 otherwise")
    ap.add_argument("--restart", type=int, default=None,
                    help="outer GMRES restart length; default 1000 for the bar (its low-frequency EFIE "
                         "converges in a staircase that restarts would lengthen), 300 for the cubes, 200 "
                         "otherwise")
    ap.add_argument("--inner-relax", type=float, default=0.1,
                    help="relaxed nested tolerance inside the FP32 correction solves: nested solve j runs to "
                         "this x (correction target) / (outer residual estimate); 0: fixed tolerance")
    ap.add_argument("--skin-cutoff", type=float, default=5.0,
                    help="skin-depth cutoff of the interior problem in skin depths (Sec. V; 0 off)")
    ap.add_argument("--precond", type=int, default=4,
                    help="preconditioner bit mask: 1 nested block-Jacobi, 2 outer block-Jacobi, 4 nested "
                         "near-region preconditioner in Schwarz form (conductive media)")
    a = ap.parse_args()
    if a.tol is None:
        a.tol = 1e-7 if a.workload == "bar" else 1e-6
    if a.restart is None:
        a.restart = {"bar": 1000, "cubes": 300}.get(a.workload, 200)
    return a


SOLVE_OPTS = {}
SETUP_OPTS = {"skin_cutoff": 0.0}


def workload_cfg(name):
    """The synthetic configuration of a request workload."""
    from workloads import cube_array_cfg, bar_cfg, sphere_cfg
    if name == "cubes":
        return cube_array_cfg()
    if name == "bar":
        return bar_cfg()
    cfg = sphere_cfg()
    cfg.ext_grid_n = 0          # the Sec. IV rule: lambda_r / 20 of the interior, 44 points per axis
    return cfg


def build_problem(cfg):
    from paper_2003_11679_amd import Problem
    p = Problem(cfg.freq)
    for o in cfg.objects:
        p.add_object(o.xyz, o.tri, eps_r=o.eps_r, mu_r=o.mu_r, sigma=o.sigma)
    p.set_grid(-1, n=cfg.ext_grid_n, near_radius=cfg.near_radius)
    if not cfg.shared_grid:
        for i, o in enumerate(cfg.objects):
            p.set_grid(i, n=o.grid_n or 0, near_radius=cfg.near_radius, share=0)
    p.set_skin_cutoff(SETUP_OPTS["skin_cutoff"])
    p.setup()
    return p


def run_request(cfg, prec, tol, timing=False):
    """One solve request; returns (problem, report, setup_s, total_s)."""
    import torch
    t0 = time.perf_counter()
    p = build_problem(cfg)
    t1 = time.perf_counter()
    if timing:
        p.set_timing(2)   # the near-field CSR products alone: two events per product
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


def spmv_model(p, media, prec):
    """Algorithmic HBM bytes of one k_spmv_far launch over the RWG rows of
    `media` (one launch per group of media): CSR values and column indices
    in the stored form (16-bit offsets from each row's first column plus
    that base when every row spans fewer than 65536 columns, else 32-bit
    indices), row pointers, x read once, y written once, and the far-part
    operands of the rows' triangles (coefficients, interpolation partials,
    slot) unless the media run without grid part."""
    s = 8 if prec == 1 else 16          # complex element
    r = 4 if prec == 1 else 8           # real element
    nnz = nrow = tris = 0
    idx = 0
    far = False
    for md in media:
        rp, cols = p.near_pattern(md)
        rows = np.nonzero(rp[1:] > rp[:-1])[0]
        b, e = rp[rows], rp[rows + 1]
        n = int(len(cols))
        span = int((cols[e - 1] - cols[b]).max()) if n else 0
        nr = len(rows)
        nnz += n
        nrow += nr
        tris += 2 * nr // 3
        idx += 2 * n + 4 * nr if span < 65536 else 4 * n
        far = far or not p.is_local(md)
    E = p.num_rwg
    b = nnz * s + idx + 8 * (nrow + 1) + E * s + nrow * s + 8 * nrow
    if far:
        b += tris * (12 * r + 5 * s + 4)
    return b, nnz


def cpu_baseline_aim(cfg, rows=24):
    """The oracle's AIM product (O-aim, same approximation as the GPU) of one
    medium for one right-hand side, timed on a bounded sample: the grid part
    (projection, FFT convolution, interpolation) of the whole medium, plus
    the precorrected near-field rows of a seeded row sample, extrapolated to
    all rows of the medium.  The medium is the first object's interior on
    its own grid (the nested operator's unit of work)."""
    from oracle.rwg import RWGMesh
    from oracle.aim import Grid, AIMOperator
    from oracle import physics as ph
    o = cfg.objects[0]
    m = RWGMesh([(o.xyz, o.tri)])
    k = ph.wavenumber(cfg.freq, o.eps_r, 1.0, o.sigma)
    n = o.grid_n if not cfg.shared_grid and o.grid_n else cfg.ext_grid_n
    if not n:
        from paper_2003_11679_amd.sie import grid_choose
        ext = float(np.max(m.xyz.max(0) - m.xyz.min(0)))
        n = grid_choose(cfg.freq, o.eps_r, 1.0, o.sigma, ext, float(np.mean(m.length)))["n"]
    rng = np.random.default_rng(11683)
    x = rng.standard_normal(m.nrwg) + 1j * rng.standard_normal(m.nrwg)
    sample = rng.choice(m.nrwg, size=min(rows, m.nrwg), replace=False)
    t0 = time.perf_counter()
    op = AIMOperator(m, Grid.enclosing(m.xyz, n), k, near_radius=cfg.near_radius, near=False)
    _ = op.far_part(x, "A") - op.far_part(x, "P") / k ** 2
    t1 = time.perf_counter()
    _ = op.near_rows(sample)
    t2 = time.perf_counter()
    per = (t1 - t0) + (t2 - t1) * m.nrwg / len(sample)
    return {"value": 1.0 / per, "unit": "SIE matvecs/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": f"oracle AIM L product of one medium (interior of object 0: {len(o.tri)} triangles, "
                      f"{m.nrwg} RWG, {n}^3 grid, near radius {cfg.near_radius}): moments and grid part "
                      f"of the whole medium {t1 - t0:.1f} s, precorrected near rows of {len(sample)} seeded "
                      f"rows {t2 - t1:.1f} s extrapolated to {m.nrwg} rows; {per:.1f} s per matvec"}


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
    1 GiB device copy (calibration of the counters) and five FP32 products
    of every interior medium of the cube array (SIE_INTERIORS: the nested
    operator's k_spmv_far launch over all 64 cubes, the dominant kernel)."""
    import torch
    from paper_2003_11679_amd import INTERIORS
    a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    SETUP_OPTS["skin_cutoff"] = args.skin_cutoff
    cfg = workload_cfg("cubes")
    p = build_problem(cfg)
    X = torch.randn(p.num_rwg, dtype=torch.complex64, device="cuda")
    Y = torch.empty_like(X)
    for _ in range(5):
        p.matvec(INTERIORS, 0, X, Y)
    torch.cuda.synchronize()
    nb, nnz = spmv_model(p, list(range(len(cfg.objects))), 1)
    print(json.dumps({"copy_bytes": 2 ** 30, "k_spmv_far_algorithmic_bytes": nb, "nnz": nnz}))


def spmv_traffic(workload):
    """Measured HBM bytes per dominant k_spmv_far<float> launch of the
    workload from the committed counter summary, if the kernel source is
    the one measured (else None)."""
    import hashlib
    import re
    prof = os.path.join(ROOT, "profiles", f"k_spmv_far__{workload}_traffic.md")
    src = os.path.join(ROOT, "paper_2003_11679_amd", "csrc", "k_grid.hip")
    if not os.path.exists(prof):
        return None
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
    request_workload(args)


def request_workload(args):
    """Solve requests of one configuration (see the module docstring)."""
    import torch
    cfg = workload_cfg(args.workload)
    prec = 1 if args.precision == "fp32" else 0
    SOLVE_OPTS.update(restart=args.restart, precond=args.precond, inner_relax=args.inner_relax)
    SETUP_OPTS["skin_cutoff"] = args.skin_cutoff
    T = sum(len(o.tri) for o in cfg.objects)
    print(f"[bench] workload {args.workload}: {len(cfg.objects)} objects, {T} triangles, precision "
          f"{args.precision}, warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    ref = None
    model = None
    for i in range(args.warmup):
        p, rep, su, tot = run_request(cfg, prec, args.tol)
        print(f"[bench] warmup {i}: setup {su:.2f}s total {tot:.2f}s {rep}", file=sys.stderr, flush=True)
        if i == 0:
            media = list(range(len(cfg.objects)))
            model = {"int": spmv_model(p, media, prec), "ext64": spmv_model(p, [-1], 0),
                     "int64": spmv_model(p, media, 0), "local": [p.is_local(m) for m in media],
                     "E": p.num_rwg}
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
    lat, matvecs, kmatvecs, setups, reps = [], 0, 0, [], []
    tm = {k: [0, 0.0] for k in ("spmv", "spmv64", "spmv_int32", "spmv_int64")}
    t0 = time.perf_counter()
    for i in range(args.steps):
        p, rep, su, tot = run_request(cfg, prec, args.tol, timing=True)
        st = p.stage_times()
        for k in tm:
            tm[k][0] += st[k][0]
            tm[k][1] += st[k][1]
        if model is None:
            media = list(range(len(cfg.objects)))
            model = {"int": spmv_model(p, media, prec), "ext64": spmv_model(p, [-1], 0),
                     "int64": spmv_model(p, media, 0), "local": [p.is_local(m) for m in media],
                     "E": p.num_rwg}
        del p            # release the request's device memory before the next one
        lat.append(tot); setups.append(su); reps.append(rep)
        matvecs += rep["matvecs"]
        kmatvecs += rep["k_matvecs"]
        print(f"[bench] step {i}: setup {su:.2f}s total {tot:.2f}s {rep}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    Tt = time.perf_counter() - t0
    # dominant kernel: the interior media's near-field product in the path's
    # precision (one launch per group of media per nested product)
    kn, kms = tm["spmv_int32"] if prec == 1 else tm["spmv_int64"]
    nbytes, nnz = model["int"] if prec == 1 else model["int64"]
    avg_ms = kms / max(kn, 1)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9 if kn else None
    # exterior products: all launches minus the interior ones, per precision
    e64n = tm["spmv64"][0] - tm["spmv_int64"][0]
    e64ms = tm["spmv64"][1] - tm["spmv_int64"][1]
    conv = all(r["converged"] for r in reps)
    names = {"cubes": "8x8 array of lossy dielectric cubes (edge 0.2 lambda0, pitch 0.4 lambda0, eps_r ~ U[2,10], "
                      "sigma ~ U[0,10] S/m, seed 11682), 196608 triangles (294912 RWG), 1 GHz, exterior grid "
                      "256^3 (FFT on the live box), one 16^3 grid per cube",
             "bar": "copper bar 100x10x5 um, sigma 5.8e7 S/m, 20088 triangles (30132 RWG), 10 GHz, 64^3 grid",
             "sphere": "dielectric sphere r = 1 m, eps_r 4, 1280 triangles (1920 RWG), 150 MHz, 44^3 grid "
                       "(the lambda_r/20 rule of Sec. IV)"}
    out = {
        "metric": "SIE matvecs/s + served solves/s, p50/p99 latency at rel err <=1e-3 vs FP64",
        "value": matvecs / Tt,
        "unit": "SIE matvecs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": Tt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64" if prec == 1 else "c128",
        "data": "synthetic",
        "config": {"workload": names[args.workload] + f", near radius {cfg.near_radius}, plane wave -z "
                               f"x-polarised, 1 RHS, GIBC solve to a relative FP64 residual of {args.tol:g}"
                               + (f", skin-depth cutoff {args.skin_cutoff:g}" if args.skin_cutoff else ""),
                   "precision": args.precision, "nnz_near_interior": int(nnz),
                   "interior_media_without_grid_part": int(sum(model["local"]))},
        "k_matvecs_per_s": kmatvecs / Tt,
        "solves_per_s": args.steps / Tt,
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
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": spmv_traffic(args.workload) if prec == 1 else None,
                     "kernel": "k_spmv_far<float> (interior media)" if prec == 1 else
                               "k_spmv_far<double> (interior media)",
                     "avg_launch_ms": avg_ms, "launches": kn, "bytes_per_launch": nbytes},
        "spmv_exterior_fp64": {"avg_launch_ms": e64ms / max(e64n, 1), "launches": e64n,
                               "bytes_per_launch": model["ext64"][0],
                               "achieved_gbs": model["ext64"][0] / (e64ms / e64n * 1e-3) / 1e9 if e64n else None},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle AIM product, bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_aim(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
