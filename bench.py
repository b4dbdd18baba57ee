#!/usr/bin/env python3
"""Benchmark: SIE matvecs/s and served solves/s of the GIBC/AIM solver on one
MI355X.

Default workload: the 8 x 8 array of lossy dielectric cubes (edge 0.2
lambda0, pitch 0.4 lambda0, eps_r ~ U[2,10], sigma ~ U[0,10] S/m; 196,608
triangles / 294,912 RWG functions, 1 GHz, exterior grid 256^3 with the FFT on
the live box, one 16^3 grid per cube, near region 11 points across).  One
step is one complete solve request: mesh topology, grids and stencils, near
lists, FP64 near-field integrals with precorrection, Green's spectra, the
factors of the constraint preconditioner, the plane wave, the solve of the
augmented EFIE (Sec. III-E, eq. sys) with nested GIBC interiors (FP32
interior stages inside FP64 refinement to the relative FP64 block residual
--tol, default 1e-6; the 64 interior grids batched into one launch per stage)
and the far field.  The FP32 currents of the first warmup request are
compared with an FP64 solve of the same request (relative error gate 1e-3).
After the timed steps five requests of the copper bar (100 x 10 x 5 um,
sigma 5.8e7 S/m, 20,088 triangles, 10 GHz, 64^3 grid, interior skin-depth
cutoff of 5 skin depths, residual 1e-7) are measured the same way, with
their own FP64 gate and kernel roofline (--no-secondary skips them).
--workload bar and sphere time those configurations instead (a bar run
measures one cube-array request after its steps).  The synthetic meshes are
generated on the host before the timed region; one request's problem is
released before the next one starts (its device memory stays with the
library's pool for the next request).

value = SIE matvecs / s over the timed steps: one SIE matvec is one L-type
AIM product (eq. AIM_Lin) of one medium for one right-hand side (the
augmented exterior product counts as one); K-type products are counted
beside it.  The 64 cubes' nested systems iterate side by side; by default
an object whose system has converged is left out of the remaining nested
products of that solve (its rows are zero) and those products are neither
computed nor counted, so a request counts ~37,000 L products instead of
~139,000 and takes ~25 % less time.  The other mode (--keep-converged 1,
every object multiplied in every nested iteration) is timed for a few
requests after the steps for comparison.  Solves/s and p50/p99 request
latency are reported too.  The
roofline object covers the near-field CSR launch class with the largest
measured time (per medium class and precision), timed with HIP events the
library records on the stream the kernel runs on.
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
    ap.add_argument("--workload", choices=["bar", "cubes", "sphere", "fft", "batch", "serve", "counters"],
                    default="cubes",
                    help="cubes (default), bar, sphere: solve requests on the cube array, copper bar or "
                         "dielectric sphere; fft: 4-field 256^3 convolution microbenchmark; "
                         "batch: 64 plane waves solved together on a 4,824-triangle copper bar; "
                         "serve: a Poisson stream of solve requests on the library's server; "
                         "counters: launches for HBM counter runs (1 GiB copy, copper-bar exterior and cube-array "
                         "interior near-field products)")
    ap.add_argument("--nrhs", type=int, default=64, help="batch workload: plane waves")
    ap.add_argument("--requests", type=int, default=8, help="serve workload: requests of the trace")
    ap.add_argument("--max-tri", type=int, default=20000, help="serve workload: triangle cap per request")
    ap.add_argument("--max-iter", type=int, default=400, help="serve workload: outer iteration cap per solve")
    ap.add_argument("--inner-max-iter", type=int, default=300, help="serve workload: nested iteration cap")
    ap.add_argument("--slots", type=int, default=4, help="serve workload: concurrent requests")
    ap.add_argument("--tol", type=float, default=None,
                    help="relative FP64 block residual of every solve; default 1e-7 for the bar (its EFIE "
                         "conditioning turns a 1e-6 residual into ~1e-3 in the currents; 1e-7 keeps FP32 "
                         "within 1e-3 of FP64), 1e-6 otherwise")
    ap.add_argument("--restart", type=int, default=None,
                    help="outer GMRES restart length; default 1000 for the bar and the cube array (their "
                         "exterior EFIE converges in a staircase that restarts would lengthen), 400 for the serve "
                         "trace (its outer cap: shorter restarts stall on electrically large conductors), 200 "
                         "otherwise")
    ap.add_argument("--inner-relax", type=float, default=0.1,
                    help="relaxed nested tolerance inside the FP32 correction solves: nested solve j runs to "
                         "this x (correction target) / (outer residual estimate); 0: fixed tolerance")
    ap.add_argument("--skin-cutoff", type=float, default=5.0,
                    help="skin-depth cutoff of the interior problem in skin depths (Sec. V; 0 off)")
    ap.add_argument("--augmented", type=int, default=1,
                    help="request workloads: 1 (default) exterior problem as the augmented EFIE with the "
                         "constraint preconditioner (Sec. III-E, eq. sys); 0 the GIBC system of the EFIE")
    ap.add_argument("--keep-converged", type=int, default=0,
                    help="1: nested solves keep multiplying the objects whose nested systems have converged "
                         "(default 0: their rows are skipped and their products not counted); the cube-array "
                         "run also times a few requests in the other mode for comparison")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the other configuration measured after the timed steps (bar requests after "
                         "the cube array, one cube-array request after the bar)")
    ap.add_argument("--precond", type=int, default=None,
                    help="preconditioner bit mask: 1 nested block-Jacobi, 2 outer block-Jacobi, 4 nested "
                         "near-region preconditioner in Schwarz form (conductive media), 8 with 4: for every "
                         "interior medium, 16 the near-region preconditioner as an exact sparse LU where the "
                         "medium's near-region matrix stays sparse (with 4: Schwarz for the others); default "
                         "12 for the cube array, 28 for the serve trace, 4 otherwise")
    a = ap.parse_args()
    if a.tol is None:
        a.tol = DEFAULT_TOL.get(a.workload, 1e-6)
    if a.restart is None:
        a.restart = {"bar": 1000, "cubes": 1000, "serve": 400}.get(a.workload, 200)
    if a.precond is None:
        a.precond = DEFAULT_PRECOND.get(a.workload, 4)
    return a


# per workload: relative FP64 block residual of the solves (the bar's EFIE
# conditioning turns a 1e-6 residual into ~1e-3 in the currents) and the
# preconditioner bits (Schwarz clusters for every interior of the cube array)
DEFAULT_TOL = {"bar": 1e-7, "cubes": 1e-6}
DEFAULT_PRECOND = {"bar": 4, "cubes": 12, "serve": 28}


SOLVE_OPTS = {}
SETUP_OPTS = {"skin_cutoff": 0.0, "augmented": False}


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
    p.set_augmented(SETUP_OPTS["augmented"])
    p.setup()
    return p


def run_request(cfg, prec, tol, timing=False, opts=None):
    """One solve request; returns (problem, report, setup_s, total_s)."""
    import torch
    t0 = time.perf_counter()
    p = build_problem(cfg)
    t1 = time.perf_counter()
    if timing:
        p.set_timing(2)   # the near-field CSR products alone: two events per product
    w = cfg.waves[0]
    p.set_planewaves(w.khat, w.e0)
    rep = p.solve(prec, tol=tol, **(SOLVE_OPTS if opts is None else opts))
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


def oracle_threads():
    """Threads the oracle's OpenMP pair integrals run on (numpy's FFTs run
    on one of them)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return min(n, int(env)) if env.isdigit() and int(env) > 0 else n


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
    return {"value": 1.0 / per, "unit": "SIE matvecs/s", "cores": oracle_threads(), "kind": "oracle",
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
    return {"value": rate, "unit": "SIE matvecs/s", "cores": oracle_threads(), "kind": "oracle",
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


def fft_measure(steps, warmup, precision):
    """4 fields of a full-occupancy 256^3 live box (complex64), FFT 512^3,
    times the Green's spectrum of k0 at 1 GHz with h = 3 lambda0 / 253:
    milliseconds per convolution with the built-in and the tuned tile
    shapes, and the achieved fraction of the HBM peak."""
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
    dt = torch.complex64 if precision == "fp32" else torch.complex128
    s = 8 if dt == torch.complex64 else 16
    gen = torch.Generator(device="cuda").manual_seed(11685)
    src = torch.randn((4, nl[2], nl[1], nl[0]), dtype=dt, device="cuda", generator=gen)
    out = torch.empty_like(src)
    import paper_2003_11679_amd as P
    fams = ("fft_y_fwd", "fft_y_inv", "fft_z")

    def timed(builtin):
        for f in fams:
            P.tuning_force(f, 0 if builtin else -1)
        for _ in range(warmup + 1):   # the first convolution tunes the tile shapes
            p.convolve(-1, src, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            p.convolve(-1, src, out)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_builtin = timed(True)
    ms = timed(False)
    for f in fams:
        P.tuning_force(f, -1)
    tuned = [{"stage": r["stage"], "us": r["us"], "choice": r["choice"]} for r in P.tuning_report()
             if r["stage"] in fams]
    nb = fft_bytes(nl, m, s, 4)
    ach = nb / (ms * 1e-3) / 1e9
    del p, src, out
    return {"ms": ms, "ms_builtin_shapes": ms_builtin, "tuning": tuned, "dtype": "c64" if s == 8 else "c128",
            "workload": f"4 fields, live box {nl}, FFT {m}, G spectrum of k0 at 1 GHz",
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": nb}}


def fft_micro(args):
    r = fft_measure(args.steps, args.warmup, args.precision)
    print(json.dumps({"metric": "4-field zero-padded FFT convolution time", "value": r["ms"], "unit": "ms",
                      "higher_is_better": False, "steps": args.steps, "warmup": args.warmup,
                      "dtype": r["dtype"], "data": "synthetic", "config": {"workload": r["workload"]},
                      "ms_builtin_shapes": r["ms_builtin_shapes"], "tuning": r["tuning"],
                      "roofline": r["roofline"]}))


def batch_workload(args):
    """64 plane waves (8 x 8 incidence grid, polarisation alternating theta /
    phi) at 4 frequencies on a copper bar of the batching meshes (100 x 10 x 5
    um, 90 x 9 x 4 divisions = 4,824 triangles, sigma 5.8e7 S/m; 1, 3, 10 and
    30 GHz; 32^3 grid, near radius 5, skin-depth cutoff): each frequency is
    one request whose 64 right-hand sides are solved together (lock-step
    GMRES, batched products: near-field values streamed once per batch), and
    the four frequencies run concurrently on the library's server.  One step
    is the whole 4 x 64 batch.  The FP32 far field of one wave at 10 GHz is
    checked against an FP64 single-wave solve."""
    import torch
    from workloads import box_mesh
    from workloads.configs import multi_rhs_waves
    from paper_2003_11679_amd import Problem, Server
    xyz, tri = box_mesh((100e-6, 10e-6, 5e-6), (90, 9, 4))
    waves = multi_rhs_waves()[:args.nrhs]
    freqs = (1e9, 3e9, 10e9, 30e9)
    prec = 1 if args.precision == "fp32" else 0
    opts = dict(tol=args.tol, restart=args.restart, precond=args.precond, inner_relax=args.inner_relax)
    khat = [w.khat for w in waves]
    e0 = [w.e0 for w in waves]
    th = np.linspace(0.0, np.pi, 37)
    rhat = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)

    def problem(f, ctx=None):
        p = Problem(f, ctx=ctx)
        p.add_object(xyz, tri, eps_r=1.0, sigma=5.8e7)
        p.set_grid(-1, n=32, near_radius=5)
        p.set_skin_cutoff(args.skin_cutoff)
        p.set_augmented(bool(args.augmented))
        return p

    def one(timing=False):
        srv = Server(max_slots=len(freqs))
        t0 = time.perf_counter()
        ts = [srv.submit(problem(f, srv.ctx), khat, e0, prec, **opts) for f in freqs]
        infos, probs = [], []
        for t in ts:
            while True:
                i = srv.poll(t)
                if i["done"]:
                    break
                time.sleep(0.002)
            infos.append(i)
            probs.append(srv.take(t))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        srv.close()
        return probs, infos, dt

    ref = None
    for i in range(args.warmup):
        probs, infos, dt = one()
        print(f"[bench] batch warmup {i}: {dt:.2f}s {[x['report'] for x in infos]}", file=sys.stderr, flush=True)
        if i == 0:
            q = problem(10e9)
            q.setup()
            q.set_planewaves(khat[5], e0[5])
            q.solve(0, **opts)
            F64 = q.far_field(rhat)
            F32 = probs[2].far_field(rhat, rhs=5)
            ref = {"rel_err_far_field": float(np.abs(F32 - F64).max() / np.abs(F64).max()),
                   "wave": 5, "freq_hz": 10e9}
            print(f"[bench] fp64 single-wave reference: {ref}", file=sys.stderr, flush=True)
            del q
        del probs
    t0 = time.perf_counter()
    matvecs = kmatvecs = 0
    reps = []
    for i in range(args.steps):
        probs, infos, dt = one()
        for x in infos:
            matvecs += x["report"]["matvecs"]
            kmatvecs += x["report"]["k_matvecs"]
            reps.append(x)
        print(f"[bench] batch step {i}: {dt:.2f}s {[x['report'] for x in infos]}", file=sys.stderr, flush=True)
        del probs
    T = time.perf_counter() - t0
    nrhs = len(waves) * len(freqs)
    print(json.dumps({"metric": "RHS-matvecs/s of batched multi-RHS, multi-frequency solves", "value": matvecs / T,
                      "unit": "RHS-matvecs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": T / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "c64+f64" if prec == 1 else "c128", "data": "synthetic",
                      "config": {"workload": f"{len(waves)} plane waves (8x8 incidence grid, alternating "
                                             "polarisation) x 4 frequencies (1, 3, 10, 30 GHz), copper bar "
                                             "100x10x5 um, 4824 triangles, 32^3 grid, near radius 5, skin-depth "
                                             f"cutoff {args.skin_cutoff:g}, solve to {args.tol:g}; frequencies "
                                             "run concurrently on the server, right-hand sides in lock step"},
                      "k_matvecs_per_s": kmatvecs / T, "rhs_solves_per_s": args.steps * nrhs / T,
                      "batches_per_s": args.steps / T,
                      "converged": all(x["status"] == 0 for x in reps),
                      "residual_fp64_max": max(x["report"]["residual"] for x in reps),
                      "fp32_vs_fp64": ref,
                      "per_frequency_s": [x["t_end_s"] - x["t_start_s"] for x in reps[-len(freqs):]]}))


def serve_workload(args):
    """The seeded Poisson request stream (50 req/s): each request a sphere,
    box or ellipsoid with its own material and frequency, on the grid of the
    Sec. IV rule (near radius 3, skin-depth cutoff), submitted at its arrival
    time to the library's server; latency = completion - arrival (queueing,
    setup and solve).  The same requests run twice, FP32 + FP64 refinement
    and plain FP64; the far fields of each request are compared between the
    two."""
    import torch
    from workloads.configs import serving_trace, serving_mesh
    from paper_2003_11679_amd import Problem, Server
    trace = serving_trace()[:args.requests]
    reqs = []
    for r in trace:
        r = dict(r)
        r["nt"] = min(r["nt"], args.max_tri)
        xyz, tri = serving_mesh(r)
        reqs.append((r, xyz, tri))
    th = np.linspace(0.0, np.pi, 37)
    rhat = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)

    def run(prec):
        srv = Server(max_slots=args.slots)
        t0 = time.perf_counter()
        tickets = []
        for r, xyz, tri in reqs:
            dt = r["t"] - trace[0]["t"] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            p = Problem(r["freq"], ctx=srv.ctx)
            p.add_object(xyz, tri, eps_r=r["eps_r"], sigma=r["sigma"])
            p.set_grid(-1, n=0, near_radius=3)
            p.set_skin_cutoff(args.skin_cutoff)
            p.set_augmented(bool(args.augmented))
            tickets.append(srv.submit(p, (0.0, 0.0, -1.0), (1.0, 0.0, 0.0), prec, tol=args.tol, restart=args.restart,
                                      precond=args.precond, max_iter=args.max_iter,
                                      inner_max_iter=args.inner_max_iter,
                                      inner_relax=args.inner_relax))
        infos = [None] * len(tickets)
        far = [None] * len(tickets)
        started = [False] * len(tickets)
        left = set(range(len(tickets)))
        while left:
            for q in sorted(left):
                i = srv.poll(tickets[q])
                if i["running"] and not started[q]:
                    started[q] = True
                    print(f"[bench] {'fp32' if prec else 'fp64'} request {q + 1}: started", file=sys.stderr,
                          flush=True)
                if i["done"]:
                    infos[q] = i
                    left.discard(q)
                    pq = srv.take(tickets[q])
                    far[q] = pq.far_field(rhat) if i["status"] in (0, -5) else None
                    del pq
                    print(f"[bench] {'fp32' if prec else 'fp64'} request {q + 1}: status {i['status']} latency "
                          f"{i['t_end_s'] - i['t_submit_s']:.2f}s run {i['t_end_s'] - i['t_start_s']:.2f}s "
                          f"{i['report']}", file=sys.stderr, flush=True)
            time.sleep(0.005)
        wall = time.perf_counter() - t0
        srv.close()
        lat = [i["t_end_s"] - i["t_submit_s"] for i in infos]
        span = max(i["t_end_s"] for i in infos) - min(i["t_submit_s"] for i in infos)
        return {"solves_per_s": len(infos) / span, "latency_p50_s": float(np.percentile(lat, 50)),
                "latency_p99_s": float(np.percentile(lat, 99)), "converged": sum(i["status"] == 0 for i in infos),
                "wall_s": wall, "busy_s": sum(i["t_end_s"] - i["t_start_s"] for i in infos)}, infos, far

    prec = 1 if args.precision == "fp32" else 0
    main, infos, far = run(prec)
    ref = None
    if prec == 1:
        ref, infos64, far64 = run(0)
        errs = [float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(far, far64)
                if a is not None and b is not None]
        ref["far_field_rel_err_max"] = max(errs) if errs else None
        ref["far_field_rel_err_median"] = float(np.median(errs)) if errs else None
    tris = [len(t) for _, _, t in reqs]
    print(json.dumps({"metric": "served solves/s, p50/p99 latency", "value": main["solves_per_s"],
                      "unit": "solves/s", "n_gpus": 1, "steps": len(infos), "warmup": 0,
                      "ms_per_step": 1e3 / main["solves_per_s"], "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "c64+f64" if prec == 1 else "c128", "data": "synthetic",
                      "config": {"workload": f"first {len(infos)} requests of the seeded 50 req/s trace "
                                             f"({min(tris)}-{max(tris)} triangles, cap {args.max_tri}), "
                                             f"{args.slots} slots, Sec. IV grid rule, near radius 3, skin-depth "
                                             f"cutoff {args.skin_cutoff:g}, solve to {args.tol:g} (caps "
                                             f"{args.max_iter} outer / {args.inner_max_iter} nested iterations, "
                                             f"outer restart {args.restart}, preconditioner {args.precond})"},
                      **main, "offered_rate": 50.0, "fp64_same_requests": ref}))


def counters_workload(args):
    """Launches for `rocprofv3 --pmc FETCH_SIZE` / `WRITE_SIZE` runs, in this
    order: a plain 1 GiB device copy three times (calibration of the
    counters); five FP64 and five FP32 exterior L products of the copper bar
    (its near-field launches are the bar requests' dominant class); five FP32
    products of every interior medium of the cube array (SIE_INTERIORS: the
    nested operator's k_spmv_far launch over all 64 cubes).  Prints the
    algorithmic bytes of each class."""
    import torch
    from paper_2003_11679_amd import INTERIORS
    a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    SETUP_OPTS["skin_cutoff"] = args.skin_cutoff
    out = {"copy_bytes": 2 ** 30}
    p = build_problem(workload_cfg("bar"))
    for prec, dt in ((0, torch.complex128), (1, torch.complex64)):
        X = torch.randn(p.num_rwg, dtype=dt, device="cuda")
        Y = torch.empty_like(X)
        for _ in range(5):
            p.matvec(-1, 0, X, Y)
        torch.cuda.synchronize()
        nb, nnz = spmv_model(p, [-1], prec)
        out[f"bar_exterior{64 if prec == 0 else 32}"] = {"bytes": nb, "nnz": nnz}
    del p
    torch.cuda.synchronize()
    cfg = workload_cfg("cubes")
    p = build_problem(cfg)
    X = torch.randn(p.num_rwg, dtype=torch.complex64, device="cuda")
    Y = torch.empty_like(X)
    for _ in range(5):
        p.matvec(INTERIORS, 0, X, Y)
    torch.cuda.synchronize()
    nb, nnz = spmv_model(p, list(range(len(cfg.objects))), 1)
    out["cubes_interior32"] = {"bytes": nb, "nnz": nnz}
    print(json.dumps(out))


TRAFFIC_FILES = {"bar": "copper_bar", "cubes": "cube_array"}


def spmv_source_sha():
    """SHA-256 of the k_spmv_far kernel and its launcher in k_grid.hip (the
    code a stored counter measurement belongs to)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2003_11679_amd", "csrc", "k_grid.hip")).read()
    a = src.index("__global__ void k_spmv_far")
    b = src.index("// y[r][row] = sum_j N[row][j] xt[j][r]")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def spmv_traffic(workload, cls):
    """Measured HBM bytes per launch of the near-field class `cls` of the
    workload from the committed counter summary, if the kernel source is
    the one measured (else None)."""
    import hashlib
    import re
    if workload not in TRAFFIC_FILES:
        return None
    prof = os.path.join(ROOT, "profiles", f"k_spmv_far__{TRAFFIC_FILES[workload]}_traffic.md")
    if not os.path.exists(prof):
        return None
    sha = spmv_source_sha()
    for m in re.finditer(r"bench-traffic: class=(\w+) bytes_per_launch=(\d+) k_spmv_far_sha256=([0-9a-f]+)",
                         open(prof).read()):
        if m.group(1) == cls and m.group(3) == sha:
            return int(m.group(2))
    return None


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


def spmv_classes(p, ncfg_objects, prec):
    """Byte models of the near-field CSR launch classes of a request."""
    media = list(range(ncfg_objects))
    return {"interior": spmv_model(p, media, prec), "interior64": spmv_model(p, media, 0),
            "exterior64": spmv_model(p, [-1], 0), "exterior32": spmv_model(p, [-1], 1),
            "local": [p.is_local(m) for m in media]}


def dominant_kernel(tm, model, prec):
    """The near-field CSR launch class with the largest measured time, with
    its HIP-event average and algorithmic bytes."""
    ext64 = (tm["spmv64"][0] - tm["spmv_int64"][0], tm["spmv64"][1] - tm["spmv_int64"][1])
    ext32 = (tm["spmv"][0] - tm["spmv64"][0] - tm["spmv_int32"][0] - tm["spmv_skip"][0],
             tm["spmv"][1] - tm["spmv64"][1] - tm["spmv_int32"][1] - tm["spmv_skip"][1])
    cls = {"interior media": (tm["spmv_int32"] if prec == 1 else tm["spmv_int64"],
                              model["interior"] if prec == 1 else model["interior64"], prec == 1),
           "exterior medium": (ext64, model["exterior64"], False)}
    if prec == 1:
        cls["exterior medium, FP32"] = (ext32, model["exterior32"], True)
    name = max(cls, key=lambda k: cls[k][0][1])
    (n, ms), (nb, nnz), fp32 = cls[name]
    avg = ms / max(n, 1)
    ach = nb / (avg * 1e-3) / 1e9 if n else None
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS if ach else None,
            "kernel": ("k_spmv_far<float> " if fp32 else "k_spmv_far<double> ") + f"({name})",
            "class": {"interior media": "interior32" if fp32 else "interior64",
                      "exterior medium": "exterior64", "exterior medium, FP32": "exterior32"}[name],
            "avg_launch_ms": avg, "launches": n, "bytes_per_launch": nb, "nnz": nnz,
            "share_of_csr_time": ms / max(tm["spmv"][1], 1e-30)}


def tuning_summary():
    """Launch shapes the tuner chose for this process's grid stages:
    stage/precision/shape -> chosen candidate and its gain over the
    built-in shape."""
    import paper_2003_11679_amd as P
    out = {}
    for r in P.tuning_report():
        key = f"{r['stage']}/{r['precision']}/" + "x".join(str(v) for v in r["shape"])
        us = r["us"]
        out[key] = {"choice": r["choice"], "us_builtin": round(us[0], 1), "us_chosen": round(us[r["choice"]], 1)}
    return out


def fp64_gate(p, tol, opts):
    """FP64 solve of the same request; relative differences of the FP32
    currents and far field from it."""
    u32, v32 = p.currents()
    th = np.linspace(0.0, np.pi, 91)
    rhat = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)
    F32 = p.far_field(rhat)
    r64 = p.solve(0, tol=tol, **opts)
    u64, v64 = p.currents()
    F64 = p.far_field(rhat)
    return {"rel_err_u": float(np.linalg.norm(u32 - u64) / np.linalg.norm(u64)),
            "rel_err_v": float(np.linalg.norm(v32 - v64) / np.linalg.norm(v64)),
            "rel_err_far_field": float(np.abs(F32 - F64).max() / np.abs(F64).max()),
            "fp64_solve": r64}


NAMES = {"cubes": "8x8 array of lossy dielectric cubes (edge 0.2 lambda0, pitch 0.4 lambda0, eps_r ~ U[2,10], "
                  "sigma ~ U[0,10] S/m, seed 11682), 196608 triangles (294912 RWG), 1 GHz, exterior grid 256^3 "
                  "(FFT on the live box), one 16^3 grid per cube",
         "bar": "copper bar 100x10x5 um, sigma 5.8e7 S/m, 20088 triangles (30132 RWG), 10 GHz, 64^3 grid",
         "sphere": "dielectric sphere r = 1 m, eps_r 4, 1280 triangles (1920 RWG), 150 MHz, 44^3 grid "
                   "(the lambda_r/20 rule of Sec. IV)"}


def nested_mode_comparison(args, cfg, prec, nreq):
    """The same request with the other keep_converged setting: with 1 every
    object's nested product is computed in every nested iteration (more L
    products per second, slower solves); with 0 the objects whose systems
    have converged are skipped."""
    import torch
    keep = 1 - args.keep_converged
    opts = dict(SOLVE_OPTS, keep_converged=keep)
    lat, mv = [], 0
    for i in range(nreq):
        p, rep, su, tot = run_request(cfg, prec, args.tol, opts=opts)
        del p
        lat.append(tot)
        mv += rep["matvecs"]
        print(f"[bench] keep_converged={keep} request {i}: total {tot:.2f}s {rep}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return {"keep_converged": keep, "requests": nreq, "request_s_mean": float(np.mean(lat)),
            "matvecs_per_request": mv // nreq, "matvecs_per_s": mv / float(np.sum(lat)),
            "solves_per_s": nreq / float(np.sum(lat))}


def secondary_request(args, name, nreq):
    """`nreq` requests of another configuration after the timed steps (its
    default options, FP32 + refinement), with the near-field kernel roofline
    and the FP64 gate of the first one."""
    import torch
    cfg = workload_cfg(name)
    opts = dict(restart=1000, precond=DEFAULT_PRECOND.get(name, 4), inner_relax=args.inner_relax)
    tol = DEFAULT_TOL.get(name, 1e-6)
    tm = {k: [0, 0.0] for k in ("spmv", "spmv64", "spmv_int32", "spmv_int64", "spmv_skip")}
    lat, reps, setups, gate, model = [], [], [], None, None
    for i in range(nreq):
        p, rep, su, tot = run_request(cfg, 1, tol, timing=True, opts=opts)
        st = p.stage_times()
        for k in tm:
            tm[k][0] += st[k][0]
            tm[k][1] += st[k][1]
        if model is None:
            model = spmv_classes(p, len(cfg.objects), 1)
        print(f"[bench] {name} request {i}: setup {su:.2f}s total {tot:.2f}s {rep}", file=sys.stderr, flush=True)
        if i == 0:
            gate = fp64_gate(p, tol, opts)
            print(f"[bench] {name} fp64 gate: {gate}", file=sys.stderr, flush=True)
        del p
        torch.cuda.synchronize()
        lat.append(tot); reps.append(rep); setups.append(su)
    roof = dominant_kernel({k: tuple(v) for k, v in tm.items()}, model, 1)
    roof["traffic"] = spmv_traffic(name, roof["class"])
    return {"workload": NAMES[name] + f", near radius {cfg.near_radius}, plane wave -z x-polarised, 1 RHS, "
                                      f"FP32 + FP64 refinement to {tol:g}"
                                      + (", augmented EFIE" if SETUP_OPTS["augmented"] else ""),
            "requests": nreq, "request_s_mean": float(np.mean(lat)), "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)), "setup_s_mean": float(np.mean(setups)),
            "matvecs_per_s": sum(r["matvecs"] for r in reps) / sum(lat),
            "k_matvecs_per_s": sum(r["k_matvecs"] for r in reps) / sum(lat),
            "converged": all(r["converged"] for r in reps), "report": reps[-1],
            "roofline": roof, "fp32_vs_fp64": gate}


def request_workload(args):
    """Solve requests of one configuration (see the module docstring)."""
    import torch
    cfg = workload_cfg(args.workload)
    prec = 1 if args.precision == "fp32" else 0
    SOLVE_OPTS.update(restart=args.restart, precond=args.precond, inner_relax=args.inner_relax,
                      keep_converged=args.keep_converged)
    SETUP_OPTS["skin_cutoff"] = args.skin_cutoff
    SETUP_OPTS["augmented"] = bool(args.augmented)
    T = sum(len(o.tri) for o in cfg.objects)
    print(f"[bench] workload {args.workload}: {len(cfg.objects)} objects, {T} triangles, precision "
          f"{args.precision}, warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    ref = None
    model = None
    for i in range(args.warmup):
        p, rep, su, tot = run_request(cfg, prec, args.tol)
        print(f"[bench] warmup {i}: setup {su:.2f}s total {tot:.2f}s {rep}", file=sys.stderr, flush=True)
        if model is None:
            model = spmv_classes(p, len(cfg.objects), prec)
        if i == 0 and prec == 1:
            ref = fp64_gate(p, args.tol, SOLVE_OPTS)
            print(f"[bench] fp64 reference: {ref}", file=sys.stderr, flush=True)
        del p
    torch.cuda.synchronize()
    lat, matvecs, kmatvecs, setups, reps = [], 0, 0, [], []
    tm = {k: [0, 0.0] for k in ("spmv", "spmv64", "spmv_int32", "spmv_int64", "spmv_skip")}
    t0 = time.perf_counter()
    for i in range(args.steps):
        p, rep, su, tot = run_request(cfg, prec, args.tol, timing=True)
        st = p.stage_times()
        for k in tm:
            tm[k][0] += st[k][0]
            tm[k][1] += st[k][1]
        if model is None:
            model = spmv_classes(p, len(cfg.objects), prec)
        del p            # release the request's device memory before the next one
        lat.append(tot); setups.append(su); reps.append(rep)
        matvecs += rep["matvecs"]
        kmatvecs += rep["k_matvecs"]
        print(f"[bench] step {i}: setup {su:.2f}s total {tot:.2f}s {rep}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    Tt = time.perf_counter() - t0
    roof = dominant_kernel({k: tuple(v) for k, v in tm.items()}, model, prec)
    roof["traffic"] = spmv_traffic(args.workload, roof["class"])
    out = {
        "metric": "SIE matvecs/s + served solves/s, p50/p99 latency at rel err <=1e-3 vs FP64",
        "value": matvecs / Tt,
        "unit": "SIE matvecs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": Tt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64" if prec == 1 else "c128",
        "data": "synthetic",
        "config": {"workload": NAMES[args.workload] + f", near radius {cfg.near_radius}, plane wave -z "
                               f"x-polarised, 1 RHS, "
                               + ("augmented EFIE (eq. sys) with nested GIBC interiors" if args.augmented
                                  else "GIBC system of the EFIE")
                               + f" solved to a relative FP64 residual of {args.tol:g}"
                               + (f", skin-depth cutoff {args.skin_cutoff:g}" if args.skin_cutoff else ""),
                   "precision": args.precision, "nnz_near_interior": int(model["interior"][1]),
                   "nnz_near_exterior": int(model["exterior64"][1]),
                   "interior_media_without_grid_part": int(sum(model["local"]))},
        "k_matvecs_per_s": kmatvecs / Tt,
        "solves_per_s": args.steps / Tt,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "setup_s_mean": float(np.mean(setups)),
        "converged": all(r["converged"] for r in reps),
        "tol": args.tol,
        "fp32_vs_fp64": ref,
        "residual_fp64_max": max(r["residual"] for r in reps),
        "outer_iters": reps[-1]["outer_iters"], "inner_iters": reps[-1]["inner_iters"],
        "refine_sweeps": reps[-1]["refine_sweeps"],
        "roofline": roof,
        "tuned_shapes": tuning_summary(),
    }
    if not args.no_secondary:
        if args.workload == "cubes":
            out["other_nested_mode"] = nested_mode_comparison(args, cfg, prec, 3)
            out["copper_bar"] = secondary_request(args, "bar", 5)
            print("[bench] FFT convolution (4 fields, 512^3)", file=sys.stderr, flush=True)
            out["fft_convolution"] = fft_measure(10, 2, "fp32")
        elif args.workload == "bar":
            out["cube_array"] = secondary_request(args, "cubes", 1)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle AIM product, bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_aim(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
