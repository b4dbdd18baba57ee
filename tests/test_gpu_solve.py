"""GPU GIBC solve against the oracle: excitation and far field, residual of
the GPU solution measured with the oracle's AIM operators, agreement with the
dense solution and with the Mie series, FP32 + FP64 refinement vs FP64."""
import numpy as np
import pytest

from cases import CASES, gpu_problem, oracle_aim, mesh_of

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KHAT = (0.0, 0.0, 1.0)
E0 = (1.0, 0.0, 0.0)


@pytest.fixture(scope="module")
def solved():
    out = {}
    for name in ("sphere2", "sphere2_lossy", "box_cond"):
        print(f"[solve {name}]", flush=True)
        p = gpu_problem(name)
        p.set_planewaves(KHAT, E0)
        r64 = p.solve(0)
        u64, v64 = p.currents()
        r32 = p.solve(1)
        u32, v32 = p.currents()
        out[name] = dict(p=p, r64=r64, r32=r32, u64=u64, v64=v64, u32=u32, v32=v32)
        print(f"  fp64 {r64}\n  fp32 {r32}", flush=True)
    return out


def _dense(name):
    from oracle.rwg import RWGMesh
    from oracle.solve import DenseProblem
    build, eps_r, sigma, freq, n, R = CASES[name]
    m = RWGMesh([build()])
    return DenseProblem(m, freq, [(eps_r, 1.0, sigma)])


def test_converged(solved):
    for name, s in solved.items():
        assert s["r64"]["converged"] and s["r64"]["residual"] <= 1e-5, (name, s["r64"])
        assert s["r32"]["converged"] and s["r32"]["residual"] <= 1e-5, (name, s["r32"])


def test_fp32_refined_matches_fp64(solved):
    """The spheres' systems are well conditioned: currents agree to 2e-5.  The
    conducting box is electrically tiny (k0 l = 0.06), its exterior EFIE
    conditioning (~1e8) turns the 1e-6 residual into ~1e-3 current
    differences along near-null directions that do not radiate; there the far
    field is compared tightly."""
    th = np.linspace(0.0, np.pi, 13)
    rhat = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)
    for name, s in solved.items():
        tol = 1e-3 if name == "box_cond" else 2e-5
        for a, b in ((s["u32"], s["u64"]), (s["v32"], s["v64"])):
            err = np.linalg.norm(a - b) / np.linalg.norm(b)
            print(f"{name}: fp32 vs fp64 currents {err:.2e}")
            assert err <= tol, (name, err)
        if name == "box_cond":
            p = s["p"]
            u, v = p.currents()
            f32 = p.far_field(rhat)
            p.solve(0)
            f64 = p.far_field(rhat)
            err = np.abs(f32 - f64).max() / np.abs(f64).max()
            print(f"{name}: fp32 vs fp64 far field {err:.2e}")
            assert err < 1e-5, (name, err)


def test_solution_satisfies_oracle_aim_system(solved):
    """Block residual of the GPU solution computed with the oracle's AIM
    operators (same approximation, independent implementation)."""
    from oracle import physics as ph
    from oracle.mom import excitation, x_matrix
    for name, s in solved.items():
        build, eps_r, sigma, freq, n, R = CASES[name]
        ext, inn = oracle_aim(name, -1), oracle_aim(name, 0)
        m = ext.mesh
        w = ph.omega(freq)
        X = x_matrix(m)
        u, v = s["u64"], s["v64"]
        e = excitation(m, ph.wavenumber(freq, 1.0), KHAT, E0)
        r1 = e - (1j * w * ph.MU0 * ext.matvec(u, "L") - (ext.matvec(v, "K") - 0.5 * X @ v))
        et = ph.eps_tilde(freq, eps_r, sigma)
        r2 = -(-(inn.matvec(u, "K") + 0.5 * X @ u) - 1j * w * et * inn.matvec(v, "L"))
        rel = np.sqrt(np.linalg.norm(r1) ** 2 + np.linalg.norm(r2) ** 2) / np.linalg.norm(e)
        assert rel < 1e-5, (name, rel)


def test_close_to_dense_solution(solved):
    """AIM solution vs the dense (unaccelerated) oracle solution on the coarse
    test grids.  The lossless eps_r = 4 sphere (12^3, near radius 3) sits near
    an interior cavity resonance (k_i a = 6.29), which amplifies the ~1e-3
    operator error of its grid in the solution.  The lossy sphere's grid
    (10^3, h = 0.29 m, near radius 2) is far coarser than the lambda/20 rule of
    Sec. IV for its interior wavenumber (|k_i| h = 7): the oracle's own AIM
    operators, assembled densely, are 1-3e-2 from the dense ones there and the
    oracle's AIM solution is 3.6e-2 (u) / 2.8e-2 (v) from the dense solution;
    the GPU solution equals the oracle's AIM one (the system-residual test).
    The conducting box (skin depth 1e-2 of an edge) has an essentially local
    interior operator; its AIM solution is 1.2e-3 (u) / 3.0e-3 (v) from the
    dense one with the oracle's own operators."""
    tols = {"sphere2_lossy": 5e-2, "sphere2": 0.1, "box_cond": 1e-2}
    for name, s in solved.items():
        dp = _dense(name)
        e = dp.rhs(KHAT, E0)
        u, v = dp.solve_block(e)
        eu = float(np.linalg.norm(s["u64"] - u) / np.linalg.norm(u))
        ev = float(np.linalg.norm(s["v64"] - v) / np.linalg.norm(v))
        print(f"{name}: |du|/|u| = {eu:.2e}, |dv|/|v| = {ev:.2e}")
        assert eu < tols[name] and ev < tols[name], (name, eu, ev)


def test_excitation_and_far_field_match_oracle(solved):
    from oracle import physics as ph
    from oracle.rwg import RWGMesh
    from oracle.farfield import far_field, directions
    s = solved["sphere2"]
    p = s["p"]
    m = RWGMesh([mesh_of("sphere2")])
    k0 = ph.wavenumber(CASES["sphere2"][3], 1.0)
    th = np.linspace(0.05, np.pi - 0.05, 9)
    rhat = directions(th, 0.3 + 0 * th)
    F = p.far_field(rhat)
    Fo = far_field(m, k0, ph.ETA0, s["u32"], s["v32"], rhat)
    assert np.abs(F - Fo).max() < 1e-10 * np.abs(Fo).max()


def test_rcs_against_mie(solved):
    from oracle import physics as ph, mie
    from oracle.farfield import directions
    s = solved["sphere2"]
    p = s["p"]
    build, eps_r, sigma, freq, n, R = CASES["sphere2"]
    k0 = ph.wavenumber(freq, 1.0)
    th = np.linspace(0.02, np.pi - 0.02, 41)
    err2 = ref2 = 0.0
    for phi in (0.0, np.pi / 2):
        F = p.far_field(directions(th, phi + 0 * th))
        r = 4 * np.pi * np.sum(np.abs(F) ** 2, axis=1)
        mr = mie.bistatic_rcs(k0, 1.0, eps_r, th, phi + 0 * th)
        err2 += np.sum((r - mr) ** 2); ref2 += np.sum(mr ** 2)
    assert np.sqrt(err2 / ref2) < 0.10


def test_relaxed_nested_tolerance(solved):
    """FP32 with the nested tolerance relaxed along the outer residual
    (inexact Krylov): same convergence test in FP64, same agreement with the
    FP64 solution as the fixed tolerance, no more nested iterations; a
    negative relaxation factor is rejected.  Runs last: it replaces the
    problems' solutions."""
    from paper_2003_11679_amd import SieError
    for name, s in solved.items():
        p = s["p"]
        r = p.solve(1, inner_relax=0.1)
        u, v = p.currents()
        print(f"{name}: relaxed {r} fixed {s['r32']}", flush=True)
        assert r["converged"] and r["residual"] <= 1e-5, (name, r)
        assert r["inner_iters"] <= s["r32"]["inner_iters"] + 5, (name, r, s["r32"])
        tol = 1e-3 if name == "box_cond" else 2e-5
        for a, b in ((u, s["u64"]), (v, s["v64"])):
            err = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert err <= tol, (name, err)
    with pytest.raises(SieError):
        solved["sphere2"]["p"].solve(1, inner_relax=-1.0)
