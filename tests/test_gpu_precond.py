"""Nested-solve preconditioner M_i = -j w eps_i L_i,NR (eq. nest2pc) in
restricted additive Schwarz form on the GPU: parity with the plain reference
built from the oracle's direct near-region operator (clusters of C^3 grid
cells with O cells of overlap, O = max(1, round(3 l / h)) for the mean RWG
edge l, C = 2 O), batched right-hand sides, identity on media whose
field does not decay within the near region, option validation, and a
solve that reaches the same solution in fewer nested iterations."""
import numpy as np
import pytest

from cases import CASES, gpu_problem, oracle_aim, vec
from schwarz_ref import clusters, schwarz_matrix
from oracle import physics as ph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _reference(name):
    op = oracle_aim(name, 0)
    build, eps_r, sigma, freq, n, R = CASES[name]
    scale = -1j * ph.omega(freq) * ph.eps_tilde(freq, eps_r, sigma)
    O = max(1, int(np.floor(3.0 * op.mesh.length.mean() / op.grid.h + 0.5)))
    cl = clusters(op.centres[op.mesh.tp], 2 * O, O)
    assert max(len(e) for _, e in cl) <= 2048
    return schwarz_matrix(scale * op.NLd.toarray(), cl), len(cl)


def test_schwarz_matches_reference():
    print("[precond schwarz bar_small]", flush=True)
    p = gpu_problem("bar_small")
    P, ncl = _reference("bar_small")
    X = np.stack([vec(p.num_rwg, 40 + r) for r in range(3)])
    ref = X @ P.T
    for dtype, tol in ((torch.complex128, 1e-9), (torch.complex64, 2e-5)):
        xd = torch.from_numpy(X).to("cuda", dtype)
        got = p.nested_precond(4, xd).cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < tol, (dtype, err)
        # one right-hand side at a time gives the same columns
        one = p.nested_precond(4, xd[1]).cpu().numpy()
        assert np.array_equal(one, got[1])
    nc, owned = p.nested_precond_clusters()
    assert nc == ncl and owned == p.num_rwg


def test_schwarz_is_identity_without_conductive_media():
    """A lossless dielectric gets no clusters: the rows pass through."""
    print("[precond schwarz sphere2]", flush=True)
    p = gpu_problem("sphere2")
    x = torch.from_numpy(vec(p.num_rwg, 5)).to("cuda", torch.complex128)
    y = p.nested_precond(4, x)
    assert torch.equal(x, y)
    assert p.nested_precond_clusters() == (0, 0)


def test_precond_options_validated():
    from paper_2003_11679_amd import SieError
    p = gpu_problem("bar_small")
    p.set_planewaves((0.0, 0.0, -1.0), (1.0, 0.0, 0.0))
    with pytest.raises(SieError):
        p.solve(0, tol=1e-6, precond=5)
    with pytest.raises(SieError):
        p.solve(0, tol=1e-6, precond=8)
    x = torch.zeros(p.num_rwg, dtype=torch.complex128, device="cuda")
    with pytest.raises(SieError):
        p.nested_precond(2, x)


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_with_schwarz_matches_unpreconditioned(prec):
    print(f"[precond solve bar_small prec {prec}]", flush=True)
    p = gpu_problem("bar_small")
    p.set_planewaves((0.0, 0.0, -1.0), (1.0, 0.0, 0.0))
    th = np.linspace(0.0, np.pi, 13)
    rhat = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)
    r0 = p.solve(prec, tol=1e-8, restart=200, precond=0)
    f0 = p.far_field(rhat)
    r4 = p.solve(prec, tol=1e-8, restart=200, precond=4)
    f4 = p.far_field(rhat)
    print(f"  none {r0}\n  schwarz {r4}", flush=True)
    assert r0["converged"] and r4["converged"]
    assert np.abs(f4 - f0).max() < 1e-5 * np.abs(f0).max()
    assert r4["inner_iters_max"] < r0["inner_iters_max"]


def test_near_lu_matches_spsolve():
    """precond 16 on the copper bar (full near list, 936 RWG functions: the
    factorisation ends in one dense front): parity with scipy's sparse solve
    of the oracle's direct near-region operator, and a solve that agrees
    with the Schwarz one in at most as many nested iterations."""
    from scipy.sparse.linalg import spsolve
    print("[precond near-region LU bar_small]", flush=True)
    p = gpu_problem("bar_small")
    op = oracle_aim("bar_small", 0)
    build, eps_r, sigma, freq, n, R = CASES["bar_small"]
    scale = -1j * ph.omega(freq) * ph.eps_tilde(freq, eps_r, sigma)
    A = (scale * op.NLd).tocsc()
    X = np.stack([vec(p.num_rwg, 50 + r) for r in range(2)])
    ref = np.stack([spsolve(A, x) for x in X])
    got = p.nested_precond(16, torch.from_numpy(X).to("cuda", torch.complex128)).cpu().numpy()
    assert np.linalg.norm(got - ref) < 1e-8 * np.linalg.norm(ref)
    nm, nnz, t = p.nested_precond_factored()
    assert nm == 1 and nnz > 0
    p.set_planewaves((0.0, 0.0, -1.0), (1.0, 0.0, 0.0))
    th = np.linspace(0.0, np.pi, 13)
    rhat = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)
    r4 = p.solve(0, tol=1e-8, restart=200, precond=4)
    f4 = p.far_field(rhat)
    r16 = p.solve(0, tol=1e-8, restart=200, precond=16)
    f16 = p.far_field(rhat)
    print(f"  schwarz {r4}\n  near LU {r16}", flush=True)
    assert r4["converged"] and r16["converged"]
    assert np.abs(f16 - f4).max() < 1e-5 * np.abs(f4).max()
    assert r16["inner_iters"] <= r4["inner_iters"]


def test_near_lu_dense_fronts_match_dense_solve():
    """precond 16 where every pair of a sphere's 3,630 RWG functions is near
    (so M_i is dense): the dissection's separators exceed 1,024 unknowns and
    the large fronts are eliminated on the device.  Parity with a dense
    solve of the same near-region matrix, and the solve of the problem with
    one nested iteration per solve."""
    from paper_2003_11679_amd import Problem
    from workloads import geodesic_sphere
    from cases import QUAD
    freq, eps_r, sigma = 150e6, 4.0, 0.2
    print("[precond near-region LU, dense fronts: geodesic sphere nu=11]", flush=True)
    xyz, tri = geodesic_sphere(11)
    p = Problem(freq)
    p.add_object(xyz, tri, eps_r=eps_r, sigma=sigma)
    p.set_grid(-1, n=8, near_radius=6)
    p.set_quadrature(**QUAD)
    p.setup()
    E = p.num_rwg
    assert E == 3630 and p.is_local(0)
    rp, cols = p.near_pattern(0)
    assert len(cols) == E * E
    scale = -1j * ph.omega(freq) * ph.eps_tilde(freq, eps_r, sigma)
    A = np.zeros((E, E), complex)
    A[np.repeat(np.arange(E), np.diff(rp)), cols] = scale * p.near_values(0, 0)
    X = np.stack([vec(E, 70 + r) for r in range(2)])
    ref = np.linalg.solve(A, X.T).T
    got = p.nested_precond(16, torch.from_numpy(X).to("cuda", torch.complex128)).cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    nm, nnz, t = p.nested_precond_factored()
    print(f"  rel err {err:.2e}, factors {nnz} off-block entries, {t:.3f} s", flush=True)
    assert err < 1e-9
    assert nm == 1 and nnz > 0
    # FP32 vectors are solved with FP32 copies of the factors
    x32 = X[0].astype(np.complex64)
    got32 = p.nested_precond(16, torch.from_numpy(x32).to("cuda")).cpu().numpy()
    ref32 = np.linalg.solve(A, x32.astype(np.complex128))
    err32 = np.linalg.norm(got32 - ref32) / np.linalg.norm(ref32)
    print(f"  FP32 factors: rel err {err32:.2e}", flush=True)
    assert err32 < 1e-6
    p.set_planewaves((0.0, 0.0, -1.0), (1.0, 0.0, 0.0))
    r = p.solve(0, tol=1e-8, restart=200, precond=16)
    print(f"  solve {r}", flush=True)
    assert r["converged"] and r["inner_iters_max"] == 1, r


def test_near_lu_options_validated():
    from paper_2003_11679_amd import SieError
    p = gpu_problem("bar_small")
    p.set_planewaves((0.0, 0.0, -1.0), (1.0, 0.0, 0.0))
    with pytest.raises(SieError):
        p.solve(0, tol=1e-6, precond=17)
    with pytest.raises(SieError):
        p.solve(0, tol=1e-6, precond=32)
    x = torch.zeros(p.num_rwg, dtype=torch.complex128, device="cuda")
    with pytest.raises(SieError):
        p.nested_precond(24, x)
