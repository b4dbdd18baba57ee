"""GPU parity of the augmented EFIE (Sec. III-E, eq. sys): the augmented
exterior product against the oracle's AIM form of it, the constraint
preconditioner against the oracle's block elimination, and augmented solves
whose block residual is measured with the oracle's operators; the constraint
preconditioner's effect on the outer iteration count."""
import numpy as np
import pytest

from cases import CASES, QUAD, oracle_aim, vec, gpu_multi, oracle_multi, multi_meshes, MULTI_OBJECTS, MULTI_FREQ

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KHAT = (0.0, 0.0, -1.0)
E0 = (1.0, 0.0, 0.0)


def _gpu_bar(augmented):
    from paper_2003_11679_amd import Problem
    build, eps_r, sigma, freq, n, R = CASES["bar_small"]
    xyz, tri = build()
    p = Problem(freq)
    p.add_object(xyz, tri, eps_r=eps_r, sigma=sigma)
    p.set_grid(-1, n=n, near_radius=R)
    p.set_quadrature(**QUAD)
    p.set_augmented(augmented)
    p.setup()
    return p


@pytest.fixture(scope="module")
def bar():
    """Reduced copper bar at 10 GHz (624 triangles, k0 h ~ 1e-3)."""
    from oracle.aefie import AugmentedAIM
    print("[augmented EFIE: bar_small]", flush=True)
    p = _gpu_bar(True)
    aa = AugmentedAIM(oracle_aim("bar_small", -1), rules=QUAD)
    return p, aa


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_setup_reports_the_schur_factors(bar):
    p, _ = bar
    info = p.augmented_info()
    assert info["on"] and info["factor_nnz"] > 0 and info["levels"] >= 1, info


def test_aug_product_matches_oracle(bar):
    """SIE_OP_AUG against AugmentedAIM: j k0 (NA + grid part) u - Dv^T (NG +
    grid part) sigma, and the weighted continuity rows."""
    p, aa = bar
    E, T = p.num_rwg, p.num_tri
    x = vec(E + T, 41)
    got = p.aug_matvec(_dev(x)).cpu().numpy()
    ref = aa.matvec(x)
    assert np.linalg.norm(got[:E] - ref[:E]) < 1e-10 * np.linalg.norm(ref[:E])
    assert np.linalg.norm(got[E:] - ref[E:]) < 1e-12 * np.linalg.norm(ref[E:])


def test_aug_product_batched_equals_single(bar):
    p, _ = bar
    E, T = p.num_rwg, p.num_tri
    X = vec(E + T, 42, nrhs=3)
    Y = p.aug_matvec(_dev(X)).cpu().numpy()
    for r in range(3):
        y = p.aug_matvec(_dev(X[r])).cpu().numpy()
        assert np.abs(Y[r] - y).max() <= 1e-12 * np.abs(y).max(), r


def test_augmented_setup_keeps_the_other_operators(bar):
    """The exterior L and K near values of an augmented setup are those of a
    plain one, bit for bit."""
    p, _ = bar
    q = _gpu_bar(False)
    for opk in (0, 1):
        assert np.array_equal(p.near_values(-1, opk), q.near_values(-1, opk)), opk


def _dense_aug(meshes, freq, materials):
    from oracle.rwg import RWGMesh
    from oracle.aefie import AugmentedProblem
    return AugmentedProblem(RWGMesh(meshes), freq, materials, rules=QUAD)


def test_constraint_preconditioner_matches_oracle(bar):
    """P^-1 r on the device (Schur factors by nested dissection) against the
    oracle's block elimination with the same direct self terms."""
    p, _ = bar
    build, eps_r, sigma, freq, n, R = CASES["bar_small"]
    dp = _dense_aug([build()], freq, [(eps_r, 1.0, sigma)])
    E, T = p.num_rwg, p.num_tri
    r = vec(E + T, 43)
    got = p.constraint_precond(_dev(r)).cpu().numpy()
    ref = dp.apply_preconditioner(r)
    assert np.linalg.norm(got - ref) < 1e-8 * np.linalg.norm(ref)
    R2 = vec(E + T, 44, nrhs=2)
    G2 = p.constraint_precond(_dev(R2)).cpu().numpy()
    for k in range(2):
        ref = dp.apply_preconditioner(R2[k])
        assert np.linalg.norm(G2[k] - ref) < 1e-8 * np.linalg.norm(ref), k


def _block_residual_aug(aa, ext, ints, X, freq, e, u, sg, v):
    """Relative residual of the augmented block system with the oracle's AIM
    operators: exterior rows of eq. sys with v kept, interior rows of eq.
    MFIE1dis."""
    from oracle import physics as ph
    E = len(u)
    w = ph.omega(freq)
    eta0 = float(np.sqrt(ph.MU0 / ph.EPS0))
    y = aa.matvec(np.concatenate([u, sg]))
    r1 = np.concatenate([e / eta0, np.zeros(len(sg))]) - y
    r1[:E] += (ext.matvec(v, "K") - 0.5 * X @ v) / eta0
    Ku = np.zeros_like(u)
    Lv = np.zeros_like(v)
    for off, n, o, eps_r, sigma in ints:
        Ku[off:off + n] = o.matvec(u[off:off + n], "K")
        Lv[off:off + n] = ph.eps_tilde(freq, eps_r, sigma) * o.matvec(v[off:off + n], "L")
    r2 = (Ku + 0.5 * X @ u) + 1j * w * Lv
    return np.sqrt(np.linalg.norm(r1) ** 2 + np.linalg.norm(r2) ** 2) / np.linalg.norm(e / eta0)


def test_augmented_solve_satisfies_oracle_system(bar):
    """FP64 and FP32 + refinement augmented solves of the copper bar: the
    oracle's AIM operators leave a block residual at the solve tolerance;
    FP32 agrees with FP64; the constraint preconditioner needs far fewer
    outer iterations than the GIBC system."""
    from oracle.rwg import RWGMesh
    from oracle.mom import excitation, x_matrix
    from oracle import physics as ph
    p, aa = bar
    build, eps_r, sigma, freq, n, R = CASES["bar_small"]
    m = RWGMesh([build()])
    X = x_matrix(m)
    e = excitation(m, ph.wavenumber(freq, 1.0), KHAT, E0)
    ints = [(0, m.nrwg, oracle_aim("bar_small", 0), eps_r, sigma)]
    ext = oracle_aim("bar_small", -1)
    p.set_planewaves(KHAT, E0)
    r64 = p.solve(0, tol=1e-9, restart=400, precond=4)
    print("augmented fp64", r64, flush=True)
    assert r64["converged"], r64
    u64, v64 = p.currents()
    s64 = p.charges()
    assert _block_residual_aug(aa, ext, ints, X, freq, e, u64, s64, v64) < 5e-9
    r32 = p.solve(1, tol=1e-9, restart=400, precond=4)
    print("augmented fp32", r32, flush=True)
    assert r32["converged"], r32
    u32, v32 = p.currents()
    assert np.linalg.norm(u32 - u64) < 1e-6 * np.linalg.norm(u64)
    q = _gpu_bar(False)
    q.set_planewaves(KHAT, E0)
    rq = q.solve(0, tol=1e-9, restart=400, precond=4)
    print("gibc fp64", rq, flush=True)
    assert r64["outer_iters"] < 0.5 * rq["outer_iters"], (r64["outer_iters"], rq["outer_iters"])
    # the two formulations solve for the same currents
    uq, _ = q.currents()
    assert np.linalg.norm(uq - u64) < 1e-3 * np.linalg.norm(u64)


@pytest.fixture(scope="module")
def multi_aug():
    from paper_2003_11679_amd import Problem
    from cases import MULTI_EXT, MULTI_INT
    print("[augmented EFIE: 3 spheres + 1 box]", flush=True)
    p = Problem(MULTI_FREQ)
    for b, eps_r, sigma in MULTI_OBJECTS:
        xyz, tri = b()
        p.add_object(xyz, tri, eps_r=eps_r, sigma=sigma)
    p.set_grid(-1, n=MULTI_EXT[0], near_radius=MULTI_EXT[1])
    for i in range(len(MULTI_OBJECTS)):
        p.set_grid(i, n=MULTI_INT[0], near_radius=MULTI_INT[1], share=0)
    p.set_quadrature(**QUAD)
    p.set_augmented(True)
    p.setup()
    return p


def test_multi_object_preconditioner_and_solve(multi_aug):
    """Several objects: the Schur complement has one block per object; the
    augmented solve leaves the oracle's block residual at the tolerance."""
    from oracle.aefie import AugmentedAIM
    from oracle.mom import excitation, x_matrix
    from oracle import physics as ph
    p = multi_aug
    m, ext, ints = oracle_multi(4)
    dp = _dense_aug(multi_meshes(4), MULTI_FREQ, [(e, 1.0, s) for _, e, s in MULTI_OBJECTS])
    E, T = p.num_rwg, p.num_tri
    r = vec(E + T, 45)
    got = p.constraint_precond(_dev(r)).cpu().numpy()
    ref = dp.apply_preconditioner(r)
    assert np.linalg.norm(got - ref) < 1e-8 * np.linalg.norm(ref)
    aa = AugmentedAIM(ext, rules=QUAD)
    x = vec(E + T, 46)
    y = p.aug_matvec(_dev(x)).cpu().numpy()
    assert np.linalg.norm(y - aa.matvec(x)) < 1e-10 * np.linalg.norm(aa.matvec(x))
    khat = (0.3, 0.0, -float(np.sqrt(1.0 - 0.09)))
    e0 = (0.0, 1.0, 0.0)
    p.set_planewaves(khat, e0)
    r64 = p.solve(0, tol=1e-8)
    print("multi augmented fp64", r64, flush=True)
    assert r64["converged"], r64
    u, v = p.currents()
    sg = p.charges()
    X = x_matrix(m)
    e = excitation(m, ph.wavenumber(MULTI_FREQ, 1.0), khat, e0)
    assert _block_residual_aug(aa, ext, ints, X, MULTI_FREQ, e, u, sg, v) < 5e-8
