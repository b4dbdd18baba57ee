"""Local forms of the interior operator on the GPU against the oracle: the
five-skin-depth cutoff (Sec. V) on a conducting box, where the interior then
has no grid part and its own cut near list (Sec. III-D-2 item a), and the
small-object bypass when every pair of a grid is near (item b)."""
import numpy as np
import pytest

from cases import QUAD, vec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FREQ, SIGMA = 1e9, 1e5          # skin depth 50 um; 5 skin depths within R h = 1 mm
BOX = ((3e-3, 2e-3, 2e-3), (6, 4, 4))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def box():
    from paper_2003_11679_amd import Problem
    from workloads import box_mesh
    from oracle.rwg import RWGMesh
    from oracle.aim import Grid, AIMOperator
    from oracle import physics as ph
    print("[conducting box with skin-depth cutoff]", flush=True)
    xyz, tri = box_mesh(*BOX)
    p = Problem(FREQ)
    p.add_object(xyz, tri, eps_r=1.0, sigma=SIGMA)
    p.set_grid(-1, n=12, near_radius=3)
    p.set_quadrature(**QUAD)
    p.set_skin_cutoff(5.0)
    p.setup()
    m = RWGMesh([(xyz, tri)])
    g = Grid.enclosing(m.xyz, 12)
    k = ph.wavenumber(FREQ, 1.0, 1.0, SIGMA)
    inner = AIMOperator(m, g, k, near_radius=3, rules=QUAD, cutoff=5.0 * ph.skin_depth(k))
    outer = AIMOperator(m, g, ph.wavenumber(FREQ, 1.0), near_radius=3, rules=QUAD)
    return p, m, inner, outer


def test_cutoff_makes_the_interior_local(box):
    p, m, inner, outer = box
    assert inner.cut_local
    assert p.is_local(0) and not p.is_local(-1)
    # the interior has the exterior grid's geometry and a near list of its own
    gi, ge = p.grid(0), p.grid(-1)
    assert gi["h"] == ge["h"] and np.array_equal(gi["n"], ge["n"])
    rp, cols = p.near_pattern(0)
    ref = inner.NA.tocsr()
    ref.sort_indices()
    assert np.array_equal(rp, ref.indptr) and np.array_equal(cols, ref.indices)
    assert len(cols) < p.near_pattern(-1)[1].size


def test_cutoff_values_and_products_match_oracle(box):
    p, m, inner, outer = box
    for opk, ref in ((0, inner.near_L()), (1, inner.NK)):
        ref = ref.tocsr(); ref.sort_indices()
        assert _rel(p.near_values(0, opk), ref.data) < 1e-10, opk
    x = vec(m.nrwg, 41)
    xd = torch.from_numpy(x).to("cuda:0")
    for name, code in (("L", 0), ("K", 1)):
        y = p.matvec(0, code, xd).cpu().numpy()
        assert _rel(y, inner.matvec(x, name)) < 1e-10, name
        y32 = p.matvec(0, code, xd.to(torch.complex64)).cpu().numpy()
        assert _rel(y32, y) < 2e-6, name
        # the exterior keeps its grid part
        ye = p.matvec(-1, code, xd).cpu().numpy()
        assert _rel(ye, outer.matvec(x, name)) < 1e-10, name
    from paper_2003_11679_amd import SieError
    with pytest.raises(SieError):
        p.convolve(0, torch.zeros((4, 4, 4, 4), dtype=torch.complex128, device="cuda:0"))


def test_cutoff_solve_satisfies_oracle_system(box):
    from oracle import physics as ph
    from oracle.mom import excitation, x_matrix
    p, m, inner, outer = box
    khat, e0 = (0.0, 0.0, -1.0), (1.0, 0.0, 0.0)
    p.set_planewaves(khat, e0)
    r = p.solve(0, tol=1e-8, precond=4)
    assert r["converged"], r
    u, v = p.currents()
    w = ph.omega(FREQ)
    X = x_matrix(m)
    e = excitation(m, ph.wavenumber(FREQ, 1.0), khat, e0)
    r1 = e - (1j * w * ph.MU0 * outer.matvec(u, "L") - (outer.matvec(v, "K") - 0.5 * X @ v))
    et = ph.eps_tilde(FREQ, 1.0, SIGMA)
    r2 = (inner.matvec(u, "K") + 0.5 * X @ u) + 1j * w * et * inner.matvec(v, "L")
    rel = np.sqrt(np.linalg.norm(r1) ** 2 + np.linalg.norm(r2) ** 2) / np.linalg.norm(e)
    assert rel < 1e-7, rel
    # the cut interior operator is the direct near-region one: the nested
    # near-region preconditioner is nearly its inverse
    assert r["inner_iters_max"] <= 3, r


def test_all_near_bypass_matches_oracle():
    from paper_2003_11679_amd import Problem
    from workloads import icosphere
    from oracle.rwg import RWGMesh
    from oracle.aim import Grid, AIMOperator
    from oracle import physics as ph
    print("[small sphere, every pair near]", flush=True)
    xyz, tri = icosphere(1)
    p = Problem(150e6)
    p.add_object(xyz, tri, eps_r=4.0, sigma=0.2)
    p.set_grid(-1, n=8, near_radius=6)
    p.set_quadrature(**QUAD)
    p.setup()
    assert p.is_local(-1) and p.is_local(0)
    m = RWGMesh([(xyz, tri)])
    g = Grid.enclosing(m.xyz, 8)
    x = vec(m.nrwg, 42)
    xd = torch.from_numpy(x).to("cuda:0")
    for medium, k in ((-1, ph.wavenumber(150e6, 1.0)), (0, ph.wavenumber(150e6, 4.0, 1.0, 0.2))):
        loc = AIMOperator(m, g, k, near_radius=6, rules=QUAD)
        full = AIMOperator(m, g, k, near_radius=6, rules=QUAD, bypass=False)
        assert loc.local and not full.local
        for name, code in (("L", 0), ("K", 1)):
            y = p.matvec(medium, code, xd).cpu().numpy()
            assert _rel(y, loc.matvec(x, name)) < 1e-10, (medium, name)
            assert _rel(y, full.matvec(x, name)) < 1e-10, (medium, name)


def test_near_lu_on_the_cut_interior(box):
    """precond 16 factors M_i = -j w eps_i L_i,NR of the cut interior exactly
    (eq. nest2pc): parity with scipy's sparse solve of the oracle's direct
    near-region operator, and one nested iteration per solve, because the
    local interior operator is M_i itself."""
    from scipy.sparse.linalg import spsolve
    from oracle import physics as ph
    p, m, inner, outer = box
    scale = -1j * ph.omega(FREQ) * ph.eps_tilde(FREQ, 1.0, SIGMA)
    A = (scale * inner.NLd).tocsc()
    X = np.stack([vec(p.num_rwg, 60 + r) for r in range(2)])
    ref = np.stack([spsolve(A, x) for x in X])
    got = p.nested_precond(16, torch.from_numpy(X).to("cuda", torch.complex128)).cpu().numpy()
    assert _rel(got, ref) < 1e-9
    one = p.nested_precond(16, torch.from_numpy(X[1]).to("cuda", torch.complex128)).cpu().numpy()
    assert np.array_equal(one, got[1])
    nm, nnz, t = p.nested_precond_factored()
    assert nm == 1 and nnz > 0, (nm, nnz, t)
    x32 = X[0].astype(np.complex64)
    got32 = p.nested_precond(16, torch.from_numpy(x32).to("cuda")).cpu().numpy()
    e32 = _rel(got32, spsolve(A, x32.astype(np.complex128)))
    print(f"  FP32 factors: rel err {e32:.2e}", flush=True)
    assert e32 < 1e-6
    p.set_planewaves((0.0, 0.0, -1.0), (1.0, 0.0, 0.0))
    r0 = p.solve(0, tol=1e-8, precond=0)
    u0, v0 = p.currents()
    for prec in (0, 1):
        r16 = p.solve(prec, tol=1e-8, precond=16)
        u16, v16 = p.currents()
        print(f"  prec {prec}: none {r0}\n  near LU {r16}", flush=True)
        assert r0["converged"] and r16["converged"]
        assert r16["inner_iters_max"] == 1, r16
        tol = 1e-6 if prec == 0 else 2e-5   # FP32 + refinement against the FP64 solve
        assert _rel(u16, u0) < tol and _rel(v16, v0) < tol
