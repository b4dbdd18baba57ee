"""AIM accuracy against the plain definition (dense Galerkin MoM of the
oracle) on the sphere configuration: 1,280 triangles, eps_r = 4, 150 MHz.

With the grid rule of Sec. IV (spacing lambda_r / 20 of the interior medium,
44 points per axis, near radius 5) the GPU's L and K products of both media
are within 1e-3 of the dense operators.  The configuration's own 16^3 grid
(h = lambda_i / 6.5) is much coarser than that rule: its interior products
are ~1e-2 from the dense ones, which the test records.  The solution error
is amplified by the interior cavity resonance next to k_i a = 6.29; the test
asserts the bound reached with the rule's grid."""
import numpy as np
import pytest

from cases import QUAD, vec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FREQ, EPS_R = 150e6, 4.0
KHAT, E0 = (0.0, 0.0, 1.0), (1.0, 0.0, 0.0)


@pytest.fixture(scope="module")
def dense():
    from oracle.rwg import RWGMesh
    from oracle.solve import DenseProblem
    from workloads import icosphere
    print("[dense oracle: 1280-triangle sphere]", flush=True)
    m = RWGMesh([icosphere(3)])
    dp = DenseProblem(m, FREQ, [(EPS_R, 1.0, 0.0)], rules=QUAD)
    u, v = dp.solve_block(dp.rhs(KHAT, E0))
    return dp, u, v


def _gpu(n):
    from paper_2003_11679_amd import Problem
    from workloads import icosphere
    xyz, tri = icosphere(3)
    p = Problem(FREQ)
    p.add_object(xyz, tri, eps_r=EPS_R)
    p.set_grid(-1, n=n, near_radius=5)     # n = 0: the rule of Sec. IV
    p.set_quadrature(**QUAD)
    p.setup()
    return p


def _op_errors(p, dp):
    x = vec(dp.mesh.nrwg, 31)
    xd = torch.from_numpy(x).to("cuda:0")
    out = {}
    for medium, L, K in ((-1, dp.L0, dp.K0), (0, dp.Li, dp.Ki)):
        for name, code, M in (("L", 0, L), ("K", 1, K)):
            y = p.matvec(medium, code, xd).cpu().numpy()
            ref = M @ x
            out[(medium, name)] = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    return out


def test_rule_grid_products_within_1e3_of_dense(dense):
    dp, _, _ = dense
    p = _gpu(0)
    g = p.grid(-1)
    print("rule grid", g["n"], g["h"], flush=True)
    assert int(g["n"][0]) == 44
    err = _op_errors(p, dp)
    print("rule grid operator errors", err, flush=True)
    for k, e in err.items():
        assert e <= 1e-3, (k, e)


def test_configuration_grid_recorded(dense):
    dp, _, _ = dense
    err = _op_errors(_gpu(16), dp)
    print("16^3 grid operator errors", err, flush=True)
    # measured: exterior (k0 h = 0.48) L 1.1e-3, K 3.2e-3; interior
    # (k_i h = 0.97) L 1.1e-2, K 2.3e-2
    assert err[(-1, "L")] < 1.5e-3 and err[(-1, "K")] < 4e-3
    assert err[(0, "L")] < 1.5e-2 and err[(0, "K")] < 3e-2


def test_rule_grid_solution_against_dense(dense):
    dp, u, v = dense
    p = _gpu(0)
    p.set_planewaves(KHAT, E0)
    for prec in (0, 1):
        r = p.solve(prec, tol=1e-8, precond=0)
        assert r["converged"], r
        ug, vg = p.currents()
        eu = float(np.linalg.norm(ug - u) / np.linalg.norm(u))
        ev = float(np.linalg.norm(vg - v) / np.linalg.norm(v))
        print(f"precision {prec}: solution error u {eu:.3e} v {ev:.3e} {r}", flush=True)
        # measured 9.73e-4 (u) and 1.25e-3 (v) in both precisions: the
        # operator errors of 3e-4 to 8e-4 amplified by the nearby resonance
        assert eu < 1.05e-3 and ev < 1.35e-3, (prec, eu, ev)
