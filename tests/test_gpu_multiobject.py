"""Several objects, each on its own grid (Sec. III-D-1: one AIM grid per
object plus the global exterior grid), against oracle operators built per
object: each medium's product, the batched product of all interiors (equal
grid shapes share one launch per stage), FP32 against FP64, and solves
whose block residual is measured with the oracle's operators (with unequal
and with equal objects, the latter solving one nested system per object)."""
import numpy as np
import pytest

from cases import gpu_multi, oracle_multi, MULTI_FREQ, vec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KHAT = (0.3, 0.0, -float(np.sqrt(1.0 - 0.09)))   # unit length
E0 = (0.0, 1.0, 0.0)


@pytest.fixture(scope="module")
def multi():
    print("[multi-object problem: 3 spheres + 1 box]", flush=True)
    return gpu_multi(4), oracle_multi(4)


def _oracle_interior(ints, x, op):
    """Block-diagonal interior product of the oracle (each object on its own
    rows)."""
    y = np.zeros_like(x)
    for off, n, o, _, _ in ints:
        y[off:off + n] = o.matvec(x[off:off + n], op)
    return y


def test_each_medium_matches_oracle(multi):
    p, (m, ext, ints) = multi
    from paper_2003_11679_amd import OP_L, OP_K
    x = vec(m.nrwg, 21)
    xd = torch.from_numpy(x).to("cuda:0")
    for i, (off, n, o, _, _) in enumerate(ints):
        for name, code in (("L", OP_L), ("K", OP_K)):
            y = p.matvec(i, code, xd).cpu().numpy()
            ref = o.matvec(x[off:off + n], name)
            err = np.linalg.norm(y[off:off + n] - ref) / np.linalg.norm(ref)
            assert err < 1e-10, (i, name, err)
            assert np.all(y[:off] == 0) and np.all(y[off + n:] == 0), (i, name)
    for name, code in (("L", OP_L), ("K", OP_K)):
        y = p.matvec(-1, code, xd).cpu().numpy()
        ref = ext.matvec(x, name)
        assert np.linalg.norm(y - ref) < 1e-10 * np.linalg.norm(ref), name


def test_batched_interiors_match_oracle_and_single_products(multi):
    p, (m, ext, ints) = multi
    from paper_2003_11679_amd import OP_L, OP_K, INTERIORS
    X = vec(m.nrwg, 22, nrhs=3)
    Xd = torch.from_numpy(X).to("cuda:0")
    for name, code in (("L", OP_L), ("K", OP_K)):
        for r in range(3):
            y = p.matvec(INTERIORS, code, Xd[r]).cpu().numpy()
            ref = _oracle_interior(ints, X[r], name)
            err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
            assert err < 1e-10, (name, r, err)
            single = sum(p.matvec(i, code, Xd[r]).cpu().numpy() for i in range(len(ints)))
            assert np.abs(y - single).max() <= 1e-12 * np.abs(single).max(), name
        # several right-hand sides in one batched launch
        Y = p.matvec(INTERIORS, code, Xd).cpu().numpy()
        for r in range(3):
            ref = _oracle_interior(ints, X[r], name)
            assert np.linalg.norm(Y[r] - ref) < 1e-10 * np.linalg.norm(ref), (name, r)
        # FP32
        Y32 = p.matvec(INTERIORS, code, Xd.to(torch.complex64)).cpu().numpy()
        assert np.linalg.norm(Y32 - Y) < 2e-6 * np.linalg.norm(Y), name


def _block_residual(m, ext, ints, u, v):
    from oracle import physics as ph
    from oracle.mom import excitation, x_matrix
    w = ph.omega(MULTI_FREQ)
    X = x_matrix(m)
    e = excitation(m, ph.wavenumber(MULTI_FREQ, 1.0), KHAT, E0)
    r1 = e - (1j * w * ph.MU0 * ext.matvec(u, "L") - (ext.matvec(v, "K") - 0.5 * X @ v))
    Lv = np.zeros_like(v)
    for off, n, o, eps_r, sigma in ints:
        Lv[off:off + n] = ph.eps_tilde(MULTI_FREQ, eps_r, sigma) * o.matvec(v[off:off + n], "L")
    r2 = -(-(_oracle_interior(ints, u, "K") + 0.5 * X @ u) - 1j * w * Lv)
    return np.sqrt(np.linalg.norm(r1) ** 2 + np.linalg.norm(r2) ** 2) / np.linalg.norm(e)


@pytest.mark.parametrize("count", [4, 3])
def test_solve_satisfies_oracle_system(count, multi):
    """count 4: unequal objects, one nested system; count 3: three equal
    spheres, one nested system per object iterated side by side."""
    if count == 4:
        p, (m, ext, ints) = multi
    else:
        print("[multi-object problem: 3 spheres]", flush=True)
        p, (m, ext, ints) = gpu_multi(3), oracle_multi(3)
    p.set_planewaves(KHAT, E0)
    r64 = p.solve(0, tol=1e-8)
    u64, v64 = p.currents()
    print(f"count {count} fp64 {r64}", flush=True)
    assert r64["converged"], r64
    assert _block_residual(m, ext, ints, u64, v64) < 1e-7
    r32 = p.solve(1, tol=1e-8)
    u32, v32 = p.currents()
    print(f"count {count} fp32 {r32}", flush=True)
    assert r32["converged"], r32
    assert np.linalg.norm(u32 - u64) < 1e-5 * np.linalg.norm(u64)
    assert np.linalg.norm(v32 - v64) < 1e-5 * np.linalg.norm(v64)
    assert r64["matvecs"] > 0 and r64["k_matvecs"] > 0


def test_skipping_converged_objects_keeps_results():
    """Equal objects (a 3 x 2 array of lossy cubes) iterate their nested
    systems side by side; once an object's system has converged its rows of
    the nested products are skipped.  The solve is the same, bit for bit in
    FP64, as one that keeps multiplying every object, and counts fewer
    L-type products."""
    from paper_2003_11679_amd import Problem
    from workloads import cube_array_cfg
    print("[3 x 2 cube array: skipping converged nested systems]", flush=True)
    cfg = cube_array_cfg(cells=4, ext_grid_n=48, int_grid_n=8, nx=3, ny=2)
    p = Problem(cfg.freq)
    for o in cfg.objects:
        p.add_object(o.xyz, o.tri, eps_r=o.eps_r, mu_r=o.mu_r, sigma=o.sigma)
    p.set_grid(-1, n=cfg.ext_grid_n, near_radius=3)
    for i, o in enumerate(cfg.objects):
        p.set_grid(i, n=o.grid_n, near_radius=3, share=0)
    p.setup()
    w = cfg.waves[0]
    p.set_planewaves(w.khat, w.e0)
    out = {}
    for keep in (1, 0):
        for prec in (0, 1):
            r = p.solve(prec, tol=1e-8, restart=300, precond=12, keep_converged=keep)
            print(f"  keep {keep} prec {prec}: {r}", flush=True)
            assert r["converged"], r
            out[keep, prec] = (r, p.currents())
    for prec in (0, 1):
        (rk, (uk, vk)), (rs, (us, vs)) = out[1, prec], out[0, prec]
        assert rs["outer_iters"] == rk["outer_iters"] and rs["inner_iters"] == rk["inner_iters"], (rs, rk)
        assert rs["matvecs"] < rk["matvecs"], (rs["matvecs"], rk["matvecs"])
        if prec == 0:
            assert np.array_equal(us, uk) and np.array_equal(vs, vk)
        else:
            assert np.linalg.norm(us - uk) <= 1e-12 * np.linalg.norm(uk)
