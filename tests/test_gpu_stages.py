"""GPU parity of the AIM stages and the full operator product against the
FP64 oracle (same seeded inputs, same quadrature orders)."""
import numpy as np
import pytest

from cases import CASES, gpu_problem, oracle_aim, vec, mesh_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module", params=["sphere2", "bar_small", "box_cond"])
def case(request):
    name = request.param
    print(f"[case {name}]", flush=True)
    return name, gpu_problem(name)


def test_topology_matches_oracle(case):
    name, p = case
    from oracle.rwg import RWGMesh
    m = RWGMesh([mesh_of(name)])
    ev, tpm = p.rwg()
    assert np.array_equal(ev, m.edge_v)
    assert np.array_equal(tpm[:, 0], m.tp) and np.array_equal(tpm[:, 1], m.tm)


@pytest.mark.parametrize("medium", [-1])
def test_stencils_bit_exact(case, medium):
    name, p = case
    op = oracle_aim(name, medium)
    g = p.grid(medium)
    assert np.allclose(g["origin"], op.grid.origin, rtol=0, atol=0)
    assert g["h"] == op.grid.h
    assert np.array_equal(p.stencils(medium), op.centres)


def test_near_pattern_matches(case):
    name, p = case
    op = oracle_aim(name, -1)
    rp, cols = p.near_pattern(-1)
    ref = op.NA.tocsr()
    ref.sort_indices()
    assert np.array_equal(rp, ref.indptr)
    assert np.array_equal(cols, ref.indices)


@pytest.mark.parametrize("medium", [-1, 0])
def test_near_values_match(case, medium):
    name, p = case
    op = oracle_aim(name, medium)
    rp, cols = p.near_pattern(medium)
    for opk, ref in ((0, op.near_L()), (1, op.NK)):
        ref = ref.tocsr(); ref.sort_indices()
        got = p.near_values(medium, opk)
        assert _rel(got, ref.data) < 1e-10, (opk, _rel(got, ref.data))


def _live(op, g):
    lo, nl = g["lo"], g["nl"]
    return (slice(lo[2], lo[2] + nl[2]), slice(lo[1], lo[1] + nl[1]), slice(lo[0], lo[0] + nl[0]))


def test_project_matches(case):
    name, p = case
    op = oracle_aim(name, -1)
    x = vec(p.num_rwg, 21)
    got = p.project(-1, _dev(x)).cpu().numpy()
    J, Q = op.project(x)
    sl = _live(op, p.grid(-1))
    ref = np.stack([J[0][sl], J[1][sl], J[2][sl], Q[sl]])
    assert _rel(got, ref) < 1e-13


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
def test_convolution_matches(case, dtype, tol):
    name, p = case
    op = oracle_aim(name, -1)
    g = p.grid(-1)
    nl = g["nl"]
    rng = np.random.default_rng(5)
    src = rng.standard_normal((4, nl[2], nl[1], nl[0])) + 1j * rng.standard_normal((4, nl[2], nl[1], nl[0]))
    got = p.convolve(-1, _dev(src, dtype)).cpu().numpy()
    sl = _live(op, g)
    n = op.grid.n
    ref = np.empty_like(src)
    for f in range(4):
        full = np.zeros((n[2], n[1], n[0]), complex)
        full[sl] = src[f]
        ref[f] = op.convolve_fft(full, "G")[sl]
    assert _rel(got, ref) < tol


def test_interpolate_matches(case):
    name, p = case
    op = oracle_aim(name, -1)
    g = p.grid(-1)
    nl = g["nl"]
    rng = np.random.default_rng(6)
    F = rng.standard_normal((4, nl[2], nl[1], nl[0])) + 1j * rng.standard_normal((4, nl[2], nl[1], nl[0]))
    got = p.interpolate(-1, _dev(F)).cpu().numpy()
    sl = _live(op, g)
    n = op.grid.n
    full = np.zeros((4, n[2], n[1], n[0]), complex)
    for f in range(4):
        full[f][sl] = F[f]
    ref = op.interpolate_vec(full[:3]) - op.interpolate_scal(full[3]) / op.k ** 2
    assert _rel(got, ref) < 1e-12


@pytest.mark.parametrize("medium", [-1, 0])
@pytest.mark.parametrize("opname,opk", [("L", 0), ("K", 1)])
def test_matvec_fp64_matches_oracle(case, medium, opname, opk):
    name, p = case
    op = oracle_aim(name, medium)
    x = vec(p.num_rwg, 31)
    got = p.matvec(medium, opk, _dev(x)).cpu().numpy()
    ref = op.matvec(x, opname)
    assert np.linalg.norm(got - ref) < 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("opname,opk", [("L", 0), ("K", 1)])
def test_matvec_fp32_close_to_fp64(case, opname, opk):
    name, p = case
    x = vec(p.num_rwg, 32)
    y64 = p.matvec(-1, opk, _dev(x)).cpu().numpy()
    y32 = p.matvec(-1, opk, _dev(x, torch.complex64)).cpu().numpy()
    assert np.linalg.norm(y32 - y64) < 2e-5 * np.linalg.norm(y64)


def test_x_operator(case):
    name, p = case
    from oracle.rwg import RWGMesh
    from oracle.mom import x_matrix
    m = RWGMesh([mesh_of(name)])
    x = vec(p.num_rwg, 33)
    got = p.matvec(-1, 2, _dev(x)).cpu().numpy()
    ref = x_matrix(m) @ x
    assert _rel(got, ref) < 1e-13


def test_stage_timer_modes(case):
    """Timing mode 1 times every stage of a product, mode 2 the near-field CSR
    product alone, 0 nothing (each call clears the totals); an unknown mode is
    rejected; timing leaves the product unchanged."""
    from paper_2003_11679_amd import SieError
    name, p = case
    x = _dev(vec(p.num_rwg, 34))
    y0 = p.matvec(-1, 0, x).cpu().numpy()
    p.set_timing(1)
    y1 = p.matvec(-1, 0, x).cpu().numpy()
    st = p.stage_times()
    for k in ("project", "fft", "interp", "spmv", "product", "spmv64"):
        assert st[k][0] == 1 and st[k][1] > 0.0, (k, st)
    p.set_timing(2)
    p.matvec(-1, 0, x)
    st = p.stage_times()
    assert st["spmv"][0] == 1 and st["spmv64"][0] == 1, st
    assert all(st[k][0] == 0 for k in ("project", "fft", "interp", "product")), st
    p.set_timing(0)
    p.matvec(-1, 0, x)
    assert all(v[0] == 0 for v in p.stage_times().values())
    with pytest.raises(SieError):
        p.set_timing(3)
    assert np.array_equal(y0, y1)


def test_device_stencil_assignment_bit_exact(case):
    """sie_stencil_assign on the device against the oracle's integer
    assignment (Sec. III-D-1 stencil anchoring), bit for bit."""
    from oracle.aim import stencil_centres
    name, p = case
    op = oracle_aim(name, -1)
    got = p.stencil_assign(-1).cpu().numpy()
    ref = stencil_centres(op.grid, op.mesh.centroid)
    assert np.array_equal(got, ref)


def test_far_field_angles_are_the_spherical_components(case):
    from oracle.farfield import far_field, directions
    from oracle import physics as ph
    name, p = case
    if name != "sphere2":
        pytest.skip("one case suffices")
    p.set_planewaves((0.0, 0.0, 1.0), (1.0, 0.0, 0.0))
    p.solve(0)
    u, v = p.currents()
    th = np.linspace(0.1, 3.0, 7); phi = np.linspace(0.0, 5.0, 7)
    et, ep = p.far_field_angles(th, phi)
    op = oracle_aim(name, -1)
    F = far_field(op.mesh, ph.wavenumber(CASES[name][3], 1.0), ph.ETA0, u, v, directions(th, phi))
    tht = np.stack([np.cos(th) * np.cos(phi), np.cos(th) * np.sin(phi), -np.sin(th)], axis=1)
    phh = np.stack([-np.sin(phi), np.cos(phi), 0 * th], axis=1)
    assert np.abs(et - np.sum(F * tht, axis=1)).max() < 1e-10 * np.abs(F).max()
    assert np.abs(ep - np.sum(F * phh, axis=1)).max() < 1e-10 * np.abs(F).max()


def test_context_keeps_the_last_error(case):
    from paper_2003_11679_amd import SieError
    name, p = case
    with pytest.raises(SieError):
        p.matvec(7, 0, torch.zeros(p.num_rwg, dtype=torch.complex128, device="cuda"))
    assert "medium" in p.last_error()
