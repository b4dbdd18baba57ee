"""Problem records for the synthetic workloads (data only).

Each builder returns a :class:`Problem`: meshes, materials, frequency, plane-wave
excitations and the grid sizes to use.  Nothing here evaluates the method.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from .meshes import icosphere, box_mesh, cube_array, geodesic_sphere, ellipsoid

C0_NOMINAL = 299792458.0   # m/s, used only to size geometry in wavelengths


@dataclass
class ObjectSpec:
    xyz: np.ndarray
    tri: np.ndarray
    eps_r: float = 1.0
    mu_r: float = 1.0
    sigma: float = 0.0
    grid_n: Optional[int] = None      # points per axis of the object's own grid


@dataclass
class PlaneWave:
    khat: Tuple[float, float, float]
    e0: Tuple[complex, complex, complex]


@dataclass
class Problem:
    name: str
    freq: float
    objects: List[ObjectSpec]
    waves: List[PlaneWave]
    ext_grid_n: int                    # points per axis of the exterior grid
    shared_grid: bool = True           # single object: interior reuses the exterior grid
    near_radius: int = 5               # Chebyshev radius in grid cells (diameter 11)
    tol: float = 1e-6
    bg_eps_r: float = 1.0
    bg_mu_r: float = 1.0
    meta: dict = field(default_factory=dict)


def sphere_cfg(level=3, radius=1.0, eps_r=4.0, sigma=0.0, freq=150e6, grid_n=16):
    """Dielectric sphere, icosphere mesh (level 3 -> 1280 triangles), x-polarised
    plane wave travelling along +z."""
    xyz, tri = icosphere(level, radius)
    return Problem(name=f"sphere_L{level}", freq=freq,
                   objects=[ObjectSpec(xyz, tri, eps_r, 1.0, sigma, grid_n)],
                   waves=[PlaneWave((0.0, 0.0, 1.0), (1.0, 0.0, 0.0))],
                   ext_grid_n=grid_n)


def bar_cfg(divisions=(180, 18, 9), size=(100e-6, 10e-6, 5e-6), sigma=5.8e7, eps_r=1.0,
            freq=10e9, grid_n=64):
    """Copper-like bar with a structured surface mesh (180x18x9 -> 20,088
    triangles), plane wave along -z polarised along x."""
    xyz, tri = box_mesh(size, divisions)
    return Problem(name="bar", freq=freq,
                   objects=[ObjectSpec(xyz, tri, eps_r, 1.0, sigma, grid_n)],
                   waves=[PlaneWave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0))],
                   ext_grid_n=grid_n)


def bar_small_cfg(divisions=(60, 6, 3), grid_n=24, **kw):
    """Reduced bar (2,232 triangles) on which a dense solve is affordable."""
    p = bar_cfg(divisions=divisions, grid_n=grid_n, **kw)
    p.name = "bar_small"
    return p


def cube_array_cfg(freq=1e9, cells=16, ext_grid_n=256, int_grid_n=16, seed=11682, nx=8, ny=8):
    """8x8 array of lossy dielectric cubes (edge 0.2 lambda0, pitch 0.4 lambda0);
    per-cube eps_r ~ U[2,10], sigma ~ U[0,10] S/m drawn row-major."""
    lam0 = C0_NOMINAL / freq
    rng = np.random.default_rng(seed)
    meshes = cube_array(nx, ny, 0.2 * lam0, 0.4 * lam0, cells)
    objs = []
    for xyz, tri in meshes:
        eps_r = rng.uniform(2.0, 10.0)
        sigma = rng.uniform(0.0, 10.0)
        objs.append(ObjectSpec(xyz, tri, eps_r, 1.0, sigma, int_grid_n))
    return Problem(name="cube_array", freq=freq, objects=objs,
                   waves=[PlaneWave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0))],
                   ext_grid_n=ext_grid_n, shared_grid=False)


def multi_rhs_waves(n_theta=8, n_phi=8):
    """Plane waves on an n_theta x n_phi incidence grid, polarisation alternating
    theta-hat / phi-hat in a checkerboard; khat = -rhat(theta, phi)."""
    waves = []
    for i in range(n_theta):
        th = (i + 0.5) * np.pi / n_theta
        for j in range(n_phi):
            ph = 2.0 * np.pi * j / n_phi
            r = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
            t = np.array([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
            p = np.array([-np.sin(ph), np.cos(ph), 0.0])
            e = t if (i + j) % 2 == 0 else p
            waves.append(PlaneWave(tuple(-r), tuple(complex(x) for x in e)))
    return waves


def batching_meshes():
    """Meshes of the multi-RHS / multi-frequency workload (sphere and bar)."""
    spheres = [("sphere5120", icosphere(4, 0.5)), ("sphere20480", geodesic_sphere(32, 0.5)),
               ("sphere50000", geodesic_sphere(50, 0.5))]
    bars = [("bar4824", box_mesh((100e-6, 10e-6, 5e-6), (90, 9, 4))),
            ("bar20088", box_mesh((100e-6, 10e-6, 5e-6), (180, 18, 9))),
            ("bar49448", box_mesh((100e-6, 10e-6, 5e-6), (285, 28, 14)))]
    return spheres, bars


def serving_trace(n=2000, rate=50.0, seed=11684):
    """Poisson request stream: arrival times and per-request parameters."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    reqs = []
    for i in range(n):
        nt = float(np.exp(rng.uniform(np.log(2e3), np.log(1e5))))
        shape = int(rng.integers(0, 3))
        eps_r = float(rng.uniform(1.0, 12.0))
        sigma = float(np.exp(rng.uniform(np.log(1e-2), np.log(5.8e7))))
        freq = float(np.exp(rng.uniform(np.log(1e9), np.log(1e11))))
        edge_scale = float(np.exp(rng.uniform(np.log(0.1), np.log(1.0))))
        aspect = rng.uniform(1.0, 4.0, size=2)
        axes = rng.uniform(1.0, 3.0, size=2)
        reqs.append(dict(t=float(t[i]), nt=nt, shape=shape, eps_r=eps_r, sigma=sigma,
                         freq=freq, edge_scale=edge_scale, aspect=aspect, axes=axes))
    return reqs


def serving_mesh(req):
    """Mesh for one serving request (sphere, box or ellipsoid of ~req['nt']
    triangles, mean edge (lambda0/sqrt(eps_r))/10 * edge_scale)."""
    lam = C0_NOMINAL / req["freq"] / np.sqrt(req["eps_r"])
    edge = lam / 10.0 * req["edge_scale"]
    nt = req["nt"]
    if req["shape"] == 0:
        nu = max(2, int(round(np.sqrt(nt / 20.0))))
        xyz, tri = geodesic_sphere(nu)
        mean_edge = 1.1 * 2 * np.pi / (np.sqrt(20 * nu * nu) * 1.0)
        return xyz * (edge / mean_edge), tri
    if req["shape"] == 1:
        ar = np.array([1.0, req["aspect"][0], req["aspect"][1]])
        area_cells = nt / 2.0
        s = np.sqrt(area_cells / (2 * (ar[0] * ar[1] + ar[1] * ar[2] + ar[2] * ar[0])))
        div = np.maximum(1, np.round(ar * s)).astype(int)
        return box_mesh(tuple(div * edge), tuple(div))
    nu = max(2, int(round(np.sqrt(nt / 20.0))))
    ax = np.array([1.0, req["axes"][0], req["axes"][1]])
    xyz, tri = geodesic_sphere(nu)
    mean_edge = 1.1 * 2 * np.pi / np.sqrt(20 * nu * nu)
    return xyz * ax * (edge / mean_edge), tri


def random_vector(n, seed, nrhs=None):
    """Seeded complex vector with N(0,1) real and imaginary parts (float64)."""
    rng = np.random.default_rng(seed)
    shape = (n,) if nrhs is None else (nrhs, n)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
