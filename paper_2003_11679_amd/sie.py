"""ctypes binding of ``libsie.so`` (include/sie.h).

Argument marshalling only: every computation runs in the HIP library.  Device
arrays are torch tensors (complex64 / complex128 on a HIP device); the stream
is torch's current stream unless one is given.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsie.so")

SIE_OK, SIE_EINVAL, SIE_ENOMEM, SIE_EMESH, SIE_EGRID, SIE_ENOCONV, SIE_EDEVICE, SIE_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32 = 0, 1
OP_L, OP_K, OP_X, OP_AUG = 0, 1, 2, 3
EXTERIOR = -1
INTERIORS = -2

_STATUS = {SIE_EINVAL: "EINVAL", SIE_ENOMEM: "ENOMEM", SIE_EMESH: "EMESH", SIE_EGRID: "EGRID",
           SIE_ENOCONV: "ENOCONV", SIE_EDEVICE: "EDEVICE", SIE_ESTATE: "ESTATE"}


class SieError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class QuadParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("touch_out", "touch_in", "close_out", "close_in", "far_out", "far_in")]


class GridParams(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("n", ctypes.c_int32), ("origin", ctypes.c_double * 3),
                ("order", ctypes.c_int32), ("near_radius", ctypes.c_int32), ("loss_ratio", ctypes.c_double),
                ("lambda_r", ctypes.c_double)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "origin"}
        d["origin"] = tuple(self.origin)
        return d


class SolverOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("inner_max_iter", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("precond", ctypes.c_int32), ("inner_relax", ctypes.c_double),
                ("keep_converged", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("inner_iters_max", ctypes.c_int32), ("refine_sweeps", ctypes.c_int32),
                ("matvecs", ctypes.c_int64), ("k_matvecs", ctypes.c_int64), ("residual", ctypes.c_double),
                ("t_setup_s", ctypes.c_double), ("t_solve_s", ctypes.c_double), ("device_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class JobInfo(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("running", ctypes.c_int32), ("status", ctypes.c_int),
                ("t_submit_s", ctypes.c_double), ("t_start_s", ctypes.c_double), ("t_end_s", ctypes.c_double),
                ("footprint", ctypes.c_size_t), ("report", Report), ("message", ctypes.c_char * 256)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n not in ("report", "message")}
        d["report"] = self.report.as_dict()
        d["message"] = self.message.decode()
        return d


_lib = None
_VP = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_DP = ctypes.POINTER(ctypes.c_double)
_CP = ctypes.POINTER(c128)

# (name, restype, argtypes): every entry point declared in include/sie.h
SIGNATURES = [
    ("sie_ctx_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_VP)]),
    ("sie_ctx_destroy", None, [_VP]),
    ("sie_ctx_trim", ctypes.c_int, [_VP]),
    ("sie_last_error", ctypes.c_char_p, []),
    ("sie_set_tuning", ctypes.c_int, [ctypes.c_int32]),
    ("sie_tuning_force", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32]),
    ("sie_tuning_report", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    ("sie_tuning_clear", ctypes.c_int, []),
    ("sie_problem_create", ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(_VP)]),
    ("sie_problem_add_object", ctypes.c_int, [_VP, _DP, ctypes.c_int64, _I32P, ctypes.c_int64,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_double, _I32P]),
    ("sie_problem_set_grid", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32]),
    ("sie_grid_choose", ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(GridParams)]),
    ("sie_problem_set_grid_params", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(GridParams), ctypes.c_int32]),
    ("sie_problem_set_quadrature", ctypes.c_int, [_VP, ctypes.POINTER(QuadParams)]),
    ("sie_problem_set_skin_cutoff", ctypes.c_int, [_VP, ctypes.c_double]),
    ("sie_medium_is_local", ctypes.c_int32, [_VP, ctypes.c_int32]),
    ("sie_problem_set_augmented", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("sie_problem_augmented_info", ctypes.c_int, [_VP, _I32P, _I64P, _I32P, _DP]),
    ("sie_constraint_precond", ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, _VP]),
    ("sie_get_charges", ctypes.c_int, [_VP, ctypes.c_int32, _CP]),
    ("sie_problem_setup", ctypes.c_int, [_VP]),
    ("sie_problem_destroy", None, [_VP]),
    ("sie_problem_num_rwg", ctypes.c_int64, [_VP]),
    ("sie_problem_num_tri", ctypes.c_int64, [_VP]),
    ("sie_get_rwg", ctypes.c_int, [_VP, _I32P, _I32P]),
    ("sie_get_grid", ctypes.c_int, [_VP, ctypes.c_int32, _DP, _DP, _I32P, _I32P, _I32P, _I32P]),
    ("sie_get_stencils", ctypes.c_int, [_VP, ctypes.c_int32, _I32P, _I64P]),
    ("sie_ctx_last_error", ctypes.c_char_p, [_VP]),
    ("sie_stencil_assign", ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP]),
    ("sie_far_field_angles", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64, _DP, _DP, _CP, _CP]),
    ("sie_get_near_pattern", ctypes.c_int, [_VP, ctypes.c_int32, _I64P, _I32P, _I64P]),
    ("sie_get_near_values", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int, _CP]),
    ("sie_get_wavenumber", ctypes.c_int, [_VP, ctypes.c_int32, _CP]),
    ("sie_matvec", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int, ctypes.c_int, ctypes.c_int32, _VP, _VP, _VP]),
    ("sie_matvec_noalloc", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP]),
    ("sie_project", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int, _VP, _VP, _VP]),
    ("sie_convolve", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int, ctypes.c_int, ctypes.c_int32, _VP, _VP, _VP]),
    ("sie_interpolate", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int, _VP, _VP, _VP]),
    ("sie_nested_precond", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int, ctypes.c_int32, _VP, _VP, _VP]),
    ("sie_nested_precond_clusters", ctypes.c_int32, [_VP, _I64P]),
    ("sie_nested_precond_factored", ctypes.c_int32, [_VP, _I64P, _DP]),
    ("sie_set_timing", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("sie_get_stage_time", ctypes.c_int, [_VP, ctypes.c_int32, _I64P, _DP]),
    ("sie_set_planewaves", ctypes.c_int, [_VP, ctypes.c_int32, _DP, _CP]),
    ("sie_solve", ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(SolverOpts), ctypes.POINTER(Report)]),
    ("sie_get_currents", ctypes.c_int, [_VP, ctypes.c_int32, _CP, _CP]),
    ("sie_far_field", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64, _DP, _CP]),
    ("sie_problem_footprint", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    ("sie_server_create", ctypes.c_int, [_VP, ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(_VP)]),
    ("sie_server_submit", ctypes.c_int, [_VP, _VP, ctypes.c_int32, _DP, _CP, ctypes.c_int,
                                         ctypes.POINTER(SolverOpts), ctypes.POINTER(ctypes.c_uint64)]),
    ("sie_server_poll", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(JobInfo)]),
    ("sie_server_take", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(_VP)]),
    ("sie_server_destroy", None, [_VP]),
]


def lib():
    """Loads libsie.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2003_11679_amd/build.py "
                               "(the HIP library is the only implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != SIE_OK:
        raise SieError(st, lib().sie_last_error().decode())
    return st


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def grid_choose(freq, eps_r, mu_r, sigma, extent, mean_edge, near_radius=5, strict=False):
    """Grid rule of Sec. IV (library side): dict of h, n, order, near radius,
    worst lossy/lossless bound ratio and lambda_r.  Host-only."""
    g = GridParams()
    _check(lib().sie_grid_choose(float(freq), float(eps_r), float(mu_r), float(sigma), float(extent),
                                 float(mean_edge), int(near_radius), int(bool(strict)), ctypes.byref(g)))
    return g.as_dict()


# Stages whose launch shapes are tuned (sie_tuning_force families).
TUNE_FAMILIES = {"fft_y_fwd": 0, "fft_y_inv": 1, "fft_z": 2, "project": 3, "interp": 4}


def set_tuning(mode):
    """Launch-shape tuning, process-wide: 1 tune on first use, 0 built-in shapes."""
    _check(lib().sie_set_tuning(int(mode)))


def tuning_force(family, candidate):
    """Testing: stage `family` (name or number) always uses `candidate` (-1: tune)."""
    f = TUNE_FAMILIES[family] if isinstance(family, str) else int(family)
    _check(lib().sie_tuning_force(f, int(candidate)))


def tuning_report():
    """The tuner's choices so far: list of dicts (stage, precision, shape, times, choice)."""
    n = ctypes.c_size_t(0)
    _check(lib().sie_tuning_report(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().sie_tuning_report(buf, n.value, None))
    out = []
    for line in buf.value.decode().splitlines():
        f = line.split()
        d = dict(kv.split("=", 1) for kv in f[1:] if "=" in kv)
        out.append({"stage": f[0], "device": int(d["dev"]), "precision": f[2],
                    "shape": [int(v) for v in d["shape"].split("x")],
                    "us": [float(v) for v in d["us"].split(",")], "choice": int(d["choice"])})
    return out


def tuning_clear():
    _check(lib().sie_tuning_clear())


class Context:
    def __init__(self, device=0):
        h = _VP()
        _check(lib().sie_ctx_create(device, ctypes.byref(h)))
        self.h = h
        self.device = device

    def trim(self):
        """Free the device memory the library keeps for reuse on this device."""
        _check(lib().sie_ctx_trim(self.h))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sie_ctx_destroy(self.h)
            self.h = None


class Problem:
    """One scattering problem: objects, grids, operators, solve."""

    def __init__(self, freq, bg_eps_r=1.0, bg_mu_r=1.0, ctx=None, device=0):
        self.ctx = ctx or Context(device)
        h = _VP()
        _check(lib().sie_problem_create(self.ctx.h, float(freq), float(bg_eps_r), float(bg_mu_r),
                                        ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None and not getattr(self, "_served", False):
            _lib.sie_problem_destroy(self.h)
            self.h = None

    # -- definition -----------------------------------------------------------
    def add_object(self, xyz, tri, eps_r=1.0, mu_r=1.0, sigma=0.0):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        oid = ctypes.c_int32()
        _check(lib().sie_problem_add_object(self.h, _ptr(xyz, ctypes.c_double), len(xyz),
                                            _ptr(tri, ctypes.c_int32), len(tri), float(eps_r), float(mu_r),
                                            float(sigma), ctypes.byref(oid)))
        return oid.value

    def set_grid(self, medium, n=0, near_radius=5, share=0):
        _check(lib().sie_problem_set_grid(self.h, medium, n, near_radius, share))

    def set_grid_params(self, medium, h=0.0, n=0, origin=None, order=2, near_radius=5, share=0):
        """Grid of a medium from explicit spacing, points per axis and first
        node (origin None: centred on the medium's objects)."""
        g = GridParams()
        g.h, g.n, g.order, g.near_radius = float(h), int(n), int(order), int(near_radius)
        o = (float("nan"),) * 3 if origin is None else tuple(float(v) for v in origin)
        for c in range(3):
            g.origin[c] = o[c]
        _check(lib().sie_problem_set_grid_params(self.h, medium, ctypes.byref(g), int(share)))

    def set_quadrature(self, **orders):
        q = QuadParams(**{k: int(v) for k, v in orders.items()})
        _check(lib().sie_problem_set_quadrature(self.h, ctypes.byref(q)))

    def set_skin_cutoff(self, skin_depths=5.0):
        _check(lib().sie_problem_set_skin_cutoff(self.h, float(skin_depths)))

    def set_augmented(self, on=True):
        """Augmented EFIE for the exterior problem (Sec. III-E), before setup."""
        _check(lib().sie_problem_set_augmented(self.h, int(bool(on))))

    def augmented_info(self):
        """(on, Schur factor entries, dissection levels, factorisation seconds)."""
        on = ctypes.c_int32(); nnz = ctypes.c_int64(); lev = ctypes.c_int32(); t = ctypes.c_double()
        _check(lib().sie_problem_augmented_info(self.h, ctypes.byref(on), ctypes.byref(nnz), ctypes.byref(lev),
                                                ctypes.byref(t)))
        return {"on": bool(on.value), "factor_nnz": int(nnz.value), "levels": int(lev.value),
                "t_factor_s": float(t.value)}

    def setup(self):
        _check(lib().sie_problem_setup(self.h))

    def footprint(self):
        """Device-memory estimate (bytes) the server admits the problem with."""
        b = ctypes.c_size_t()
        _check(lib().sie_problem_footprint(self.h, ctypes.byref(b)))
        return b.value

    def is_local(self, medium):
        """True if the medium runs without grid part (skin-depth cutoff within
        the near region, or every pair near)."""
        r = lib().sie_medium_is_local(self.h, medium)
        if r < 0:
            _check(r)
        return bool(r)

    # -- queries --------------------------------------------------------------
    @property
    def num_rwg(self):
        return lib().sie_problem_num_rwg(self.h)

    @property
    def num_tri(self):
        return lib().sie_problem_num_tri(self.h)

    def rwg(self):
        E = self.num_rwg
        ev = np.empty((E, 2), np.int32); tpm = np.empty((E, 2), np.int32)
        _check(lib().sie_get_rwg(self.h, _ptr(ev, ctypes.c_int32), _ptr(tpm, ctypes.c_int32)))
        return ev, tpm

    def grid(self, medium=EXTERIOR):
        o = np.empty(3); h = np.empty(1)
        n, lo, nl, m = (np.empty(3, np.int32) for _ in range(4))
        _check(lib().sie_get_grid(self.h, medium, _ptr(o, ctypes.c_double), _ptr(h, ctypes.c_double),
                                  _ptr(n, ctypes.c_int32), _ptr(lo, ctypes.c_int32), _ptr(nl, ctypes.c_int32),
                                  _ptr(m, ctypes.c_int32)))
        return {"origin": o, "h": float(h[0]), "n": n, "lo": lo, "nl": nl, "m": m}

    def stencils(self, medium=EXTERIOR):
        cnt = ctypes.c_int64()
        _check(lib().sie_get_stencils(self.h, medium, None, ctypes.byref(cnt)))
        out = np.empty((cnt.value, 3), np.int32)
        _check(lib().sie_get_stencils(self.h, medium, _ptr(out, ctypes.c_int32), ctypes.byref(cnt)))
        return out

    def stencil_assign(self, medium=EXTERIOR, stream=None):
        """Stencil centres recomputed on the device: int32 tensor [nt][3]."""
        import torch
        nt = len(self.stencils(medium))
        out = torch.empty((nt, 3), dtype=torch.int32, device="cuda")
        _check(lib().sie_stencil_assign(self.h, medium, _VP(out.data_ptr()), _stream(stream)))
        return out

    def last_error(self):
        """Message of the last failing call on this problem's context."""
        return lib().sie_ctx_last_error(self.ctx.h).decode()

    def near_pattern(self, medium=EXTERIOR):
        nnz = ctypes.c_int64()
        _check(lib().sie_get_near_pattern(self.h, medium, None, None, ctypes.byref(nnz)))
        rp = np.empty(self.num_rwg + 1, np.int64)
        cols = np.empty(max(nnz.value, 1), np.int32)
        _check(lib().sie_get_near_pattern(self.h, medium, _ptr(rp, ctypes.c_int64), _ptr(cols, ctypes.c_int32),
                                          ctypes.byref(nnz)))
        return rp, cols[:nnz.value]

    def near_values(self, medium, op):
        rp, cols = self.near_pattern(medium)
        out = np.empty((max(len(cols), 1), 2))
        _check(lib().sie_get_near_values(self.h, medium, op, out.ctypes.data_as(_CP)))
        return (out[:, 0] + 1j * out[:, 1])[:len(cols)]

    def wavenumber(self, medium=EXTERIOR):
        k = c128()
        _check(lib().sie_get_wavenumber(self.h, medium, ctypes.byref(k)))
        return complex(k.re, k.im)

    # -- hot path -------------------------------------------------------------
    @staticmethod
    def _prec_of(t):
        import torch
        if t.dtype == torch.complex128:
            return FP64
        if t.dtype == torch.complex64:
            return FP32
        raise TypeError("device vectors must be complex64 or complex128")

    def matvec(self, medium, op, x, y=None, stream=None):
        """y = Op x for x of shape [E] or [nrhs, E] on the device."""
        import torch
        prec = self._prec_of(x)
        x = x.contiguous()
        if y is None:
            y = torch.empty_like(x)
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _check(lib().sie_matvec(self.h, medium, op, prec, nrhs, _VP(x.data_ptr()), _VP(y.data_ptr()),
                                _stream(stream)))
        return y

    def matvec_noalloc(self, medium, op, x, y, stream=None):
        """y = Op x for one right-hand side x [E] on the device, through the
        allocation-free entry point (y must be preallocated)."""
        prec = self._prec_of(x)
        if not (x.is_contiguous() and y.is_contiguous() and x.dim() == 1 and y.shape == x.shape
                and y.dtype == x.dtype):
            raise ValueError("x and y must be contiguous vectors of one shape and dtype")
        _check(lib().sie_matvec_noalloc(self.h, medium, op, prec, _VP(x.data_ptr()), _VP(y.data_ptr()),
                                        _stream(stream)))
        return y

    def aug_matvec(self, x, y=None, stream=None):
        """Exterior rows of the augmented EFIE (SIE_OP_AUG, FP64) for x of
        shape [E + T] or [nrhs, E + T] on the device."""
        import torch
        x = x.contiguous()
        if x.dtype != torch.complex128:
            raise ValueError("the augmented product takes complex128")
        if y is None:
            y = torch.empty_like(x)
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _check(lib().sie_matvec(self.h, -1, OP_AUG, FP64, nrhs, _VP(x.data_ptr()), _VP(y.data_ptr()),
                                _stream(stream)))
        return y

    def constraint_precond(self, x, y=None, stream=None):
        """Constraint preconditioner of the augmented EFIE, y = P^-1 x for x of
        shape [E + T] or [nrhs, E + T] (complex128) on the device."""
        import torch
        x = x.contiguous()
        if x.dtype != torch.complex128:
            raise ValueError("the constraint preconditioner takes complex128")
        if y is None:
            y = torch.empty_like(x)
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _check(lib().sie_constraint_precond(self.h, nrhs, _VP(x.data_ptr()), _VP(y.data_ptr()), _stream(stream)))
        return y

    def nested_precond(self, precond, x, y=None, stream=None):
        """y = nested-solve preconditioner (1 block-Jacobi, 4 / 12 Schwarz
        clusters, 16 exact near-region LU, 20 / 28 LU where it applies and
        clusters elsewhere) applied to x of shape [E] or [nrhs, E] on the
        device."""
        import torch
        prec = self._prec_of(x)
        x = x.contiguous()
        if y is None:
            y = torch.empty_like(x)
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _check(lib().sie_nested_precond(self.h, precond, prec, nrhs, _VP(x.data_ptr()), _VP(y.data_ptr()),
                                        _stream(stream)))
        return y

    def nested_precond_clusters(self):
        """(clusters, owned RWG rows) of the built Schwarz preconditioner,
        (-1, 0) before it is built."""
        owned = ctypes.c_int64(0)
        n = lib().sie_nested_precond_clusters(self.h, ctypes.byref(owned))
        return int(n), int(owned.value)

    def nested_precond_factored(self):
        """(media with an exact near-region LU, factor entries, factor
        seconds); media -1 before it is built."""
        nnz = ctypes.c_int64(0)
        t = ctypes.c_double(0.0)
        n = lib().sie_nested_precond_factored(self.h, ctypes.byref(nnz), ctypes.byref(t))
        return int(n), int(nnz.value), float(t.value)

    def project(self, medium, x, stream=None):
        import torch
        g = self.grid(medium)
        nl = g["nl"]
        out = torch.empty((4, nl[2], nl[1], nl[0]), dtype=x.dtype, device=x.device)
        _check(lib().sie_project(self.h, medium, self._prec_of(x), _VP(x.contiguous().data_ptr()),
                                 _VP(out.data_ptr()), _stream(stream)))
        return out

    def convolve(self, medium, grid_in, out=None, op=OP_L, stream=None):
        """Zero-padded FFT convolution of grid_in [F][nl_z][nl_y][nl_x] on the
        live box: op OP_L, each field with G; op OP_K, the 3 fields J to
        grad G x J."""
        import torch
        grid_in = grid_in.contiguous()
        if out is None:
            out = torch.empty_like(grid_in)
        _check(lib().sie_convolve(self.h, medium, op, self._prec_of(grid_in), grid_in.shape[0],
                                  _VP(grid_in.data_ptr()), _VP(out.data_ptr()), _stream(stream)))
        return out

    def interpolate(self, medium, grid, stream=None):
        import torch
        y = torch.empty(self.num_rwg, dtype=grid.dtype, device=grid.device)
        _check(lib().sie_interpolate(self.h, medium, self._prec_of(grid), _VP(grid.contiguous().data_ptr()),
                                     _VP(y.data_ptr()), _stream(stream)))
        return y

    STAGES = ("project", "fft", "interp", "spmv", "product", "spmv64", "spmv_int32", "spmv_int64", "spmv_skip")

    def set_timing(self, on=True):
        """True/1: time every stage; 2: the near-field CSR product alone; False/0: off."""
        _check(lib().sie_set_timing(self.h, int(on)))

    def stage_times(self):
        """{stage: (launches, total_ms)} of the stage timers."""
        out = {}
        for i, name in enumerate(self.STAGES):
            n = ctypes.c_int64(); ms = ctypes.c_double()
            _check(lib().sie_get_stage_time(self.h, i, ctypes.byref(n), ctypes.byref(ms)))
            out[name] = (n.value, ms.value)
        return out

    # -- solve ----------------------------------------------------------------
    def set_planewaves(self, khat, e0):
        khat = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
        e0 = np.atleast_2d(np.asarray(e0, dtype=np.complex128))
        ee = np.ascontiguousarray(np.stack([e0.real, e0.imag], axis=-1))
        _check(lib().sie_set_planewaves(self.h, len(khat), _ptr(khat, ctypes.c_double), ee.ctypes.data_as(_CP)))

    def solve(self, precision=FP64, **opts):
        o = SolverOpts(**opts) if opts else None
        r = Report()
        st = lib().sie_solve(self.h, precision, ctypes.byref(o) if o else None, ctypes.byref(r))
        if st not in (SIE_OK, SIE_ENOCONV):
            _check(st)
        d = r.as_dict()
        d["converged"] = st == SIE_OK
        return d

    def currents(self, rhs=0):
        E = self.num_rwg
        u = np.empty((E, 2)); v = np.empty((E, 2))
        _check(lib().sie_get_currents(self.h, rhs, u.ctypes.data_as(_CP), v.ctypes.data_as(_CP)))
        return u[:, 0] + 1j * u[:, 1], v[:, 0] + 1j * v[:, 1]

    def charges(self, rhs=0):
        """sigma = c0 rho per triangle of an augmented solve."""
        T = self.num_tri
        sg = np.empty((T, 2))
        _check(lib().sie_get_charges(self.h, rhs, sg.ctypes.data_as(_CP)))
        return sg[:, 0] + 1j * sg[:, 1]

    def far_field_angles(self, theta, phi, rhs=0):
        """(E_theta, E_phi) far-field amplitudes at the directions (theta, phi)."""
        th = np.ascontiguousarray(np.atleast_1d(theta), dtype=np.float64)
        ph = np.ascontiguousarray(np.atleast_1d(phi), dtype=np.float64)
        if th.shape != ph.shape:
            raise ValueError("theta and phi must have one shape")
        a = np.empty((len(th), 2)); b = np.empty((len(th), 2))
        _check(lib().sie_far_field_angles(self.h, rhs, len(th), _ptr(th, ctypes.c_double),
                                          _ptr(ph, ctypes.c_double), a.ctypes.data_as(_CP), b.ctypes.data_as(_CP)))
        return a[:, 0] + 1j * a[:, 1], b[:, 0] + 1j * b[:, 1]

    def far_field(self, rhat, rhs=0):
        rhat = np.ascontiguousarray(np.atleast_2d(rhat), dtype=np.float64)
        out = np.empty((len(rhat), 3, 2))
        _check(lib().sie_far_field(self.h, rhs, len(rhat), _ptr(rhat, ctypes.c_double), out.ctypes.data_as(_CP)))
        return out[..., 0] + 1j * out[..., 1]


class Server:
    """Continuous batching of independent solve requests on one device: the
    library's worker threads admit requests first-in first-out within a
    device-memory budget and run setup, plane waves and solve concurrently."""

    def __init__(self, hbm_budget_bytes=0, max_slots=4, ctx=None, device=0):
        self.ctx = ctx or Context(device)
        h = _VP()
        _check(lib().sie_server_create(self.ctx.h, int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
        self.h = h
        self._owned = {}

    def submit(self, problem, khat, e0, precision=FP32, **opts):
        """Queues `problem` (ownership passes to the server until take());
        returns the ticket."""
        khat = np.ascontiguousarray(np.atleast_2d(khat), dtype=np.float64)
        e0 = np.atleast_2d(np.asarray(e0, dtype=np.complex128))
        ee = np.ascontiguousarray(np.stack([e0.real, e0.imag], axis=-1))
        o = SolverOpts(**opts) if opts else None
        t = ctypes.c_uint64()
        _check(lib().sie_server_submit(self.h, problem.h, len(khat), _ptr(khat, ctypes.c_double),
                                       ee.ctypes.data_as(_CP), precision, ctypes.byref(o) if o else None,
                                       ctypes.byref(t)))
        self._owned[t.value] = problem
        problem._served = True
        return t.value

    def poll(self, ticket):
        info = JobInfo()
        _check(lib().sie_server_poll(self.h, ticket, ctypes.byref(info)))
        return info.as_dict()

    def take(self, ticket):
        """Waits for the request and hands its problem back."""
        out = _VP()
        _check(lib().sie_server_take(self.h, ticket, ctypes.byref(out)))
        p = self._owned.pop(ticket)
        p._served = False
        return p

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sie_server_destroy(self.h)
            for p in self._owned.values():
                p.h = None          # destroyed by the server
            self._owned.clear()
            self.h = None

    def __del__(self):
        self.close()

