"""Loader for the oracle's plain-C pair integrals (``oracle/csrc/pairint.c``).

Builds ``oracle/_build/libpairint.so`` with gcc (no fast-math, no FMA
contraction) when it is missing or older than its source.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "pairint.c")
_OUT = os.path.join(_HERE, "_build", "libpairint.so")
_lib = None


def build(force=False):
    if (not force and os.path.exists(_OUT)
            and os.path.getmtime(_OUT) >= os.path.getmtime(_SRC)):
        return _OUT
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    tmp = _OUT + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp",
                           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _OUT)
    return _OUT


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        ll = ctypes.POINTER(ctypes.c_longlong)
        _lib.oracle_pair_blocks.argtypes = [d, d, d, d, ctypes.c_longlong, ll, ll,
                                            ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int, d, d, ctypes.c_int, d, d,
                                            ctypes.c_int, d, d, d, d, d]
        _lib.oracle_pair_blocks.restype = None
        _lib.oracle_static_pot.argtypes = [d, d, d]
        _lib.oracle_static_pot.restype = None
        _lib.oracle_polar_pot.argtypes = [d, d, ctypes.c_double, ctypes.c_double, d, d, d]
        _lib.oracle_polar_pot.restype = None
    return _lib


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


# Gauss-Legendre order of the strong-loss (polar) inner scheme, per radial
# interval and per angular piece.
POLAR_NG = 8


def _gl():
    x, w = np.polynomial.legendre.leggauss(POLAR_NG)
    return np.ascontiguousarray(x), np.ascontiguousarray(w)


def pair_blocks_c(mesh, k, tl, sl, rule_out, rule_in, polar=False):
    """C version of :func:`oracle.mom.pair_blocks_np`: returns (A, Phi, K) local
    blocks [P,3,3] complex.  polar: the strong-loss inner scheme instead of
    the inner rule."""
    L = lib()
    tl = np.ascontiguousarray(tl, dtype=np.int64)
    sl = np.ascontiguousarray(sl, dtype=np.int64)
    P = len(tl)
    bo, wo = (np.ascontiguousarray(x, dtype=np.float64) for x in rule_out)
    bi, wi = (np.ascontiguousarray(x, dtype=np.float64) for x in rule_in)
    if len(wi) > 256:
        raise ValueError("inner rule limited to 256 points")
    verts = np.ascontiguousarray(mesh.verts, dtype=np.float64)
    area = np.ascontiguousarray(mesh.area, dtype=np.float64)
    sgn = np.ascontiguousarray(mesh.tri_sign, dtype=np.float64)
    ln = np.ascontiguousarray(mesh.tri_len, dtype=np.float64)
    A = np.empty((P, 3, 3, 2)); Ph = np.empty((P, 3, 3, 2)); K = np.empty((P, 3, 3, 2))
    k = complex(k)
    gx, gw = _gl()
    L.oracle_pair_blocks(_p(verts), _p(area), _p(sgn), _p(ln), P,
                         _p(tl, ctypes.c_longlong), _p(sl, ctypes.c_longlong),
                         k.real, k.imag, len(wo), _p(bo), _p(wo), len(wi), _p(bi), _p(wi),
                         1 if polar else 0, _p(gx), _p(gw),
                         _p(A), _p(Ph), _p(K))
    c = lambda x: x[..., 0] + 1j * x[..., 1]
    return c(A), c(Ph), c(K)


def polar_pot_c(v, r, k):
    """Strong-loss inner integrals of triangle v [3,3] at r: (S, V[3], Gv[3])."""
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(9)
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(3)
    gx, gw = _gl()
    out = np.empty(14)
    k = complex(k)
    lib().oracle_polar_pot(_p(v), _p(r), k.real, k.imag, _p(gx), _p(gw), _p(out))
    c = out[0::2] + 1j * out[1::2]
    return c[0], c[1:4], c[4:7]


def static_pot_c(v, r):
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(9)
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(3)
    out = np.empty(7)
    lib().oracle_static_pot(_p(v), _p(r), _p(out))
    return out[0], out[1:4], out[4:7]
