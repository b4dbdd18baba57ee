"""Plain reference of the nested-solve preconditioner in Schwarz form (test
infrastructure): M_i = -j w eps_i L_i,NR (eq. nest2pc) from the oracle's
direct near-region operator, clusters of C^3 grid cells (cell of the stencil
centre of T+) owning their RWG functions and extending O cells on every
side; y[own] = inv(M[ext, ext])[own, :] x[ext]."""
import numpy as np


def clusters(cells, C=2, O=1):
    """cells: [E][3] integer cell per RWG.  Returns [(own, ext)] index arrays."""
    key = cells // C
    keys, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.ravel()
    out = []
    for q in range(len(keys)):
        own = np.nonzero(inv == q)[0]
        lo = keys[q] * C - O
        hi = keys[q] * C + C - 1 + O
        ext = np.nonzero(np.all((cells >= lo) & (cells <= hi), axis=1))[0]
        out.append((own, ext))
    return out


def schwarz_matrix(M, cl):
    """Dense matrix of the restricted additive Schwarz preconditioner."""
    E = M.shape[0]
    P = np.zeros((E, E), np.complex128)
    for own, ext in cl:
        Bi = np.linalg.inv(M[np.ix_(ext, ext)])
        P[np.ix_(own, ext)] = Bi[np.searchsorted(ext, own), :]
    return P
