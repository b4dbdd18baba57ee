"""Pins of the Schwarz-form preconditioner reference used by the GPU parity
tests: one cluster over everything is the exact inverse; clusters partition
the rows; with no overlap and a block-diagonal operator it is exact."""
import numpy as np

from schwarz_ref import clusters, schwarz_matrix


def _cells(E, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(1, 9, size=(E, 3))


def test_single_cluster_is_exact_inverse():
    rng = np.random.default_rng(1)
    E = 40
    M = rng.standard_normal((E, E)) + 1j * rng.standard_normal((E, E)) + 8 * np.eye(E)
    cells = _cells(E, 2)
    P = schwarz_matrix(M, clusters(cells, C=64, O=0))
    assert np.abs(P @ M - np.eye(E)).max() < 1e-12


def test_clusters_partition_rows_and_contain_owned():
    cells = _cells(300, 3)
    cl = clusters(cells, C=2, O=1)
    own = np.concatenate([o for o, _ in cl])
    assert np.array_equal(np.sort(own), np.arange(300))
    for o, e in cl:
        assert np.all(np.isin(o, e))
        # extended box: every member within O cells of the owned box
        lo = (cells[o[0]] // 2) * 2 - 1
        assert np.all(cells[e] >= lo) and np.all(cells[e] <= lo + 3)


def test_block_diagonal_operator_without_overlap_is_exact():
    rng = np.random.default_rng(4)
    cells = _cells(120, 5)
    cl = clusters(cells, C=2, O=0)
    E = len(cells)
    M = np.zeros((E, E), complex)
    for own, _ in cl:
        n = len(own)
        M[np.ix_(own, own)] = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    P = schwarz_matrix(M, cl)
    assert np.abs(P @ M - np.eye(E)).max() < 1e-10
