"""The seeded input generator: geometry rules of the synthetic molecules and
of their conformer ensembles (same topology and elements, redrawn angles and
torsions)."""
import numpy as np
import pytest

from paper_2607_20766_amd import molgen


def _bonds(xyz):
    d = np.linalg.norm(xyz[:, None] - xyz[None], axis=-1)
    i, j = np.nonzero(np.triu(np.abs(d - molgen.BOND) < 1e-3, 1))
    return set(zip(i.tolist(), j.tolist())), d


def _graph_dist(n, bonds):
    D = np.full((n, n), 99, int)
    np.fill_diagonal(D, 0)
    for i, j in bonds:
        D[i, j] = D[j, i] = 1
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def test_library_rules():
    L = molgen.library(3, 40, 10, 50, workers=1)
    for m in range(L.n_mols):
        xyz = L.mol(m).xyz.astype(np.float64)
        n = xyz.shape[0]
        bonds, d = _bonds(xyz)
        assert len(bonds) == n - 1          # a tree
        D = _graph_dist(n, bonds)
        assert D.max() < 99                 # connected
        far = D >= 3
        assert np.all(d[far] >= molgen.NONBONDED_MIN - 1e-3)


def test_conformers_keep_topology_and_elements():
    C, g = molgen.conformer_library(9, 60, 10, 40, 4, workers=1)
    assert g.tolist() == list(range(0, 241, 4))
    for m in range(60):
        sets = [C.mol(4 * m + c) for c in range(4)]
        b0, _ = _bonds(sets[0].xyz.astype(np.float64))
        n = sets[0].n_atoms
        D = _graph_dist(n, b0)
        for s in sets[1:]:
            assert np.array_equal(s.element, sets[0].element)
            b, d = _bonds(s.xyz.astype(np.float64))
            assert b == b0                              # same bonded pairs
            assert np.all(d[D >= 3] >= molgen.NONBONDED_MIN - 1e-3)
        # torsions redrawn: the shapes differ (beyond a rigid motion)
        if n >= 6:
            d0 = np.linalg.norm(sets[0].xyz[:, None] - sets[0].xyz[None], axis=-1)
            d1 = np.linalg.norm(sets[1].xyz[:, None] - sets[1].xyz[None], axis=-1)
            assert np.abs(d0 - d1).max() > 0.1


def test_conformers_are_reproducible_and_chunk_invariant():
    a, _ = molgen.conformer_library(9, 30, 10, 40, 3, workers=1)
    b, _ = molgen.conformer_library(9, 30, 10, 40, 3, workers=1)
    assert np.array_equal(a.xyz, b.xyz)
