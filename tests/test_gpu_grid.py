"""GPU dense-grid quadrature (the reference of the accuracy comparison)
against the FP64 oracle's grid, and the IS estimator against the GPU grid
within its standard error."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_20766_amd import molgen
from paper_2607_20766_amd.engine import Engine, Molecules, ShapeError
from tests import cases
from tests.gpu_common import oracle_mol, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    require_gpu()
    return Engine(0)


def test_grid_matches_oracle(eng):
    qa, qb = cases.config0()
    print("case: grid h=0.25, config0 pair", flush=True)
    g = eng.shape_grid_integrals(eng.molecules(qa), eng.molecules(qb), h=0.25, pad=6.5)
    r = O.grid_integrals(oracle_mol(O, qa), oracle_mol(O, qb), h=0.25, pad=6.5)
    for (k, v), rv in zip(g.items(), r.values()):
        assert v == pytest.approx(rv, rel=1e-11), k


def test_grid_reads_the_molecule_range(eng):
    """A one-molecule set whose atoms start inside a larger array."""
    L = molgen.library(71, 3, 12, 20, workers=1)
    full = eng.molecules(L)
    m = 1
    sub = Molecules(full.offsets[m:m + 2].contiguous(), full.xyz, full.alpha, None,
                    int(L.offsets[m + 1] - L.offsets[m]))
    alone = eng.molecules(L.mol(m))
    q = eng.molecules(molgen.molecule(1, 0, 15))
    a = eng.shape_grid_integrals(sub, q, h=0.3)
    b = eng.shape_grid_integrals(alone, q, h=0.3)
    assert a == b


def test_is_agrees_with_grid_within_se(eng):
    qa, qb = cases.config0()
    A, B = eng.molecules(qa, mol_id=[0]), eng.molecules(qb, mol_id=[1])
    g = eng.shape_grid_integrals(A, B, h=0.15, pad=6.5)
    est = eng.shape_estimate(A, B, 200000, 200000, seed=4)
    for k_is, k_se, k_g in (("O_ab", "se_O_ab", "O_ab"), ("O_aa", "se_O_aa", "O_aa"),
                            ("O_bb", "se_O_bb", "O_bb"), ("V_a", "se_V_a", "V_a"),
                            ("V_b", "se_V_b", "V_b")):
        z = (est[k_is] - g[k_g]) / est[k_se]
        assert abs(z) < 4.5, (k_is, z)
    # the first-order channel of the estimator is unbiased for the exact Eq. fo
    assert est["Ofo_ab_is"] == pytest.approx(g["Ofo_ab"], rel=0.02)


def test_grid_rejects_invalid_data(eng):
    qa, qb = cases.config0()
    bad = molgen.MolSet.concat([qb])
    bad.radius[3] = 0.0
    with pytest.raises(ShapeError):
        eng.shape_grid_integrals(eng.molecules(qa), eng.molecules(bad), h=0.5)
