"""The allocation-free estimate (shape_estimate_noalloc, fixed device scratch)
against shape_estimate on the same inputs, through the C ABI: the same
kernels on the same prepared records, so every field agrees bit for bit; two
calls in a row, the second smaller, so a stale record or partial sum of the
first call would show.  Also against the FP64 oracle on identical samples
(Eqs. expectation, var, union-is; 1e-5 relative)."""
import numpy as np
import pytest
import torch

from paper_2607_20766_amd import molgen
from paper_2607_20766_amd.engine import RESULT_FIELDS, Engine, ShapeError
from tests.gpu_common import oracle_mol, rel_err, require_gpu

pytestmark = pytest.mark.gpu

SE_FIELDS = {"se_O_ab", "se_O_aa", "se_O_bb", "se_V_a", "se_V_b", "se_T", "se_T_full"}


def _same(got, ref):
    for k in RESULT_FIELDS:
        assert got[k] == ref[k] or (np.isnan(got[k]) and np.isnan(ref[k])), (k, got[k], ref[k])
    assert got["n_a"] == ref["n_a"] and got["n_b"] == ref["n_b"]


def _vs_oracle(O, got, a, b, n_a, n_b, id_a, id_b):
    ref = O.estimate(oracle_mol(O, a), oracle_mol(O, b), n_a, n_b, seed=0, id_a=id_a,
                     id_b=id_b)
    for k in ("O_ab", "O_aa", "O_bb", "V_a", "V_b", "T"):
        assert rel_err(got[k], ref[k]) <= 1e-5, (k, got[k], ref[k])
    for k in ("se_O_ab", "se_T"):
        assert rel_err(got[k], ref[k]) <= 1e-4, (k, got[k], ref[k])


def test_noalloc_matches_estimate_two_calls(oracle):
    require_gpu()
    print("noalloc: 20/24-atom pair, n 20000/20000; then 12/9-atom pair, n 6000/4000",
          flush=True)
    eng = Engine(0)
    cases = [((0, 0, 20), (0, 1, 24), 20000, 20000),
             ((7, 3, 12), (7, 4, 9), 6000, 4000)]
    for (sa, ia, na_atoms), (sb, ib, nb_atoms), n_a, n_b in cases:
        a = molgen.molecule(sa, ia, na_atoms)
        b = molgen.molecule(sb, ib, nb_atoms)
        A = eng.molecules(a, mol_id=[ia])
        B = eng.molecules(b, mol_id=[ib])
        got = eng.shape_estimate_noalloc(A, B, n_a, n_b, seed=0)
        ref = eng.shape_estimate(A, B, n_a, n_b, seed=0)
        _same(got, ref)
        _vs_oracle(oracle, got, a, b, n_a, n_b, ia, ib)
    torch.cuda.synchronize()


def test_noalloc_rejects_sizes_beyond_its_limit():
    require_gpu()
    print("noalloc: limits (host-side checks only)", flush=True)
    eng = Engine(0)
    a = molgen.molecule(0, 0, 20)
    A = eng.molecules(a, mol_id=[0])
    with pytest.raises(ShapeError) as e:
        eng.shape_estimate_noalloc(A, A, (1 << 24) + 2, 1000)
    assert e.value.code == -2
    # a one-molecule set whose arrays hold more atoms than the fixed staging
    big = molgen.molecule(0, 5, 20)
    Big = eng.molecules(big, mol_id=[5])
    pad = torch.zeros(300 - Big.n_atoms, 3, device=Big.xyz.device)
    Big.xyz = torch.cat([Big.xyz, pad]).contiguous()
    Big.alpha = torch.cat([Big.alpha, torch.ones(300 - Big.alpha.numel(),
                                                 device=Big.xyz.device)]).contiguous()
    with pytest.raises(ShapeError) as e:
        eng.shape_estimate_noalloc(A, Big, 1000, 1000)
    assert e.value.code == -2
    # the entry point still works after the rejected calls
    got = eng.shape_estimate_noalloc(A, A, 2048, 2048)
    assert got["T"] == 1.0
