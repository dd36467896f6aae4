"""The screening kernel tracks the union complement q = prod(1 - o_i) with one
FMA per atom (q <- q - q o) and takes u = 1 - q; alignment uses the
cancellation-free recurrence u <- u + o - u o, which keeps u's relative
precision where every o_i is small.  At screening poses (both molecules
centred in their principal frames, overlapping) the samples where u is small
carry little weight, so the q form changes the estimates by far less than
the 1e-5 parity bar.  This checks that on the CPU: the side-A estimate of
O_AB (Eqs. IS and the bounded weight w = u/m) from the same oracle samples,
with u evaluated in FP32 in the kernel's atom order by each form, against
the same estimate in FP64.  Occupancies are rounded to FP32 once; products
of FP32 values are exact in FP64, so each FMA is emulated by one rounding."""
import numpy as np

import oracle as O
from paper_2607_20766_amd import molgen
from paper_2607_20766_amd.engine import LAMBDA_P27

f32 = np.float32


def _occ(xyz, alpha, r):
    d2 = ((r[:, None, :] - xyz[None, :, :]) ** 2).sum(-1)
    return np.exp(-alpha[None, :] * d2)  # FP64, [samples][atoms]


def _u_forms(o64):
    """u from FP32 occupancies: exact (FP64), q form and recurrence (FP32)."""
    o = o64.astype(f32)
    u_exact = 1.0 - np.prod(1.0 - o64, axis=1)
    q = np.ones(o.shape[0], f32)
    u = np.zeros(o.shape[0], f32)
    for i in range(o.shape[1]):
        oi = o[:, i]
        q = (q.astype(np.float64) - q.astype(np.float64) * oi).astype(f32)
        s = (u + oi).astype(f32)
        u = (s.astype(np.float64) - u.astype(np.float64) * oi).astype(f32)
    return u_exact, (f32(1) - q).astype(np.float64), u.astype(np.float64)


def test_union_complement_form_is_far_below_the_parity_bar():
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(1, 24, 10, 50, workers=1)
    qa = O.alpha_from_radius(q.radius, LAMBDA_P27)
    la = O.alpha_from_radius(L.radius, LAMBDA_P27)
    worst = {"q": 0.0, "rec": 0.0}
    for m in range(L.n_mols):
        bx = L.xyz[L.offsets[m]:L.offsets[m + 1]].astype(np.float64)
        ba = la[L.offsets[m]:L.offsets[m + 1]]
        ax = q.xyz.astype(np.float64)
        v, Z, _ = O.mol_prep(ax, qa)
        r = O.sample_points(ax, qa, 7, 0, 0, 4096)
        oA, oB = _occ(ax, qa, r), _occ(bx, ba, r)
        mA = oA.astype(f32).astype(np.float64).sum(1)
        uA = _u_forms(oA)
        uB = _u_forms(oB)
        est = [Z * np.mean(np.minimum(uA[k] / mA, 1.0) * uB[k]) for k in range(3)]
        worst["q"] = max(worst["q"], abs(est[1] - est[0]) / est[0])
        worst["rec"] = max(worst["rec"], abs(est[2] - est[0]) / est[0])
    assert worst["q"] < 1e-6, worst
    assert worst["rec"] < 1e-6, worst
