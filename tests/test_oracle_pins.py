"""Pins of the oracle parts that the estimator, screening and alignment
tests only used, never fixed: the standard errors of the Tanimoto (section
"Confidence-bounded screening": the delta-method SE(T) that drives every stop,
and the full propagation that adds the self-overlap errors), the rule of the
seeded budgets, the parameter checks of the rounds, the Adam steps of the
alignment drivers, and the integer sampling thresholds (section
"Importance-sampling estimator": exact draws from the normalised mixture).
Each pin comes from outside the code it checks: numerical differentiation,
numpy's sample statistics, the exact inclusion-exclusion value, rounds
enumerated by hand, torch.optim.Adam, exact rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from paper_2607_20766_amd import molgen
from tests import cases


def _om(O, m):
    return cases.oracle_mol(O, m)


def test_se_T_is_the_delta_method_by_central_differences(oracle):
    """SE(T) = |dT/dO_AB| SE(O_AB) with T(x) = x / (O_AA + O_BB - x); the
    derivative taken numerically (central differences, Richardson-refined),
    not from its closed form."""
    for (sa, na), (sb, nb), shift in (((40, 5), (41, 4), 0.4), ((0, 20), (1, 24), 0.0)):
        A = _om(oracle, cases.small(sa, na) if na < 10 else cases.config0()[0])
        B = _om(oracle, cases.small(sb, nb) if nb < 10 else cases.config0()[1])
        B = (B[0] + np.float32(shift), B[1])
        r = oracle.estimate(A, B, 3000, 2000, seed=11, id_a=3, id_b=4)
        S = r["O_aa"] + r["O_bb"]

        def T(x):
            return x / (S - x)

        x = r["O_ab"]
        h = 1e-3 * x
        d1 = (T(x + h) - T(x - h)) / (2 * h)
        d2 = (T(x + h / 2) - T(x - h / 2)) / h
        dT = (4 * d2 - d1) / 3
        assert r["T"] == pytest.approx(T(x), rel=1e-14)
        assert r["se_T"] == pytest.approx(abs(dT) * r["se_O_ab"], rel=1e-9)


def test_se_O_ab_from_per_sample_integrands(oracle):
    """SE(O_AB) = 1/2 sqrt(SE_A^2 + SE_B^2) with SE_P = Z_P s_P / sqrt(n_P),
    s_P numpy's sample standard deviation (n - 1) of w_P u_Q over P's own
    samples, rebuilt here from the sample points and the densities."""
    a, b = cases.config0()
    A, B = _om(oracle, a), _om(oracle, b)
    na, nb, seed = 4000, 3000, 21
    sides = []
    for P, Q, idp, n in ((A, B, 5, na), (B, A, 6, nb)):
        Z = oracle.mol_prep(*P)[1]
        r = oracle.sample_points(*P, idp, seed, 0, n)
        mP, uP = oracle.densities(*P, r)
        _, uQ = oracle.densities(*Q, r)
        f = uP / mP * uQ
        sides.append((Z * f.mean(), Z * np.std(f, ddof=1) / np.sqrt(n), Z, uP / mP * uP))
    r = oracle.estimate(A, B, na, nb, seed=seed, id_a=5, id_b=6)
    assert r["O_ab_from_a"] == pytest.approx(sides[0][0], rel=1e-12)
    assert r["O_ab_from_b"] == pytest.approx(sides[1][0], rel=1e-12)
    assert r["O_ab"] == pytest.approx(0.5 * (sides[0][0] + sides[1][0]), rel=1e-12)
    assert r["se_O_ab"] == pytest.approx(0.5 * np.hypot(sides[0][1], sides[1][1]), rel=1e-10)
    Za, fa = sides[0][2], sides[0][3]
    assert r["O_aa"] == pytest.approx(Za * fa.mean(), rel=1e-12)
    assert r["se_O_aa"] == pytest.approx(Za * np.std(fa, ddof=1) / np.sqrt(na), rel=1e-10)


@pytest.mark.parametrize("sa,sb,shift", [(40, 41, 0.4), (44, 45, 0.0)])
def test_se_T_full_is_calibrated_against_the_exact_tanimoto(oracle, sa, sb, shift):
    """Over 400 seeds the z-scores (T - T_exact) / SE(T)_full, T_exact from
    the full inclusion-exclusion series, have mean ~0 and variance ~1.  Left
    out, the covariance of O_AB with the self-overlaps halves the variance
    of z on these pairs, and a flipped sign of that term cuts it to a third:
    either falls outside the band."""
    A = _om(oracle, cases.small(sa, 5))
    B = _om(oracle, cases.small(sb, 4))
    B = (B[0] + np.float32(shift), B[1])
    Oab, Oaa, Obb = oracle.incexc(A, B), oracle.incexc(A, A), oracle.incexc(B, B)
    T_exact = Oab / (Oaa + Obb - Oab)
    z = np.array([(r["T"] - T_exact) / r["se_T_full"] for r in
                  (oracle.estimate(A, B, 1000, 1000, seed=7000 + s, id_a=1, id_b=2)
                   for s in range(400))])
    assert abs(z.mean()) < 0.2
    assert 0.82 < z.var() < 1.2


def _library_pair():
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(1, 6, 10, 50)
    return q, L


def test_seeded_budget_rounds_enumerated_by_hand(oracle):
    """n_start defers the first stop test until the pair has drawn n_start
    samples, in whole rounds, never past the cap.  With tau so large that
    every test passes, the pair stops at the first tested round: 512 per
    round, cap 4096, budgets 0, 1, 512, 513, 1300, 1536, 1537, 4096, 9999 ->
    512, 512, 512, 1024, 1536, 1536, 2048, 4096, 4096.  With tau so small
    that no test passes, every pair runs to the cap."""
    q, L = _library_pair()
    Q = _om(oracle, q)
    la = oracle.alpha_from_radius(L.radius, cases.LAMBDA)
    budgets = np.array([0, 1, 512, 513, 1300, 1536, 1537, 4096, 9999], np.int32)
    expect = [512, 512, 512, 1024, 1536, 1536, 2048, 4096, 4096]
    pairs = np.zeros(budgets.size, np.int32) + 2
    out = oracle.screen(Q, 999, L.offsets, L.xyz, la, pairs=pairs, mode=1, round_per_pair=512,
                        cap_per_pair=4096, tau=1e9, seed=3, n_start=budgets)
    assert out[:, 5].astype(int).tolist() == expect
    out = oracle.screen(Q, 999, L.offsets, L.xyz, la, pairs=pairs, mode=1, round_per_pair=512,
                        cap_per_pair=4096, tau=1e-9, seed=3, n_start=budgets)
    assert np.all(out[:, 5] == 4096)
    # with a budget and a reachable tau the pair stops at the first round at or
    # past its budget whose SE(T) meets tau: the fixed-count estimates decide
    a, b = L.offsets[2], L.offsets[3]
    se = [oracle.estimate(Q, (L.xyz[a:b], la[a:b]), 256 * k, 256 * k, seed=3, id_a=999,
                          id_b=2)["se_T"] for k in range(1, 17)]
    tau = se[5] * 1.0000001   # met from round 6 on at the latest
    for budget in (0, 1024, 2560):
        first = budget // 512 + (budget % 512 > 0)
        k = next(k for k in range(max(first, 1), 17) if se[k - 1] <= tau or k == 16)
        out = oracle.screen(Q, 999, L.offsets, L.xyz, la, pairs=pairs[:1], mode=1,
                            round_per_pair=512, cap_per_pair=8192, tau=tau, seed=3,
                            n_start=np.array([budget], np.int32))
        assert int(out[0, 5]) == 512 * k
        assert out[0, 1] == se[k - 1]


def test_screen_rejects_parameters_the_rounds_cannot_follow(oracle):
    q, L = _library_pair()
    Q = _om(oracle, q)
    la = oracle.alpha_from_radius(L.radius, cases.LAMBDA)
    bad = [dict(mode=1, round_per_pair=512, cap_per_pair=1000),   # cap not whole rounds
           dict(mode=1, round_per_pair=1, cap_per_pair=4),         # half a sample per side
           dict(mode=1, round_per_pair=513, cap_per_pair=1026),    # odd round
           dict(mode=1, round_per_pair=512, cap_per_pair=256),     # cap below one round
           dict(mode=1, round_per_pair=512, cap_per_pair=4096, tau=0.0),
           dict(mode=0, n_fixed=1),
           dict(mode=2)]
    for kw in bad:
        with pytest.raises(ValueError):
            oracle.screen(Q, 999, L.offsets, L.xyz, la, seed=1, **kw)
    with pytest.raises(ValueError):
        oracle.screen(Q, 999, L.offsets, L.xyz, la, mode=1, round_per_pair=514,
                      cap_per_pair=1028, antithetic=True)   # odd antithetic half-round


def test_screen_pair_outside_the_library_scores_nothing(oracle):
    q, L = _library_pair()
    Q = _om(oracle, q)
    la = oracle.alpha_from_radius(L.radius, cases.LAMBDA)
    out = oracle.screen(Q, 999, L.offsets, L.xyz, la, pairs=np.array([1, -1, 6, 4], np.int32),
                        mode=0, n_fixed=256, seed=1)
    assert np.all(np.isnan(out[[1, 2], :5])) and np.all(out[[1, 2], 5] == 0)
    assert np.all(np.isfinite(out[[0, 3]]))


def _adam_by_torch(grad_fn, pose0, n_steps, lr):
    """Ascent on T: torch.optim.Adam (float64, betas 0.9/0.999, eps 1e-8) on
    -dT/dpose, quaternion renormalised after each step."""
    x = torch.tensor(pose0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([x], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(n_steps):
        g = grad_fn(x.detach().numpy().copy())
        opt.zero_grad()
        x.grad = torch.from_numpy(-g)
        opt.step()
        with torch.no_grad():
            x[:4] /= torch.linalg.norm(x[:4])
    return x.detach().numpy()


def test_union_alignment_adam_steps_match_torch_adam(oracle):
    """The union alignment driver's Adam (section "Differentiable alignment
    and the hybrid pipeline") step for step against torch.optim.Adam fed the
    driver's own recorded gradients."""
    A = _om(oracle, cases.small(50, 7))
    B = _om(oracle, cases.small(51, 6))
    pose0 = np.array([0.9, 0.1, -0.2, 0.3, 0.4, -0.3, 0.2])

    def grad(p):
        return oracle.align_grad(A, B, p[None], n_samples=512, seed=2, id_a=1, id_b=2)[1][0]

    for steps in (1, 2, 5):
        ref = _adam_by_torch(grad, pose0, steps, 0.05)
        got, _ = oracle.align_adam(A, B, pose0[None], n_steps=steps, lr=0.05, n_samples=512,
                                   seed=2, id_a=1, id_b=2)
        np.testing.assert_allclose(got[0], ref, rtol=1e-12, atol=1e-14)


def test_first_order_alignment_adam_steps_match_torch_adam(oracle):
    A = _om(oracle, cases.small(52, 8))
    B = _om(oracle, cases.small(53, 9))
    pose0 = np.array([0.7, -0.3, 0.2, 0.1, -0.5, 0.6, 0.1])

    def grad(p):
        return oracle.fo_align_grad(A, B, p[None])[1][0]

    for steps in (1, 3, 6):
        ref = _adam_by_torch(grad, pose0, steps, 0.05)
        got, _ = oracle.fo_align_adam(A, B, pose0[None], n_steps=steps, lr=0.05)
        np.testing.assert_allclose(got[0], ref, rtol=1e-12, atol=1e-14)


def test_thresholds_by_exact_rational_arithmetic(oracle):
    """thr_i = floor(2^32 * (v_0 + .. + v_i) / Z) with the running sums in
    atom order: recomputed from the FP64 sums with exact rationals, so the
    floor is taken on the exact quotient rather than its rounding."""
    for m in (cases.config0()[0], cases.config0()[1], molgen.molecule(7, 7, 50),
              molgen.molecule(8, 3, 2)):
        xyz, alpha = _om(oracle, m)
        v, Z, thr = oracle.mol_prep(xyz, alpha)
        run, exact = 0.0, []
        for i in range(v.size - 1):
            run = run + float(v[i])          # the FP64 running sum, in order
            q = Fraction(run) / Fraction(Z)
            exact.append(min(2**32 - 1, (q * 2**32).__floor__()))
        assert thr.astype(np.int64).tolist() == exact


def test_component_is_the_count_of_thresholds_at_or_below_the_word(oracle):
    """j = #{i : x0 >= thr_i} (a word equal to a threshold selects the upper
    component): from the Philox words themselves and numpy's searchsorted
    on the thresholds."""
    m = molgen.molecule(9, 1, 33)
    xyz, alpha = _om(oracle, m)
    _, _, thr = oracle.mol_prep(xyz, alpha)
    mol_id, seed, k0, n = 77, 0x1234_5678_9ABC, 1000, 4000
    _, comp = oracle.sample_points(xyz, alpha, mol_id, seed, k0, n, return_component=True)
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
    x0 = np.empty(n, np.uint32)
    for i in range(n):
        k = k0 + i
        x0[i] = oracle.philox(np.array([k & 0xFFFFFFFF, k >> 32, mol_id, 0], np.uint32), key)[0]
    assert np.array_equal(comp, np.searchsorted(thr, x0, side="right"))
