"""Pins of the oracle estimator against what the paper and the mathematics fix:
the inclusion-exclusion series (Eq. incexc) in closed form for small
molecules, dense-grid quadrature of Eq. union-overlap, the first-order closed
form (Eq. fo) and its variance (Eq. var), the bound on the union-estimator
variance, the n^-1/2 error decay, the calibration of the reported standard
errors, and exact symmetries."""
import numpy as np
import pytest

from tests import cases


def _om(O, m):
    return cases.oracle_mol(O, m)


def test_union_pointwise_equals_series(oracle):
    """1 - prod(1 - o_i) equals the full alternating series of Eq. incexc."""
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 9, 12):
        A = _om(oracle, cases.small(2, n))
        pts = rng.normal(size=(20, 3)) * 2.0
        m, u = oracle.densities(*A, pts)
        for k in range(pts.shape[0]):
            s = oracle.union_series_at(A, pts[k])
            assert abs(s - u[k]) <= 1e-13
        assert np.all(u <= m + 1e-15) and np.all(u >= 0) and np.all(u <= 1)


def test_incexc_matches_grid(oracle):
    """Two independent exact references agree: the 2^N-term series integrated
    term by term with the Gaussian product theorem, and trapezoid quadrature."""
    for n_a, n_b in ((3, 4), (5, 5)):
        A = _om(oracle, cases.small(3, n_a))
        B = _om(oracle, cases.small(4, n_b))
        g = oracle.grid_integrals(A, B, h=0.15)
        assert oracle.incexc(A, B) == pytest.approx(g["uAuB"], rel=1e-9)
        assert oracle.incexc(A, A) == pytest.approx(g["uA2"], rel=1e-9)
        assert oracle.incexc(A) == pytest.approx(g["uA"], rel=1e-9)
        assert oracle.fo_overlap(A, B) == pytest.approx(g["mAmB"], rel=1e-11)


def test_grid_converged(oracle):
    A, B = (_om(oracle, m) for m in cases.config0())
    g1 = oracle.grid_integrals(A, B, h=0.2)
    g2 = oracle.grid_integrals(A, B, h=0.1)
    for k in g1:
        assert g1[k] == pytest.approx(g2[k], rel=1e-9)


def test_single_atom_reduces_to_first_order(oracle):
    """One atom: u = o = m, so w = 1, V = Z exactly and the union overlap is
    the first-order closed form."""
    A = (np.zeros((1, 3), np.float32), np.array([0.8], np.float32))
    B = (np.array([[1.1, -0.4, 0.3]], np.float32), np.array([1.0], np.float32))
    r = oracle.estimate(A, B, 50000, 50000, seed=4, id_a=1, id_b=2)
    Za = (np.pi / np.float64(np.float32(0.8))) ** 1.5
    assert r["V_a"] == pytest.approx(Za, rel=1e-14)
    assert r["se_V_a"] < 1e-12 * Za
    fo = oracle.fo_overlap(A, B)
    assert abs(r["O_ab"] - fo) < 4.5 * r["se_O_ab"]
    assert r["O_ab"] == pytest.approx(r["Ofo_ab_is"], rel=1e-14)
    # int o^2 = (pi / (2 alpha))^(3/2)
    assert abs(r["O_aa"] - (np.pi / (2 * np.float64(np.float32(0.8)))) ** 1.5) < 4.5 * r["se_O_aa"]


@pytest.mark.parametrize("na,nb,seed", [(3, 4, 0), (5, 5, 1), (4, 2, 2)])
def test_is_unbiased_vs_incexc(oracle, na, nb, seed):
    A = _om(oracle, cases.small(10 + seed, na))
    B = _om(oracle, cases.small(20 + seed, nb))
    # put B near A so that the overlap is substantial
    B = (B[0] + np.float32(0.7), B[1])
    r = oracle.estimate(A, B, 100000, 100000, seed=seed, id_a=5, id_b=6)
    assert abs(r["O_ab"] - oracle.incexc(A, B)) < 4.5 * r["se_O_ab"]
    assert abs(r["O_aa"] - oracle.incexc(A, A)) < 4.5 * r["se_O_aa"]
    assert abs(r["O_bb"] - oracle.incexc(B, B)) < 4.5 * r["se_O_bb"]
    assert abs(r["V_a"] - oracle.incexc(A)) < 4.5 * r["se_V_a"]
    assert abs(r["V_b"] - oracle.incexc(B)) < 4.5 * r["se_V_b"]


def test_config0_pair_vs_grid(oracle):
    """20- and 24-atom molecules: union IS within 4.5 SE of grid quadrature."""
    A, B = (_om(oracle, m) for m in cases.config0())
    r = oracle.estimate(A, B, 100000, 100000, seed=0, id_a=0, id_b=1)
    g = oracle.grid_integrals(A, B, h=0.2)
    assert abs(r["O_ab"] - g["uAuB"]) < 4.5 * r["se_O_ab"]
    assert abs(r["O_aa"] - g["uA2"]) < 4.5 * r["se_O_aa"]
    assert abs(r["O_bb"] - g["uB2"]) < 4.5 * r["se_O_bb"]
    assert abs(r["V_a"] - g["uA"]) < 4.5 * r["se_V_a"]
    assert abs(r["V_b"] - g["uB"]) < 4.5 * r["se_V_b"]
    # the union never exceeds first order (pointwise m >= u)
    assert g["uAuB"] < g["mAmB"] and g["uA2"] < g["mA2"]
    T = g["uAuB"] / (g["uA2"] + g["uB2"] - g["uAuB"])
    assert abs(r["T"] - T) < 4.5 * r["se_T_full"]


def test_first_order_channel_mean_and_variance(oracle):
    """The FO channel estimates Eq. fo; its per-sample variance is Eq. var with
    E_q[m_B^2] from the triple-Gaussian closed form."""
    A, B = (_om(oracle, m) for m in cases.config0())
    n = 100000
    Za = oracle.mol_prep(*A)[1]
    fo = oracle.fo_overlap(A, B)
    Em = fo / Za
    Em2 = oracle.fo_second_moment(A, B) / Za
    se = Za * np.sqrt((Em2 - Em**2) / n)
    # side-A FO channel: Z_A times the mean of m_B over samples of q_A
    pts = oracle.sample_points(*A, 0, 7, 0, n)
    mB, _ = oracle.densities(*B, pts)
    assert abs(Za * mB.mean() - fo) < 4.5 * se
    assert np.var(mB, ddof=1) == pytest.approx(Em2 - Em**2, rel=0.05)
    # and the estimator reports the same channel, symmetrised
    Zb = oracle.mol_prep(*B)[1]
    mA, _ = oracle.densities(*A, oracle.sample_points(*B, 1, 7, 0, n))
    r = oracle.estimate(A, B, n, n, seed=7, id_a=0, id_b=1)
    assert r["Ofo_ab_is"] == pytest.approx(0.5 * (Za * mB.mean() + Zb * mA.mean()),
                                           rel=1e-12)


def test_se_decays_as_inverse_sqrt_n(oracle):
    A, B = (_om(oracle, m) for m in cases.config0())
    s = []
    for n in (4096, 16384, 65536):
        r = oracle.estimate(A, B, n, n, seed=1, id_a=0, id_b=1)
        s.append(r["se_O_ab"])
    slope = np.polyfit(np.log([4096, 16384, 65536]), np.log(s), 1)[0]
    assert slope == pytest.approx(-0.5, abs=0.03)


def test_union_variance_bound(oracle):
    """0 <= w_A u_B <= 1 gives Var <= Z^2/(4n) for each side."""
    A, B = (_om(oracle, m) for m in cases.config0())
    n = 20000
    r = oracle.estimate(A, B, n, n, seed=2, id_a=0, id_b=1)
    Za = oracle.mol_prep(*A)[1]
    Zb = oracle.mol_prep(*B)[1]
    assert r["se_O_aa"] <= Za / (2 * np.sqrt(n))
    assert r["se_O_bb"] <= Zb / (2 * np.sqrt(n))
    assert r["se_V_a"] <= Za / (2 * np.sqrt(n))
    assert 2 * r["se_O_ab"] <= np.hypot(Za, Zb) / (2 * np.sqrt(n))


def test_standard_errors_calibrated(oracle):
    """z-scores of the union overlap against the exact series over 150 seeds
    are ~N(0, 1)."""
    A = _om(oracle, cases.small(30, 5))
    B = _om(oracle, cases.small(31, 4))
    B = (B[0] + np.float32(0.5), B[1])
    exact = oracle.incexc(A, B)
    exact_aa = oracle.incexc(A, A)
    z, za = [], []
    for s in range(150):
        r = oracle.estimate(A, B, 1500, 1500, seed=1000 + s, id_a=1, id_b=2)
        z.append((r["O_ab"] - exact) / r["se_O_ab"])
        za.append((r["O_aa"] - exact_aa) / r["se_O_aa"])
    for zz in (np.array(z), np.array(za)):
        assert abs(zz.mean()) < 0.35
        assert 0.7 < zz.var() < 1.4


def test_pair_symmetries(oracle):
    A, B = (_om(oracle, m) for m in cases.config0())
    r1 = oracle.estimate(A, B, 3000, 3000, seed=5, id_a=10, id_b=20)
    r2 = oracle.estimate(B, A, 3000, 3000, seed=5, id_a=20, id_b=10)
    assert r1["T"] == r2["T"]
    assert r1["O_ab"] == r2["O_ab"]
    assert r1["O_aa"] == r2["O_bb"]
    rs = oracle.estimate(A, A, 3000, 3000, seed=5, id_a=10, id_b=10)
    assert rs["T"] == 1.0
    assert rs["O_ab"] == rs["O_aa"] == rs["O_bb"]


def test_weights_bounded(oracle):
    A, B = (_om(oracle, m) for m in cases.config0())
    pts = oracle.sample_points(*A, 0, 0, 0, 20000)
    m, u = oracle.densities(*A, pts)
    w = u / m
    assert np.all(w >= 0) and np.all(w <= 1)
    assert m.min() > np.exp(-15.0)


def test_screen_fixed_matches_estimate(oracle):
    from paper_2607_20766_amd import molgen
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(1, 40, 10, 50)
    Q = _om(oracle, q)
    la = oracle.alpha_from_radius(L.radius, cases.LAMBDA)
    out = oracle.screen(Q, 999, L.offsets, L.xyz, la, pairs=np.array([3, 17], np.int32),
                        mode=0, n_fixed=1024, seed=9)
    for row, m in zip(out, (3, 17)):
        a, b = L.offsets[m], L.offsets[m + 1]
        r = oracle.estimate(Q, (L.xyz[a:b], la[a:b]), 1024, 1024, seed=9, id_a=999, id_b=m)
        assert row[0] == r["T"] and row[1] == r["se_T"] and row[2] == r["O_ab"]
        assert row[5] == 2048


def test_screen_adaptive_stopping(oracle):
    from paper_2607_20766_amd import molgen
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(1, 24, 10, 50)
    Q = _om(oracle, q)
    la = oracle.alpha_from_radius(L.radius, cases.LAMBDA)
    tau, cap = 0.01, 8192
    out = oracle.screen(Q, 999, L.offsets, L.xyz, la, mode=1, round_per_pair=512,
                        cap_per_pair=cap, tau=tau, seed=3)
    n_used = out[:, 5]
    assert np.all(n_used % 512 == 0) and np.all(n_used >= 512) and np.all(n_used <= cap)
    assert np.all((out[:, 1] <= tau) | (n_used == cap))
    # a pair that stopped early did not meet tau one round earlier
    for p in range(len(n_used)):
        n = int(n_used[p])
        a, b = L.offsets[p], L.offsets[p + 1]
        r = oracle.estimate(Q, (L.xyz[a:b], la[a:b]), n // 2, n // 2, seed=3, id_a=999, id_b=p)
        assert r["T"] == out[p, 0] and r["se_T"] == out[p, 1]
        if n > 512:
            r0 = oracle.estimate(Q, (L.xyz[a:b], la[a:b]), n // 2 - 256, n // 2 - 256,
                                 seed=3, id_a=999, id_b=p)
            assert r0["se_T"] > tau


# --- antithetic sampling (section "Importance-sampling estimator": each draw
# paired with its reflection about its component's centre) -----------------

def test_antithetic_pairs_are_reflections(oracle):
    m = cases.small(3, 9)
    xyz, al = cases.oracle_mol(oracle, m)
    r, comp = oracle.sample_points(xyz, al, 5, 7, 0, 2000, return_component=True,
                                   antithetic=True)
    iid, comp_iid = oracle.sample_points(xyz, al, 5, 7, 0, 1000, return_component=True)
    assert np.array_equal(comp[0::2], comp[1::2])
    assert np.array_equal(comp[0::2], comp_iid)        # pair p uses Philox block p
    assert np.array_equal(r[0::2], iid)
    c = xyz.astype(np.float64)[comp[0::2]]
    assert np.allclose(r[0::2] + r[1::2], 2 * c, rtol=0, atol=1e-12)


def test_antithetic_fo_channel_unbiased(oracle):
    """Over many seeds the antithetic first-order estimate scatters about
    the closed form (Eq. fo) with no bias beyond its replicate error."""
    a, b = cases.small(4, 5), cases.small(5, 6)
    A, B = cases.oracle_mol(oracle, a), cases.oracle_mol(oracle, b)
    exact = oracle.fo_overlap(A, B)
    d = np.asarray([oracle.estimate(A, B, 400, 400, seed=seed, antithetic=True)["Ofo_ab_is"]
                    - exact for seed in range(600)])
    assert abs(d.mean()) < 4.5 * d.std(ddof=1) / np.sqrt(d.size)


def test_antithetic_union_within_se_of_grid(oracle):
    a, b = cases.config0()
    A, B = cases.oracle_mol(oracle, a), cases.oracle_mol(oracle, b)
    g = oracle.grid_integrals(A, B, h=0.2, pad=6.5)
    r = oracle.estimate(A, B, 40000, 40000, seed=3, antithetic=True)
    assert abs(r["O_ab"] - g["uAuB"]) <= 4.5 * r["se_O_ab"]
    assert abs(r["V_a"] - g["uA"]) <= 4.5 * r["se_V_a"]
    assert abs(r["O_aa"] - g["uA2"]) <= 4.5 * r["se_O_aa"]


def test_antithetic_se_calibrated_on_union(oracle):
    """z-scores of the antithetic union overlap against a long reference run
    have unit spread over seeds."""
    a, b = cases.small(6, 5), cases.small(7, 5)
    A, B = cases.oracle_mol(oracle, a), cases.oracle_mol(oracle, b)
    ref = oracle.estimate(A, B, 2000000, 2000000, seed=10**6, antithetic=True)["O_ab"]
    z = []
    for seed in range(500):
        r = oracle.estimate(A, B, 512, 512, seed=seed, antithetic=True)
        z.append((r["O_ab"] - ref) / r["se_O_ab"])
    z = np.asarray(z)
    assert abs(z.mean()) < 0.2
    assert 0.88 < z.std(ddof=1) < 1.12
