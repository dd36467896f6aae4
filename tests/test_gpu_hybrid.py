"""GPU parity of the hybrid pipeline (first-order alignment, then union
scoring) against the FP64 oracle: T_FO and its pose gradient, the alignment
starts, Adam trajectories, best start, moved coordinates, and the pipeline
end to end."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_20766_amd import molgen
from paper_2607_20766_amd.engine import LAMBDA_P27, SHAPE_SCREEN_ADAPTIVE, Engine, ShapeError
from paper_2607_20766_amd.hybrid import HybridScreen
from tests.gpu_common import compare_adaptive, oracle_mol, require_gpu

pytestmark = pytest.mark.gpu

QUERY_ID = 0xFFFFFF00


@pytest.fixture(scope="module")
def eng():
    require_gpu()
    return Engine(0)


@pytest.fixture(scope="module")
def pairs():
    A = molgen.library(61, 6, 15, 45, workers=1)
    B = molgen.library(62, 6, 15, 45, workers=1)
    return A, B


def _rot(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _poses(n_pairs, n_starts, seed=3):
    p = molgen.random_poses(seed, n_pairs, n_starts).astype(np.float32)
    p[..., 4:] *= 0.5
    return p


def test_value_and_gradient_match_oracle(eng, pairs):
    A, B = pairs
    dA, dB = eng.molecules(A), eng.molecules(B)
    poses = _poses(A.n_mols, 4)
    dp = torch.from_numpy(poses.copy()).cuda()
    print("case: T_FO and gradient, 6 pairs x 4 poses", flush=True)
    T, g = eng.shape_fo_align(dA, dB, dp, n_steps=0, need_grad=True)
    T, g = T.cpu().numpy(), g.cpu().numpy()
    assert np.array_equal(dp.cpu().numpy(), poses)   # no step: poses unchanged
    for p in range(A.n_mols):
        Tr, gr = O.fo_align_grad(oracle_mol(O, A.mol(p)), oracle_mol(O, B.mol(p)),
                                 poses[p].astype(np.float64))
        assert np.abs(T[p] - Tr).max() <= 1e-5 * np.abs(Tr).max()
        assert np.abs(g[p] - gr).max() <= 1e-4 * np.abs(gr).max(), (p, g[p], gr)


def test_starts_match_oracle(eng, pairs):
    A, B = pairs
    dA, dB = eng.molecules(A), eng.molecules(B)
    st = eng.shape_fo_starts(dA, dB, n_random=3, seed=9).cpu().numpy()
    assert st.shape == (A.n_mols, 8, 7)
    for p in range(A.n_mols):
        ref = O.fo_starts(oracle_mol(O, A.mol(p)), oracle_mol(O, B.mol(p)), pair_id=p,
                          n_random=3, seed=9)
        for s in range(8):
            assert np.abs(_rot(st[p, s, :4]) - _rot(ref[s, :4])).max() <= 1e-5, (p, s)
            assert np.abs(st[p, s, 4:] - ref[s, 4:]).max() <= 1e-4, (p, s)


def test_shared_query_broadcasts(eng, pairs):
    """A single A molecule serves every pair, as the same molecule repeated."""
    _, B = pairs
    q = molgen.molecule(1, 0, 30)
    Q = eng.molecules(q)
    Qrep = eng.molecules(molgen.MolSet.concat([q] * B.n_mols))
    dB = eng.molecules(B)
    s1 = eng.shape_fo_starts(Q, dB, n_random=2, seed=1)
    s2 = eng.shape_fo_starts(Qrep, dB, n_random=2, seed=1)
    assert torch.equal(s1, s2)
    T1, _ = eng.shape_fo_align(Q, dB, s1, n_steps=5)
    T2, _ = eng.shape_fo_align(Qrep, dB, s2, n_steps=5)
    assert torch.equal(T1, T2) and torch.equal(s1, s2)


@pytest.mark.parametrize("steps", [10, 60])
def test_adam_matches_oracle(eng, pairs, steps):
    A, B = pairs
    dA, dB = eng.molecules(A), eng.molecules(B)
    poses = _poses(A.n_mols, 3, seed=5)
    dp = torch.from_numpy(poses.copy()).cuda()
    print(f"case: first-order Adam, {steps} steps", flush=True)
    T, _ = eng.shape_fo_align(dA, dB, dp, n_steps=steps, lr=0.05)
    T, pg = T.cpu().numpy(), dp.cpu().numpy()
    for p in range(A.n_mols):
        pr, Tr = O.fo_align_adam(oracle_mol(O, A.mol(p)), oracle_mol(O, B.mol(p)),
                                 poses[p].astype(np.float64), n_steps=steps, lr=0.05)
        if steps <= 10:
            # FP32 and FP64 trajectories stay together over a few steps
            assert np.abs(pg[p] - pr).max() <= 1e-3, (p, pg[p], pr)
            assert np.abs(T[p] - Tr).max() <= 1e-4
        # and reach the same optimum value from every start
        assert np.abs(T[p].max() - Tr.max()) <= 2e-3
        assert np.all(T[p] >= O.fo_align_grad(oracle_mol(O, A.mol(p)), oracle_mol(O, B.mol(p)),
                                              poses[p].astype(np.float64))[0] - 1e-3)


def test_best_pose_and_apply_pose(eng, pairs):
    _, B = pairs
    rng = np.random.default_rng(2)
    T = rng.uniform(size=(B.n_mols, 5)).astype(np.float32)
    T[1, :] = np.nan
    T[2, 3] = np.nan
    T[3, 1] = T[3, 4] = 2.0       # tie: the lower index wins
    pose = _poses(B.n_mols, 5, seed=8)
    bp, bT = eng.shape_best_pose(torch.from_numpy(T).cuda(), torch.from_numpy(pose).cuda())
    bp, bT = bp.cpu().numpy(), bT.cpu().numpy()
    for p in range(B.n_mols):
        key = np.where(np.isnan(T[p]), -np.inf, T[p])
        b = int(np.argmax(key)) if np.isfinite(key).any() else 0
        assert np.array_equal(bp[p], pose[p, b]), p
    dB = eng.molecules(B)
    moved = eng.shape_apply_pose(dB, torch.from_numpy(pose[:, 0].copy()).cuda()).cpu().numpy()
    for p in range(B.n_mols):
        a0, a1 = B.offsets[p], B.offsets[p + 1]
        want = B.xyz[a0:a1].astype(np.float64) @ _rot(pose[p, 0, :4]).T + pose[p, 0, 4:]
        assert np.abs(moved[a0:a1] - want).max() <= 1e-5


def test_hybrid_screen_end_to_end(eng):
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(63, 77, 10, 50, workers=1)
    Q = eng.molecules(q, mol_id=[QUERY_ID])
    lib = eng.molecules(L)
    hs = HybridScreen(eng, n_random=3, n_steps=40, lr=0.05, seed=2)
    print("case: hybrid screen, 77 molecules", flush=True)
    bufs = hs.screen(Q, lib)
    out = {k: v.cpu().numpy() for k, v in bufs["out"].items()}
    # the scores are those of the union screen of the superposed library
    direct = eng.shape_screen(Q, hs.moved(lib, bufs), mode=SHAPE_SCREEN_ADAPTIVE, seed=2)
    for k in out:
        assert np.array_equal(out[k], direct[k].cpu().numpy()), k
    # alignment raised the first-order Tanimoto over the given pose for every pair
    ident = torch.zeros(L.n_mols, 1, 7, device="cuda")
    ident[:, 0, 0] = 1.0
    T0, _ = eng.shape_fo_align(Q, lib, ident, n_steps=0)
    bT = bufs["best_T_fo"].cpu().numpy()
    assert np.all(bT >= T0.cpu().numpy()[:, 0] - 1e-6)
    # and the union Tanimoto on average
    plain = eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, seed=2)["T"].cpu().numpy()
    assert out["T"].mean() > plain.mean()
    assert np.all(np.abs(out["se_T"]) <= 0.005 * (1 + 1e-6) + (out["n_used"] == 65536))


def _oracle_hybrid_poses(q, L, n_random, n_steps, lr, seed):
    """The first stage of the hybrid pipeline in the oracle: the starts of
    each pair, first-order Adam from every start, the best final start."""
    oq = oracle_mol(O, q)
    poses = np.empty((L.n_mols, 7))
    for m in range(L.n_mols):
        om = oracle_mol(O, L.mol(m))
        st = O.fo_starts(oq, om, pair_id=m, n_random=n_random, seed=seed)
        pr, Tr = O.fo_align_adam(oq, om, st, n_steps=n_steps, lr=lr)
        poses[m] = pr[int(np.argmax(Tr))]
    return poses


def test_superposed_union_scores_match_oracle(eng):
    """The union stage of the hybrid pipeline on superposed pairs: poses from
    the oracle's own first-order alignment, applied by shape_apply_pose and
    scored by the adaptive union screen on the GPU; the oracle moves the
    library itself (FP64 rotation of the same FP32 pose) and screens it.
    Parity as for any adaptive screen, at poses far from the given ones."""
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(63, 40, 10, 50, workers=1)
    tau, cap, seed = 0.005, 65536, 2
    print("case: union IS of superposed pairs (oracle alignment)", flush=True)
    poses = _oracle_hybrid_poses(q, L, 3, 40, 0.05, seed).astype(np.float32)
    Q = eng.molecules(q, mol_id=[QUERY_ID])
    lib = eng.molecules(L)
    hs = HybridScreen(eng, seed=seed)
    bufs = hs.buffers(lib)
    bufs["best_pose"].copy_(torch.from_numpy(poses))
    eng.shape_apply_pose(lib, bufs["best_pose"], out=bufs["xyz"])
    g = eng.shape_screen(Q, hs.moved(lib, bufs), mode=SHAPE_SCREEN_ADAPTIVE, tau=tau,
                         cap_per_pair=cap, seed=seed)
    g = {k: v.cpu().numpy() for k, v in g.items()}
    moved = L.xyz.astype(np.float64).copy()
    for m in range(L.n_mols):
        a0, a1 = L.offsets[m], L.offsets[m + 1]
        moved[a0:a1] = moved[a0:a1] @ _rot(poses[m, :4]).T + poses[m, 4:].astype(np.float64)
    Lm = molgen.MolSet(L.offsets, moved.astype(np.float32), L.radius, L.element)
    la = O.alpha_from_radius(L.radius, LAMBDA_P27)
    r = O.screen(oracle_mol(O, q), QUERY_ID, Lm.offsets, Lm.xyz, la, mode=1, round_per_pair=512,
                 cap_per_pair=cap, tau=tau, seed=seed)
    compare_adaptive(g, r, q, Lm, tau, cap, seed, QUERY_ID)
    # the superposition raised the union Tanimoto over the given poses
    plain = O.screen(oracle_mol(O, q), QUERY_ID, L.offsets, L.xyz, la, mode=1, tau=tau,
                     cap_per_pair=cap, seed=seed)
    assert r[:, 0].mean() > plain[:, 0].mean()


def test_invalid_molecule_gives_nan(eng, pairs):
    A, B = pairs
    Bbad = molgen.MolSet.concat([B.mol(p) for p in range(B.n_mols)])
    Bbad.xyz[Bbad.offsets[2] + 1, 0] = np.nan
    dA, dB = eng.molecules(A), eng.molecules(Bbad)
    st = eng.shape_fo_starts(dA, dB, n_random=1)
    T, _ = eng.shape_fo_align(dA, dB, st, n_steps=3)
    T = T.cpu().numpy()
    assert np.all(np.isnan(T[2])) and np.isfinite(np.delete(T, 2, axis=0)).all()
    with pytest.raises(ShapeError):
        eng.shape_check_data()
    with pytest.raises(ShapeError):
        eng.shape_fo_align(dA, eng.molecules(molgen.library(1, 3, 10, 20, workers=1)), st[:3],
                           n_steps=1)


def test_degenerate_molecules(eng):
    """1-, 2- and 3-atom molecules (isotropic or axial mixtures: the principal
    frame is not unique) and the 256-atom maximum: starts and first-order
    Adam stay finite, never end below their start, and from the given pose
    (a unique trajectory) end at the oracle's T within 1e-3.  (Looser than
    for drug-sized molecules: rotations about a symmetry axis have a zero
    gradient, whose FP32 rounding noise Adam rescales to full steps.)"""
    q = molgen.molecule(8, 0, 3)
    L = molgen.MolSet.concat([molgen.molecule(9, i, n) for i, n in enumerate((1, 2, 3, 40, 256))])
    Q = eng.molecules(q, mol_id=[QUERY_ID])
    lib = eng.molecules(L)
    print("case: degenerate molecules, first-order alignment", flush=True)
    st = eng.shape_fo_starts(Q, lib, 3, 0)
    st0 = st.cpu().numpy().copy()
    T, _ = eng.shape_fo_align(Q, lib, st, 10, 0.05)
    T, pg = T.cpu().numpy(), st.cpu().numpy()
    assert np.all(np.isfinite(st0)) and np.all(np.isfinite(T)) and np.all(np.isfinite(pg))
    oq = oracle_mol(O, q)
    for p in range(L.n_mols):
        om = oracle_mol(O, L.mol(p))
        T0 = O.fo_align_grad(oq, om, st0[p].astype(np.float64))[0]
        assert np.all(T[p] >= T0 - 1e-3), (p, T[p], T0)
        pr, Tr = O.fo_align_adam(oq, om, st0[p, :1].astype(np.float64), n_steps=10, lr=0.05)
        assert abs(T[p, 0] - Tr[0]) <= 1e-3, (p, T[p, 0], Tr[0])


def test_group_max(eng):
    rng = np.random.default_rng(4)
    T = rng.uniform(size=40).astype(np.float32)
    T[3:6] = np.nan                   # group 1 all NaN
    T[7] = np.nan
    T[10] = T[12] = 5.0               # tie in group 3: the lower entry
    off = np.array([0, 3, 6, 6, 10, 15, 40], np.int32)   # group 2 empty
    bT, bi = eng.shape_group_max(torch.from_numpy(T).cuda(), torch.from_numpy(off).cuda())
    bT, bi = bT.cpu().numpy(), bi.cpu().numpy()
    eng.shape_check_data()   # every group inside T: no data error
    for gi in range(off.size - 1):
        seg = T[off[gi]:off[gi + 1]]
        key = np.where(np.isnan(seg), -np.inf, seg)
        if seg.size == 0 or np.all(np.isnan(seg)):
            assert np.isnan(bT[gi]) and bi[gi] == -1
        else:
            j = int(np.argmax(key))
            assert bi[gi] == off[gi] + j and bT[gi] == seg[j]


def test_group_max_bounds_its_reads(eng):
    """Offsets outside T (or reversed) read nothing: NaN and -1, reported as
    a data error; the other groups are unaffected."""
    T = torch.arange(10, dtype=torch.float32, device="cuda")
    off = torch.tensor([0, 4, 12, 8, 10], dtype=torch.int32, device="cuda")
    bT, bi = eng.shape_group_max(T, off)
    bT, bi = bT.cpu().numpy(), bi.cpu().numpy()
    assert bT[0] == 3.0 and bi[0] == 3
    assert np.isnan(bT[1]) and bi[1] == -1      # runs past the end of T
    assert np.isnan(bT[2]) and bi[2] == -1      # reversed
    assert bT[3] == 9.0 and bi[3] == 9
    with pytest.raises(ShapeError):
        eng.shape_check_data()


@pytest.mark.parametrize("aligned", [False, True])
def test_ensemble_screen_takes_the_best_conformer(eng, aligned):
    from paper_2607_20766_amd.hybrid import EnsembleScreen
    C, goff = molgen.conformer_library(5, 40, 10, 40, 4, workers=1)
    q = molgen.molecule(1, 0, 30)
    Q = eng.molecules(q, mol_id=[QUERY_ID])
    lib = eng.molecules(C)
    hs = HybridScreen(eng, n_random=1, n_steps=20, seed=1) if aligned else None
    es = EnsembleScreen(eng, hybrid=hs, seed=1)
    print(f"case: conformer ensemble, aligned={aligned}", flush=True)
    bufs = es.screen(Q, lib, torch.from_numpy(goff).cuda())
    T = bufs["out"]["T"].cpu().numpy().reshape(40, 4)
    best = bufs["best_T"].cpu().numpy()
    ent = bufs["best_entry"].cpu().numpy()
    assert np.array_equal(best, T.max(1))
    assert np.array_equal(ent, np.arange(40) * 4 + T.argmax(1))
    assert np.all(best >= T[:, 0])
    if not aligned:
        # every conformer's union score against the oracle, and the maximum
        # over each molecule's conformers against the host maximum of the
        # oracle's scores (section on limitations: max over conformers)
        out = {k: v.cpu().numpy() for k, v in bufs["out"].items()}
        la = O.alpha_from_radius(C.radius, LAMBDA_P27)
        r = O.screen(oracle_mol(O, q), QUERY_ID, C.offsets, C.xyz, la, mode=1, tau=0.005,
                     cap_per_pair=65536, seed=1)
        compare_adaptive(out, r, q, C, 0.005, 65536, 1, QUERY_ID)
        Tr = r[:, 0].reshape(40, 4)
        assert np.all(np.abs(best - Tr.max(1)) <= 1e-5 * np.abs(Tr.max(1)))
        # the same conformer wins unless the oracle's top two lie within the
        # parity tolerance of each other
        top2 = np.sort(Tr, 1)[:, -2:]
        clear = top2[:, 1] - top2[:, 0] > 2e-5 * top2[:, 1]
        assert np.array_equal((ent - np.arange(40) * 4)[clear], Tr.argmax(1)[clear])


@pytest.mark.parametrize("a_atoms,b_atoms,n_starts", [((3, 16), (10, 50), 1),
                                                      ((50, 64), (10, 50), 6),
                                                      ((20, 30), (10, 50), 19),
                                                      ((3, 16), (70, 90), 8),
                                                      ((70, 80), (10, 50), 5)])
def test_every_launch_shape_matches_oracle(eng, a_atoms, b_atoms, n_starts):
    """The alignment kernel's launch shapes: one start per 16-lane row with
    A's atoms in 1 to 4 rows per lane (up to 16, 32, 48, 64 atoms), start
    counts that leave spare rows or need a second workgroup (19 = 16 + 3),
    library molecules past 64 atoms (70-90; four or more atoms per lane in
    the moves), and A past 64 atoms, which takes the one-start-per-wave
    kernel.  T_FO and the gradient at the given poses, then 5 Adam steps,
    against the oracle."""
    A = molgen.library(64, 3, *a_atoms, workers=1)
    B = molgen.library(65, 3, *b_atoms, workers=1)
    dA, dB = eng.molecules(A), eng.molecules(B)
    poses = _poses(A.n_mols, n_starts, seed=11)
    print(f"case: first-order alignment, A {a_atoms}, B {b_atoms} atoms, {n_starts} starts",
          flush=True)
    T, g = eng.shape_fo_align(dA, dB, torch.from_numpy(poses.copy()).cuda(), n_steps=0,
                              need_grad=True)
    T, g = T.cpu().numpy(), g.cpu().numpy()
    dp = torch.from_numpy(poses.copy()).cuda()
    T5, _ = eng.shape_fo_align(dA, dB, dp, n_steps=5, lr=0.05)
    T5, p5 = T5.cpu().numpy(), dp.cpu().numpy()
    for p in range(A.n_mols):
        oa, ob = oracle_mol(O, A.mol(p)), oracle_mol(O, B.mol(p))
        Tr, gr = O.fo_align_grad(oa, ob, poses[p].astype(np.float64))
        assert np.abs(T[p] - Tr).max() <= 1e-5 * np.abs(Tr).max(), (p, T[p], Tr)
        assert np.abs(g[p] - gr).max() <= 1e-4 * np.abs(gr).max(), (p, g[p], gr)
        pr, Tr5 = O.fo_align_adam(oa, ob, poses[p].astype(np.float64), n_steps=5, lr=0.05)
        assert np.abs(p5[p] - pr).max() <= 1e-3, (p, p5[p], pr)
        assert np.abs(T5[p] - Tr5).max() <= 1e-4, (p, T5[p], Tr5)


def test_long_first_order_alignment_in_launch_order_same_bits(eng):
    """At least 16 library molecules per compute unit are aligned on the
    query largest first (row layout); T, gradients and final poses equal
    those of the same molecules aligned in calls of 1,000, which keep the
    plain numbering, bit for bit."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    n = 16 * n_cu + 37
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(34, n, 1, 90, workers=4)
    Q = eng.molecules(q, mol_id=[QUERY_ID])
    lib = eng.molecules(L)
    dev = eng.torch_device
    p0 = torch.from_numpy(_poses(n, 8, seed=6)).to(dev)
    print(f"case: {n} molecules", flush=True)
    pose = p0.clone()
    T, g = eng.shape_fo_align(Q, lib, pose, 5, 0.05, need_grad=True)
    parts = []
    for a in range(0, n, 1000):
        idx = np.arange(a, min(n, a + 1000))
        sub = eng.molecules(L.subset(idx))
        pc = p0[a:a + len(idx)].clone()
        Tc, gc = eng.shape_fo_align(Q, sub, pc, 5, 0.05, need_grad=True)
        parts.append([x.cpu().numpy() for x in (Tc, gc, pc)])
    for k, full in enumerate((T, g, pose)):
        got = np.concatenate([p[k] for p in parts])
        assert np.array_equal(full.cpu().numpy(), got), k
    assert np.all(np.isfinite(T.cpu().numpy()))
