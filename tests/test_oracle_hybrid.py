"""Pins of the oracle's hybrid pipeline (section "Differentiable alignment and
the hybrid pipeline"): the first-order aligned Tanimoto against an
independent evaluation (moved coordinates through the closed-form Eq. fo),
its pose gradient against central differences, the principal-axis starts
against numpy's eigen-decomposition, uniformity of the random starts, exact
recovery of a rigidly moved copy by a principal start, and Adam."""
import numpy as np
import pytest

from paper_2607_20766_amd import molgen
from tests import cases


def _pair(O, na=18, nb=22, seed=0):
    A = cases.oracle_mol(O, molgen.molecule(6, 2 * seed, na))
    B = cases.oracle_mol(O, molgen.molecule(6, 2 * seed + 1, nb))
    return A, B


def _rot(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _t_fo_direct(O, A, B, pose):
    """T_FO from the moved coordinates and the closed-form overlap."""
    moved = (B[0].astype(np.float64) @ _rot(pose[:4]).T + pose[4:]).astype(np.float64)
    # or_fo_overlap reads float32 coordinates: compare at float32-representable poses
    Bm = (moved.astype(np.float32), B[1])
    o_ab = O.fo_overlap(A, Bm)
    return o_ab / (O.fo_overlap(A, A) + O.fo_overlap(B, B) - o_ab), moved


def _poses(seed, n):
    p = molgen.random_poses(seed, 1, n).reshape(-1, 7).astype(np.float64)
    p[:, 4:] *= 0.5
    return p


def test_value_matches_closed_form_on_moved_coordinates(oracle):
    A, B = _pair(oracle)
    # poses whose moved coordinates are exact in float32: axis rotations by
    # quarter turns and binary translations
    poses = np.array([[1, 0, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0.5, -0.25, 1.0],
                      [0.5 ** 0.5, 0, 0.5 ** 0.5, 0, 0.125, 0, 0]])
    T, _ = oracle.fo_align_grad(A, B, poses)
    for p in range(3):
        Td, moved = _t_fo_direct(oracle, A, B, poses[p])
        if np.array_equal(moved.astype(np.float32).astype(np.float64), moved):
            assert T[p] == pytest.approx(Td, rel=1e-12)
        else:
            assert T[p] == pytest.approx(Td, rel=1e-6)


def test_gradient_matches_central_differences(oracle):
    A, B = _pair(oracle)
    poses = _poses(7, 3)
    T, g = oracle.fo_align_grad(A, B, poses)

    def central(p, h):
        fd = np.zeros(7)
        for i in range(7):
            e = np.zeros(7)
            e[i] = h
            Tp, _ = oracle.fo_align_grad(A, B, poses[p] + e)
            Tm, _ = oracle.fo_align_grad(A, B, poses[p] - e)
            fd[i] = (Tp[0] - Tm[0]) / (2 * h)
        return fd

    for p in range(poses.shape[0]):
        d1, d2 = central(p, 1e-3), central(p, 5e-4)
        rich = (4 * d2 - d1) / 3
        assert np.abs(g[p] - rich).max() <= 1e-6 * np.abs(g[p]).max(), (g[p], rich)
        # T depends on q only through q/|q|
        assert abs(np.dot(g[p, :4], poses[p, :4])) <= 1e-10 * np.abs(g[p]).max()


def _mixture_frame(M):
    xyz, alpha = M[0].astype(np.float64), M[1].astype(np.float64)
    v = (np.pi / alpha) ** 1.5
    w = v / v.sum()
    mu = w @ xyz
    d = xyz - mu
    C = (w[:, None] * d).T @ d
    ev, U = np.linalg.eigh(C)
    return mu, U[:, ::-1], ev[::-1]


def test_principal_starts_map_axes(oracle):
    A, B = _pair(oracle, 25, 30, seed=1)
    st = oracle.fo_starts(A, B, pair_id=3, n_random=0, seed=0)
    assert st.shape == (5, 7)
    assert np.array_equal(st[0], [1, 0, 0, 0, 0, 0, 0])
    muA, UA, _ = _mixture_frame(A)
    muB, UB, _ = _mixture_frame(B)
    signs = set()
    for s in range(1, 5):
        R = _rot(st[s, :4])
        assert np.linalg.norm(st[s, :4]) == pytest.approx(1.0, abs=1e-12)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)
        # each principal axis of B goes onto the same-rank axis of A (up to sign)
        proj = UA.T @ R @ UB
        assert np.allclose(np.abs(proj), np.eye(3), atol=1e-9)
        signs.add(tuple(np.sign(np.diag(proj)).astype(int)))
        # means coincide
        assert np.allclose(R @ muB + st[s, 4:], muA, atol=1e-12)
    # the four proper sign patterns, each once
    d = np.linalg.det(UA) * np.linalg.det(UB)
    assert len(signs) == 4 and all(np.isclose(np.prod(s_), d) for s_ in signs)


def test_random_starts_are_uniform_rotations(oracle):
    A, B = _pair(oracle)
    st = oracle.fo_starts(A, B, pair_id=0, n_random=3000, seed=5)[5:]
    assert np.allclose(np.linalg.norm(st[:, :4], axis=1), 1.0, atol=1e-12)
    Rs = np.stack([_rot(q) for q in st[:, :4]])
    # Haar measure on SO(3): E[R] = 0 and E[R_ij^2] = 1/3
    assert np.abs(Rs.mean(0)).max() < 0.05
    assert np.abs((Rs ** 2).mean(0) - 1 / 3).max() < 0.03
    again = oracle.fo_starts(A, B, pair_id=0, n_random=3000, seed=5)[5:]
    assert np.array_equal(st, again)
    other = oracle.fo_starts(A, B, pair_id=1, n_random=4, seed=5)[5:]
    assert not np.allclose(other, st[:4])


def test_principal_start_recovers_a_moved_copy(oracle):
    """B = A rotated and shifted: one principal start superposes it exactly
    (T_FO = 1); Adam, whose first steps have length ~lr whatever the
    gradient, stays within lr of it."""
    A, _ = _pair(oracle, 24, 10, seed=2)
    q = np.array([0.3, -0.5, 0.7, 0.2])
    R = _rot(q)
    shift = np.array([1.5, -2.0, 0.75])
    Bxyz = (A[0].astype(np.float64) @ R.T + shift).astype(np.float32)
    B = (Bxyz, A[1])
    st = oracle.fo_starts(A, B, n_random=0)
    T, _ = oracle.fo_align_grad(A, B, st)
    assert T.max() == pytest.approx(1.0, abs=1e-6)
    pose, Tf = oracle.fo_align_adam(A, B, st[[int(np.argmax(T))]], n_steps=20, lr=0.01)
    assert Tf[0] > 0.999


def test_adam_recovers_a_perturbed_copy(oracle):
    A, _ = _pair(oracle, 20, 10, seed=3)
    B = A
    # start a small rotation and shift away from the superposition
    th = 0.3
    pose0 = np.array([[np.cos(th / 2), np.sin(th / 2) * 0.6, np.sin(th / 2) * 0.8, 0.0,
                       0.6, -0.4, 0.3]])
    T0, _ = oracle.fo_align_grad(A, B, pose0)
    pose, Tf = oracle.fo_align_adam(A, B, pose0, n_steps=150, lr=0.02)
    assert T0[0] < 0.9
    assert Tf[0] > 0.999
