"""Pins of the oracle's alignment gradient (Eq. grad with common random
numbers) and its Adam optimiser: central finite differences, invariances, and
recovery of a rigidly moved copy (the paper's displaced-copy experiment on a
synthetic molecule)."""
import numpy as np
import pytest

from paper_2607_20766_amd import molgen
from tests import cases


def _pair(O, na=18, nb=22, seed=0):
    A = cases.oracle_mol(O, molgen.molecule(3, 2 * seed, na))
    B = cases.oracle_mol(O, molgen.molecule(3, 2 * seed + 1, nb))
    return A, B


def test_gradient_matches_central_differences(oracle):
    A, B = _pair(oracle)
    poses = molgen.random_poses(3, 1, 4).reshape(-1, 7).astype(np.float64)
    poses[:, 4:] *= 0.5
    T, g, _ = oracle.align_grad(A, B, poses, n_samples=512, seed=1, id_a=0, id_b=1)
    def central(p, h):
        fd = np.zeros(7)
        for i in range(7):
            e = np.zeros(7)
            e[i] = h
            Tp, _, _ = oracle.align_grad(A, B, poses[p] + e, n_samples=512, seed=1, id_a=0, id_b=1)
            Tm, _, _ = oracle.align_grad(A, B, poses[p] - e, n_samples=512, seed=1, id_a=0, id_b=1)
            fd[i] = (Tp[0] - Tm[0]) / (2 * h)
        return fd

    for p in range(poses.shape[0]):
        d1 = central(p, 1e-3)
        d2 = central(p, 5e-4)
        # h = 1e-3 central differences carry an O(h^2) error of ~1e-5 relative
        assert np.abs(g[p] - d1).max() <= 5e-5 * np.abs(g[p]).max(), (g[p], d1)
        # Richardson extrapolation removes it: O(h^4)
        rich = (4 * d2 - d1) / 3
        assert np.abs(g[p] - rich).max() <= 1e-6 * np.abs(g[p]).max(), (g[p], rich)


def test_gradient_tangent_to_quaternion_scale(oracle):
    """T depends on q only through q/|q|: T(cq) = T(q) and dT/dq . q = 0."""
    A, B = _pair(oracle)
    pose = molgen.random_poses(4, 1, 1).reshape(7).astype(np.float64)
    T1, g, _ = oracle.align_grad(A, B, pose, n_samples=256, seed=2)
    p2 = pose.copy()
    p2[:4] *= 3.0
    T2, g2, _ = oracle.align_grad(A, B, p2, n_samples=256, seed=2)
    assert T1[0] == pytest.approx(T2[0], rel=1e-13)
    assert abs(np.dot(g[0, :4], pose[:4])) <= 1e-12 * np.abs(g[0]).max()
    assert np.allclose(g2[0, :4] * 3.0, g[0, :4], rtol=1e-10, atol=1e-14)


def test_translation_covariance(oracle):
    """Moving A by s and B's translation by s leaves T unchanged."""
    A, B = _pair(oracle)
    pose = molgen.random_poses(5, 1, 1).reshape(7).astype(np.float64)
    s = np.array([0.5, -0.25, 0.125], np.float32)  # exact in binary
    T1, g1, _ = oracle.align_grad(A, B, pose, n_samples=256, seed=3)
    A2 = (A[0] + s, A[1])
    p2 = pose.copy()
    p2[4:] += s
    T2, g2, _ = oracle.align_grad(A2, B, p2, n_samples=256, seed=3)
    assert T1[0] == pytest.approx(T2[0], rel=2e-6)
    assert np.allclose(g1, g2, rtol=1e-4, atol=1e-6 * np.abs(g1).max())


def test_displaced_copy_recovered(oracle):
    """B is A rotated by a random rotation; multi-start Adam (16 uniform
    quaternions, t ~ N(0, 1), 60 steps, lr 0.05, 2048 samples) superposes it to
    T close to 1 (the paper recovers a displaced copy to T = 1.00)."""
    Am = molgen.molecule(6, 0, 15)
    A = cases.oracle_mol(oracle, Am)
    q = np.array([0.3, -0.5, 0.7, 0.4])
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    B = ((A[0].astype(np.float64) @ R).astype(np.float32), A[1].copy())  # R^T applied
    starts = molgen.random_poses(6, 1, 16).reshape(-1, 7)
    T0, _, _ = oracle.align_grad(A, B, starts.astype(np.float64), n_samples=2048,
                                 seed=0, id_a=0, id_b=1)
    pose, T = oracle.align_adam(A, B, starts, n_steps=60, lr=0.05, n_samples=2048,
                                seed=0, id_a=0, id_b=1)
    assert T.max() > 0.97
    assert T.max() > T0.max() + 0.1
