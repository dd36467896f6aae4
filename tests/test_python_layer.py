"""The Python layer on the CPU, over an oracle-backed stand-in for the
engine: ShapeAlignFn (the torch.autograd.Function around shape_align_grad)
passes the engine's pathwise gradient through autograd, that gradient is the
derivative of the Function's own forward, and a torch optimiser driving poses
through it recovers a displaced rigid copy.  The stand-in has the engine's
shape_align_grad interface; the values come from the FP64 oracle."""
import numpy as np
import torch

import oracle as O
from paper_2607_20766_amd import molgen
from paper_2607_20766_amd.engine import LAMBDA_P27, ShapeAlignFn


class OracleAlignEngine:
    """shape_align_grad of the engine, computed by the oracle: A and B are
    lists of oracle molecules (xyz, alpha), one per pair."""

    def shape_align_grad(self, A, B, pose, O_aa, O_bb, n_samples=2048, seed=0,
                         need_grad=True, stream=None):
        P, S = pose.shape[0], pose.shape[1]
        T = torch.zeros(P, S, dtype=torch.float64)
        g = torch.zeros(P, S, 7, dtype=torch.float64)
        for p in range(P):
            Tp, gp, _ = O.align_grad(A[p], B[p], pose[p].numpy().astype(np.float64),
                                     n_samples=n_samples, seed=seed, id_a=2 * p, id_b=2 * p + 1)
            T[p] = torch.from_numpy(Tp)
            g[p] = torch.from_numpy(gp)
        return T, (g if need_grad else None)


def _pairs(n, seed):
    L = molgen.library(seed, 2 * n, 8, 14, workers=1)
    mols = [(L.mol(i).xyz, O.alpha_from_radius(L.mol(i).radius, LAMBDA_P27))
            for i in range(2 * n)]
    return mols[0::2], mols[1::2]


def _poses(n_pairs, n_starts, seed):
    p = molgen.random_poses(seed, n_pairs, n_starts).astype(np.float64)
    p[..., 4:] *= 0.5
    return torch.from_numpy(p)


def test_backward_is_incoming_gradient_times_pose_gradient():
    A, B = _pairs(2, 71)
    eng = OracleAlignEngine()
    pose = _poses(2, 3, 4).requires_grad_(True)
    w = torch.from_numpy(np.random.default_rng(0).normal(size=(2, 3)))
    T = ShapeAlignFn.apply(pose, eng, A, B, None, None, 512, 0)
    (w * T).sum().backward()
    _, g = eng.shape_align_grad(A, B, pose.detach(), None, None, 512, 0)
    assert torch.equal(pose.grad, w.unsqueeze(-1) * g)


def test_gradient_is_the_derivative_of_the_forward():
    """Central differences of w . T(pose + h d) through the Function (common
    random numbers: T is smooth in the pose) against <grad, d>."""
    A, B = _pairs(2, 72)
    eng = OracleAlignEngine()
    pose = _poses(2, 2, 5)
    rng = np.random.default_rng(1)
    w = torch.from_numpy(rng.normal(size=(2, 2)))
    d = torch.from_numpy(rng.normal(size=(2, 2, 7)))
    x = pose.clone().requires_grad_(True)
    (w * ShapeAlignFn.apply(x, eng, A, B, None, None, 512, 0)).sum().backward()
    h = 1e-5
    f = lambda p: float((w * ShapeAlignFn.apply(p, eng, A, B, None, None, 512, 0)).sum())
    fd = (f(pose + h * d) - f(pose - h * d)) / (2 * h)
    an = float((x.grad * d).sum())
    assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)


def test_torch_adam_through_the_function_recovers_a_displaced_copy():
    """B is A moved by a small rotation and translation; torch.optim.Adam on
    -T from the identity pose brings T close to 1."""
    L = molgen.library(73, 1, 12, 12, workers=1)
    xa = L.mol(0).xyz.astype(np.float64)
    alpha = O.alpha_from_radius(L.mol(0).radius, LAMBDA_P27)
    th = 0.25
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    xb = (xa - xa.mean(0)) @ R.T + xa.mean(0) + np.array([0.4, -0.3, 0.2])
    A, B = [(xa.astype(np.float32), alpha)], [(xb.astype(np.float32), alpha)]
    eng = OracleAlignEngine()
    pose = torch.tensor([[[1.0, 0, 0, 0, 0, 0, 0]]], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pose], lr=0.05)
    T0 = None
    for _ in range(60):
        opt.zero_grad()
        T = ShapeAlignFn.apply(pose, eng, A, B, None, None, 512, 0)
        T0 = float(T.detach()) if T0 is None else T0
        (-T.sum()).backward()
        opt.step()
    T1 = float(ShapeAlignFn.apply(pose.detach(), eng, A, B, None, None, 512, 0))
    assert T0 < 0.8 and T1 > 0.95, (T0, T1)


def test_seed_budget_rule():
    """Budgets from a predicted per-sample SE scale sigma: SE(T) = sigma / sqrt(n)
    reaches tau at n = (sigma / tau)^2, taken in whole rounds within
    [round, cap]."""
    from types import SimpleNamespace

    from paper_2607_20766_amd.surrogate import Triage

    cfg = SimpleNamespace(tau=0.005, round_per_pair=512, cap_per_pair=65536)
    need = np.array([1.0, 511.0, 512.5, 4095.0, 4097.0, 65535.0, 1e6])
    sigma = cfg.tau * np.sqrt(need)
    n = Triage.seed_budget(cfg, np.log(sigma))
    want = np.array([512, 512, 1024, 4096, 4608, 65536, 65536])
    assert np.array_equal(n, want), n
    # every budget meets the target at its own sigma, unless capped
    se = sigma / np.sqrt(n)
    assert np.all((se <= cfg.tau * (1 + 1e-12)) | (n == cfg.cap_per_pair))
