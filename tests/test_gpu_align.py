"""GPU parity of the alignment path (shape_self_overlap, shape_align_grad,
shape_adam_pose / shape_align) against the FP64 oracle: values 1e-5, gradients
1e-4 of the pose's largest component, central differences 2e-3, final Adam T
1e-3 absolute; displaced-copy recovery."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_20766_amd import molgen
from paper_2607_20766_amd.engine import Engine, LAMBDA_P27, ShapeAlignFn
from tests.gpu_common import oracle_mol, rel_err, require_gpu

pytestmark = pytest.mark.gpu
NS = 2048


@pytest.fixture(scope="module")
def eng():
    require_gpu()
    return Engine(0)


def _pairs(n_pairs, seed=3):
    rng = np.random.default_rng(seed)
    A, B = [], []
    for p in range(n_pairs):
        A.append(molgen.molecule(seed, 2 * p, int(rng.integers(15, 46))))
        B.append(molgen.molecule(seed, 2 * p + 1, int(rng.integers(15, 46))))
    return molgen.MolSet.concat(A), molgen.MolSet.concat(B)


def _gpu_sets(eng, A, B):
    ida = np.arange(A.n_mols, dtype=np.uint32) * 2
    idb = ida + 1
    return eng.molecules(A, mol_id=ida), eng.molecules(B, mol_id=idb), ida, idb


def test_align_grad_matches_oracle(eng):
    n_pairs, n_starts = 12, 4
    A, B = _pairs(n_pairs)
    gA, gB, ida, idb = _gpu_sets(eng, A, B)
    poses = molgen.random_poses(3, n_pairs, n_starts)
    poses[..., 4:] *= 0.5
    pose = torch.from_numpy(poses).cuda()
    Oaa = eng.shape_self_overlap(gA, NS, seed=0)
    Obb = eng.shape_self_overlap(gB, NS, seed=0)
    T, g = eng.shape_align_grad(gA, gB, pose, Oaa, Obb, NS, seed=0)
    T, g, Oaa, Obb = (x.cpu().numpy() for x in (T, g, Oaa, Obb))
    for p in range(n_pairs):
        print(f"case: pair {p}", flush=True)
        Ap, Bp = A.mol(p), B.mol(p)
        Tr, gr, selfo = O.align_grad(oracle_mol(O, Ap), oracle_mol(O, Bp),
                                     poses[p].astype(np.float64), n_samples=NS, seed=0,
                                     id_a=int(ida[p]), id_b=int(idb[p]))
        assert rel_err(Oaa[p], selfo[0]) <= 1e-5 and rel_err(Obb[p], selfo[1]) <= 1e-5
        assert np.all(rel_err(T[p], Tr, floor=1e-4) <= 1e-5), (T[p], Tr)
        for s in range(n_starts):
            scale = np.abs(gr[s]).max()
            assert np.abs(g[p, s] - gr[s]).max() <= 1e-4 * scale + 1e-7, (g[p, s], gr[s])


def test_align_grad_central_differences(eng):
    A, B = _pairs(4, seed=5)
    gA, gB, _, _ = _gpu_sets(eng, A, B)
    poses = molgen.random_poses(5, 4, 2)
    poses[..., 4:] *= 0.5
    pose = torch.from_numpy(poses).cuda()
    Oaa = eng.shape_self_overlap(gA, NS)
    Obb = eng.shape_self_overlap(gB, NS)
    _, g = eng.shape_align_grad(gA, gB, pose, Oaa, Obb, NS)
    g = g.cpu().numpy()
    h = 1e-3
    fd = np.zeros_like(g)
    for c in range(7):
        e = torch.zeros_like(pose)
        e[..., c] = h
        Tp, _ = eng.shape_align_grad(gA, gB, pose + e, Oaa, Obb, NS, need_grad=False)
        Tm, _ = eng.shape_align_grad(gA, gB, pose - e, Oaa, Obb, NS, need_grad=False)
        fd[..., c] = ((Tp.double() - Tm.double()) / (2 * h)).cpu().numpy()
    scale = np.abs(g).max(axis=-1, keepdims=True)
    assert np.all(np.abs(g - fd) <= 2e-3 * scale + 2e-5), np.abs(g - fd).max()


def test_autograd_function(eng):
    A, B = _pairs(3, seed=7)
    gA, gB, _, _ = _gpu_sets(eng, A, B)
    pose = torch.from_numpy(molgen.random_poses(7, 3, 5)).cuda().requires_grad_(True)
    Oaa = eng.shape_self_overlap(gA, NS)
    Obb = eng.shape_self_overlap(gB, NS)
    T = ShapeAlignFn.apply(pose, eng, gA, gB, Oaa, Obb, NS, 0)
    w = torch.arange(15, dtype=torch.float32, device="cuda").reshape(3, 5)
    (T * w).sum().backward()
    _, g = eng.shape_align_grad(gA, gB, pose.detach(), Oaa, Obb, NS)
    assert torch.allclose(pose.grad, w.unsqueeze(-1) * g)


def test_adam_matches_oracle(eng):
    n_pairs, n_starts, steps = 3, 4, 60
    A, B = _pairs(n_pairs, seed=9)
    gA, gB, ida, idb = _gpu_sets(eng, A, B)
    poses = molgen.random_poses(9, n_pairs, n_starts)
    pose = torch.from_numpy(poses.copy()).cuda()
    T, best = eng.shape_align(gA, gB, pose, n_samples=NS, n_steps=steps, lr=0.05, seed=0)
    T = T.cpu().numpy()
    best = best.cpu().numpy()
    for p in range(n_pairs):
        print(f"case: adam pair {p}", flush=True)
        _, Tr = O.align_adam(oracle_mol(O, A.mol(p)), oracle_mol(O, B.mol(p)), poses[p],
                             n_steps=steps, lr=0.05, n_samples=NS, seed=0,
                             id_a=int(ida[p]), id_b=int(idb[p]))
        assert np.all(np.abs(T[p] - Tr) <= 1e-3), (T[p], Tr)
        assert best[p] == int(np.argmax(T[p]))


def test_fused_optimisation_equals_step_by_step(eng):
    """shape_align runs all Adam steps inside one launch; the same steps as
    shape_align_grad + shape_adam_pose in turn give the same bits."""
    n_pairs, n_starts, steps = 5, 6, 12
    A, B = _pairs(n_pairs, seed=13)
    gA, gB, _, _ = _gpu_sets(eng, A, B)
    poses = molgen.random_poses(13, n_pairs, n_starts)
    fused = torch.from_numpy(poses.copy()).cuda()
    print("case: fused alignment vs step by step", flush=True)
    T_f, best = eng.shape_align(gA, gB, fused, n_samples=NS, n_steps=steps, lr=0.05, seed=2)
    pose = torch.from_numpy(poses.copy()).cuda()
    Oaa = eng.shape_self_overlap(gA, NS, seed=2)
    Obb = eng.shape_self_overlap(gB, NS, seed=2)
    m, v = torch.zeros_like(pose), torch.zeros_like(pose)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(steps):
        _, g = eng.shape_align_grad(gA, gB, pose, Oaa, Obb, NS, seed=2)
        eng.shape_adam_pose(pose, g, m, v, step, lr=0.05)
    T_s, _ = eng.shape_align_grad(gA, gB, pose, Oaa, Obb, NS, seed=2, need_grad=False)
    torch.cuda.synchronize()
    assert torch.equal(fused, pose)
    assert torch.equal(T_f, T_s)
    assert torch.equal(best.long(), T_s.argmax(dim=1))


def test_displaced_copy_recovered(eng):
    """B = A under a random rotation; 16 starts, 60 Adam steps: best T ~ 1
    (the molecule of the oracle's displaced-copy pin)."""
    a = molgen.molecule(6, 0, 15)
    q = np.array([0.3, -0.5, 0.7, 0.4])
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    b = molgen.MolSet(a.offsets.copy(), (a.xyz.astype(np.float64) @ R).astype(np.float32),
                      a.radius.copy(), a.element.copy())
    gA = eng.molecules(a, mol_id=[0])
    gB = eng.molecules(b, mol_id=[1])
    pose = torch.from_numpy(molgen.random_poses(6, 1, 16)).cuda()
    Oaa = eng.shape_self_overlap(gA, NS)
    Obb = eng.shape_self_overlap(gB, NS)
    T0, _ = eng.shape_align_grad(gA, gB, pose, Oaa, Obb, NS, need_grad=False)
    T, best = eng.shape_align(gA, gB, pose, n_samples=NS, n_steps=60, lr=0.05)
    assert float(T.max()) > 0.97
    assert float(T.max()) > float(T0.max()) + 0.1


def test_long_alignments_in_launch_order_same_bits(eng):
    """At least 4 pairs per compute unit are aligned largest pair first (the
    order comes from the atom counts); T, gradients, final poses and best
    starts equal those of the same pairs aligned in calls of 500, which keep
    the plain order, bit for bit (shape_align_grad and shape_align)."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    n = 4 * n_cu + 37
    A = molgen.library(32, n, 5, 60, workers=4)
    B = molgen.library(33, n, 1, 70, workers=4)
    ida = np.arange(n, dtype=np.uint32) * 2
    gA, gB = eng.molecules(A, mol_id=ida), eng.molecules(B, mol_id=ida + 1)
    dev = eng.torch_device
    poses = torch.from_numpy(molgen.random_poses(5, n, 3)).to(dev)
    saa, sbb = eng.shape_self_overlap(gA, 256), eng.shape_self_overlap(gB, 256)
    print(f"case: {n} pairs", flush=True)
    T, g = eng.shape_align_grad(gA, gB, poses, saa, sbb, 256)
    pose_f = poses.clone()
    Tf, best = eng.shape_align(gA, gB, pose_f, n_samples=256, n_steps=3, lr=0.05)
    parts = []
    for a in range(0, n, 500):
        idx = np.arange(a, min(n, a + 500))
        cA = eng.molecules(A.subset(idx), mol_id=ida[idx])
        cB = eng.molecules(B.subset(idx), mol_id=ida[idx] + 1)
        sl = slice(a, a + len(idx))
        Tc, gc = eng.shape_align_grad(cA, cB, poses[sl].contiguous(), saa[sl].contiguous(),
                                      sbb[sl].contiguous(), 256)
        pc = poses[sl].clone()
        Tfc, bc = eng.shape_align(cA, cB, pc, n_samples=256, n_steps=3, lr=0.05)
        parts.append([x.cpu().numpy() for x in (Tc, gc, pc, Tfc, bc)])
    for k, full in enumerate((T, g, pose_f, Tf, best)):
        got = np.concatenate([p[k] for p in parts])
        assert np.array_equal(full.cpu().numpy(), got), k
    assert np.all(np.isfinite(T.cpu().numpy()))
