"""Pins of the oracle's surrogate parts against library routines: features
against numpy's symmetric eigensolver and the Eq. fo self-overlap; the FP64
MLP, its loss gradient and Adam against torch CPU float64 autograd and
torch.optim.Adam."""
import numpy as np
import pytest
import torch

from paper_2607_20766_amd import molgen
from tests import cases


def test_features_definition(oracle):
    L = molgen.library(21, 40, 10, 50, workers=1)
    a = oracle.alpha_from_radius(L.radius, cases.LAMBDA)
    F = oracle.features(L.offsets, L.xyz, a)
    for m in (0, 7, 39):
        s, e = L.offsets[m], L.offsets[m + 1]
        c = L.xyz[s:e].astype(np.float64)
        al = a[s:e].astype(np.float64)
        v = (np.pi / al) ** 1.5
        pi = v / v.sum()
        mu = pi @ c
        cov = (pi[:, None, None] * (c[:, :, None] * c[:, None, :]
                                    + np.eye(3)[None] / (2 * al[:, None, None]))).sum(0)
        cov -= np.outer(mu, mu)
        ev = np.sort(np.linalg.eigvalsh(cov))[::-1]
        assert np.allclose(F[m, 16:19], np.sqrt(ev), rtol=1e-12)
        d = np.linalg.norm(c - mu, axis=1)
        h = np.bincount(np.minimum((d / 0.5).astype(int), 15), minlength=16)
        assert np.array_equal(F[m, :16], h)
        # width classes are the four element types of the generator
        counts = np.bincount(np.array([3, 1, 2, 0])[L.element[s:e]], minlength=4)
        el_by_alpha = np.array([(al < 0.767).sum(), ((al >= 0.767) & (al < 0.893)).sum(),
                                ((al >= 0.893) & (al < 0.995)).sum(), (al >= 0.995).sum()])
        assert np.array_equal(F[m, 19:23], el_by_alpha)
        assert np.array_equal(np.sort(F[m, 19:23]), np.sort(counts))
        assert F[m, 23] == pytest.approx(oracle.fo_overlap((L.xyz[s:e], a[s:e]),
                                                           (L.xyz[s:e], a[s:e])), rel=1e-14)


def _torch_mlp(width, params):
    Ws, off = [], 0
    for i in range(len(width) - 1):
        n_in, n_out = width[i], width[i + 1]
        W = torch.tensor(params[off:off + n_in * n_out].reshape(n_in, n_out), requires_grad=True)
        off += n_in * n_out
        b = torch.tensor(params[off:off + n_out], requires_grad=True)
        off += n_out
        Ws.append((W, b))
    return Ws


def _torch_forward(Ws, x):
    h = x
    for i, (W, b) in enumerate(Ws):
        h = h @ W + b
        if i + 1 < len(Ws):
            h = torch.relu(h)
    return h


def test_mlp_matches_torch_autograd(oracle):
    width = [12, 16, 16, 3]
    rng = np.random.default_rng(0)
    P = oracle.mlp_nparams(width)
    params = rng.normal(size=P) * 0.3
    x = rng.normal(size=(10, 12))
    t = rng.normal(size=(10, 3))
    lw = np.array([1.0, 0.5, 2.0])
    y = oracle.mlp_forward(width, params, x)
    loss, g = oracle.mlp_loss_grad(width, params, x, t, lw)
    Ws = _torch_mlp(width, params)
    yt = _torch_forward(Ws, torch.tensor(x))
    assert np.allclose(y, yt.detach().numpy(), rtol=1e-13, atol=1e-13)
    lt = ((yt - torch.tensor(t)) ** 2 * torch.tensor(lw)).mean(0).sum()
    lt.backward()
    gt = np.concatenate([np.concatenate([W.grad.numpy().ravel(), b.grad.numpy()]) for W, b in Ws])
    assert loss == pytest.approx(lt.item(), rel=1e-13)
    assert np.allclose(g, gt, rtol=1e-12, atol=1e-14)


def test_adam_matches_torch(oracle):
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    pt = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=50)
        oracle.adam(p, g, m, v, t, 0.01)
        pt.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(p, pt.detach().numpy(), rtol=1e-13, atol=1e-15)
