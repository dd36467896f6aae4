"""Shared helpers of the GPU parity tests (HIP path vs FP64 oracle)."""
import numpy as np
import pytest
import torch

import oracle as O

from paper_2607_20766_amd.engine import LAMBDA_P27


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def rel_err(got, ref, floor=0.0):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def oracle_mol(O, ms):
    return (ms.xyz, O.alpha_from_radius(ms.radius, LAMBDA_P27))


def compare_screen(g, r, idx=None, tol=1e-5, se_tol=1e-4):
    if idx is None:
        idx = np.arange(r.shape[0])
    assert np.all(rel_err(g["T"][idx], r[:, 0]) <= tol), np.max(rel_err(g["T"][idx], r[:, 0]))
    assert np.all(rel_err(g["O_ab"][idx], r[:, 2], floor=1e-3) <= tol)
    assert np.all(rel_err(g["O_aa"][idx], r[:, 3]) <= tol)
    assert np.all(rel_err(g["O_bb"][idx], r[:, 4]) <= tol)
    assert np.all(rel_err(g["se_T"][idx], r[:, 1], floor=1e-9) <= se_tol)


def compare_adaptive(g, r, q, L, tau, cap, seed, query_id, idx=None, min_same=0.9):
    """GPU adaptive screen vs oracle.screen(mode=1) on pairs idx.  Both decide
    in FP64 after the same rounds; a decision may differ only where SE(T)
    sits within FP32 rounding of tau: at the first round where the two
    differ (the smaller sample count) the oracle's SE(T) must be that close
    to tau, and the GPU's values are then compared with the oracle's fixed
    estimate at the GPU's own sample count."""
    if idx is None:
        idx = np.arange(r.shape[0])
    n_g = g["n_used"][idx].astype(np.int64)
    n_r = r[:, 5].astype(np.int64)
    same = n_g == n_r
    assert same.mean() >= min_same, same.mean()
    compare_screen(g, r[same], idx=idx[same])
    oq = oracle_mol(O, q)
    for j in np.nonzero(~same)[0]:
        m = int(idx[j])
        a0, a1 = L.offsets[m], L.offsets[m + 1]
        om = (L.xyz[a0:a1], O.alpha_from_radius(L.radius[a0:a1], LAMBDA_P27))
        n_flip = int(min(n_g[j], n_r[j]))
        at_flip = O.estimate(oq, om, n_flip // 2, n_flip // 2, seed=seed, id_a=query_id, id_b=m)
        assert abs(at_flip["se_T"] - tau) <= 1e-4 * tau, (m, n_g[j], n_r[j], at_flip["se_T"])
        ref = O.estimate(oq, om, int(n_g[j]) // 2, int(n_g[j]) // 2, seed=seed, id_a=query_id,
                         id_b=m)
        row = np.array([[ref["T"], ref["se_T"], ref["O_ab"], ref["O_aa"], ref["O_bb"],
                         n_g[j]]])
        compare_screen(g, row, idx=np.array([m]))
    assert np.all((g["se_T"][idx] <= tau * (1 + 1e-6)) | (n_g == cap))
