"""FP64 CPU oracle for the IS shape-overlap estimator (TEST INFRASTRUCTURE).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does.  The C source
(shape_oracle.c) follows the paper's definitions step by step; this module is
argument marshalling through ctypes and nothing else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# Eq. occ with the width convention of the synthetic workloads: a Gaussian
# height p = 2.7 in the Grant-Pickup form alpha = pi (3p/(4 pi R^3))^(2/3)
# equals the unit-height form alpha = kappa/(lambda R^2) with lambda = p^(-2/3).
LAMBDA_P27 = 2.7 ** (-2.0 / 3.0)

RESULT_FIELDS = ("O_ab", "O_aa", "O_bb", "V_a", "V_b", "T",
                 "se_O_ab", "se_O_aa", "se_O_bb", "se_V_a", "se_V_b", "se_T",
                 "se_T_full", "O_ab_from_a", "O_ab_from_b", "Ofo_ab_is",
                 "Ofo_aa_is", "Ofo_bb_is", "n_a", "n_b")

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_d = ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.or_norm_inv.argtypes = [_d]
        L.or_norm_inv.restype = _d
        L.or_alpha_from_radius.argtypes = [_f32p, _i64, _d, _f32p]
        L.or_mol_prep.argtypes = [_i, _f32p, _f32p, _f64p, _f64p, _u32p]
        L.or_sample_points.argtypes = [_i, _f32p, _f32p, _u32, _u64, _u64, _i64, _i, _f64p,
                                       _vp]
        L.or_densities.argtypes = [_i, _f32p, _f32p, _i64, _f64p, _f64p, _f64p]
        L.or_estimate.argtypes = [_i, _f32p, _f32p, _u32, _i, _f32p, _f32p, _u32,
                                  _i64, _i64, _u64, _i, _f64p]
        L.or_screen.argtypes = [_i, _f32p, _f32p, _u32, ctypes.c_int32, _i32p, _f32p, _f32p,
                                _vp, _vp,
                                ctypes.c_int32, _i, _i64, _i64, _i64, _d, _u64, _i, _vp, _i,
                                _f64p]
        L.or_fo_overlap.argtypes = [_i, _f32p, _f32p, _i, _f32p, _f32p]
        L.or_fo_overlap.restype = _d
        L.or_fo_second_moment.argtypes = [_i, _f32p, _f32p, _i, _f32p, _f32p]
        L.or_fo_second_moment.restype = _d
        L.or_incexc.argtypes = [_i, _f32p, _f32p, _i, _vp, _vp]
        L.or_incexc.restype = _d
        L.or_union_series_at.argtypes = [_i, _f32p, _f32p, _f64p]
        L.or_union_series_at.restype = _d
        L.or_grid_integrals.argtypes = [_i, _f32p, _f32p, _i, _f32p, _f32p, _d, _d, _i, _f64p]
        L.or_align_grad.argtypes = [_i, _f32p, _f32p, _u32, _i, _f32p, _f32p, _u32,
                                    _i64, _u64, ctypes.c_int32, _f64p, _f64p, _f64p, _f64p]
        L.or_align_adam.argtypes = [_i, _f32p, _f32p, _u32, _i, _f32p, _f32p, _u32,
                                    _i64, _u64, ctypes.c_int32, _f64p, ctypes.c_int32, _d,
                                    _f64p, _f64p]
        L.or_fo_align_grad.argtypes = [_i, _f32p, _f32p, _i, _f32p, _f32p, ctypes.c_int32,
                                       _f64p, _f64p, _vp]
        L.or_fo_align_adam.argtypes = [_i, _f32p, _f32p, _i, _f32p, _f32p, ctypes.c_int32,
                                       _f64p, ctypes.c_int32, _d, _f64p, _f64p]
        L.or_fo_starts.argtypes = [_i, _f32p, _f32p, _i, _f32p, _f32p, _u32, ctypes.c_int32,
                                   _u64, _f64p]
        L.or_features.argtypes = [ctypes.c_int32, _i32p, _f32p, _f32p, _f64p]
        L.or_mlp_nparams.argtypes = [_i, _i32p]
        L.or_mlp_nparams.restype = _i64
        L.or_mlp_forward.argtypes = [_i, _i32p, _f64p, ctypes.c_int32, _f64p, _f64p]
        L.or_mlp_loss_grad.argtypes = [_i, _i32p, _f64p, ctypes.c_int32, _f64p, _f64p, _f64p,
                                       _f64p, _f64p]
        L.or_adam.argtypes = [_i64, _f64p, _f64p, _f64p, _f64p, ctypes.c_int32, _d, _d, _d, _d]
        L.or_adam.restype = None
        L.or_num_threads.restype = _i
        _lib = L
    return _lib


def _mol(xyz, alpha):
    xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    alpha = np.ascontiguousarray(alpha, np.float32).reshape(-1)
    if xyz.shape[0] != alpha.shape[0]:
        raise ValueError("xyz and alpha disagree in atom count")
    return xyz, alpha


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def norm_inv(u: float) -> float:
    return lib().or_norm_inv(float(u))


def alpha_from_radius(radius, lam: float = LAMBDA_P27) -> np.ndarray:
    r = np.ascontiguousarray(radius, np.float32).reshape(-1)
    out = np.zeros_like(r)
    lib().or_alpha_from_radius(r, r.size, float(lam), out)
    return out


def mol_prep(xyz, alpha):
    xyz, alpha = _mol(xyz, alpha)
    n = alpha.size
    v = np.zeros(n)
    Z = np.zeros(1)
    thr = np.zeros(max(n - 1, 1), np.uint32)
    lib().or_mol_prep(n, xyz, alpha, v, Z, thr)
    return v, float(Z[0]), thr[: n - 1]


def sample_points(xyz, alpha, mol_id, seed, k0, n, return_component=False, antithetic=False):
    xyz, alpha = _mol(xyz, alpha)
    r = np.zeros((n, 3))
    comp = np.zeros(n, np.int32)
    lib().or_sample_points(alpha.size, xyz, alpha, mol_id, seed, k0, n, int(bool(antithetic)),
                           r, comp.ctypes.data)
    return (r, comp) if return_component else r


def densities(xyz, alpha, r):
    xyz, alpha = _mol(xyz, alpha)
    r = np.ascontiguousarray(r, np.float64).reshape(-1, 3)
    m = np.zeros(r.shape[0])
    u = np.zeros(r.shape[0])
    lib().or_densities(alpha.size, xyz, alpha, r.shape[0], r, m, u)
    return m, u


def estimate(A, B, n_a, n_b, seed=0, id_a=0, id_b=1, antithetic=False) -> dict:
    """A, B: (xyz, alpha) tuples.  Returns the FP64 result fields.
    antithetic: samples 2p, 2p+1 are a draw and its reflection; standard
    errors from the pair means."""
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    out = np.zeros(20)
    rc = lib().or_estimate(aa.size, xa, aa, id_a, ab.size, xb, ab, id_b, n_a, n_b,
                           seed, int(bool(antithetic)), out)
    if rc:
        raise RuntimeError(f"oracle estimate failed ({rc})")
    d = dict(zip(RESULT_FIELDS, out.tolist()))
    d["n_a"] = int(d["n_a"])
    d["n_b"] = int(d["n_b"])
    return d


def screen(query, id_q, lib_off, lib_xyz, lib_alpha, lib_id=None, pairs=None,
           mode=0, n_fixed=4096, round_per_pair=512, cap_per_pair=65536,
           tau=0.005, seed=0, n_threads=0, n_start=None, antithetic=False):
    """Returns [n_pairs, 6] = T, se_T, O_ab, O_aa, O_bb, n_used (pair total).
    A pair index outside the library gives NaN and n_used 0.  Raises
    ValueError for parameters the rounds cannot follow (odd or non-positive
    rounds, a cap that is not a whole number of rounds, tau <= 0)."""
    xq, aq = _mol(*query)
    off = np.ascontiguousarray(lib_off, np.int32)
    lx = np.ascontiguousarray(lib_xyz, np.float32).reshape(-1, 3)
    la = np.ascontiguousarray(lib_alpha, np.float32)
    ids = None if lib_id is None else np.ascontiguousarray(lib_id, np.uint32)
    pr = None if pairs is None else np.ascontiguousarray(pairs, np.int32)
    n_pairs = off.size - 1 if pr is None else pr.size
    ns = None if n_start is None else np.ascontiguousarray(n_start, np.int32)
    out = np.zeros((n_pairs, 6))
    rc = lib().or_screen(aq.size, xq, aq, id_q, off.size - 1, off, lx, la,
                         None if ids is None else ids.ctypes.data,
                         None if pr is None else pr.ctypes.data, n_pairs, mode,
                         n_fixed, round_per_pair, cap_per_pair, tau, seed,
                         n_threads, None if ns is None else ns.ctypes.data,
                         int(bool(antithetic)), out)
    if rc == -2:
        raise ValueError("oracle screen: parameters outside the rules of the rounds")
    if rc:
        raise RuntimeError("oracle screen failed")
    return out


def fo_overlap(A, B) -> float:
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    return lib().or_fo_overlap(aa.size, xa, aa, ab.size, xb, ab)


def fo_second_moment(A, B) -> float:
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    return lib().or_fo_second_moment(aa.size, xa, aa, ab.size, xb, ab)


def incexc(A, B=None) -> float:
    """int u_A u_B by the full inclusion-exclusion series; int u_A if B is None."""
    xa, aa = _mol(*A)
    if B is None:
        return lib().or_incexc(aa.size, xa, aa, 0, None, None)
    xb, ab = _mol(*B)
    return lib().or_incexc(aa.size, xa, aa, ab.size, xb.ctypes.data, ab.ctypes.data)


def union_series_at(A, r) -> float:
    xa, aa = _mol(*A)
    return lib().or_union_series_at(aa.size, xa, aa, np.ascontiguousarray(r, np.float64))


GRID_FIELDS = ("uAuB", "uA2", "uB2", "uA", "uB", "mAmB", "mA2", "mB2")


def grid_integrals(A, B, h=0.2, pad=6.5, n_threads=0) -> dict:
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    out = np.zeros(8)
    rc = lib().or_grid_integrals(aa.size, xa, aa, ab.size, xb, ab, h, pad, n_threads, out)
    if rc:
        raise RuntimeError("oracle grid failed")
    return dict(zip(GRID_FIELDS, out.tolist()))


def align_grad(A, B, poses, n_samples=2048, seed=0, id_a=0, id_b=1):
    """T and dT/dpose at each pose [P, 7]; also (O_aa, O_bb)."""
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    poses = np.ascontiguousarray(poses, np.float64).reshape(-1, 7)
    T = np.zeros(poses.shape[0])
    g = np.zeros((poses.shape[0], 7))
    selfo = np.zeros(2)
    rc = lib().or_align_grad(aa.size, xa, aa, id_a, ab.size, xb, ab, id_b, n_samples,
                             seed, poses.shape[0], poses, T, g, selfo)
    if rc:
        raise RuntimeError("oracle align_grad failed")
    return T, g, selfo


def align_adam(A, B, pose0, n_steps=60, lr=0.05, n_samples=2048, seed=0, id_a=0,
               id_b=1):
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    pose0 = np.ascontiguousarray(pose0, np.float64).reshape(-1, 7)
    pose = np.zeros_like(pose0)
    T = np.zeros(pose0.shape[0])
    rc = lib().or_align_adam(aa.size, xa, aa, id_a, ab.size, xb, ab, id_b, n_samples,
                             seed, pose0.shape[0], pose0, n_steps, lr, pose, T)
    if rc:
        raise RuntimeError("oracle align_adam failed")
    return pose, T



def fo_align_grad(A, B, poses):
    """First-order aligned Tanimoto T_FO and dT_FO/dpose at each pose [P, 7]
    (hybrid pipeline: the alignment objective)."""
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    poses = np.ascontiguousarray(poses, np.float64).reshape(-1, 7)
    T = np.zeros(poses.shape[0])
    g = np.zeros((poses.shape[0], 7))
    if lib().or_fo_align_grad(aa.size, xa, aa, ab.size, xb, ab, poses.shape[0], poses, T,
                              g.ctypes.data_as(ctypes.c_void_p)):
        raise RuntimeError("oracle fo_align_grad failed")
    return T, g


def fo_align_adam(A, B, pose0, n_steps=60, lr=0.05):
    """Adam on -T_FO from each start [S, 7]: final poses and T_FO there."""
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    pose0 = np.ascontiguousarray(pose0, np.float64).reshape(-1, 7)
    pose = np.zeros_like(pose0)
    T = np.zeros(pose0.shape[0])
    if lib().or_fo_align_adam(aa.size, xa, aa, ab.size, xb, ab, pose0.shape[0], pose0,
                              int(n_steps), float(lr), pose, T):
        raise RuntimeError("oracle fo_align_adam failed")
    return pose, T


def fo_starts(A, B, pair_id=0, n_random=3, seed=0):
    """Alignment starts [5 + n_random, 7]: identity, the four proper
    principal-axis alignments, random rotations about B's mean."""
    xa, aa = _mol(*A)
    xb, ab = _mol(*B)
    out = np.zeros((5 + int(n_random), 7))
    if lib().or_fo_starts(aa.size, xa, aa, ab.size, xb, ab, int(pair_id), int(n_random),
                          int(seed), out):
        raise RuntimeError("oracle fo_starts failed")
    return out

def num_threads() -> int:
    return lib().or_num_threads()


# ----------------------------------------------------------------------------
# Surrogate (learned triage): features, MLP and Adam in FP64.
# ----------------------------------------------------------------------------
FEATURES = 24


def features(offsets, xyz, alpha) -> np.ndarray:
    """[n_mols, 24] per-molecule features (see shape_oracle.c)."""
    off = np.ascontiguousarray(offsets, np.int32)
    x = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    a = np.ascontiguousarray(alpha, np.float32)
    out = np.zeros((off.size - 1, FEATURES))
    if lib().or_features(off.size - 1, off, x, a, out):
        raise RuntimeError("oracle features failed")
    return out


def mlp_nparams(width) -> int:
    w = np.ascontiguousarray(width, np.int32)
    return int(lib().or_mlp_nparams(w.size - 1, w))


def mlp_forward(width, params, x) -> np.ndarray:
    w = np.ascontiguousarray(width, np.int32)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros((x.shape[0], int(w[-1])))
    lib().or_mlp_forward(w.size - 1, w, np.ascontiguousarray(params, np.float64), x.shape[0],
                         x, y)
    return y


def mlp_loss_grad(width, params, x, target, loss_weights):
    w = np.ascontiguousarray(width, np.int32)
    x = np.ascontiguousarray(x, np.float64)
    g = np.zeros(mlp_nparams(width))
    loss = np.zeros(1)
    lib().or_mlp_loss_grad(w.size - 1, w, np.ascontiguousarray(params, np.float64), x.shape[0],
                           x, np.ascontiguousarray(target, np.float64),
                           np.ascontiguousarray(loss_weights, np.float64), loss, g)
    return float(loss[0]), g


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In place on p, m, v (float64 arrays)."""
    lib().or_adam(p.size, p, np.ascontiguousarray(g, np.float64), m, v, int(t), lr, b1, b2, eps)
