"""Thin Python binding of the C ABI in include/shape_is.h.

Argument marshalling only: torch provides device memory and the HIP stream,
every step of the computation runs in the HIP library.  The library must be
built (``python -m paper_2607_20766_amd.build``); there is no fallback.
"""
from __future__ import annotations

import contextlib
import ctypes
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshape_is.so")

SHAPE_OK = 0
SHAPE_SCREEN_FIXED = 0
SHAPE_SCREEN_ADAPTIVE = 1
SHAPE_MAX_ATOMS = 256
SHAPE_SCREEN_VARIANTS = 8
# (side-A, side-B) points per lane of each screening-kernel tile variant, in
# the library's variant order (names the kernel instance in profiles)
SCREEN_VARIANT_SHAPES = ((4, 2), (2, 2), (4, 1), (4, 4), (8, 2), (2, 1), (8, 4), (2, 4))
SHAPE_E_UNSUPPORTED = -5

# Eq. occ width convention of the synthetic workloads: a Gaussian height
# p = 2.7 in the Grant-Pickup width corresponds to lambda = p^(-2/3).
LAMBDA_P27 = 2.7 ** (-2.0 / 3.0)

ERRORS = {-1: "SHAPE_E_INVAL", -2: "SHAPE_E_RANGE", -3: "SHAPE_E_NOMEM",
          -4: "SHAPE_E_HIP", -5: "SHAPE_E_UNSUPPORTED", -6: "SHAPE_E_DATA"}


@contextlib.contextmanager
def profile_range(name: str):
    """A named roctx range (shape_range_push/pop) around a block of calls."""
    L = load_library()
    rc = L.shape_range_push(name.encode())
    if rc != SHAPE_OK:
        raise ShapeError(rc, L.shape_last_error(None).decode(errors="replace"))
    try:
        yield
    finally:
        L.shape_range_pop()


def tune_cache_file(path: str | None):
    """Back the process-wide tuning cache with a text file (read now, new
    choices appended); None detaches it."""
    L = load_library()
    rc = L.shape_tune_cache_file(None if path is None else os.fsencode(path))
    if rc != SHAPE_OK:
        raise ShapeError(rc, L.shape_last_error(None).decode(errors="replace"))


def tune_cache_clear():
    """Forget every remembered tuning choice of this process."""
    load_library().shape_tune_cache_clear()


def tune_cache_size() -> int:
    return int(load_library().shape_tune_cache_size())


class ShapeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class ShapeMols(ctypes.Structure):
    _fields_ = [("n_mols", ctypes.c_int32), ("max_atoms", ctypes.c_int32),
                ("n_atoms", ctypes.c_int64), ("atom_offset", ctypes.c_void_p),
                ("xyz", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("mol_id", ctypes.c_void_p)]


RESULT_FIELDS = ("O_ab", "O_aa", "O_bb", "V_a", "V_b", "T",
                 "se_O_ab", "se_O_aa", "se_O_bb", "se_V_a", "se_V_b", "se_T",
                 "se_T_full", "O_ab_from_a", "O_ab_from_b", "Ofo_ab_is",
                 "Ofo_aa_is", "Ofo_bb_is")


# shape_grid_integrals outputs: union overlaps, union volumes, first-order overlaps
GRID_FIELDS = ("O_ab", "O_aa", "O_bb", "V_a", "V_b", "Ofo_ab", "Ofo_aa", "Ofo_bb")


class ShapeResult(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in RESULT_FIELDS] + [
        ("n_a", ctypes.c_int64), ("n_b", ctypes.c_int64)]


class ShapeScreenParams(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("n_per_side", ctypes.c_int32),
                ("round_per_pair", ctypes.c_int32), ("cap_per_pair", ctypes.c_int32),
                ("tau", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("n_start", ctypes.c_void_p)]


class ShapeScreenOut(ctypes.Structure):
    _fields_ = [("T", ctypes.c_void_p), ("se_T", ctypes.c_void_p),
                ("O_ab", ctypes.c_void_p), ("O_aa", ctypes.c_void_p),
                ("O_bb", ctypes.c_void_p), ("n_used", ctypes.c_void_p)]


_lib = None


def load_library():
    """Load libshape_is.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2607_20766_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64, d = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_uint64, ctypes.c_double)
        L.shape_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.shape_destroy.argtypes = [vp]
        L.shape_destroy.restype = None
        L.shape_last_error.argtypes = [vp]
        L.shape_last_error.restype = ctypes.c_char_p
        L.shape_version.restype = ctypes.c_char_p
        L.shape_alpha_from_radius.argtypes = [vp, vp, i64, d, vp, vp]
        L.shape_estimate.argtypes = [vp, ctypes.POINTER(ShapeMols), ctypes.POINTER(ShapeMols),
                                     i64, i64, u64, vp, ctypes.POINTER(ShapeResult)]
        L.shape_estimate_noalloc.argtypes = [vp, ctypes.POINTER(ShapeMols),
                                             ctypes.POINTER(ShapeMols), i64, i64, u64, vp,
                                             ctypes.POINTER(ShapeResult)]
        L.shape_sample_points.argtypes = [vp, ctypes.POINTER(ShapeMols), i32, i64, i32, u64,
                                          vp, vp, vp, vp, vp]
        L.shape_screen.argtypes = [vp, ctypes.POINTER(ShapeMols), ctypes.POINTER(ShapeMols),
                                   vp, i32, ctypes.POINTER(ShapeScreenParams), vp,
                                   ctypes.POINTER(ShapeScreenOut)]
        L.shape_check_data.argtypes = [vp, vp]
        L.shape_fail_allocations.argtypes = [vp, i32]
        L.shape_range_push.argtypes = [ctypes.c_char_p]
        L.shape_range_pop.argtypes = []
        L.shape_tune_cache_file.argtypes = [ctypes.c_char_p]
        L.shape_tune_cache_clear.argtypes = []
        L.shape_tune_cache_size.argtypes = []
        L.shape_tune_cache_size.restype = i32
        L.shape_screen_tune.argtypes = [vp, ctypes.POINTER(ShapeMols),
                                        ctypes.POINTER(ShapeMols), vp, i32,
                                        ctypes.POINTER(ShapeScreenParams), vp, vp, vp]
        L.shape_prepare_cache.argtypes = [vp, ctypes.c_int]
        L.shape_set_sampling.argtypes = [vp, i32]
        L.shape_get_sampling.argtypes = [vp]
        L.shape_get_sampling.restype = i32
        L.shape_screen_set_variant.argtypes = [vp, i32]
        L.shape_screen_get_variant.argtypes = [vp]
        L.shape_screen_get_variant.restype = i32
        L.shape_graph_begin.argtypes = [vp, vp]
        L.shape_graph_end.argtypes = [vp, vp, ctypes.POINTER(vp)]
        L.shape_graph_launch.argtypes = [vp, vp, vp]
        L.shape_graph_destroy.argtypes = [vp]
        L.shape_graph_destroy.restype = None
        L.shape_memory_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                        ctypes.POINTER(i32)]
        L.shape_self_overlap.argtypes = [vp, ctypes.POINTER(ShapeMols), i32, u64, vp, vp]
        L.shape_align_grad.argtypes = [vp, ctypes.POINTER(ShapeMols), ctypes.POINTER(ShapeMols),
                                       i32, vp, vp, vp, i32, u64, vp, vp, vp]
        L.shape_adam_pose.argtypes = [vp, vp, vp, vp, vp, i64, vp, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
        L.shape_align.argtypes = [vp, ctypes.POINTER(ShapeMols), ctypes.POINTER(ShapeMols), i32,
                                  vp, i32, i32, ctypes.c_float, u64, vp, vp, vp]
        L.shape_grid_integrals.argtypes = [vp, ctypes.POINTER(ShapeMols),
                                           ctypes.POINTER(ShapeMols), d, d, vp,
                                           ctypes.POINTER(d)]
        L.shape_fo_starts.argtypes = [vp, ctypes.POINTER(ShapeMols), ctypes.POINTER(ShapeMols),
                                      i32, u64, vp, vp]
        L.shape_fo_align.argtypes = [vp, ctypes.POINTER(ShapeMols), ctypes.POINTER(ShapeMols),
                                     i32, vp, i32, ctypes.c_float, vp, vp, vp]
        L.shape_best_pose.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
        L.shape_apply_pose.argtypes = [vp, ctypes.POINTER(ShapeMols), vp, vp, vp]
        L.shape_group_max.argtypes = [vp, vp, i64, vp, i32, vp, vp, vp]
        L.shape_features.argtypes = [vp, ctypes.POINTER(ShapeMols), vp, vp]
        L.shape_pair_features.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp]
        L.shape_mlp_infer.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
        L.shape_mlp_forward.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                                        vp, vp, vp]
        L.shape_fo_overlap.argtypes = [vp, ctypes.POINTER(ShapeMols), ctypes.POINTER(ShapeMols),
                                       vp, i32, vp, vp]
        L.shape_gemm.argtypes = [vp, i32, i32, i32, vp, i64, i64, vp, i64, i64, vp, i64, vp, vp,
                                 i64, ctypes.c_uint32, vp]
        L.shape_colsum.argtypes = [vp, i32, i32, vp, i64, vp, vp]
        L.shape_mlp_backward.argtypes = [vp, i32, vp, i32, vp, vp, vp, ctypes.c_uint32, vp, vp]
        L.shape_mlp_pack.argtypes = [vp, vp, vp, vp]
        L.shape_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp,
                                           ctypes.POINTER(ShapeMlpAdam), vp, vp, vp]
        L.shape_colsum_set.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.shape_gemm_set.argtypes = [vp, i32, ctypes.POINTER(ShapeGemmDesc), vp]
        L.shape_mse.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.shape_adam.argtypes = [vp, vp, vp, vp, vp, i64, vp, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, vp]
        L.shape_topk.argtypes = [vp, vp, i32, i32, vp, vp]
        L.shape_seed_budget.argtypes = [vp, vp, i64, vp, i32, d, d, d, i32, i32, vp, vp]
        L.shape_peak_rates.argtypes = [vp, vp, ctypes.POINTER(d)]
        L.shape_timing_enable.argtypes = [vp, ctypes.c_int]
        L.shape_timing_read.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i64), ctypes.c_int]
        _lib = L
    return _lib


class ShapeGemmDesc(ctypes.Structure):
    """shape_gemm_desc: one product of shape_gemm_set."""
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("bias", ctypes.c_void_p), ("gate", ctypes.c_void_p),
                ("sam", ctypes.c_int64), ("sak", ctypes.c_int64), ("sbk", ctypes.c_int64),
                ("sbn", ctypes.c_int64), ("scm", ctypes.c_int64), ("sgm", ctypes.c_int64),
                ("M", ctypes.c_int32), ("N", ctypes.c_int32), ("K", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class ShapeMlpAdam(ctypes.Structure):
    """shape_mlp_adam: optimiser state of the fused training step."""
    _fields_ = [("params", ctypes.c_void_p), ("m", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("step", ctypes.c_void_p), ("packed", ctypes.c_void_p),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


SHAPE_MLP_PACK_BYTES = 598016
SHAPE_MLP_STEP_MAX_ROWS = 65536


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _shape_ok(t, shape):
    return t.dim() == len(shape) and all(s is None or t.shape[i] == s
                                         for i, s in enumerate(shape))


def _check_out(t, name, dtype, shape, device):
    """An output the library writes: it must already be what the kernel
    writes (no converted copy could carry the results back)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if not _shape_ok(t, shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


class _Args:
    """Input tensors of one library call on one stream: shapes and devices
    checked, dtype and layout converted on the device if needed; every
    converted copy is tied to the stream (record_stream) so that its memory
    is not reused before the queued work that reads it has run."""

    def __init__(self, eng: "Engine", stream):
        self.device = eng.torch_device
        self.stream = stream   # None: the device's current stream

    def __call__(self, t, name, dtype, shape=None, numel=None, optional=False):
        if t is None:
            if optional:
                return None
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a tensor")
        if shape is not None and not _shape_ok(t, shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, expected {self.device}")
        c = t.to(dtype).contiguous()
        if c.data_ptr() != t.data_ptr() or c.dtype != t.dtype:
            c.record_stream(self.stream if self.stream is not None
                            else torch.cuda.current_stream(self.device))
        return c

    def out(self, t, name, dtype, shape):
        return _check_out(t, name, dtype, shape, self.device)


@dataclasses.dataclass
class Molecules:
    """A molecule set resident on the device (CSR layout, see shape_mols)."""

    offsets: torch.Tensor  # int32 [n_mols + 1]
    xyz: torch.Tensor      # float32 [n_atoms, 3]
    alpha: torch.Tensor    # float32 [n_atoms]
    mol_id: torch.Tensor | None  # int32 [n_mols] (bit pattern of uint32 ids) or None
    max_atoms: int

    @property
    def n_mols(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    def validate(self, device, name="molecules"):
        """The layout the C ABI reads: int32 offsets [n_mols + 1], float32
        xyz [n_atoms, 3] and alpha [n_atoms], int32 ids [n_mols] or None,
        contiguous on `device` (values are checked by the kernels)."""
        n = self.n_mols
        if n < 1:
            raise ValueError(f"{name}: no molecules")
        if not 1 <= int(self.max_atoms) <= SHAPE_MAX_ATOMS:
            raise ValueError(f"{name}: max_atoms {self.max_atoms} outside [1, {SHAPE_MAX_ATOMS}]")
        _check_out(self.offsets, f"{name}.offsets", torch.int32, (n + 1,), device)
        _check_out(self.xyz, f"{name}.xyz", torch.float32, (None, 3), device)
        _check_out(self.alpha, f"{name}.alpha", torch.float32, (self.n_atoms,), device)
        if self.mol_id is not None:
            _check_out(self.mol_id, f"{name}.mol_id", torch.int32, (n,), device)
        return self

    def c_struct(self) -> ShapeMols:
        return ShapeMols(self.n_mols, self.max_atoms, self.n_atoms,
                         self.offsets.data_ptr(), self.xyz.data_ptr(),
                         self.alpha.data_ptr(),
                         None if self.mol_id is None else self.mol_id.data_ptr())


class Engine:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0):
        L = load_library()
        self.device = device
        self._ctx = ctypes.c_void_p()
        rc = L.shape_create(ctypes.byref(self._ctx), device)
        if rc != SHAPE_OK:
            raise ShapeError(rc, L.shape_last_error(None).decode())
        self.torch_device = torch.device("cuda", device)

    def close(self):
        if self._ctx:
            load_library().shape_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != SHAPE_OK:
            raise ShapeError(rc, load_library().shape_last_error(self._ctx).decode())

    def _mols(self, *sets):
        return [m.validate(self.torch_device, name).c_struct() for name, m in sets]

    # -- molecule upload -------------------------------------------------------
    def alpha_from_radius(self, radius: torch.Tensor, lam: float = LAMBDA_P27,
                          stream=None) -> torch.Tensor:
        radius = _Args(self, stream)(radius, "radius", torch.float32)
        alpha = torch.empty_like(radius)
        self._check(load_library().shape_alpha_from_radius(
            self._ctx, _ptr(radius), radius.numel(), float(lam), _ptr(alpha), _stream(stream)))
        return alpha

    def molecules(self, molset, lam: float = LAMBDA_P27, mol_id=None) -> Molecules:
        """Upload a host MolSet (geometry + radii); widths come from
        shape_alpha_from_radius on the device."""
        dev = self.torch_device
        off = torch.from_numpy(np.ascontiguousarray(molset.offsets, np.int32)).to(dev)
        xyz = torch.from_numpy(np.ascontiguousarray(molset.xyz, np.float32)).to(dev)
        rad = torch.from_numpy(np.ascontiguousarray(molset.radius, np.float32)).to(dev)
        alpha = self.alpha_from_radius(rad, lam)
        ids = None
        if mol_id is not None:
            ids = torch.from_numpy(
                np.ascontiguousarray(np.asarray(mol_id, np.uint32).view(np.int32))).to(dev)
        max_atoms = int(np.max(np.diff(molset.offsets))) if molset.n_mols else 1
        return Molecules(off, xyz, alpha, ids, max_atoms)

    # -- estimator ---------------------------------------------------------------
    def shape_estimate(self, A: Molecules, B: Molecules, n_a: int, n_b: int,
                       seed: int = 0, stream=None) -> dict:
        res = ShapeResult()
        a, b = self._mols(("A", A), ("B", B))
        self._check(load_library().shape_estimate(self._ctx, ctypes.byref(a), ctypes.byref(b),
                                                  int(n_a), int(n_b), int(seed),
                                                  _stream(stream), ctypes.byref(res)))
        out = {f: getattr(res, f) for f in RESULT_FIELDS}
        out["n_a"], out["n_b"] = res.n_a, res.n_b
        return out

    def shape_estimate_noalloc(self, A: Molecules, B: Molecules, n_a: int, n_b: int,
                               seed: int = 0, stream=None) -> dict:
        """shape_estimate through the allocation-free entry point (fixed
        scratch in the library; n_a, n_b <= 2^24, at most 256 atoms per set)."""
        res = ShapeResult()
        a, b = self._mols(("A", A), ("B", B))
        self._check(load_library().shape_estimate_noalloc(
            self._ctx, ctypes.byref(a), ctypes.byref(b), int(n_a), int(n_b), int(seed),
            _stream(stream), ctypes.byref(res)))
        out = {f: getattr(res, f) for f in RESULT_FIELDS}
        out["n_a"], out["n_b"] = res.n_a, res.n_b
        return out

    def shape_sample_points(self, M: Molecules, mol: int, k0: int, n: int, seed: int = 0,
                            stream=None) -> dict:
        """The GPU's sampling steps for molecule `mol` of M, samples k0..k0+n-1:
        thresholds (uint32 bit patterns in int32 [atoms]), Philox words
        [n, 4], components [n] and points [n, 3] (device tensors)."""
        (m,) = self._mols(("M", M))
        dev = self.torch_device
        na = (int(M.offsets[mol + 1].item() - M.offsets[mol].item())
              if 0 <= mol < M.n_mols else 1)
        out = {"thr": torch.empty(max(na, 1), dtype=torch.int32, device=dev),
               "words": torch.empty(max(n, 1), 4, dtype=torch.int32, device=dev),
               "comp": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
               "r": torch.empty(max(n, 1), 3, dtype=torch.float32, device=dev)}
        self._check(load_library().shape_sample_points(
            self._ctx, ctypes.byref(m), int(mol), int(k0), int(n), int(seed), _stream(stream),
            _ptr(out["thr"]), _ptr(out["words"]), _ptr(out["comp"]), _ptr(out["r"])))
        out["thr"] = out["thr"][:na]
        for k in ("words", "comp", "r"):
            out[k] = out[k][:n]
        return out

    def _screen_call(self, query, lib, pairs, n_pairs, n_start, stream):
        """Checked pair list and budgets of a screen: (pairs or None, n,
        n_start or None, molecule structs)."""
        arg = _Args(self, stream)
        q, l_ = self._mols(("query", query), ("lib", lib))
        if pairs is not None:
            pairs = arg(pairs, "pairs", torch.int32, shape=(None,))
            n = int(pairs.numel())
        else:
            n = lib.n_mols if n_pairs is None else int(n_pairs)
        n_start = arg(n_start, "n_start", torch.int32, numel=n, optional=True)
        return pairs, n, n_start, q, l_

    def shape_screen(self, query: Molecules, lib: Molecules, *, mode: int = SHAPE_SCREEN_FIXED,
                     n_per_side: int = 4096, round_per_pair: int = 512,
                     cap_per_pair: int = 65536, tau: float = 0.005, seed: int = 0,
                     pairs: torch.Tensor | None = None, n_pairs: int | None = None,
                     n_start: torch.Tensor | None = None, out: dict | None = None,
                     stream=None) -> dict:
        """Screen the query against library molecules; returns device tensors
        T, se_T, O_ab, O_aa, O_bb (float32) and n_used (int32) per pair."""
        pairs, n, n_start, q, l_ = self._screen_call(query, lib, pairs, n_pairs, n_start, stream)
        dev = self.torch_device
        if out is None:
            out = {k: torch.empty(n, dtype=torch.float32, device=dev)
                   for k in ("T", "se_T", "O_ab", "O_aa", "O_bb")}
            out["n_used"] = torch.empty(n, dtype=torch.int32, device=dev)
        for k in ("T", "se_T", "O_ab", "O_aa", "O_bb", "n_used"):
            if k in ("T", "se_T") and out.get(k) is None:
                raise ValueError(f"out[{k!r}] is required")
            _check_out(out.get(k), f"out[{k!r}]",
                       torch.int32 if k == "n_used" else torch.float32, (n,), dev)
        prm = ShapeScreenParams(mode, n_per_side, round_per_pair, cap_per_pair, tau, seed,
                                None if n_start is None else n_start.data_ptr())
        o = ShapeScreenOut(*(out[k].data_ptr() if out.get(k) is not None else None
                             for k in ("T", "se_T", "O_ab", "O_aa", "O_bb", "n_used")))
        self._check(load_library().shape_screen(self._ctx, ctypes.byref(q), ctypes.byref(l_),
                                                _ptr(pairs), n, ctypes.byref(prm),
                                                _stream(stream), ctypes.byref(o)))
        return out

    def shape_screen_tune(self, query: Molecules, lib: Molecules, *,
                          mode: int = SHAPE_SCREEN_ADAPTIVE, n_per_side: int = 4096,
                          round_per_pair: int = 512, cap_per_pair: int = 65536,
                          tau: float = 0.005, seed: int = 0, pairs: torch.Tensor | None = None,
                          n_pairs: int | None = None, n_start: torch.Tensor | None = None,
                          stream=None):
        """Time every tile variant of the screening kernel on this workload,
        keep the fastest for later screens; returns (best, [ms per variant]).
        A workload of a kind tuned before in this process (or read from the
        tuning-cache file) reuses that choice without timing: ms are -1."""
        pairs, n, n_start, q, l_ = self._screen_call(query, lib, pairs, n_pairs, n_start, stream)
        prm = ShapeScreenParams(mode, n_per_side, round_per_pair, cap_per_pair, tau, seed,
                                None if n_start is None else n_start.data_ptr())
        ms = (ctypes.c_float * SHAPE_SCREEN_VARIANTS)()
        best = ctypes.c_int32(-1)
        self._check(load_library().shape_screen_tune(
            self._ctx, ctypes.byref(q), ctypes.byref(l_), _ptr(pairs), n, ctypes.byref(prm),
            _stream(stream), ms, ctypes.byref(best)))
        return int(best.value), [float(x) for x in ms]

    def sampling(self, antithetic: bool | None = None) -> bool:
        """Select antithetic (True) or i.i.d. (False) sampling if given;
        return whether antithetic sampling is on."""
        L = load_library()
        if antithetic is not None:
            self._check(L.shape_set_sampling(self._ctx, 1 if antithetic else 0))
        return int(L.shape_get_sampling(self._ctx)) == 1

    def prepare_cache(self, enable: bool = True):
        """Reuse the preparation of an unchanged molecule set across calls
        (see shape_prepare_cache); enabling also forgets earlier ones."""
        self._check(load_library().shape_prepare_cache(self._ctx, int(enable)))

    def fail_allocations(self, n: int):
        """Make the next n scratch allocations of this context fail as out of
        memory (shape_fail_allocations; tests of error handling)."""
        self._check(load_library().shape_fail_allocations(self._ctx, int(n)))

    def screen_variant(self, variant: int | None = None) -> int:
        """Select the screening tile variant (-1 = default) if given; return
        the current one."""
        L = load_library()
        if variant is not None:
            self._check(L.shape_screen_set_variant(self._ctx, int(variant)))
        return int(L.shape_screen_get_variant(self._ctx))

    # -- graphs ----------------------------------------------------------------
    def capture(self, fn, stream=None, warmup: bool = True) -> "Graph":
        """Record the library calls that fn() makes into a HIP graph.

        fn must only issue calls of this engine (and torch kernels) on the
        current stream, reading and writing tensors allocated beforehand and
        kept alive as long as the graph: a replay reuses the captured device
        addresses.  With warmup, fn runs once uncaptured first so that the
        library's scratch is already large enough."""
        if warmup:
            fn()
        torch.cuda.synchronize(self.torch_device)
        s = stream if stream is not None else torch.cuda.Stream(self.torch_device)
        L = load_library()
        handle = ctypes.c_void_p()
        with torch.cuda.stream(s):
            self._check(L.shape_graph_begin(self._ctx, _stream(s)))
            try:
                fn()
            except BaseException:
                L.shape_graph_end(self._ctx, _stream(s), ctypes.byref(handle))
                if handle:
                    L.shape_graph_destroy(handle)
                raise
            self._check(L.shape_graph_end(self._ctx, _stream(s), ctypes.byref(handle)))
        return Graph(self, handle)

    def memory_info(self) -> dict:
        """Scratch bytes in use, retired scratch kept for live graphs, and
        the number of live graphs of this context."""
        held, retired, live = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        self._check(load_library().shape_memory_info(self._ctx, ctypes.byref(held),
                                                     ctypes.byref(retired), ctypes.byref(live)))
        return {"scratch_bytes": held.value, "retired_bytes": retired.value,
                "live_graphs": live.value}

    # -- alignment -------------------------------------------------------------
    def shape_self_overlap(self, M: Molecules, n_samples: int = 2048, seed: int = 0,
                           stream=None) -> torch.Tensor:
        (m,) = self._mols(("M", M))
        out = torch.empty(M.n_mols, dtype=torch.float32, device=self.torch_device)
        self._check(load_library().shape_self_overlap(self._ctx, ctypes.byref(m), int(n_samples),
                                                      int(seed), _stream(stream), _ptr(out)))
        return out

    def shape_align_grad(self, A: Molecules, B: Molecules, pose: torch.Tensor,
                         O_aa: torch.Tensor, O_bb: torch.Tensor, n_samples: int = 2048,
                         seed: int = 0, need_grad: bool = True, stream=None):
        """T [pairs, starts] and dT/dpose [pairs, starts, 7] (None if not needed)."""
        arg = _Args(self, stream)
        a, b = self._mols(("A", A), ("B", B))
        pairs = A.n_mols
        pose = arg(pose, "pose", torch.float32, shape=(pairs, None, 7))
        starts = pose.shape[1]
        O_aa = arg(O_aa, "O_aa", torch.float32, numel=pairs)
        O_bb = arg(O_bb, "O_bb", torch.float32, numel=pairs)
        T = torch.empty(pairs, starts, dtype=torch.float32, device=self.torch_device)
        g = (torch.empty(pairs, starts, 7, dtype=torch.float32, device=self.torch_device)
             if need_grad else None)
        self._check(load_library().shape_align_grad(
            self._ctx, ctypes.byref(a), ctypes.byref(b), starts, _ptr(pose), _ptr(O_aa),
            _ptr(O_bb), int(n_samples), int(seed), _stream(stream), _ptr(T), _ptr(g)))
        return T, g

    def shape_adam_pose(self, pose, dT, m, v, step, lr=0.05, beta1=0.9, beta2=0.999, eps=1e-8,
                        stream=None):
        arg = _Args(self, stream)
        shape = (None, 7) if pose.dim() == 2 else (None, None, 7)
        pose = arg.out(pose, "pose", torch.float32, shape)
        m = arg.out(m, "m", torch.float32, tuple(pose.shape))
        v = arg.out(v, "v", torch.float32, tuple(pose.shape))
        step = arg.out(step, "step", torch.int32, (1,))
        dT = arg(dT, "dT_dpose", torch.float32, numel=pose.numel())
        self._check(load_library().shape_adam_pose(
            self._ctx, _ptr(pose), _ptr(dT), _ptr(m), _ptr(v), pose.numel() // 7, _ptr(step),
            float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))

    def shape_align(self, A: Molecules, B: Molecules, pose: torch.Tensor, n_samples: int = 2048,
                    n_steps: int = 60, lr: float = 0.05, seed: int = 0, stream=None):
        """Multi-start Adam alignment in place on `pose` [pairs, starts, 7];
        returns (T at the final poses [pairs, starts], best start [pairs])."""
        a, b = self._mols(("A", A), ("B", B))
        pairs = A.n_mols
        _check_out(pose, "pose", torch.float32, (pairs, None, 7), self.torch_device)
        starts = pose.shape[1]
        T = torch.empty(pairs, starts, dtype=torch.float32, device=self.torch_device)
        best = torch.empty(pairs, dtype=torch.int32, device=self.torch_device)
        self._check(load_library().shape_align(
            self._ctx, ctypes.byref(a), ctypes.byref(b), starts, _ptr(pose), int(n_samples),
            int(n_steps), float(lr), int(seed), _stream(stream), _ptr(T), _ptr(best)))
        return T, best

    # -- grid reference ------------------------------------------------------------
    def shape_grid_integrals(self, A: Molecules, B: Molecules, h: float = 0.2,
                             pad: float = 6.5, stream=None) -> dict:
        """Trapezoid-rule integrals of one pair on a cubic grid (FP64)."""
        out = (ctypes.c_double * 8)()
        a, b = self._mols(("A", A), ("B", B))
        self._check(load_library().shape_grid_integrals(self._ctx, ctypes.byref(a),
                                                        ctypes.byref(b), float(h), float(pad),
                                                        _stream(stream), out))
        return dict(zip(GRID_FIELDS, list(out)))

    # -- hybrid pipeline: first-order alignment ---------------------------------
    def shape_fo_starts(self, A: Molecules, B: Molecules, n_random: int = 3, seed: int = 0,
                        out=None, stream=None) -> torch.Tensor:
        """Alignment starts [pairs, 5 + n_random, 7]: given pose, four
        principal-axis alignments, random rotations."""
        a, b = self._mols(("A", A), ("B", B))
        shape = (B.n_mols, 5 + int(n_random), 7)
        if out is None:
            out = torch.empty(*shape, dtype=torch.float32, device=self.torch_device)
        _check_out(out, "out", torch.float32, shape, self.torch_device)
        self._check(load_library().shape_fo_starts(self._ctx, ctypes.byref(a), ctypes.byref(b),
                                                   int(n_random), int(seed), _stream(stream),
                                                   _ptr(out)))
        return out

    def shape_fo_align(self, A: Molecules, B: Molecules, pose: torch.Tensor, n_steps: int = 50,
                       lr: float = 0.05, T=None, need_grad: bool = False, stream=None):
        """Adam on the first-order Tanimoto from each start; pose
        [pairs, starts, 7] is updated in place.  Returns (T [pairs, starts],
        dT/dpose at the final poses or None)."""
        a, b = self._mols(("A", A), ("B", B))
        dev = self.torch_device
        _check_out(pose, "pose", torch.float32, (B.n_mols, None, 7), dev)
        pairs, starts = pose.shape[0], pose.shape[1]
        if T is None:
            T = torch.empty(pairs, starts, dtype=torch.float32, device=dev)
        _check_out(T, "T", torch.float32, (pairs, starts), dev)
        g = (torch.empty(pairs, starts, 7, dtype=torch.float32, device=dev)
             if need_grad else None)
        self._check(load_library().shape_fo_align(self._ctx, ctypes.byref(a), ctypes.byref(b),
                                                  starts, _ptr(pose), int(n_steps), float(lr),
                                                  _stream(stream), _ptr(T), _ptr(g)))
        return T, g

    def shape_best_pose(self, T: torch.Tensor, pose: torch.Tensor, best_pose=None, best_T=None,
                        stream=None):
        arg = _Args(self, stream)
        T = arg(T, "T", torch.float32, shape=(None, None))
        pairs, starts = T.shape
        pose = arg(pose, "pose", torch.float32, shape=(pairs, starts, 7))
        if best_pose is None:
            best_pose = torch.empty(pairs, 7, dtype=torch.float32, device=self.torch_device)
        if best_T is None:
            best_T = torch.empty(pairs, dtype=torch.float32, device=self.torch_device)
        arg.out(best_pose, "best_pose", torch.float32, (pairs, 7))
        arg.out(best_T, "best_T", torch.float32, (pairs,))
        self._check(load_library().shape_best_pose(self._ctx, pairs, starts, _ptr(T), _ptr(pose),
                                                   _stream(stream), _ptr(best_pose),
                                                   _ptr(best_T)))
        return best_pose, best_T

    def shape_group_max(self, T: torch.Tensor, group_offset: torch.Tensor, best_T=None,
                        best_idx=None, stream=None):
        """Max over each group of consecutive entries (conformer ensembles):
        (best T [groups], its entry [groups]); a group reaching outside T
        gives NaN and -1 (bounded in the kernel, reported by
        shape_check_data)."""
        arg = _Args(self, stream)
        group_offset = arg(group_offset, "group_offset", torch.int32, shape=(None,))
        T = arg(T, "T", torch.float32)
        g = group_offset.numel() - 1
        if best_T is None:
            best_T = torch.empty(g, dtype=torch.float32, device=self.torch_device)
        if best_idx is None:
            best_idx = torch.empty(g, dtype=torch.int32, device=self.torch_device)
        arg.out(best_T, "best_T", torch.float32, (g,))
        arg.out(best_idx, "best_idx", torch.int32, (g,))
        self._check(load_library().shape_group_max(self._ctx, _ptr(T), T.numel(),
                                                   _ptr(group_offset), g, _stream(stream),
                                                   _ptr(best_T), _ptr(best_idx)))
        return best_T, best_idx

    def shape_apply_pose(self, M: Molecules, pose: torch.Tensor, out=None,
                         stream=None) -> torch.Tensor:
        arg = _Args(self, stream)
        (m,) = self._mols(("M", M))
        pose = arg(pose, "pose", torch.float32, shape=(M.n_mols, 7))
        if out is None:
            out = torch.empty_like(M.xyz)
        arg.out(out, "out", torch.float32, tuple(M.xyz.shape))
        self._check(load_library().shape_apply_pose(self._ctx, ctypes.byref(m), _ptr(pose),
                                                    _stream(stream), _ptr(out)))
        return out

    def shape_features(self, M: Molecules, out=None, stream=None) -> torch.Tensor:
        (m,) = self._mols(("M", M))
        if out is None:
            out = torch.empty(M.n_mols, 24, dtype=torch.float32, device=self.torch_device)
        _check_out(out, "out", torch.float32, (M.n_mols, 24), self.torch_device)
        self._check(load_library().shape_features(self._ctx, ctypes.byref(m), _stream(stream),
                                                  _ptr(out)))
        return out

    def shape_fo_overlap(self, query: Molecules, lib: Molecules, pairs=None, n_pairs=None,
                         out=None, stream=None) -> torch.Tensor:
        arg = _Args(self, stream)
        q, l_ = self._mols(("query", query), ("lib", lib))
        if pairs is not None:
            pairs = arg(pairs, "pairs", torch.int32, shape=(None,))
            n = pairs.numel()
        else:
            n = lib.n_mols if n_pairs is None else int(n_pairs)
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=self.torch_device)
        arg.out(out, "out", torch.float32, (n,))
        self._check(load_library().shape_fo_overlap(self._ctx, ctypes.byref(q), ctypes.byref(l_),
                                                    _ptr(pairs), n, _stream(stream), _ptr(out)))
        return out

    def _pair_args(self, arg, f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross, params=None):
        """Checked inputs of the pair-feature calls; returns them with n."""
        f_q = arg(f_q, "f_q", torch.float32, shape=(None, 24))
        f_lib = arg(f_lib, "f_lib", torch.float32, shape=(None, 24))
        if idx is not None:
            idx = arg(idx, "idx", torch.int32, shape=(None,))
            n = idx.numel()
        elif n is None:
            n = f_lib.shape[0]
        elif int(n) > f_lib.shape[0]:
            raise ValueError(f"n = {n} exceeds the {f_lib.shape[0]} rows of f_lib")
        n = int(n)
        qidx = arg(qidx, "qidx", torch.int32, numel=n, optional=True)
        if qidx is None and f_q.shape[0] < 1:
            raise ValueError("f_q has no row")
        fo_cross = arg(fo_cross, "fo_cross", torch.float32, numel=n, optional=True)
        mean = arg(mean, "mean", torch.float32, numel=96)
        inv_std = arg(inv_std, "inv_std", torch.float32, numel=96)
        if params is not None:
            from .surrogate import n_params
            params = arg(params, "params", torch.float32, numel=n_params())
        return f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross, params

    def shape_pair_features(self, f_q, f_lib, mean, inv_std, idx=None, qidx=None, n=None,
                            fo_cross=None, out=None, stream=None) -> torch.Tensor:
        arg = _Args(self, stream)
        f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross, _ = self._pair_args(
            arg, f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross)
        if out is None:
            out = torch.empty(n, 96, dtype=torch.float32, device=self.torch_device)
        arg.out(out, "out", torch.float32, (n, 96))
        self._check(load_library().shape_pair_features(
            self._ctx, _ptr(f_q), _ptr(f_lib), _ptr(qidx), _ptr(idx), n, _ptr(fo_cross),
            _ptr(mean), _ptr(inv_std), _stream(stream), _ptr(out)))
        return out

    def shape_mlp_infer(self, f_q, f_lib, mean, inv_std, params, idx=None, qidx=None, n=None,
                        fo_cross=None, out=None, stream=None) -> torch.Tensor:
        """Fused pair features + 96-256-256-256-2 network (BF16): [n, 2]."""
        arg = _Args(self, stream)
        f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross, params = self._pair_args(
            arg, f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross, params)
        if out is None:
            out = torch.empty(n, 2, dtype=torch.float32, device=self.torch_device)
        arg.out(out, "out", torch.float32, (n, 2))
        self._check(load_library().shape_mlp_infer(
            self._ctx, _ptr(f_q), _ptr(f_lib), _ptr(qidx), _ptr(idx), n, _ptr(fo_cross),
            _ptr(mean), _ptr(inv_std), _ptr(params), _stream(stream), _ptr(out)))
        return out

    def shape_mlp_forward(self, f_q, f_lib, mean, inv_std, params, x, h, out, idx=None,
                          qidx=None, n=None, fo_cross=None, stream=None):
        """Training forward: shape_mlp_infer's output in out [n, 2], plus the
        standardised features x [n, 96] and hidden activations h[0..2]
        [n, 256] (FP32, after ReLU) that the backward pass reads."""
        arg = _Args(self, stream)
        f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross, params = self._pair_args(
            arg, f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross, params)
        arg.out(out, "out", torch.float32, (n, 2))
        arg.out(x, "x", torch.float32, (n, 96))
        for i in range(3):
            arg.out(h[i], f"h[{i}]", torch.float32, (n, 256))
        self._check(load_library().shape_mlp_forward(
            self._ctx, _ptr(f_q), _ptr(f_lib), _ptr(qidx), _ptr(idx), n, _ptr(fo_cross),
            _ptr(mean), _ptr(inv_std), _ptr(params), _stream(stream), _ptr(x), _ptr(h[0]),
            _ptr(h[1]), _ptr(h[2]), _ptr(out)))
        return out

    def shape_mlp_pack(self, params, packed=None, stream=None):
        """The network's weights in the two bf16 layouts of the fused
        training step (shape_mlp_pack); returns packed (int16 tensor of
        SHAPE_MLP_PACK_BYTES)."""
        from .surrogate import n_params
        arg = _Args(self, stream)
        params = arg(params, "params", torch.float32, numel=n_params())
        if packed is None:
            packed = torch.empty(SHAPE_MLP_PACK_BYTES // 2, dtype=torch.int16,
                                 device=self.torch_device)
        arg.out(packed, "packed", torch.int16, (SHAPE_MLP_PACK_BYTES // 2,))
        self._check(load_library().shape_mlp_pack(self._ctx, _ptr(params), _stream(stream),
                                                  _ptr(packed)))
        return packed

    def shape_mlp_train_step(self, f_q, f_lib, mean, inv_std, target, loss_w, params, m, v,
                             step, packed, lr, beta1=0.9, beta2=0.999, eps=1e-8, idx=None,
                             qidx=None, n=None, fo_cross=None, grad=None, loss=None,
                             stream=None):
        """One fused training step of the surrogate (shape_mlp_train_step):
        params, m, v, step and packed are updated in place; returns the loss
        tensor [1] (loss if given).  grad (optional) receives dloss/dparams."""
        from .surrogate import n_params
        arg = _Args(self, stream)
        f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross, _ = self._pair_args(
            arg, f_q, f_lib, mean, inv_std, idx, qidx, n, fo_cross)
        target = arg(target, "target", torch.float32, shape=(n, 2))
        loss_w = arg(loss_w, "loss_w", torch.float32, numel=2)
        npar = n_params()
        for t, name in ((params, "params"), (m, "m"), (v, "v")):
            arg.out(t, name, torch.float32, (npar,))
        arg.out(step, "step", torch.int32, (1,))
        arg.out(packed, "packed", torch.int16, (SHAPE_MLP_PACK_BYTES // 2,))
        if grad is not None:
            arg.out(grad, "grad", torch.float32, (npar,))
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.torch_device)
        arg.out(loss, "loss", torch.float32, (1,))
        opt = ShapeMlpAdam(params.data_ptr(), m.data_ptr(), v.data_ptr(), step.data_ptr(),
                           packed.data_ptr(), float(lr), float(beta1), float(beta2), float(eps))
        self._check(load_library().shape_mlp_train_step(
            self._ctx, _ptr(f_q), _ptr(f_lib), _ptr(qidx), _ptr(idx), n, _ptr(fo_cross),
            _ptr(mean), _ptr(inv_std), _ptr(target), _ptr(loss_w), ctypes.byref(opt),
            _stream(stream), _ptr(grad), _ptr(loss)))
        return loss

    def _strided(self, t, name, rows, cols, s_row, s_col, optional=False):
        """An operand addressed by the caller's own strides from its first
        element: float32 on the engine's device, used as it is (no copy,
        which would change what the strides address), and every element
        (r s_row + c s_col) inside the memory behind the tensor."""
        if t is None:
            if optional:
                return None
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a tensor")
        if t.dtype != torch.float32:
            raise ValueError(f"{name} has dtype {t.dtype}, expected torch.float32")
        if s_row < 0 or s_col < 0:
            raise ValueError(f"{name}: negative stride")
        avail = t.untyped_storage().nbytes() // 4 - t.storage_offset()
        last = (rows - 1) * s_row + (cols - 1) * s_col
        if last >= avail:
            raise ValueError(f"{name}: element {last} lies past the {avail} elements behind it")
        if t.device != self.torch_device:
            raise ValueError(f"{name} is on {t.device}, expected {self.torch_device}")
        return t

    def _gemm_checked(self, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, bias, gate, sgm):
        M, N, K = int(M), int(N), int(K)
        A = self._strided(A, "A", M, K, int(sam), int(sak))
        B = self._strided(B, "B", K, N, int(sbk), int(sbn))
        self._strided(C, "C", M, N, int(scm), 1)
        bias = self._strided(bias, "bias", 1, N, 0, 1, optional=True)
        gate = self._strided(gate, "gate", M, N, int(sgm), 1, optional=True)
        return A, B, bias, gate

    def shape_gemm(self, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, bias=None, gate=None, sgm=0,
                   bf16=True, relu=False, stream=None):
        A, B, bias, gate = self._gemm_checked(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, bias,
                                              gate, sgm)
        flags = (1 if bf16 else 0) | (2 if relu else 0)
        self._check(load_library().shape_gemm(
            self._ctx, int(M), int(N), int(K), _ptr(A), int(sam), int(sak), _ptr(B), int(sbk),
            int(sbn), _ptr(C), int(scm), _ptr(bias), _ptr(gate), int(sgm), flags,
            _stream(stream)))

    def shape_gemm_set(self, products, stream=None):
        """Several products in one call (shape_gemm_set): products is a list
        of dicts with shape_gemm's arguments (M, N, K, A, sam, sak, B, sbk,
        sbn, C, scm and optionally bias, gate, sgm, bf16, relu)."""
        n = len(products)
        arr = (ShapeGemmDesc * n)()
        for d, p in zip(arr, products):
            A, B, bias, gate = self._gemm_checked(
                p["M"], p["N"], p["K"], p["A"], p["sam"], p["sak"], p["B"], p["sbk"],
                p["sbn"], p["C"], p["scm"], p.get("bias"), p.get("gate"), p.get("sgm", 0))
            d.A, d.B, d.C = A.data_ptr(), B.data_ptr(), p["C"].data_ptr()
            d.bias = bias.data_ptr() if bias is not None else None
            d.gate = gate.data_ptr() if gate is not None else None
            d.sam, d.sak, d.sbk, d.sbn = int(p["sam"]), int(p["sak"]), int(p["sbk"]), int(p["sbn"])
            d.scm, d.sgm = int(p["scm"]), int(p.get("sgm", 0))
            d.M, d.N, d.K = int(p["M"]), int(p["N"]), int(p["K"])
            d.flags = (1 if p.get("bf16", True) else 0) | (2 if p.get("relu", False) else 0)
        self._check(load_library().shape_gemm_set(self._ctx, n, arr, _stream(stream)))

    def shape_mlp_backward(self, width, params, acts, dout, grad, bf16=True, stream=None):
        """dloss/dparams of a dense ReLU network (shape_mlp_backward): acts
        = [inputs, hidden outputs after ReLU ...] ([batch, width[l]] each),
        dout = dloss/doutput [batch, width[-1]]; grad in params' layout."""
        arg = _Args(self, stream)
        width = [int(w) for w in width]
        L = len(width) - 1
        if len(acts) != L:
            raise ValueError(f"acts holds {len(acts)} arrays, expected {L}")
        batch = int(dout.shape[0])
        from .surrogate import n_params
        npar = n_params(width)
        params = arg(params, "params", torch.float32, numel=npar)
        arg.out(grad, "grad", torch.float32, tuple(grad.shape))
        if grad.numel() != npar:
            raise ValueError(f"grad has {grad.numel()} elements, expected {npar}")
        dout = arg(dout, "dout", torch.float32, shape=(batch, width[-1]))
        acts = [arg(a, f"acts[{l}]", torch.float32, shape=(batch, width[l]))
                for l, a in enumerate(acts)]
        w_arr = (ctypes.c_int32 * (L + 1))(*width)
        a_arr = (ctypes.c_void_p * L)(*[a.data_ptr() for a in acts])
        v = lambda a: ctypes.cast(a, ctypes.c_void_p)
        self._check(load_library().shape_mlp_backward(
            self._ctx, L, v(w_arr), batch, _ptr(params), v(a_arr), _ptr(dout),
            1 if bf16 else 0, _stream(stream), _ptr(grad)))

    def shape_colsum(self, A, M, N, lda, out, stream=None):
        arg = _Args(self, stream)
        A = self._strided(A, "A", int(M), int(N), int(lda), 1)
        arg.out(out, "out", torch.float32, (int(N),))
        self._check(load_library().shape_colsum(self._ctx, int(M), int(N), _ptr(A), int(lda),
                                                _ptr(out), _stream(stream)))

    def shape_colsum_set(self, mats, stream=None):
        """Column sums of several matrices in one launch: mats is a list of
        (A, M, N, lda, out) with device float tensors A and out."""
        arg = _Args(self, stream)
        n = len(mats)
        for A, M, N, lda, out in mats:
            self._strided(A, "A", int(M), int(N), int(lda), 1)
            arg.out(out, "out", torch.float32, (int(N),))
        Ms = (ctypes.c_int32 * n)(*[int(m[1]) for m in mats])
        Ns = (ctypes.c_int32 * n)(*[int(m[2]) for m in mats])
        ldas = (ctypes.c_int64 * n)(*[int(m[3]) for m in mats])
        As = (ctypes.c_void_p * n)(*[m[0].data_ptr() for m in mats])
        outs = (ctypes.c_void_p * n)(*[m[4].data_ptr() for m in mats])
        v = lambda a: ctypes.cast(a, ctypes.c_void_p)
        self._check(load_library().shape_colsum_set(self._ctx, n, v(Ms), v(Ns), v(As), v(ldas),
                                                    v(outs), _stream(stream)))

    def shape_mse(self, y, t, w, grad, loss, stream=None):
        arg = _Args(self, stream)
        y = arg(y, "y", torch.float32, shape=(None, None))
        B, N = y.shape
        t = arg(t, "t", torch.float32, shape=(B, N))
        w = arg(w, "w", torch.float32, numel=N)
        arg.out(grad, "grad", torch.float32, (B, N))
        arg.out(loss, "loss", torch.float32, (1,))
        self._check(load_library().shape_mse(self._ctx, int(B), int(N), _ptr(y), _ptr(t),
                                             _ptr(w), _stream(stream), _ptr(grad), _ptr(loss)))

    def shape_adam(self, p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        arg = _Args(self, stream)
        arg.out(p, "p", torch.float32, tuple(p.shape))
        arg.out(m, "m", torch.float32, tuple(p.shape))
        arg.out(v, "v", torch.float32, tuple(p.shape))
        arg.out(step, "step", torch.int32, (1,))
        g = arg(g, "g", torch.float32, numel=p.numel())
        self._check(load_library().shape_adam(self._ctx, _ptr(p), _ptr(g), _ptr(m), _ptr(v),
                                               p.numel(), _ptr(step), float(lr), float(beta1),
                                               float(beta2), float(eps), _stream(stream)))

    def shape_topk(self, score, k, out=None, stream=None) -> torch.Tensor:
        arg = _Args(self, stream)
        score = arg(score, "score", torch.float32)
        if out is None:
            out = torch.empty(int(k), dtype=torch.int32, device=self.torch_device)
        arg.out(out, "out", torch.int32, (int(k),))
        self._check(load_library().shape_topk(self._ctx, _ptr(score), score.numel(), int(k),
                                              _stream(stream), _ptr(out)))
        return out

    def shape_seed_budget(self, raw, y_mean, y_std, tau, round_per_pair, cap_per_pair, idx=None,
                          k=None, out=None, stream=None) -> torch.Tensor:
        """Sample budgets n = (exp(raw[:, 1] y_std + y_mean) / tau)^2 in whole
        rounds within [round, cap], for rows idx (device int32 [k])."""
        arg = _Args(self, stream)
        _check_out(raw, "raw", torch.float32, (None, None), self.torch_device)
        if raw.shape[1] < 2:
            raise ValueError("raw needs at least two columns")
        if idx is not None:
            idx = arg(idx, "idx", torch.int32, shape=(None,))
            k = idx.numel()
        elif k is None:
            k = raw.shape[0]
        elif int(k) > raw.shape[0]:
            raise ValueError("k exceeds the rows of raw")
        if out is None:
            out = torch.empty(int(k), dtype=torch.int32, device=self.torch_device)
        arg.out(out, "out", torch.int32, (int(k),))
        self._check(load_library().shape_seed_budget(
            self._ctx, _ptr(raw), int(raw.stride(0)), _ptr(idx), int(k), float(y_mean),
            float(y_std), float(tau), int(round_per_pair), int(cap_per_pair), _stream(stream),
            _ptr(out)))
        return out

    def peak_rates(self, stream=None) -> dict:
        """Measured issue rates: FP32 FMA (VGPR operands), v_exp_f32 and
        v_mad_u64_u32 lane operations per second, LDS bytes read per second,
        FP32 FMA lane operations per second with SGPR operands."""
        out = (ctypes.c_double * 5)()
        self._check(load_library().shape_peak_rates(self._ctx, _stream(stream), out))
        return {"fma_lane_ops_per_s": out[0], "exp_lane_ops_per_s": out[1],
                "mad_u64_u32_lane_ops_per_s": out[2], "lds_read_bytes_per_s": out[3],
                "fma_sgpr_operand_lane_ops_per_s": out[4]}

    def shape_timing_enable(self, enable: bool = True):
        self._check(load_library().shape_timing_enable(self._ctx, int(enable)))

    def shape_timing_read(self, reset: bool = True):
        """(summed dominant-kernel milliseconds, launches) since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(load_library().shape_timing_read(self._ctx, ctypes.byref(ms),
                                                     ctypes.byref(n), int(reset)))
        return ms.value, n.value

    def shape_check_data(self, stream=None):
        self._check(load_library().shape_check_data(self._ctx, _stream(stream)))


class ShapeAlignFn(torch.autograd.Function):
    """T(pose) with the library's pathwise gradient (common random numbers).

    forward(pose [pairs, starts, 7]) runs shape_align_grad once and keeps
    dT/dpose; backward multiplies it by the incoming gradient.
    """

    @staticmethod
    def forward(ctx, pose, engine, A, B, O_aa, O_bb, n_samples=2048, seed=0):
        T, g = engine.shape_align_grad(A, B, pose.detach(), O_aa, O_bb, n_samples, seed,
                                       need_grad=True)
        ctx.save_for_backward(g)
        return T

    @staticmethod
    def backward(ctx, grad_T):
        (g,) = ctx.saved_tensors
        return grad_T.unsqueeze(-1) * g, None, None, None, None, None, None, None


class Graph:
    """An executable HIP graph of engine calls (see Engine.capture)."""

    def __init__(self, eng: Engine, handle: ctypes.c_void_p):
        self._eng = eng
        self._handle = handle

    def replay(self, stream=None):
        if not self._handle:
            raise ValueError("graph is closed")
        self._eng._check(load_library().shape_graph_launch(self._eng._ctx, self._handle,
                                                           _stream(stream)))

    def close(self):
        if self._handle:
            load_library().shape_graph_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
