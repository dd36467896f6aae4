"""Hybrid screening pipeline (section "Differentiable alignment and the
hybrid pipeline"): every library molecule is rigidly aligned on the query by
the analytic first-order overlap (Eq. fo) — Adam from the given pose, the
four proper principal-axis alignments and random rotations, best start kept
— and the superposed pair is then scored by confidence-bounded union IS.

Every arithmetic step runs in the HIP library (starts, alignment, choice of
the best start, moving the coordinates, IS); this module orders the calls
and owns the buffers, so a whole screen can be captured as one graph.
"""
from __future__ import annotations

import torch

from .engine import SHAPE_SCREEN_ADAPTIVE, Engine, Molecules


class HybridScreen:
    def __init__(self, eng: Engine, n_random: int = 3, n_steps: int = 50, lr: float = 0.05,
                 seed: int = 0, tau: float = 0.005, round_per_pair: int = 512,
                 cap_per_pair: int = 65536):
        self.eng = eng
        self.n_random = n_random
        self.n_steps = n_steps
        self.lr = lr
        self.seed = seed
        self.tau = tau
        self.round_per_pair = round_per_pair
        self.cap_per_pair = cap_per_pair

    @property
    def n_starts(self) -> int:
        return 5 + self.n_random

    def buffers(self, lib: Molecules) -> dict:
        """Device buffers of one screen of `lib` (allocation-free calls)."""
        dev = self.eng.torch_device
        n = lib.n_mols
        f32 = dict(dtype=torch.float32, device=dev)
        out = {k: torch.empty(n, **f32) for k in ("T", "se_T", "O_ab", "O_aa", "O_bb")}
        out["n_used"] = torch.empty(n, dtype=torch.int32, device=dev)
        return {"pose": torch.empty(n, self.n_starts, 7, **f32),
                "T_fo": torch.empty(n, self.n_starts, **f32),
                "best_pose": torch.empty(n, 7, **f32), "best_T_fo": torch.empty(n, **f32),
                "xyz": torch.empty_like(lib.xyz), "out": out}

    def moved(self, lib: Molecules, bufs: dict) -> Molecules:
        """The library at its aligned poses (same ids, widths, layout)."""
        return Molecules(lib.offsets, bufs["xyz"], lib.alpha, lib.mol_id, lib.max_atoms)

    def screen(self, query: Molecules, lib: Molecules, bufs: dict | None = None) -> dict:
        """Align, then score.  Returns bufs: best_pose, best_T_fo (aligned
        first-order Tanimoto), xyz (moved library) and out (IS outputs of
        the superposed pairs: T, se_T, O_ab, O_aa, O_bb, n_used)."""
        e = self.eng
        if bufs is None:
            bufs = self.buffers(lib)
        e.shape_fo_starts(query, lib, self.n_random, self.seed, out=bufs["pose"])
        e.shape_fo_align(query, lib, bufs["pose"], self.n_steps, self.lr, T=bufs["T_fo"])
        e.shape_best_pose(bufs["T_fo"], bufs["pose"], best_pose=bufs["best_pose"],
                          best_T=bufs["best_T_fo"])
        e.shape_apply_pose(lib, bufs["best_pose"], out=bufs["xyz"])
        e.shape_screen(query, self.moved(lib, bufs), mode=SHAPE_SCREEN_ADAPTIVE,
                       round_per_pair=self.round_per_pair, cap_per_pair=self.cap_per_pair,
                       tau=self.tau, seed=self.seed, out=bufs["out"])
        return bufs


class EnsembleScreen:
    """Conformer ensembles (max over conformers, the paper's accuracy lever):
    every conformer of every library molecule is scored against the query —
    at its given pose, or first aligned by the hybrid pipeline — and each
    molecule keeps its best conformer (shape_group_max)."""

    def __init__(self, eng: Engine, hybrid: HybridScreen | None = None, tau: float = 0.005,
                 round_per_pair: int = 512, cap_per_pair: int = 65536, seed: int = 0):
        self.eng = eng
        self.hybrid = hybrid
        self.tau = tau
        self.round_per_pair = round_per_pair
        self.cap_per_pair = cap_per_pair
        self.seed = seed

    def buffers(self, conf_lib: Molecules, n_mols: int) -> dict:
        dev = self.eng.torch_device
        n = conf_lib.n_mols
        if self.hybrid is not None:
            b = self.hybrid.buffers(conf_lib)
        else:
            f32 = dict(dtype=torch.float32, device=dev)
            out = {k: torch.empty(n, **f32) for k in ("T", "se_T", "O_ab", "O_aa", "O_bb")}
            out["n_used"] = torch.empty(n, dtype=torch.int32, device=dev)
            b = {"out": out}
        b["best_T"] = torch.empty(n_mols, dtype=torch.float32, device=dev)
        b["best_entry"] = torch.empty(n_mols, dtype=torch.int32, device=dev)
        return b

    def screen(self, query: Molecules, conf_lib: Molecules, group_offset: torch.Tensor,
               bufs: dict | None = None) -> dict:
        """Returns bufs with best_T and best_entry per molecule and the
        per-conformer IS outputs in out."""
        n_mols = group_offset.numel() - 1
        if bufs is None:
            bufs = self.buffers(conf_lib, n_mols)
        if self.hybrid is not None:
            self.hybrid.screen(query, conf_lib, bufs)
        else:
            self.eng.shape_screen(query, conf_lib, mode=SHAPE_SCREEN_ADAPTIVE,
                                  round_per_pair=self.round_per_pair,
                                  cap_per_pair=self.cap_per_pair, tau=self.tau, seed=self.seed,
                                  out=bufs["out"])
        self.eng.shape_group_max(bufs["out"]["T"], group_offset, best_T=bufs["best_T"],
                                 best_idx=bufs["best_entry"])
        return bufs
