"""Resumable screening of a large library (checkpoint and resume).

A pair's samples are keyed by (seed, molecule ids, sample counter) and its
adaptive rounds depend on that pair alone (section "Confidence-bounded
screening": each pair draws rounds until its own SE(T) reaches tau or the
cap), so a screen split into chunks of pairs gives every pair the bits of
one whole-library screen.  screen_in_chunks runs the chunks in order and,
after each, writes the outputs so far and the next chunk's index to a
safetensors file; called again with the same file it continues from there.
A pair's own work is bounded by the cap (at most 65,536 samples per pair at
the default settings), so the pair is the unit of resumption.
"""
from __future__ import annotations

import os

import numpy as np
import torch

from .engine import SHAPE_SCREEN_ADAPTIVE, Engine, Molecules

KEYS = ("T", "se_T", "O_ab", "O_aa", "O_bb", "n_used")


def _params_tensor(kw: dict) -> torch.Tensor:
    """The screen's parameters, stored with the state so that a resume with
    other parameters is refused."""
    return torch.tensor([float(kw.get("mode", SHAPE_SCREEN_ADAPTIVE)),
                         float(kw.get("n_per_side", 4096)), float(kw.get("round_per_pair", 512)),
                         float(kw.get("cap_per_pair", 65536)), float(kw.get("tau", 0.005)),
                         float(kw.get("seed", 0))], dtype=torch.float64)


def screen_in_chunks(eng: Engine, query: Molecules, lib: Molecules, chunk: int,
                     state_path: str | None = None, stop_after: int | None = None,
                     **kw) -> dict | None:
    """Screen the query against every library molecule in chunks of `chunk`
    pairs (shape_screen with a pair list).  With state_path, progress is
    saved after each chunk and a previous run's state is resumed.
    stop_after: return None after that many chunks of this call (an
    interruption, for tests).  Returns host arrays of every output once the
    library is done."""
    from safetensors.torch import load_file, save_file
    n = lib.n_mols
    if chunk < 1:
        raise ValueError("chunk must be >= 1")
    params = _params_tensor(kw)
    out = {k: np.empty(n, np.int32 if k == "n_used" else np.float32) for k in KEYS}
    start = 0
    if state_path and os.path.exists(state_path):
        st = load_file(state_path)
        if int(st["n_lib"].item()) != n or int(st["chunk"].item()) != chunk or \
                not torch.equal(st["params"], params):
            raise ValueError(f"{state_path} belongs to another screen")
        start = int(st["next"].item())
        for k in KEYS:
            out[k][:start * chunk] = st[k].numpy()[:start * chunk]
    n_chunks = (n + chunk - 1) // chunk
    done = 0
    for c in range(start, n_chunks):
        if stop_after is not None and done == stop_after:
            return None
        lo, hi = c * chunk, min(n, (c + 1) * chunk)
        pairs = torch.arange(lo, hi, dtype=torch.int32, device=eng.torch_device)
        res = eng.shape_screen(query, lib, pairs=pairs, **kw)
        for k in KEYS:
            out[k][lo:hi] = res[k].cpu().numpy()
        done += 1
        if state_path:
            st = {k: torch.from_numpy(out[k].copy()) for k in KEYS}
            st.update(n_lib=torch.tensor(n), chunk=torch.tensor(chunk),
                      next=torch.tensor(c + 1), params=params)
            tmp = state_path + ".tmp"
            save_file(st, tmp)
            os.replace(tmp, state_path)
    return out
