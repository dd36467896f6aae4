"""Learned triage for confidence-bounded screening.

A small MLP (96 -> 256 -> 256 -> 256 -> 2, ReLU, BF16 operands with FP32
accumulation on the matrix cores) predicts, from cheap pair features, the
shape Tanimoto of a (query, library) pair and the per-sample scale of its
standard error, log(SE(T) sqrt(n)).  Trained on labels produced by the IS
screening kernel itself, it ranks a library so that confidence-bounded IS
refines only the head of the ranking, with per-pair sample budgets seeded
from the predicted scale (n = (sigma / tau)^2).  IS is both the fallback and
the arbiter: every reported Tanimoto comes from IS.

Every arithmetic step runs in the HIP library (features, pair features,
dense layers, loss, Adam, top-k, IS); this module orders the calls.  Small
host-side steps are bookkeeping on at most a few MB (feature statistics from
a subsample, label transforms, budget rounding).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .engine import (SHAPE_MLP_STEP_MAX_ROWS, SHAPE_SCREEN_ADAPTIVE, Engine, Molecules,
                     profile_range)

WIDTH = (96, 256, 256, 256, 2)


def n_params(width=WIDTH) -> int:
    return sum(width[i] * width[i + 1] + width[i + 1] for i in range(len(width) - 1))


def init_params(seed: int, width=WIDTH) -> np.ndarray:
    """He-uniform weights, zero biases, packed W_0, b_0, W_1, b_1, ... with
    W_l row-major [in][out] (random numbers drawn on the host and passed in)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 0x31C])))
    parts = []
    for i in range(len(width) - 1):
        bound = math.sqrt(6.0 / width[i])
        parts.append(rng.uniform(-bound, bound, size=width[i] * width[i + 1]))
        parts.append(np.zeros(width[i + 1]))
    return np.concatenate(parts).astype(np.float32)


class MLP:
    """Dense ReLU network whose forward, backward, loss and Adam run in the
    library's kernels (shape_gemm, shape_colsum, shape_mse, shape_adam)."""

    def __init__(self, eng: Engine, params: np.ndarray, width=WIDTH, bf16: bool = True):
        self.eng = eng
        self.width = tuple(width)
        self.bf16 = bf16
        dev = eng.torch_device
        self.params = torch.from_numpy(np.ascontiguousarray(params, np.float32)).to(dev)
        assert self.params.numel() == n_params(width)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.packed = None   # bf16 packings of the weights for the fused training step
        self._acts = {}

    def _views(self, flat):
        out, off = [], 0
        for i in range(len(self.width) - 1):
            n_in, n_out = self.width[i], self.width[i + 1]
            W = flat[off:off + n_in * n_out]
            off += n_in * n_out
            b = flat[off:off + n_out]
            off += n_out
            out.append((W, b))
        return out

    def _buffers(self, B):
        if B not in self._acts:
            dev = self.eng.torch_device
            self._acts[B] = {
                "h": [torch.empty(B, w, dtype=torch.float32, device=dev) for w in self.width[1:]],
                "dout": torch.empty(B, self.width[-1], dtype=torch.float32, device=dev),
                "loss": torch.empty(1, dtype=torch.float32, device=dev),
            }
        return self._acts[B]

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x: [B, width[0]] float32 on the device -> [B, width[-1]]."""
        B = x.shape[0]
        buf = self._buffers(B)
        h = x
        L = len(self.width) - 1
        for l, (W, b) in enumerate(self._views(self.params)):
            n_in, n_out = self.width[l], self.width[l + 1]
            out = buf["h"][l]
            self.eng.shape_gemm(B, n_out, n_in, h, n_in, 1, W, n_out, 1, out, n_out, bias=b,
                                bf16=self.bf16, relu=(l + 1 < L))
            h = out
        return h

    def backward(self, x: torch.Tensor, dout: torch.Tensor):
        """Gradient of the loss w.r.t. the parameters into self.grad, given
        d loss / d output (the activations of the last forward are reused):
        one shape_mlp_backward call."""
        buf = self._buffers(x.shape[0])
        acts = [x] + buf["h"][:-1]
        self.eng.shape_mlp_backward(self.width, self.params, acts, dout, self.grad,
                                    bf16=self.bf16)

    def loss_grad(self, x, target, loss_weights, loss_out=None):
        """Forward, weighted MSE and backward; returns the loss tensor [1]
        (loss_out if given)."""
        self.forward(x)
        return self.loss_grad_after_forward(x, target, loss_weights, loss_out)

    def loss_grad_after_forward(self, x, target, loss_weights, loss_out=None):
        """Weighted MSE and backward, given that the activation buffers of
        batch x.shape[0] hold the forward of x (forward, or the fused
        shape_mlp_forward); returns the loss tensor [1] (loss_out if given:
        the loss is written there directly)."""
        buf = self._buffers(x.shape[0])
        dout = buf["dout"]
        loss = buf["loss"] if loss_out is None else loss_out
        self.eng.shape_mse(buf["h"][-1], target, loss_weights, dout, loss)
        self.backward(x, dout)
        return loss

    def fused_step_ok(self, batch: int) -> bool:
        """Whether shape_mlp_train_step takes this network and batch."""
        return (self.bf16 and self.width == WIDTH and batch % 32 == 0
                and 32 <= batch <= SHAPE_MLP_STEP_MAX_ROWS)

    def pack(self):
        """Pack the current parameters for train_step (after any change to
        self.params made outside train_step)."""
        self.packed = self.eng.shape_mlp_pack(self.params, self.packed)

    def train_step(self, f_q, f_lib, mean, inv_std, target, loss_weights, lr, idx=None,
                   qidx=None, fo_cross=None, loss_out=None, beta1=0.9, beta2=0.999, eps=1e-8):
        """Features, forward, loss, backward and Adam of one minibatch in two
        launches (shape_mlp_train_step; self.packed must be current: pack());
        the bits of forward + loss_grad_after_forward + adam_step."""
        return self.eng.shape_mlp_train_step(
            f_q, f_lib, mean, inv_std, target, loss_weights, self.params, self.m, self.v,
            self.step, self.packed, lr, beta1, beta2, eps, idx=idx, qidx=qidx,
            fo_cross=fo_cross, grad=self.grad, loss=loss_out)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.eng.shape_adam(self.params, self.grad, self.m, self.v, self.step, lr, beta1, beta2,
                            eps)

    def predict(self, x: torch.Tensor, chunk: int = 65536) -> torch.Tensor:
        out = torch.empty(x.shape[0], self.width[-1], dtype=torch.float32,
                          device=self.eng.torch_device)
        for s in range(0, x.shape[0], chunk):
            e = min(s + chunk, x.shape[0])
            out[s:e].copy_(self.forward(x[s:e]))
        return out


class Triage:
    """Surrogate-seeded confidence-bounded screening.

    Training data are (query, library molecule) pairs given by index arrays
    into per-molecule feature tables; minibatches are assembled on the device
    by shape_pair_features.  Labels (host arrays) come from adaptive IS.
    """

    def __init__(self, eng: Engine, seed: int = 0, bf16: bool = True, tau: float = 0.005,
                 round_per_pair: int = 512, cap_per_pair: int = 65536, use_fo: bool = True):
        self.eng = eng
        # use the pair's analytic first-order overlap (Eq. fo) in two feature slots
        self.use_fo = use_fo
        self.mlp = MLP(eng, init_params(seed), bf16=bf16)
        dev = eng.torch_device
        self.mean = torch.zeros(96, dtype=torch.float32, device=dev)
        self.inv_std = torch.ones(96, dtype=torch.float32, device=dev)
        self.y_mean = np.zeros(2)
        self.y_std = np.ones(2)
        self.tau = tau
        self.round_per_pair = round_per_pair
        self.cap_per_pair = cap_per_pair

    # -- labels and features -----------------------------------------------------
    def labels(self, query: Molecules, lib: Molecules, seed: int = 0):
        """IS labels of one query against the library: T and
        log(SE(T) sqrt(n_used)) (the per-sample scale) from adaptive screening."""
        out = self.eng.shape_screen(query, lib, mode=SHAPE_SCREEN_ADAPTIVE,
                                    round_per_pair=self.round_per_pair,
                                    cap_per_pair=self.cap_per_pair, tau=self.tau, seed=seed)
        T = out["T"].cpu().numpy().astype(np.float64)
        se = out["se_T"].cpu().numpy().astype(np.float64)
        n = out["n_used"].cpu().numpy().astype(np.float64)
        return T, np.log(se * np.sqrt(n)), n

    def labels_many(self, queries, lib: Molecules, seed: int = 0, n_streams: int = 4,
                    fo: bool = False):
        """labels() for several queries (Molecules, each one molecule) at
        once: the screens go round-robin to n_streams library contexts on
        their own streams, so one screen's ramp and tail overlap the next
        one's work, with one synchronisation at the end.  Same kernels, seeds
        and tile variant as labels(), so the same values.  Returns T, the
        log scale and n_used as [n_queries, n_lib] arrays (and the
        first-order cross-overlaps if fo)."""
        dev = self.eng.torch_device
        n_q, n = len(queries), lib.n_mols
        f32 = dict(dtype=torch.float32, device=dev)
        T = torch.empty(n_q, n, **f32)
        se = torch.empty(n_q, n, **f32)
        nu = torch.empty(n_q, n, dtype=torch.int32, device=dev)
        fo_out = torch.empty(n_q, n, **f32) if fo else None
        helpers = [Engine(self.eng.device) for _ in range(max(n_streams, 1) - 1)]
        engs = [self.eng] + helpers
        for e in helpers:
            e.screen_variant(self.eng.screen_variant())
            e.sampling(self.eng.sampling())
        streams = [torch.cuda.Stream(device=dev) for _ in engs]
        cur = torch.cuda.current_stream(dev)
        for st in streams:
            st.wait_stream(cur)   # the uploads of the queries and the library
        try:
            for e in engs:
                e.prepare_cache(True)   # the library is prepared once per context
            for i, q in enumerate(queries):
                k = i % len(engs)
                out = {"T": T[i], "se_T": se[i], "n_used": nu[i]}
                engs[k].shape_screen(q, lib, mode=SHAPE_SCREEN_ADAPTIVE,
                                     round_per_pair=self.round_per_pair,
                                     cap_per_pair=self.cap_per_pair, tau=self.tau, seed=seed,
                                     out=out, stream=streams[k])
                if fo:
                    engs[k].shape_fo_overlap(q, lib, out=fo_out[i], stream=streams[k])
            for st in streams:
                cur.wait_stream(st)
            torch.cuda.synchronize(dev)
        finally:
            for e in engs:
                e.prepare_cache(False)
            for e in helpers:
                e.close()
        Tn = T.cpu().numpy().astype(np.float64)
        sen = se.cpu().numpy().astype(np.float64)
        nn = nu.cpu().numpy().astype(np.float64)
        res = (Tn, np.log(sen * np.sqrt(nn)), nn)
        return res + (fo_out.cpu().numpy(),) if fo else res

    def fo_overlap(self, query: Molecules, lib: Molecules):
        """First-order cross-overlaps of the query with every library molecule
        (device) when the model uses them, else None."""
        return self.eng.shape_fo_overlap(query, lib) if self.use_fo else None

    def fit_standardisation(self, f_q, f_lib, qidx: np.ndarray, midx: np.ndarray,
                            fo: np.ndarray | None = None, n_sample: int = 65536, seed: int = 0):
        """Mean and standard deviation of the 96 raw pair features over a
        random subsample of the training pairs."""
        dev = self.eng.torch_device
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 0x57D])))
        sel = rng.choice(qidx.size, size=min(n_sample, qidx.size), replace=False)
        zero = torch.zeros(96, dtype=torch.float32, device=dev)
        one = torch.ones(96, dtype=torch.float32, device=dev)
        fo_sel = None
        if self.use_fo:
            fo_sel = torch.from_numpy(np.ascontiguousarray(fo[sel], np.float32)).to(dev)
        raw = self.eng.shape_pair_features(
            f_q, f_lib, zero, one, idx=torch.from_numpy(midx[sel].astype(np.int32)).to(dev),
            qidx=torch.from_numpy(qidx[sel].astype(np.int32)).to(dev),
            fo_cross=fo_sel).cpu().numpy()
        mu = raw.astype(np.float64).mean(0)
        sd = raw.astype(np.float64).std(0)
        sd[sd < 1e-6] = 1.0
        self.mean.copy_(torch.from_numpy(mu.astype(np.float32)))
        self.inv_std.copy_(torch.from_numpy((1.0 / sd).astype(np.float32)))

    # -- checkpoints ---------------------------------------------------------------
    def state_dict(self) -> dict:
        """Everything training and screening read: network parameters, Adam
        moments and step counter, feature standardisation and label
        statistics, as CPU tensors."""
        m = self.mlp
        return {
            "params": m.params.detach().cpu().clone(), "adam_m": m.m.detach().cpu().clone(),
            "adam_v": m.v.detach().cpu().clone(), "adam_step": m.step.detach().cpu().clone(),
            "feat_mean": self.mean.detach().cpu().clone(),
            "feat_inv_std": self.inv_std.detach().cpu().clone(),
            "y_mean": torch.from_numpy(np.asarray(self.y_mean, np.float64)),
            "y_std": torch.from_numpy(np.asarray(self.y_std, np.float64)),
            "width": torch.tensor(self.mlp.width, dtype=torch.int64),
        }

    def load_state_dict(self, sd: dict):
        m = self.mlp
        if tuple(int(w) for w in sd["width"]) != m.width:
            raise ValueError(f"checkpoint widths {tuple(sd['width'].tolist())} != {m.width}")
        for dst, key in ((m.params, "params"), (m.m, "adam_m"), (m.v, "adam_v"),
                         (m.step, "adam_step"), (self.mean, "feat_mean"),
                         (self.inv_std, "feat_inv_std")):
            src = sd[key]
            if src.shape != dst.shape or src.dtype != dst.dtype:
                raise ValueError(f"checkpoint {key}: {tuple(src.shape)} {src.dtype}, expected "
                                 f"{tuple(dst.shape)} {dst.dtype}")
            dst.copy_(src)
        self.y_mean = sd["y_mean"].numpy().copy()
        self.y_std = sd["y_std"].numpy().copy()
        m.packed = None   # repacked by the next training run

    def save(self, path: str):
        """Checkpoint to a safetensors file (tensors only, nothing executable)."""
        from safetensors.torch import save_file
        save_file(self.state_dict(), path)

    def load(self, path: str):
        from safetensors.torch import load_file
        self.load_state_dict(load_file(path))

    # -- training --------------------------------------------------------------------
    def train(self, f_q, f_lib, qidx: np.ndarray, midx: np.ndarray, Y: np.ndarray,
              fo: np.ndarray | None = None, epochs: int = 8, batch: int = 4096,
              lr: float = 1e-3, seed: int = 0, log=None, graph: bool = True,
              fused_forward: bool = True, fused_step: bool = True, start_epoch: int = 0):
        """Minibatch Adam on the weighted MSE of standardised labels Y [n, 2].

        Each epoch's shuffle is drawn on the device (seeded generator) and
        its rows gathered there into fixed buffers, so after the first
        (eager) epoch the whole epoch of steps is
        captured once as a HIP graph and replayed (graph=True): identical
        kernels and results, without a host round trip per launch; the loss
        history is read once at the end.  fused_step: each
        minibatch in the two launches of shape_mlp_train_step (BF16 network
        of the default widths, batch a multiple of 32); else fused_forward:
        its features and forward in one kernel (shape_mlp_forward), then the
        loss, backward and Adam calls.  All three give the same bits.

        start_epoch resumes a run (after load_state_dict of its checkpoint):
        the shuffles of the epochs before it are drawn and skipped, so
        train(epochs=a) + checkpoint + train(epochs=b, start_epoch=a) ends
        with the bits of train(epochs=a + b) (the history returned covers
        the resumed epochs)."""
        dev = self.eng.torch_device
        self.y_mean = Y.mean(0)
        self.y_std = Y.std(0)
        Ys = ((Y - self.y_mean) / self.y_std).astype(np.float32)
        lw = torch.ones(2, dtype=torch.float32, device=dev)
        n = qidx.size
        nb = n // batch
        # each epoch's shuffle is drawn on the device from a seeded generator
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(np.random.SeedSequence([int(seed), 0x7EA]).generate_state(1)[0]))
        for _ in range(int(start_epoch)):
            torch.randperm(qidx.size, generator=gen, device=dev)
        xb = torch.empty(batch, 96, dtype=torch.float32, device=dev)
        losses = torch.empty(max(nb, 1), dtype=torch.float32, device=dev)
        rows = nb * batch
        q_ep = torch.empty(rows, dtype=torch.int32, device=dev)
        m_ep = torch.empty(rows, dtype=torch.int32, device=dev)
        y_ep = torch.empty(rows, 2, dtype=torch.float32, device=dev)
        fo_ep = torch.empty(rows, dtype=torch.float32, device=dev) if self.use_fo else None

        fused = fused_forward and self.mlp.bf16 and self.mlp.width == WIDTH
        one_call = fused_step and self.mlp.fused_step_ok(batch)
        if one_call:
            self.mlp.pack()

        def epoch_steps():
            for b in range(nb):
                s, e = b * batch, (b + 1) * batch
                fo_b = None if fo_ep is None else fo_ep[s:e]
                if one_call:
                    self.mlp.train_step(f_q, f_lib, self.mean, self.inv_std, y_ep[s:e], lw, lr,
                                        idx=m_ep[s:e], qidx=q_ep[s:e], fo_cross=fo_b,
                                        loss_out=losses[b:b + 1])
                    continue
                if fused:
                    acts = self.mlp._buffers(batch)["h"]
                    self.eng.shape_mlp_forward(f_q, f_lib, self.mean, self.inv_std,
                                               self.mlp.params, xb, acts[:3], acts[3],
                                               idx=m_ep[s:e], qidx=q_ep[s:e], fo_cross=fo_b)
                    self.mlp.loss_grad_after_forward(xb, y_ep[s:e], lw, losses[b:b + 1])
                else:
                    self.eng.shape_pair_features(f_q, f_lib, self.mean, self.inv_std,
                                                 idx=m_ep[s:e], qidx=q_ep[s:e], out=xb,
                                                 fo_cross=fo_b)
                    self.mlp.loss_grad(xb, y_ep[s:e], lw, losses[b:b + 1])
                self.mlp.adam_step(lr)

        # the training rows stay on the device; an epoch draws its
        # permutation there and gathers its rows
        q_all = torch.from_numpy(qidx.astype(np.int32)).to(dev)
        m_all = torch.from_numpy(midx.astype(np.int32)).to(dev)
        y_all = torch.from_numpy(np.ascontiguousarray(Ys)).to(dev)
        fo_all = (torch.from_numpy(np.ascontiguousarray(fo, np.float32)).to(dev)
                  if fo_ep is not None else None)
        loss_hist = torch.empty(epochs, max(nb, 1), dtype=torch.float32, device=dev)
        g = None
        try:
            for ep in range(epochs):
                perm_dev = torch.randperm(n, generator=gen, device=dev)[:rows]
                torch.index_select(q_all, 0, perm_dev, out=q_ep)
                torch.index_select(m_all, 0, perm_dev, out=m_ep)
                torch.index_select(y_all, 0, perm_dev, out=y_ep)
                if fo_ep is not None:
                    torch.index_select(fo_all, 0, perm_dev, out=fo_ep)
                with profile_range(f"triage.epoch {start_epoch + ep}"):
                    if graph and ep > 0 and nb > 0:
                        if g is None:
                            g = self.eng.capture(epoch_steps, warmup=False)
                        g.replay()
                    else:
                        epoch_steps()
                loss_hist[ep].copy_(losses)
                if log:
                    log(f"epoch {ep}: loss {float(losses.cpu().numpy().mean()):.4f}")
            hist = loss_hist.cpu().numpy()
        finally:
            if g is not None:
                g.close()
        return [float(h.mean()) for h in hist]

        return history

    def predict_raw(self, f_q, f_lib, fo=None, chunk: int = 65536, fused: bool = True,
                    out=None):
        """Standardised network outputs [n, 2] on the device for the query
        against every library row (fo: first-order cross-overlaps, device).
        fused: one kernel for features and all layers (BF16 network of the
        standard width); otherwise features, then one GEMM per layer."""
        dev = self.eng.torch_device
        n = f_lib.shape[0]
        if out is None:
            out = torch.empty(n, 2, dtype=torch.float32, device=dev)
        if fused and self.mlp.bf16 and self.mlp.width == WIDTH:
            return self.eng.shape_mlp_infer(f_q, f_lib, self.mean, self.inv_std,
                                            self.mlp.params, n=n, fo_cross=fo, out=out)
        xb = torch.empty(min(chunk, n), 96, dtype=torch.float32, device=dev)
        for s in range(0, n, chunk):
            e = min(s + chunk, n)
            x = xb[: e - s]
            self.eng.shape_pair_features(f_q, f_lib[s:e], self.mean, self.inv_std, out=x,
                                         n=e - s, fo_cross=None if fo is None else fo[s:e])
            out[s:e].copy_(self.mlp.forward(x))
        return out

    def to_labels(self, raw: np.ndarray):
        """(predicted T, predicted log SE scale) from standardised outputs."""
        y = raw.astype(np.float64) * self.y_std + self.y_mean
        return y[:, 0], y[:, 1]

    # -- screening ---------------------------------------------------------------
    def seed_budget(self, log_scale: np.ndarray) -> np.ndarray:
        """Host statement of the budget rule that shape_seed_budget applies on
        the device (used to check it): n = (sigma / tau)^2 samples per pair,
        in whole rounds within [round, cap]."""
        n = np.exp(2.0 * log_scale) / self.tau ** 2
        n = np.ceil(n / self.round_per_pair) * self.round_per_pair
        return np.clip(n, self.round_per_pair, self.cap_per_pair).astype(np.int32)

    def screen_buffers(self, n: int, frac: float = 0.05) -> dict:
        """Device buffers of one screen of an n-molecule library (for calls
        that must not allocate, e.g. inside a captured graph)."""
        dev = self.eng.torch_device
        k = max(1, int(round(frac * n)))
        f32 = dict(dtype=torch.float32, device=dev)
        out = {key: torch.empty(k, **f32) for key in ("T", "se_T", "O_ab", "O_aa", "O_bb")}
        out["n_used"] = torch.empty(k, dtype=torch.int32, device=dev)
        return {"n": n, "k": k, "fo": torch.empty(n, **f32) if self.use_fo else None,
                "raw": torch.empty(n, 2, **f32), "score": torch.empty(n, **f32),
                "top": torch.empty(k, dtype=torch.int32, device=dev),
                "budget": torch.empty(k, dtype=torch.int32, device=dev), "out": out}

    def screen(self, query: Molecules, lib: Molecules, f_q, f_lib, frac: float = 0.05,
               seed: int = 0, bufs: dict | None = None):
        """Rank the library by predicted T, refine the top `frac` by adaptive
        IS with budgets seeded from the predicted SE scale.  Returns
        (refined library indices [k] (device, increasing), IS outputs, raw
        network outputs [n, 2]).  Every step runs on the device without a
        host round trip; bufs (from screen_buffers) receives the results."""
        n = lib.n_mols
        if bufs is None:
            bufs = self.screen_buffers(n, frac)
        assert bufs["n"] == n
        k = bufs["k"]
        with profile_range("triage.screen"):
            fo = (self.eng.shape_fo_overlap(query, lib, out=bufs["fo"]) if self.use_fo
                  else None)
            raw = self.predict_raw(f_q, f_lib, fo, out=bufs["raw"])
            bufs["score"].copy_(raw[:, 0])
            top = self.eng.shape_topk(bufs["score"], k, out=bufs["top"])
            budget = self.eng.shape_seed_budget(raw, self.y_mean[1], self.y_std[1], self.tau,
                                                self.round_per_pair, self.cap_per_pair,
                                                idx=top, out=bufs["budget"])
            out = self.eng.shape_screen(query, lib, mode=SHAPE_SCREEN_ADAPTIVE, pairs=top,
                                        round_per_pair=self.round_per_pair,
                                        cap_per_pair=self.cap_per_pair, tau=self.tau,
                                        seed=seed, n_start=budget, out=bufs["out"])
        return top, out, raw
