#!/usr/bin/env python3
"""Benchmark of the IS shape-overlap engine on one MI355X.

Step = one confidence-bounded screen (section "Confidence-bounded
screening"): a 30-atom query against the 100,000-molecule synthetic library
(10-50 heavy atoms, principal frames), rounds of 512 samples per pair until
the Tanimoto SE is at most 0.005 or 65,536 samples are used.  The headline
value is Tanimoto pairs/s at SE <= 0.005; the same run reports atom
evaluations/s, a fixed-budget screen (4096 samples per side) for comparison,
the dominant kernel against its ALU roofline and the FP64 CPU oracle timed on
a bounded sample of the same workload.

Inputs are resident in HBM before timing starts.  One JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Tanimoto pairs/s at SE≤0.005 (plain IS vs surrogate+IS); atom-evals/s"
QUERY_ID = 0xFFFFFF00
N_LIB = 100000
TAU = 0.005
ROUND = 512
CAP = 65536
N_FIXED = 4096

# Roofline of the density loop (bound by FP32 vector arithmetic, not HBM).
# Algorithmic work of one atom evaluation (o_i at one point plus its m/u
# update): 13 FP32 flops -- r - c (3 sub), |r - c|^2 (1 mul + 2 fma = 5),
# times alpha (1 mul), m += o (1 add), u + o (1 - u) (1 sub + 1 fma = 3) --
# and one exponential, which is not counted as a flop.  Peak: the published
# FP32 vector rate of the MI355X, 157.3 TFLOP/s.
FLOPS_PER_EVAL = 13
PEAK_BF16_TFLOPS = 2500.0   # dense BF16 matrix-core peak of MI355X
PEAK_FP32_TFLOPS = 157.3
# Per launch of the adaptive screening kernel on this workload (deterministic
# for a given kernel build), from the rocprofv3 summaries in profiles/:
# HBM bytes (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, scaled by a 1 GiB copy of
# known size) and executed wave instructions (SQ_INSTS_VALU,
# SQ_INSTS_VALU_TRANS_F32).  None until taken on the current kernel.
TRAFFIC_BYTES = 48951.3 * 1024 * 2.0 + 7670.2 * 1024 * 1.0
VALU_INSTS = 6483674909
TRANS_INSTS = 744223320
COUNTER_SOURCE = "profiles/k_screen_100k_library_counters.md"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def atom_evals(n_side, na, nb):
    """Atom evaluations the kernel performs per pair and the plain-equivalent
    count.  Side A (query samples, cached query densities): n_side * N_B
    partner evaluations.  Side B (library samples): n_side * N_A partner and
    n_side * N_B own evaluations.  Plain estimator: 2 n_side (N_A + N_B)."""
    other = n_side * nb + n_side * na
    own = n_side * nb
    plain = 2 * n_side * (na + nb)
    return other, own, plain


def cpu_baseline(q, L, target_s=15.0):
    """FP64 oracle on the host cores, adaptive screening of a bounded prefix of
    the library (batches of 64 pairs until target_s of wall time)."""
    import oracle as O
    from paper_2607_20766_amd.engine import LAMBDA_P27

    qa = (q.xyz, O.alpha_from_radius(q.radius, LAMBDA_P27))
    la = O.alpha_from_radius(L.radius, LAMBDA_P27)
    threads = O.num_threads()
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < target_s and done < L.n_mols:
        idx = np.arange(done, min(done + 64, L.n_mols), dtype=np.int32)
        O.screen(qa, QUERY_ID, L.offsets, L.xyz, la, pairs=idx, mode=1,
                 round_per_pair=ROUND, cap_per_pair=CAP, tau=TAU, seed=0)
        done += idx.size
    dt = time.perf_counter() - t0
    # the same work on one thread, over a shorter prefix
    done1 = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < target_s / 4 and done1 < L.n_mols:
        idx = np.arange(done1, min(done1 + 8, L.n_mols), dtype=np.int32)
        O.screen(qa, QUERY_ID, L.offsets, L.xyz, la, pairs=idx, mode=1,
                 round_per_pair=ROUND, cap_per_pair=CAP, tau=TAU, seed=0, n_threads=1)
        done1 += idx.size
    dt1 = time.perf_counter() - t1
    return {"value": done / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "cpu_model": host_cpu_model(),
            "sample": f"adaptive screen (tau {TAU}, rounds of {ROUND}, cap {CAP}) of "
                      f"library molecules 0..{done - 1} ({done} pairs) against the "
                      f"30-atom query, FP64, {dt:.1f} s on {threads} threads",
            "value_one_thread": done1 / dt1,
            "sample_one_thread": f"molecules 0..{done1 - 1} ({done1} pairs), {dt1:.1f} s"}


def issue_fraction(kernel_ms, peaks):
    """Issue-slot use of the screening kernel: executed VALU wave
    instructions per launch (counters), the transcendental ones weighted by
    the measured cost of v_exp_f32 in FMA issue slots, x 64 lanes, per second
    of kernel time, against the measured FMA issue rate of the same chip."""
    exp_cost = peaks["fma_lane_ops_per_s"] / peaks["exp_lane_ops_per_s"]
    out = {"peak_fma_lane_ops_per_s": peaks["fma_lane_ops_per_s"],
           "exp_cost_fma_slots": exp_cost, "counters": COUNTER_SOURCE}
    if VALU_INSTS is None or TRANS_INSTS is None:
        out.update({"valu_insts_per_launch": None, "frac": None})
        return out
    slots = (VALU_INSTS - TRANS_INSTS) + TRANS_INSTS * exp_cost
    rate = slots * 64 / (kernel_ms * 1e-3)
    out.update({"valu_insts_per_launch": VALU_INSTS, "trans_insts_per_launch": TRANS_INSTS,
                "issue_lane_slots_per_s": rate, "frac": rate / peaks["fma_lane_ops_per_s"]})
    return out


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_align(eng, n_pairs, n_starts=16, n_steps=60, n_samples=2048, lr=0.05):
    """Multi-start rigid alignment (section "Differentiable alignment and the
    hybrid pipeline"): n_pairs pairs of 15-45-atom molecules, 16 starts each
    (uniform quaternions, t ~ N(0, 1 A^2)), 60 Adam steps on -T with 2048
    common-random-number samples per step, one shape_align call."""
    import torch

    from paper_2607_20766_amd import molgen

    log(f"alignment workload: {n_pairs} pairs x {n_starts} starts")
    A = molgen.library(30, n_pairs, 15, 45)
    B = molgen.library(31, n_pairs, 15, 45)
    ida = np.arange(n_pairs, dtype=np.uint32) * 2
    gA = eng.molecules(A, mol_id=ida)
    gB = eng.molecules(B, mol_id=ida + 1)
    poses0 = torch.from_numpy(molgen.random_poses(3, n_pairs, n_starts)).to(eng.torch_device)
    pose = poses0.clone()
    eng.shape_align(gA, gB, pose, n_samples=n_samples, n_steps=2, lr=lr)  # warm-up
    pose.copy_(poses0)
    torch.cuda.synchronize()
    eng.shape_timing_enable(True)
    eng.shape_timing_read(reset=True)
    t0 = time.perf_counter()
    T, best = eng.shape_align(gA, gB, pose, n_samples=n_samples, n_steps=n_steps, lr=lr)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, _ = eng.shape_timing_read(reset=True)
    eng.shape_timing_enable(False)
    T0, _ = eng.shape_align_grad(gA, gB, poses0, eng.shape_self_overlap(gA, n_samples),
                                 eng.shape_self_overlap(gB, n_samples), n_samples,
                                 need_grad=False)
    nb = B.sizes().astype(np.int64)
    evals = int((nb * n_samples * n_starts).sum()) * (n_steps + 1)
    Tb = T.max(dim=1).values.cpu().numpy()
    return {
        "workload": f"{n_pairs} pairs (15-45 atoms) x {n_starts} starts, {n_steps} Adam "
                    f"steps, lr {lr}, {n_samples} CRN samples per step, FP32",
        "pairs_per_s": n_pairs / wall,
        "ms_per_alignment_call": wall * 1e3,
        "kernel_ms": kern_ms,
        "pose_steps_per_s": n_pairs * n_starts * n_steps / wall,
        "adjoint_atom_evals_per_s": evals / wall,
        "mean_best_T_start": float(T0.max(dim=1).values.mean()),
        "mean_best_T_final": float(Tb.mean()),
    }


def bench_accuracy(eng, n_mols=12, n_samples=200000, h=0.15):
    """Accuracy panel (section "Accuracy: the union estimator is unbiased;
    first order over-counts") on synthetic drug-like molecules: union IS
    (2e5 samples) vs the GPU grid reference, and the first-order over-count
    of the union volume and self-overlap."""
    import torch

    from paper_2607_20766_amd import molgen

    rel_v, rel_o, z_v, ratio_v, ratio_o = [], [], [], [], []
    t_grid = 0.0
    pts = 0
    for i in range(n_mols):
        m = molgen.molecule(12, i, 15 + (i * 30) // max(1, n_mols - 1))
        M = eng.molecules(m, mol_id=[i])
        est = eng.shape_estimate(M, M, n_samples, n_samples, seed=i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = eng.shape_grid_integrals(M, M, h=h, pad=6.5)
        t_grid += time.perf_counter() - t0
        ext = m.xyz.max(0) - m.xyz.min(0) + 13.0
        pts += int(np.prod(np.ceil(ext / h) + 1))
        rel_v.append(abs(est["V_a"] / g["V_a"] - 1))
        rel_o.append(abs(est["O_aa"] / g["O_aa"] - 1))
        z_v.append((est["V_a"] - g["V_a"]) / est["se_V_a"])
        # first order: Z = int m (volume), int m^2 (self-overlap)
        alpha = eng.alpha_from_radius(torch.from_numpy(m.radius).cuda()).cpu().numpy()
        Z = float(np.sum((np.pi / alpha.astype(np.float64)) ** 1.5))
        ratio_v.append(Z / g["V_a"])
        ratio_o.append(g["Ofo_aa"] / g["O_aa"])
    return {
        "workload": f"{n_mols} synthetic molecules (15-45 atoms): union IS with "
                    f"{n_samples} samples vs GPU trapezoid grid (h {h} A, pad 6.5 A, FP64)",
        "mean_rel_err_volume": float(np.mean(rel_v)),
        "max_rel_err_volume": float(np.max(rel_v)),
        "mean_rel_err_self_overlap": float(np.mean(rel_o)),
        "max_rel_err_self_overlap": float(np.max(rel_o)),
        "max_abs_z_volume": float(np.max(np.abs(z_v))),
        "first_order_over_union_volume_mean": float(np.mean(ratio_v)),
        "first_order_over_union_volume_range": [float(np.min(ratio_v)), float(np.max(ratio_v))],
        "first_order_over_union_self_overlap_mean": float(np.mean(ratio_o)),
        "grid_points_per_s": pts / t_grid,
    }


def bench_hybrid(eng, Q, lib, n_random=3, n_steps=50):
    """Hybrid pipeline (section "Differentiable alignment and the hybrid
    pipeline"): each library molecule aligned on the query by first-order
    Adam (the given pose, 4 principal-axis and n_random random starts,
    n_steps steps, lr 0.05), best start kept, superposed pair scored by
    adaptive union IS.  The whole pipeline is one HIP graph."""
    import torch

    from paper_2607_20766_amd.engine import SHAPE_SCREEN_ADAPTIVE
    from paper_2607_20766_amd.hybrid import HybridScreen

    n = lib.n_mols
    hs = HybridScreen(eng, n_random=n_random, n_steps=n_steps, lr=0.05, seed=0, tau=TAU,
                      round_per_pair=ROUND, cap_per_pair=CAP)
    bufs = hs.buffers(lib)
    log("hybrid: first-order alignment + union IS")
    hs.screen(Q, lib, bufs)
    torch.cuda.synchronize()
    g = eng.capture(lambda: hs.screen(Q, lib, bufs))
    t = []
    for _ in range(3):
        t0 = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    g.close()
    t_all = float(np.median(t))
    # stage times (direct launches, HIP events on the current stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    eng.shape_fo_starts(Q, lib, n_random, 0, out=bufs["pose"])
    eng.shape_fo_align(Q, lib, bufs["pose"], n_steps, 0.05, T=bufs["T_fo"])
    ev[1].record()
    eng.shape_best_pose(bufs["T_fo"], bufs["pose"], best_pose=bufs["best_pose"],
                        best_T=bufs["best_T_fo"])
    eng.shape_apply_pose(lib, bufs["best_pose"], out=bufs["xyz"])
    ev[2].record()
    out = eng.shape_screen(Q, hs.moved(lib, bufs), mode=SHAPE_SCREEN_ADAPTIVE,
                           round_per_pair=ROUND, cap_per_pair=CAP, tau=TAU, seed=0,
                           out=bufs["out"])
    ev[3].record()
    torch.cuda.synchronize()
    ident = torch.zeros(n, 1, 7, device=eng.torch_device)
    ident[:, 0, 0] = 1.0
    T0, _ = eng.shape_fo_align(Q, lib, ident, n_steps=0)
    plain = eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=ROUND,
                             cap_per_pair=CAP, tau=TAU, seed=0)
    T_al = out["T"].cpu().numpy()
    T_pl = plain["T"].cpu().numpy()
    n_starts = 5 + n_random
    fo_terms = float(n_starts * (n_steps + 1)) * float(
        (Q.n_atoms * (lib.offsets[1:] - lib.offsets[:-1]).to(torch.int64)).sum().item())
    return {
        "workload": f"{n} library molecules vs a 30-atom query: first-order alignment from "
                    f"{n_starts} starts x {n_steps} Adam steps (lr 0.05), best start, then "
                    f"adaptive union IS (tau {TAU}) of the superposed pairs; one HIP graph",
        "pairs_per_s": n / t_all,
        "ms_per_screen": t_all * 1e3,
        "ms_alignment": ev[0].elapsed_time(ev[1]),
        "ms_best_and_move": ev[1].elapsed_time(ev[2]),
        "ms_union_is": ev[2].elapsed_time(ev[3]),
        "fo_pair_terms_per_s": fo_terms / (ev[0].elapsed_time(ev[1]) * 1e-3),
        "mean_T_fo_given_pose": float(T0.mean().item()),
        "mean_T_fo_aligned": float(bufs["best_T_fo"].mean().item()),
        "mean_T_union_given_pose": float(np.nanmean(T_pl)),
        "mean_T_union_aligned": float(np.nanmean(T_al)),
        "is_samples_aligned": int(out["n_used"].cpu().numpy().astype(np.int64).sum()),
    }


def bench_ensemble(eng, Q, n_mols=5000, n_conf=10):
    """Conformer ensembles (max over conformers): n_mols molecules x n_conf
    conformers screened against the query, at their given poses and after
    hybrid first-order alignment; each molecule keeps its best conformer."""
    import torch

    from paper_2607_20766_amd import molgen
    from paper_2607_20766_amd.hybrid import EnsembleScreen, HybridScreen

    log(f"ensemble: generating {n_mols} x {n_conf} conformers")
    C, goff = molgen.conformer_library(13, n_mols, 10, 50, n_conf)
    lib = eng.molecules(C)
    goff_d = torch.from_numpy(goff).to(eng.torch_device)
    res = {"workload": f"{n_mols} molecules x {n_conf} conformers (10-50 atoms) vs a 30-atom "
                       f"query; adaptive union IS (tau {TAU}) of every conformer, max per "
                       f"molecule; also with hybrid first-order alignment (8 starts x 50 steps)"}
    for name, hs in (("given_pose", None),
                     ("aligned", HybridScreen(eng, n_random=3, n_steps=50, tau=TAU,
                                              round_per_pair=ROUND, cap_per_pair=CAP))):
        es = EnsembleScreen(eng, hybrid=hs, tau=TAU, round_per_pair=ROUND, cap_per_pair=CAP)
        bufs = es.buffers(lib, n_mols)
        es.screen(Q, lib, goff_d, bufs)
        torch.cuda.synchronize()
        g = eng.capture(lambda: es.screen(Q, lib, goff_d, bufs))
        t = []
        for _ in range(3):
            t0 = time.perf_counter()
            g.replay()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        g.close()
        T = bufs["out"]["T"].cpu().numpy().reshape(n_mols, n_conf)
        best = bufs["best_T"].cpu().numpy()
        res[name] = {
            "molecules_per_s": n_mols / float(np.median(t)),
            "conformer_pairs_per_s": n_mols * n_conf / float(np.median(t)),
            "ms_per_screen": float(np.median(t)) * 1e3,
            "mean_best_T": float(np.mean(best)),
            "mean_T_conformer0": float(np.mean(T[:, 0])),
            "frac_best_not_conformer0": float(np.mean(np.argmax(T, 1) != 0)),
        }
    return res


def train_step_timing(eng, f_q, f_lib, tr, batch=4096, steps=64):
    """Kernel time of one fused training step (its two launches, HIP events
    around the call) on a scratch network with the trained statistics, and
    its BF16 products against the dense MFMA peak."""
    import torch

    from paper_2607_20766_amd.surrogate import MLP, WIDTH, init_params
    dev = eng.torch_device
    net = MLP(eng, init_params(1))
    net.pack()
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    qi = torch.randint(0, f_q.shape[0], (batch,), generator=g, device=dev, dtype=torch.int32)
    mi = torch.randint(0, f_lib.shape[0], (batch,), generator=g, device=dev, dtype=torch.int32)
    y = torch.randn(batch, 2, generator=g, device=dev)
    fo = torch.rand(batch, generator=g, device=dev) * 40
    lw = torch.ones(2, device=dev)
    for _ in range(4):
        net.train_step(f_q, f_lib, tr.mean, tr.inv_std, y, lw, 1e-3, idx=mi, qidx=qi, fo_cross=fo)
    eng.shape_timing_enable(True)
    eng.shape_timing_read(reset=True)
    for _ in range(steps):
        net.train_step(f_q, f_lib, tr.mean, tr.inv_std, y, lw, 1e-3, idx=mi, qidx=qi, fo_cross=fo)
    torch.cuda.synchronize()
    kern_ms, launches = eng.shape_timing_read(reset=True)
    eng.shape_timing_enable(False)
    step_us = kern_ms / max(launches, 1) * 1e3
    # multiply-adds per row: forward, input gradients (layers 3..1), weight gradients
    macs = sum(i * o for i, o in zip(WIDTH[:-1], WIDTH[1:]))
    macs_in = sum(i * o for i, o in zip(WIDTH[1:-1], WIDTH[2:]))
    flops = 2.0 * batch * (2 * macs + macs_in)
    achieved = flops / (step_us * 1e-6) / 1e12
    return {"batch": batch, "kernel_us_per_step": step_us, "launches_per_step": 2,
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_BF16_TFLOPS,
                         "flops_per_step": flops,
                         "note": "BF16 products of one step (forward, input gradients, weight "
                                 "gradients) / kernel time of its two launches, against the "
                                 "dense BF16 matrix-core peak"}}


def bench_triage(eng, n_lib, n_queries=256, n_train_lib=3907, epochs=10):
    """Learned triage: a BF16 MLP trained on ~10^6 IS-labelled pairs (256
    queries x 3907 molecules) ranks an n_lib-molecule library against a
    held-out 30-atom query; the top 5 % are refined by adaptive IS with
    budgets seeded from the predicted SE scale.  Compared with plain adaptive
    IS over the whole library (same tau, rounds, cap)."""
    import scipy.stats
    import torch

    from paper_2607_20766_amd import molgen
    from paper_2607_20766_amd.engine import SHAPE_SCREEN_ADAPTIVE, SHAPE_SCREEN_FIXED
    from paper_2607_20766_amd.surrogate import Triage

    log("triage: training set labels")
    Lt = molgen.library(40, n_train_lib, 10, 50)
    Qs = molgen.library(41, n_queries, 10, 50)
    lib_t = eng.molecules(Lt)
    f_lib_t = eng.shape_features(lib_t)
    f_q = eng.shape_features(eng.molecules(Qs))
    tr = Triage(eng, seed=0)
    t0 = time.perf_counter()
    # one adaptive screen per training query (query-major rows), spread over
    # four contexts and streams
    qs = [eng.molecules(Qs.mol(i), mol_id=[0xFFFF0000 + i]) for i in range(Qs.n_mols)]
    T, s_, _, FO = tr.labels_many(qs, lib_t, fo=True)
    qi = np.repeat(np.arange(Qs.n_mols), Lt.n_mols)
    mi = np.tile(np.arange(Lt.n_mols), Qs.n_mols)
    Y = np.stack([T.ravel(), s_.ravel()], 1)
    FO = FO.ravel()
    t_labels = time.perf_counter() - t0
    tr.fit_standardisation(f_q, f_lib_t, qi, mi, fo=FO)
    t0 = time.perf_counter()
    hist = tr.train(f_q, f_lib_t, qi, mi, Y, fo=FO, epochs=epochs, batch=4096, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    step = train_step_timing(eng, f_q, f_lib_t, tr)

    log(f"triage: {n_lib}-molecule library")
    qt = molgen.molecule(5, 0, 30)
    L = molgen.library(5, n_lib, 10, 50)
    Q = eng.molecules(qt, mol_id=[QUERY_ID])
    lib = eng.molecules(L)

    dev = eng.torch_device
    f_qt = torch.empty(1, 24, dtype=torch.float32, device=dev)
    f_l = torch.empty(n_lib, 24, dtype=torch.float32, device=dev)
    bufs = tr.screen_buffers(n_lib, frac=0.05)
    plain_out = {k: torch.empty(n_lib, dtype=torch.float32, device=dev)
                 for k in ("T", "se_T", "O_ab", "O_aa", "O_bb")}
    plain_out["n_used"] = torch.empty(n_lib, dtype=torch.int32, device=dev)

    def run_triage():
        # library features are recomputed each time (query-independent, but
        # counted here); each molecule set is prepared once per screen
        eng.prepare_cache(True)
        eng.shape_features(Q, out=f_qt)
        eng.shape_features(lib, out=f_l)
        r = tr.screen(Q, lib, f_qt, f_l, frac=0.05, bufs=bufs)
        eng.prepare_cache(False)
        return r

    def run_plain():
        return eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=ROUND,
                                cap_per_pair=CAP, tau=TAU, seed=0, out=plain_out)

    def wall(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return float(np.median(t)), r

    # plain fixed-budget comparator: the smallest multiple of 512 samples per
    # side at which >= 99 % of a 10^4-pair pilot reach SE(T) <= tau (the
    # pilot at 4096 per side predicts it by the n^-1/2 law; it is then
    # checked and raised by 512 until the pilot meets it)
    log("triage: fixed-budget comparator")
    n_pilot = min(10000, n_lib)
    pilot = eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_FIXED, n_per_side=4096, seed=3,
                             n_pairs=n_pilot)
    se_p = pilot["se_T"].cpu().numpy().astype(np.float64)
    need = 4096.0 * (se_p / TAU) ** 2
    n_fix = int(np.ceil(np.nanquantile(need, 0.99) / 512.0) * 512)
    n_fix = max(512, min(n_fix, 1 << 20))
    while True:
        chk = eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_FIXED, n_per_side=n_fix, seed=3,
                               n_pairs=n_pilot)
        frac_ok = float(np.mean(chk["se_T"].cpu().numpy() <= TAU))
        if frac_ok >= 0.99 or n_fix >= (1 << 20):
            break
        n_fix += 512
    fixed_out = {k: torch.empty_like(v) for k, v in plain_out.items()}

    def run_fixed():
        return eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_FIXED, n_per_side=n_fix, seed=0,
                                out=fixed_out)

    # direct launches, then each pipeline as one HIP graph
    t_fixed, _ = wall(run_fixed, reps=1)
    t_plain_direct, _ = wall(run_plain)
    t_tri_direct, _ = wall(run_triage)
    g_plain = eng.capture(run_plain)
    g_tri = eng.capture(run_triage)
    t_plain, _ = wall(g_plain.replay)
    t_tri, _ = wall(g_tri.replay)
    g_plain.close()
    g_tri.close()
    plain = plain_out
    top, out, raw = bufs["top"], bufs["out"], bufs["raw"]
    T_plain = plain["T"].cpu().numpy()
    n_plain = int(plain["n_used"].cpu().numpy().astype(np.int64).sum())
    n_tri = int(out["n_used"].cpu().numpy().astype(np.int64).sum())
    k1 = n_lib // 100
    true_top = set(np.argsort(-T_plain, kind="stable")[:k1].tolist())
    top = top.cpu().numpy()
    n_plain_top = int(plain["n_used"].cpu().numpy().astype(np.int64)[top].sum())
    T_ref = out["T"].cpu().numpy()
    got = set(top[np.argsort(-T_ref, kind="stable")[:k1]].tolist())
    T_hat, _ = tr.to_labels(raw.cpu().numpy())
    fo_t = eng.shape_fo_overlap(Q, lib).cpu().numpy()
    fq = eng.shape_features(Q).cpu().numpy()[0]
    fl = eng.shape_features(lib).cpu().numpy()
    T_fo = fo_t / (fq[23] + fl[:, 23] - fo_t)
    fo_top = set(np.argsort(-T_fo, kind="stable")[: n_lib // 20].tolist())
    return {
        "workload": f"MLP 96-256-256-256-2 (BF16 MFMA, FP32 accumulation) trained on "
                    f"{qi.size} IS-labelled pairs ({n_queries} queries x {n_train_lib}), "
                    f"{epochs} epochs; held-out 30-atom query vs {n_lib} molecules; top 5 % "
                    f"refined by adaptive IS (tau {TAU}) with seeded budgets",
        "pairs_per_s_surrogate_is": n_lib / t_tri,
        "pairs_per_s_plain_adaptive_is": n_lib / t_plain,
        "speedup": t_plain / t_tri,
        "fixed_budget_per_side": n_fix,
        "fixed_budget_pilot_frac_at_tau": frac_ok,
        "pairs_per_s_plain_fixed_is": n_lib / t_fixed,
        "speedup_vs_fixed": t_fixed / t_tri,
        "ms_surrogate_is": t_tri * 1e3,
        "ms_plain_adaptive_is": t_plain * 1e3,
        "ms_surrogate_is_direct_launches": t_tri_direct * 1e3,
        "ms_plain_adaptive_is_direct_launches": t_plain_direct * 1e3,
        "is_samples_surrogate_is": n_tri,
        "is_samples_plain": n_plain,
        # plain adaptive IS's samples on the same refined pairs: the seeded
        # budgets' overshoot (or saving) against rounds from the start
        "is_samples_plain_on_refined_pairs": n_plain_top,
        "recall_top1pct": len(true_top & got) / k1,
        "mae_T_surrogate_vs_is": float(np.abs(T_hat - T_plain).mean()),
        "spearman_surrogate_vs_is": float(scipy.stats.spearmanr(T_hat, T_plain)[0]),
        "recall_top1pct_within_fo_tanimoto_top5pct": len(true_top & fo_top) / k1,
        "train_s": t_train,
        "train_step": step,
        "label_s": t_labels,
        "final_train_loss": hist[-1],
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--library", type=int, default=N_LIB)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the converged-ranking comparison (untimed)")
    ap.add_argument("--no-align", action="store_true", help="skip the alignment workload")
    ap.add_argument("--align-pairs", type=int, default=10000)
    ap.add_argument("--no-triage", action="store_true", help="skip the learned-triage workload")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the conformer-ensemble workload")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the IS-vs-grid accuracy panel")
    ap.add_argument("--no-hybrid", action="store_true",
                    help="skip the first-order-alignment + union-IS workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device three times (a plain copy of known "
                         "size for scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--triage-library", type=int, default=1000000)
    ap.add_argument("--tune-cache", default=None,
                    help="text file that keeps the screening kernel's tuning choices across runs")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure the instruction issue rates (FP32 FMA, v_exp_f32, "
                         "v_mad_u64_u32, LDS reads) and exit")
    ap.add_argument("--only", choices=("align", "hybrid", "triage", "ensemble", "accuracy"),
                    help="run one secondary workload alone (for profiling) and print its "
                         "section")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures a single GPU (--gpus 1): screening pairs shard across "
              "GPUs without communication, and the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        a = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 4}))
        return

    from paper_2607_20766_amd import molgen
    from paper_2607_20766_amd.engine import (SCREEN_VARIANT_SHAPES, SHAPE_SCREEN_ADAPTIVE,
                                             SHAPE_SCREEN_FIXED, Engine, tune_cache_file)
    if args.tune_cache:
        tune_cache_file(args.tune_cache)

    if args.peaks:
        eng = Engine(0)
        r = eng.peak_rates()
        r["device"] = torch.cuda.get_device_name(0)
        r["compute_units"] = torch.cuda.get_device_properties(0).multi_processor_count
        print(json.dumps(r), flush=True)
        return
    if args.only in ("align", "accuracy", "triage"):
        eng = Engine(0)
        fn = {"align": lambda: bench_align(eng, args.align_pairs),
              "accuracy": lambda: bench_accuracy(eng),
              "triage": lambda: bench_triage(eng, args.triage_library)}[args.only]
        print(json.dumps({"section": args.only, args.only: fn()}), flush=True)
        return

    log("generating workload")
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(1, args.library, 10, 50)
    sizes = L.sizes().astype(np.int64)
    na = q.n_atoms
    log(f"library: {L.n_mols} molecules, {L.n_atoms} atoms")

    eng = Engine(0)
    Q = eng.molecules(q, mol_id=[QUERY_ID])
    lib = eng.molecules(L)
    dev = eng.torch_device
    if args.only in ("hybrid", "ensemble"):
        fn = {"hybrid": lambda: bench_hybrid(eng, Q, lib),
              "ensemble": lambda: bench_ensemble(eng, Q)}[args.only]
        print(json.dumps({"section": args.only, args.only: fn()}), flush=True)
        return
    n = L.n_mols
    out = {k: torch.empty(n, dtype=torch.float32, device=dev)
           for k in ("T", "se_T", "O_ab", "O_aa", "O_bb")}
    out["n_used"] = torch.empty(n, dtype=torch.int32, device=dev)
    out_f = {k: torch.empty_like(v) for k, v in out.items()}

    def adaptive():
        eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=ROUND,
                         cap_per_pair=CAP, tau=TAU, seed=0, out=out)

    def fixed():
        eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_FIXED, n_per_side=N_FIXED, seed=0,
                         out=out_f)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        eng.shape_timing_enable(True)
        eng.shape_timing_read(reset=True)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(steps):
            fn()
        stop.record()
        torch.cuda.synchronize()
        kern_ms, launches = eng.shape_timing_read(reset=True)
        eng.shape_timing_enable(False)
        return start.elapsed_time(stop) / steps, kern_ms / max(launches, 1)

    # work granularity of the screening kernel, autotuned on this workload
    # (every variant gives bit-identical results; untimed set-up)
    log("measuring instruction issue rates")
    peaks = eng.peak_rates()
    log("tuning the screening kernel")
    best, tune_ms = eng.shape_screen_tune(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE,
                                          round_per_pair=ROUND, cap_per_pair=CAP, tau=TAU,
                                          seed=0)
    log(f"tile variant {best}: " + ", ".join(f"{t:.2f}" for t in tune_ms) + " ms")

    log("timing adaptive screen (direct launches; kernel events)")
    ms_eager, kern_ms = timed(adaptive, args.steps, args.warmup)
    eng.shape_check_data()
    # the step's launches (preparation, query cache, screen) as one HIP graph
    graph = eng.capture(adaptive)

    def replay():
        graph.replay()

    log("timing adaptive screen (graph replays)")
    ms_step, _ = timed(replay, args.steps, args.warmup)
    graph.close()
    eng.shape_check_data()
    n_used = out["n_used"].cpu().numpy().astype(np.int64)
    se_T = out["se_T"].cpu().numpy()
    n_side = n_used // 2
    other, own, plain = atom_evals(n_side, na, sizes)
    ev_other, ev_own, ev_plain = int(other.sum()), int(own.sum()), int(plain.sum())
    evals = ev_other + ev_own
    achieved = evals * FLOPS_PER_EVAL / (kern_ms * 1e-3) / 1e12

    log("timing fixed-budget screen")
    ms_fixed, kern_fixed = timed(fixed, args.steps, args.warmup)
    nf = np.full(n, N_FIXED, np.int64)
    fo, fown, fplain = atom_evals(nf, na, sizes)
    se_fixed = out_f["se_T"].cpu().numpy()

    res = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"confidence-bounded screen: 30-atom query vs {n} synthetic "
                        f"molecules (10-50 heavy atoms, principal frames), rounds of "
                        f"{ROUND} Philox samples per pair until SE(T)<={TAU} or {CAP} "
                        f"samples, FP32 with FP64 reductions",
            "library": n, "query_atoms": na, "tau": TAU, "round_per_pair": ROUND,
            "cap_per_pair": CAP,
        },
        "ms_per_step_direct_launches": ms_eager,
        "tuning": {"variant": best, "ms_per_variant": tune_ms},
        "atom_evals_per_s": (ev_other + ev_own) / (ms_step * 1e-3),
        "plain_equivalent_atom_evals_per_s": ev_plain / (ms_step * 1e-3),
        "samples_per_step": int(n_used.sum()),
        "pairs_at_tau": float(np.mean(se_T <= TAU)),
        "pairs_at_cap": float(np.mean(n_used >= CAP)),
        "roofline": {
            "kernel": "k_screen<%d, %d> (adaptive)" % SCREEN_VARIANT_SHAPES[best],
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": TRAFFIC_BYTES,
            "kernel_ms": kern_ms,
            "atom_evals_per_launch": evals,
            "flops_per_atom_eval": FLOPS_PER_EVAL,
            "note": f"{FLOPS_PER_EVAL} algorithmic FP32 flops per atom evaluation x "
                    "evaluations per launch / HIP-event kernel time, against the published "
                    "157.3 TFLOP/s FP32 vector peak (which counts packed FMAs); traffic = "
                    "HBM bytes per launch from rocprofv3 counters scaled by a plain copy",
            "issue": issue_fraction(kern_ms, peaks),
        },
        "fixed_budget": {
            "n_per_side": N_FIXED,
            "pairs_per_s": n / (ms_fixed * 1e-3),
            "ms_per_step": ms_fixed,
            "kernel_ms": kern_fixed,
            "atom_evals_per_s": int((fo + fown).sum()) / (ms_fixed * 1e-3),
            "plain_equivalent_atom_evals_per_s": int(fplain.sum()) / (ms_fixed * 1e-3),
            "pairs_at_tau": float(np.mean(se_fixed <= TAU)),
            "samples_per_step": int(2 * N_FIXED * n),
        },
    }

    # antithetic sampling (the paper's second standard variance control):
    # same rounds, stopping rule and cap; standard errors from pair means
    log("timing adaptive screen, antithetic sampling")
    eng.sampling(True)
    out_a = {k: torch.empty_like(v) for k, v in out.items()}

    def adaptive_anti():
        eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=ROUND,
                         cap_per_pair=CAP, tau=TAU, seed=0, out=out_a)

    ms_anti, kern_anti = timed(adaptive_anti, args.steps, args.warmup)
    eng.sampling(False)
    n_used_a = out_a["n_used"].cpu().numpy().astype(np.int64)
    res["antithetic"] = {
        "pairs_per_s": n / (ms_anti * 1e-3),
        "ms_per_step": ms_anti,
        "kernel_ms": kern_anti,
        "samples_per_step": int(n_used_a.sum()),
        "samples_vs_iid": float(n_used_a.sum() / n_used.sum()),
        "pairs_at_tau": float(np.mean(out_a["se_T"].cpu().numpy() <= TAU)),
    }

    if not args.no_quality:
        # converged ranking: 2^16 samples per side (untimed)
        log("converged reference ranking")
        ref = eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_FIXED, n_per_side=65536, seed=1)
        t_ref = ref["T"].cpu().numpy()
        import scipy.stats
        t_ad = out["T"].cpu().numpy()
        t_fx = out_f["T"].cpu().numpy()
        res["quality"] = {
            "spearman_adaptive_vs_converged": float(scipy.stats.spearmanr(t_ad, t_ref)[0]),
            "spearman_fixed_vs_converged": float(scipy.stats.spearmanr(t_fx, t_ref)[0]),
            "samples_adaptive_over_fixed": float(n_used.sum() / (2 * N_FIXED * n)),
            "converged": "fixed 65,536 samples per side, independent seed",
        }

    if not args.no_align:
        res["align"] = bench_align(eng, args.align_pairs)

    if not args.no_hybrid:
        res["hybrid"] = bench_hybrid(eng, Q, lib)

    if not args.no_accuracy:
        res["accuracy"] = bench_accuracy(eng)

    if not args.no_ensemble:
        res["ensemble"] = bench_ensemble(eng, Q)

    if not args.no_triage:
        res["triage"] = bench_triage(eng, args.triage_library)
    res["peaks"] = peaks

    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(q, L, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
