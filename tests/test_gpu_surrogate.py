"""GPU parity of the learned-triage kernels (shape_features, shape_gemm,
shape_colsum, shape_mse, shape_adam, shape_topk) against the FP64 oracle and
exact host references, and the gain of surrogate-seeded screening over plain
confidence-bounded IS on a small library."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_20766_amd import molgen
from paper_2607_20766_amd.engine import (LAMBDA_P27, SHAPE_SCREEN_ADAPTIVE, Engine, Molecules,
                                         ShapeError)
from paper_2607_20766_amd.surrogate import MLP, WIDTH, Triage, init_params, n_params
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    require_gpu()
    return Engine(0)


def bf16_round(x):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_features_match_oracle(eng):
    L = molgen.MolSet.concat([molgen.library(21, 200, 10, 50, workers=1),
                              molgen.molecule(22, 0, 1), molgen.molecule(22, 1, 256)])
    lib = eng.molecules(L)
    g = eng.shape_features(lib).cpu().numpy().astype(np.float64)
    r = O.features(L.offsets, L.xyz, O.alpha_from_radius(L.radius, LAMBDA_P27))
    assert np.array_equal(g[:, 19:23], r[:, 19:23])
    # histogram: identical except a count moved between neighbouring bins for
    # an atom within rounding of a bin edge
    diff = g[:, :16] - r[:, :16]
    assert np.all(diff.sum(1) == 0) and np.abs(diff).sum() <= 2
    assert np.allclose(g[:, 16:19], r[:, 16:19], rtol=1e-5, atol=1e-6)
    assert np.allclose(g[:, 23], r[:, 23], rtol=1e-5)


def test_large_library_features_in_launch_order_same_bits(eng):
    """From 512 molecules per compute unit on, the features kernel takes the
    molecules in descending order of their squared atom count (four to a
    wave); every row equals the row of the same molecule in a call of 5,000
    molecules, which keeps the plain order, bit for bit.  1- to 96-atom
    molecules drawn with repeats from 3,000; two invalid ones give NaN rows
    and the data-error flag."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    n = 512 * n_cu + 77
    L0 = molgen.library(27, 3000, 1, 96, workers=4)
    L = L0.subset(np.random.default_rng(27).integers(0, L0.n_mols, n))
    L.xyz[L.offsets[17] + 2, 1] = np.nan
    lib = eng.molecules(L)
    lib.alpha[int(L.offsets[n - 5])] = -1.0
    print(f"features of {n} molecules", flush=True)
    full = eng.shape_features(lib).cpu().numpy()
    with pytest.raises(ShapeError):
        eng.shape_check_data()
    eng.shape_check_data()
    bad = [17, n - 5]
    assert np.isnan(full[bad]).all()
    assert np.isfinite(np.delete(full, bad, 0)).all()
    parts = []
    for a in range(0, n, 5000):
        b = min(n, a + 5000)
        o0, o1 = int(L.offsets[a]), int(L.offsets[b])
        part = Molecules((lib.offsets[a:b + 1] - o0).contiguous(), lib.xyz[o0:o1],
                         lib.alpha[o0:o1], None, lib.max_atoms)
        parts.append(eng.shape_features(part).cpu().numpy())
    with pytest.raises(ShapeError):
        eng.shape_check_data()
    eng.shape_check_data()
    plain = np.concatenate(parts)
    assert np.array_equal(full, plain, equal_nan=True)


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("M,N,K", [(37, 70, 45), (256, 2, 256), (5, 300, 96), (64, 64, 4096)])
def test_gemm_matches_host(eng, bf16, M, N, K):
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.normal(size=(M, K)).astype(np.float32)
    Bt = rng.normal(size=(N, K)).astype(np.float32)  # B given transposed: B(k, n) = Bt[n, k]
    bias = rng.normal(size=N).astype(np.float32)
    gate = rng.normal(size=(M, N)).astype(np.float32)
    dA, dBt, db, dg = (torch.from_numpy(x).cuda() for x in (A, Bt, bias, gate))
    C = torch.empty(M, N, dtype=torch.float32, device="cuda")
    eng.shape_gemm(M, N, K, dA, K, 1, dBt, 1, K, C, N, bias=db, bf16=bf16, relu=True)
    Ar, Br = (bf16_round(A), bf16_round(Bt).T) if bf16 else (A.astype(np.float64),
                                                           Bt.T.astype(np.float64))
    ref = np.maximum(Ar @ Br + bias, 0.0)
    scale = np.abs(Ar).max() * np.abs(Br).max() * K
    assert np.abs(C.cpu().numpy() - ref).max() <= 2e-7 * scale + 1e-6
    # gate epilogue, A given transposed
    At = np.ascontiguousarray(A.T)
    eng.shape_gemm(M, N, K, torch.from_numpy(At).cuda(), 1, M, dBt, 1, K, C, N, gate=dg, sgm=N,
                   bf16=bf16)
    ref2 = (Ar @ Br) * (gate > 0)
    assert np.abs(C.cpu().numpy() - ref2).max() <= 2e-7 * scale + 1e-6


def test_colsum_mse_adam(eng):
    rng = np.random.default_rng(4)
    A = rng.normal(size=(1000, 7)).astype(np.float32)
    out = torch.empty(7, dtype=torch.float32, device="cuda")
    eng.shape_colsum(torch.from_numpy(A).cuda(), 1000, 7, 7, out)
    assert np.allclose(out.cpu().numpy(), A.astype(np.float64).sum(0), rtol=1e-6, atol=1e-5)
    y = rng.normal(size=(513, 2)).astype(np.float32)
    t = rng.normal(size=(513, 2)).astype(np.float32)
    w = np.array([1.0, 0.5], np.float32)
    grad = torch.empty(513, 2, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    eng.shape_mse(torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda(),
                  torch.from_numpy(w).cuda(), grad, loss)
    e = y.astype(np.float64) - t
    assert loss.item() == pytest.approx((w * e * e).mean(0).sum(), rel=1e-6)
    assert np.allclose(grad.cpu().numpy(), 2 * w * e / 513, rtol=1e-5, atol=1e-9)
    p = rng.normal(size=300)
    m = np.zeros(300)
    v = np.zeros(300)
    dp, dm, dv = (torch.from_numpy(x.astype(np.float32)).cuda() for x in (p, m, v))
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t_ in range(1, 6):
        g = rng.normal(size=300)
        O.adam(p, g, m, v, t_, 0.01)
        eng.shape_adam(dp, torch.from_numpy(g.astype(np.float32)).cuda(), dm, dv, step, 0.01)
    assert int(step.item()) == 5
    assert np.allclose(dp.cpu().numpy(), p, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("bf16,tol", [(False, 2e-5), (True, 3e-2)])
def test_mlp_matches_oracle(eng, bf16, tol):
    width = list(WIDTH)
    params = init_params(3)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(300, 96)).astype(np.float32)
    t = rng.normal(size=(300, 2)).astype(np.float32)
    lw = np.array([1.0, 1.0])
    net = MLP(eng, params, bf16=bf16)
    dx = torch.from_numpy(x).cuda()
    y = net.forward(dx).cpu().numpy()
    yr = O.mlp_forward(width, params.astype(np.float64), x)
    assert np.abs(y - yr).max() <= tol * np.abs(yr).max()
    loss = net.loss_grad(dx, torch.from_numpy(t).cuda(),
                         torch.from_numpy(lw.astype(np.float32)).cuda()).item()
    lr_, gr = O.mlp_loss_grad(width, params.astype(np.float64), x, t, lw)
    g = net.grad.cpu().numpy().astype(np.float64)
    assert loss == pytest.approx(lr_, rel=tol)
    assert np.abs(g - gr).max() <= tol * np.abs(gr).max()
    assert np.dot(g, gr) / (np.linalg.norm(g) * np.linalg.norm(gr)) > 1 - tol
    if not bf16:
        # element by element: relative to each entry, with a floor for entries
        # that are themselves sums cancelling to near zero (FP32 accumulation
        # over the 300-row batch leaves ~1e-6 of the layer's largest entry)
        off = 0
        for i, o in zip(width[:-1], width[1:]):
            for n_el in (i * o, o):
                seg = slice(off, off + n_el)
                floor = 1e-6 * np.abs(gr[seg]).max()
                assert np.all(np.abs(g[seg] - gr[seg]) <= 2e-5 * np.abs(gr[seg]) + floor), \
                    (i, o, n_el, np.max(np.abs(g[seg] - gr[seg]) / (np.abs(gr[seg]) + 1e-30)))
                off += n_el


def test_topk_exact(eng):
    rng = np.random.default_rng(6)
    for n, k in ((1000, 37), (70000, 3500), (5, 5), (300, 1), (1000000, 50000)):
        s = rng.normal(size=n).astype(np.float32)
        s[rng.integers(0, n, n // 10)] = 0.5   # ties
        s[rng.integers(0, n, 3)] = np.nan
        s[rng.integers(0, n, 2)] = -np.inf
        got = eng.shape_topk(torch.from_numpy(s).cuda(), k).cpu().numpy()
        key = np.where(np.isnan(s), -np.inf, s)
        order = np.lexsort((np.arange(n), -key))  # descending score, then index
        want = np.sort(order[:k])
        assert np.array_equal(got, want), (n, k)


def test_topk_degenerate_scores(eng):
    """Top-k when every radix digit is shared: all scores equal, all NaN
    (NaN ranks lowest), k = n, and one score above a sea of equal ones; ties
    go to the lower index."""
    cases = [(np.full(5000, 0.25, np.float32), 123), (np.full(777, np.nan, np.float32), 7),
             (np.full(300, -1.0, np.float32), 300)]
    one = np.full(100000, 3.0, np.float32)
    one[54321] = 3.0000002
    cases.append((one, 10))
    for s, k in cases:
        got = eng.shape_topk(torch.from_numpy(s).cuda(), k).cpu().numpy()
        key = np.where(np.isnan(s), -np.inf, s)
        want = np.sort(np.lexsort((np.arange(s.size), -key))[:k])
        assert np.array_equal(got, want), (s.size, k)


@pytest.mark.parametrize("shift", [(0.0, 0.0, 0.0), (120.0, -75.0, 40.0)])
def test_fo_overlap_matches_oracle(eng, shift):
    """First-order cross overlaps (Eq. fo) against the oracle's closed form
    at 1e-5, also with query and library moved together far from the origin
    (the kernel's expanded distances are taken about the query's centroid)."""
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(11, 50, 10, 50, workers=1)
    d = np.asarray(shift, np.float32)
    q.xyz = (q.xyz + d).astype(np.float32)
    L.xyz = (L.xyz + d).astype(np.float32)
    Q = eng.molecules(q)
    lib = eng.molecules(L)
    g = eng.shape_fo_overlap(Q, lib).cpu().numpy()
    qa = (q.xyz, O.alpha_from_radius(q.radius, LAMBDA_P27))
    la = O.alpha_from_radius(L.radius, LAMBDA_P27)
    ref = [O.fo_overlap(qa, (L.xyz[L.offsets[m]:L.offsets[m + 1]],
                             la[L.offsets[m]:L.offsets[m + 1]])) for m in range(L.n_mols)]
    assert np.allclose(g, ref, rtol=1e-5)


@pytest.mark.parametrize("q_atoms", [1, 16, 17, 32, 33, 64, 65, 256])
def test_fo_overlap_every_lane_layout(eng, q_atoms):
    """The cross-overlap kernel's lane layouts: query atoms per lane group
    16 (4 phases over the library atoms), 32 (2 phases), 64 (1 phase), and
    blocks of 64 beyond 64 atoms; library molecules of 1 to 256 atoms, a
    ragged pair count and a pairs list with repeats, against the oracle's
    closed form (Eq. fo) at 1e-5."""
    q = molgen.molecule(80, q_atoms, q_atoms)
    L = molgen.MolSet.concat([molgen.molecule(81, i, n) for i, n in
                              enumerate((1, 2, 15, 16, 17, 31, 33, 50, 63, 64, 65, 128, 256))])
    Q = eng.molecules(q)
    lib = eng.molecules(L)
    pairs = torch.tensor([12, 0, 5, 5, 11, 3, 7], dtype=torch.int32, device="cuda")
    print(f"case: first-order cross overlap, query {q_atoms} atoms", flush=True)
    g_all = eng.shape_fo_overlap(Q, lib).cpu().numpy()
    g_sub = eng.shape_fo_overlap(Q, lib, pairs=pairs).cpu().numpy()
    qa = (q.xyz, O.alpha_from_radius(q.radius, LAMBDA_P27))
    la = O.alpha_from_radius(L.radius, LAMBDA_P27)
    ref = np.array([O.fo_overlap(qa, (L.xyz[L.offsets[m]:L.offsets[m + 1]],
                                      la[L.offsets[m]:L.offsets[m + 1]]))
                    for m in range(L.n_mols)])
    assert np.all(np.abs(g_all - ref) <= 1e-5 * ref), np.max(np.abs(g_all - ref) / ref)
    assert np.array_equal(g_sub, g_all[pairs.cpu().numpy()])


def test_triage_gain(eng):
    """Surrogate-seeded screening spends far fewer IS samples than plain
    confidence-bounded IS over the whole library, keeps the top 1 %, and
    predicts the union Tanimoto closely."""
    tr = Triage(eng, seed=0)
    Lt = molgen.library(40, 2000, 10, 50, workers=2)
    Qs = molgen.library(41, 24, 10, 50, workers=1)
    lib_t = eng.molecules(Lt)
    f_lib_t = eng.shape_features(lib_t)
    f_q = eng.shape_features(eng.molecules(Qs))
    qi, mi, Y, FO = [], [], [], []
    for i in range(Qs.n_mols):
        q = eng.molecules(Qs.mol(i), mol_id=[0xFFFF0000 + i])
        T, s, _ = tr.labels(q, lib_t)
        FO.append(eng.shape_fo_overlap(q, lib_t).cpu().numpy())
        qi.append(np.full(Lt.n_mols, i))
        mi.append(np.arange(Lt.n_mols))
        Y.append(np.stack([T, s], 1))
    qi, mi, Y, FO = (np.concatenate(x) for x in (qi, mi, Y, FO))
    tr.fit_standardisation(f_q, f_lib_t, qi, mi, fo=FO)
    hist = tr.train(f_q, f_lib_t, qi, mi, Y, fo=FO, epochs=8, batch=2048, lr=1e-3)
    assert hist[-1] < 0.5 * hist[0]
    # held-out query and library
    qt = molgen.molecule(5, 0, 30)
    L = molgen.library(5, 20000, 10, 50, workers=2)
    Q = eng.molecules(qt, mol_id=[0xFFFFFF00])
    lib = eng.molecules(L)
    f_qt = eng.shape_features(Q)
    f_l = eng.shape_features(lib)
    plain = eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, tau=0.005, cap_per_pair=65536)
    T_plain = plain["T"].cpu().numpy()
    n_plain = int(plain["n_used"].cpu().numpy().astype(np.int64).sum())
    top, out, raw = tr.screen(Q, lib, f_qt, f_l, frac=0.05)
    n_tri = int(out["n_used"].cpu().numpy().astype(np.int64).sum())
    k1 = len(T_plain) // 100
    true_top = set(np.argsort(-T_plain, kind="stable")[:k1].tolist())
    top = top.cpu().numpy()
    T_ref = out["T"].cpu().numpy()
    got_top = set(top[np.argsort(-T_ref, kind="stable")[:k1]].tolist())
    recall = len(true_top & got_top) / k1
    T_hat, _ = tr.to_labels(raw.cpu().numpy())
    mae = float(np.abs(T_hat - T_plain).mean())
    print(f"recall@1% {recall:.3f}  MAE {mae:.4f}  samples {n_tri} vs {n_plain}", flush=True)
    assert n_tri < 0.2 * n_plain
    assert recall >= 0.98
    # far better than predicting the mean (whose MAE is ~0.8 of the spread)
    assert mae < 0.5 * float(T_plain.std())
    # every refined pair met the target or its cap
    se = out["se_T"].cpu().numpy()
    n_used = out["n_used"].cpu().numpy()
    assert np.all((se <= 0.005 * (1 + 1e-6)) | (n_used == 65536))


@pytest.mark.parametrize("n,with_fo,with_idx", [(1000, True, False), (300, False, True),
                                                (128, True, True), (1, False, False)])
def test_fused_inference_matches_layers(eng, n, with_fo, with_idx):
    """shape_mlp_infer equals shape_pair_features + one BF16 GEMM per layer,
    bit for bit (same roundings, same accumulation order)."""
    rng = np.random.default_rng(n)
    n_lib = n + 37
    f_q = rng.normal(size=(3, 24)).astype(np.float32)
    f_lib = rng.normal(size=(n_lib, 24)).astype(np.float32)
    f_q[:, 23] = rng.uniform(50, 100, 3)
    f_lib[:, 23] = rng.uniform(50, 100, n_lib)
    mean = rng.normal(size=96).astype(np.float32)
    inv_std = rng.uniform(0.5, 2.0, 96).astype(np.float32)
    params = init_params(7)
    params[params.size // 2:] *= 1.5   # nonzero biases somewhere
    params = params + rng.normal(scale=0.01, size=params.size).astype(np.float32)
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    fq, fl, mu, isd = d(f_q), d(f_lib), d(mean), d(inv_std)
    idx = d(rng.integers(0, n_lib, n).astype(np.int32)) if with_idx else None
    qidx = d(rng.integers(0, 3, n).astype(np.int32)) if with_idx else None
    fo = d(rng.uniform(1, 40, n).astype(np.float32)) if with_fo else None
    print(f"case: fused inference n={n} fo={with_fo} idx={with_idx}", flush=True)
    x = eng.shape_pair_features(fq, fl, mu, isd, idx=idx, qidx=qidx, n=n, fo_cross=fo)
    net = MLP(eng, params, bf16=True)
    y_layers = net.forward(x).clone()
    y_fused = eng.shape_mlp_infer(fq, fl, mu, isd, net.params, idx=idx, qidx=qidx, n=n,
                                  fo_cross=fo)
    torch.cuda.synchronize()
    assert y_fused.shape == (n, 2)
    assert torch.equal(y_fused, y_layers)
    assert torch.isfinite(y_fused).all()
    # the training forward: same output, plus the features and activations
    # that the layers wrote
    h_layers = [h[:n].clone() for h in net._buffers(n)["h"][:3]]
    xf = torch.full((n, 96), np.nan, device="cuda")
    hf = [torch.full((n, 256), np.nan, device="cuda") for _ in range(3)]
    yf = torch.full((n, 2), np.nan, device="cuda")
    eng.shape_mlp_forward(fq, fl, mu, isd, net.params, xf, hf, yf, idx=idx, qidx=qidx, n=n,
                          fo_cross=fo)
    torch.cuda.synchronize()
    assert torch.equal(yf, y_layers) and torch.equal(xf, x)
    for l in range(3):
        assert torch.equal(hf[l], h_layers[l]), l


def test_gemm_set_equals_gemm(eng):
    """Several products in one shape_gemm_set call give each product
    shape_gemm's bits: weight-gradient shapes (split K), a product without
    split K with bias, ReLU and gate, and two that do not fit the batched
    kernel (FP32 operands; 128 x 128 tiles) and run as by shape_gemm."""
    rng = np.random.default_rng(41)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    specs = [
        dict(M=256, N=256, K=4096, at=True, bf16=True),     # Xt dZ, split K
        dict(M=96, N=256, K=4096, at=True, bf16=True),
        dict(M=256, N=2, K=4096, at=True, bf16=True),
        dict(M=300, N=70, K=45, at=False, bf16=True, bias=True, relu=True, gate=True),
        dict(M=64, N=64, K=100, at=False, bf16=False),      # FP32: shape_gemm path
        dict(M=4096, N=512, K=64, at=False, bf16=True),     # 128 x 128 tiles
    ]
    prods, refs = [], []
    for sp in specs:
        M, N, K = sp["M"], sp["N"], sp["K"]
        if sp["at"]:   # A(m, k) = X[k][m]
            A = d(rng.normal(size=(K, M)))
            sam, sak = 1, M
        else:
            A = d(rng.normal(size=(M, K)))
            sam, sak = K, 1
        B = d(rng.normal(size=(K, N)))
        bias = d(rng.normal(size=N)) if sp.get("bias") else None
        gate = d(rng.normal(size=(M, N))) if sp.get("gate") else None
        ref = torch.empty(M, N, device="cuda")
        eng.shape_gemm(M, N, K, A, sam, sak, B, N, 1, ref, N, bias=bias, gate=gate,
                       sgm=N, bf16=sp["bf16"], relu=sp.get("relu", False))
        refs.append(ref)
        prods.append(dict(M=M, N=N, K=K, A=A, sam=sam, sak=sak, B=B, sbk=N, sbn=1,
                          C=torch.full((M, N), np.nan, device="cuda"), scm=N, bias=bias,
                          gate=gate, sgm=N, bf16=sp["bf16"], relu=sp.get("relu", False)))
    print("case: 6 products in one shape_gemm_set call", flush=True)
    eng.shape_gemm_set(prods)
    torch.cuda.synchronize()
    for p, ref in zip(prods, refs):
        assert torch.equal(p["C"], ref), (p["M"], p["N"], p["K"])
    with pytest.raises(ShapeError):
        eng.shape_gemm_set(prods + prods[:3])   # 9 > 8 products


def test_labels_many_equals_labels(eng):
    """Label screens spread over several contexts and streams give each
    query the values of its own labels() call."""
    Lt = molgen.library(42, 300, 10, 50, workers=1)
    Qs = molgen.library(43, 6, 10, 50, workers=1)
    lib = eng.molecules(Lt)
    qs = [eng.molecules(Qs.mol(i), mol_id=[0xFFFF0000 + i]) for i in range(Qs.n_mols)]
    tr = Triage(eng, seed=0)
    print("case: labels of 6 queries on 4 streams", flush=True)
    T, ls, n, fo = tr.labels_many(qs, lib, fo=True)
    for i, q in enumerate(qs):
        Ti, lsi, ni = tr.labels(q, lib)
        assert np.array_equal(T[i], Ti) and np.array_equal(n[i], ni), i
        assert np.array_equal(ls[i], lsi), i
        assert np.array_equal(fo[i], eng.shape_fo_overlap(q, lib).cpu().numpy()), i


def test_colsum_set_equals_colsum(eng):
    """One launch for several matrices gives each column sum the bits of
    shape_colsum: row counts below, at and far above the 16 chunks of 32 rows
    a workgroup forms at once, ragged column counts, a padded row stride."""
    rng = np.random.default_rng(31)
    shapes = [(4096, 256, 256), (4096, 2, 2), (37, 70, 75), (1, 1, 1), (513, 129, 130),
              (20000, 65, 65)]
    mats, want = [], []
    for M, N, lda in shapes:
        A = torch.from_numpy(rng.normal(size=(M, lda)).astype(np.float32)).cuda()
        ref = torch.empty(N, dtype=torch.float32, device="cuda")
        eng.shape_colsum(A, M, N, lda, ref)
        mats.append((A, M, N, lda, torch.full((N,), np.nan, device="cuda")))
        want.append(ref)
    print("case: column sums of 6 matrices in one launch", flush=True)
    eng.shape_colsum_set(mats)
    torch.cuda.synchronize()
    for (A, M, N, lda, out), ref in zip(mats, want):
        assert torch.equal(out, ref), (M, N, lda)
    with pytest.raises(ShapeError):
        eng.shape_colsum_set(mats + mats[:3])   # 9 > 8 matrices


def test_training_with_fused_forward_equals_layers(eng):
    """Training whose minibatch forward is one shape_mlp_forward kernel, and
    training whose whole minibatch step is one shape_mlp_train_step call,
    give the loss history, parameters, Adam moments and step count of the
    per-layer path, bit for bit."""
    rng = np.random.default_rng(23)
    n_q, n_l, n = 3, 700, 5000
    f_q = rng.normal(size=(n_q, 24)).astype(np.float32)
    f_l = rng.normal(size=(n_l, 24)).astype(np.float32)
    f_q[:, 23] = rng.uniform(50, 100, n_q)
    f_l[:, 23] = rng.uniform(50, 100, n_l)
    fq, fl = torch.from_numpy(f_q).cuda(), torch.from_numpy(f_l).cuda()
    qi, mi = rng.integers(0, n_q, n), rng.integers(0, n_l, n)
    Y = rng.normal(size=(n, 2))
    FO = rng.uniform(1, 40, n)
    res = []
    for fused, one_call in ((False, False), (True, False), (True, True)):
        print(f"case: training, fused forward={fused}, fused step={one_call}", flush=True)
        tr = Triage(eng, seed=4)
        tr.fit_standardisation(fq, fl, qi, mi, fo=FO)
        hist = tr.train(fq, fl, qi, mi, Y, fo=FO, epochs=2, batch=1024, lr=1e-3,
                        fused_forward=fused, fused_step=one_call)
        res.append((hist, tr.mlp.params.cpu().numpy().copy(), tr.mlp.m.cpu().numpy().copy(),
                    tr.mlp.v.cpu().numpy().copy(), int(tr.mlp.step.item())))
    for r in res[1:]:
        assert r[0] == res[0][0]
        for a, b in zip(r[1:], res[0][1:]):
            assert np.array_equal(a, b)


def test_graph_training_equals_eager(eng):
    """Epochs replayed from one captured HIP graph train exactly as eager
    launches do (loss history and final parameters bit for bit)."""
    rng = np.random.default_rng(21)
    n_q, n_l, n = 3, 700, 5000
    f_q = rng.normal(size=(n_q, 24)).astype(np.float32)
    f_l = rng.normal(size=(n_l, 24)).astype(np.float32)
    f_q[:, 23] = rng.uniform(50, 100, n_q)
    f_l[:, 23] = rng.uniform(50, 100, n_l)
    fq, fl = torch.from_numpy(f_q).cuda(), torch.from_numpy(f_l).cuda()
    qi, mi = rng.integers(0, n_q, n), rng.integers(0, n_l, n)
    Y = rng.normal(size=(n, 2))
    FO = rng.uniform(1, 40, n)
    res = []
    for graph in (False, True):
        print(f"case: training, graph={graph}", flush=True)
        tr = Triage(eng, seed=3)
        tr.fit_standardisation(fq, fl, qi, mi, fo=FO)
        hist = tr.train(fq, fl, qi, mi, Y, fo=FO, epochs=3, batch=1024, lr=1e-3, graph=graph)
        res.append((hist, tr.mlp.params.cpu().numpy().copy()))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1])


def test_seed_budget_matches_host_rule(eng):
    tr = Triage(eng, seed=0)
    tr.y_mean = np.array([0.3, -1.7])
    tr.y_std = np.array([0.2, 0.8])
    rng = np.random.default_rng(9)
    raw = rng.normal(scale=2.0, size=(5000, 2)).astype(np.float32)
    raw[17, 1] = np.nan
    raw[18, 1] = 1e30
    raw[19, 1] = -1e30
    idx = rng.permutation(5000)[:1234].astype(np.int32)
    draw = torch.from_numpy(raw).cuda()
    got = eng.shape_seed_budget(draw, tr.y_mean[1], tr.y_std[1], tr.tau, tr.round_per_pair,
                                tr.cap_per_pair, idx=torch.from_numpy(idx).cuda())
    ls = raw[idx].astype(np.float64)[:, 1] * tr.y_std[1] + tr.y_mean[1]
    with np.errstate(over="ignore", invalid="ignore"):
        want = tr.seed_budget(ls)
    want[np.isnan(ls)] = tr.cap_per_pair
    assert np.array_equal(got.cpu().numpy(), want)
    full = eng.shape_seed_budget(draw, tr.y_mean[1], tr.y_std[1], tr.tau, tr.round_per_pair,
                                 tr.cap_per_pair).cpu().numpy()
    assert full[17] == tr.cap_per_pair and full[18] == tr.cap_per_pair
    assert full[19] == tr.round_per_pair


def _backward_by_layers(eng, width, params, acts, dout, grad, bf16):
    """The backward pass composed from the single products: input gradients
    with shape_gemm (ReLU gate), every weight gradient with shape_gemm_set,
    every bias gradient with shape_colsum_set."""
    B = dout.shape[0]
    L = len(width) - 1
    offs = [0]
    for i, o in zip(width[:-1], width[1:]):
        offs.append(offs[-1] + i * o + o)
    dz, wg, bg = dout, [], []
    for l in range(L - 1, -1, -1):
        n_in, n_out = width[l], width[l + 1]
        gW = grad[offs[l]:offs[l] + n_in * n_out]
        gb = grad[offs[l] + n_in * n_out:offs[l + 1]]
        wg.append(dict(M=n_in, N=n_out, K=B, A=acts[l], sam=1, sak=n_in, B=dz, sbk=n_out,
                       sbn=1, C=gW, scm=n_out, bf16=bf16))
        bg.append((dz, B, n_out, n_out, gb))
        if l > 0:
            dn = torch.empty(B, n_in, dtype=torch.float32, device="cuda")
            eng.shape_gemm(B, n_in, n_out, dz, n_out, 1, params[offs[l]:offs[l] + n_in * n_out],
                           1, n_out, dn, n_in, gate=acts[l], sgm=n_in, bf16=bf16)
            dz = dn
    eng.shape_gemm_set(wg)
    eng.shape_colsum_set(bg)


@pytest.mark.parametrize("width,B", [(WIDTH, 4096), (WIDTH, 300), ((5, 37, 3), 1),
                                     ((7, 2), 1000), ((33, 65, 129, 17, 8, 4), 777)])
@pytest.mark.parametrize("bf16", [True, False])
def test_mlp_backward_equals_layer_calls(eng, width, B, bf16):
    """shape_mlp_backward gives the bits of the per-layer calls it replaces,
    for the network's own shape and ragged ones (widths off the tiles, a
    single layer, a single row)."""
    width = list(width)
    rng = np.random.default_rng(41)
    params = torch.from_numpy(init_params(9, width)).cuda()
    acts = [torch.from_numpy(rng.normal(size=(B, width[0])).astype(np.float32)).cuda()]
    for w in width[1:-1]:
        h = rng.normal(size=(B, w)).astype(np.float32)
        acts.append(torch.from_numpy(np.maximum(h, 0)).cuda())   # post-ReLU: zeros gate
    dout = torch.from_numpy(rng.normal(size=(B, width[-1])).astype(np.float32)).cuda()
    print(f"case: MLP backward {width} batch {B} bf16={bf16}", flush=True)
    ref = torch.full((n_params(width),), np.nan, device="cuda")
    _backward_by_layers(eng, width, params, acts, dout, ref, bf16)
    got = torch.full_like(ref, np.nan)
    eng.shape_mlp_backward(width, params, acts, dout, got, bf16=bf16)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    with pytest.raises(ValueError):
        eng.shape_mlp_backward(width, params, acts[:-1], dout, got)


@pytest.mark.parametrize("n", [32, 64, 576, 1024, 4096, 4128, 8192, 65536])
def test_train_step_equals_calls(eng, n):
    """shape_mlp_train_step against shape_mlp_forward, shape_mse,
    shape_mlp_backward and shape_adam over three consecutive steps: loss,
    gradient, parameters, moments, step counter and the repacked weights bit
    for bit.  Batches of one workgroup, of a half-filled last loss block
    (576 rows, ragged split-K chunks), of single-chunk weight gradients (64),
    of the training batch (4096) and beyond it (8192: split-K chunks that
    differ between layers), a single 32-row workgroup, 4,128 rows (a
    loss block of one 32-row wave; 26 split-K chunks of 160 rows, the last
    one shorter) and the largest batch (up to 128 chunks per weight tile,
    bias and loss sums over several staging passes)."""
    rng = np.random.default_rng(50 + n)
    n_q, n_l = 3, 20000
    f_q = rng.normal(size=(n_q, 24)).astype(np.float32)
    f_l = rng.normal(size=(n_l, 24)).astype(np.float32)
    f_q[:, 23] = rng.uniform(50, 100, n_q)
    f_l[:, 23] = rng.uniform(50, 100, n_l)
    fq, fl = torch.from_numpy(f_q).cuda(), torch.from_numpy(f_l).cuda()
    mean = torch.from_numpy(rng.normal(size=96).astype(np.float32) * 0.3).cuda()
    inv_std = torch.from_numpy(rng.uniform(0.5, 1.5, 96).astype(np.float32)).cuda()
    lw = torch.tensor([1.0, 0.5], dtype=torch.float32, device="cuda")
    params = init_params(7)
    ref, fus = MLP(eng, params), MLP(eng, params)
    fus.pack()
    xb = torch.empty(n, 96, dtype=torch.float32, device="cuda")
    for it in range(3):
        qi = torch.from_numpy(rng.integers(0, n_q, n).astype(np.int32)).cuda()
        mi = torch.from_numpy(rng.integers(0, n_l, n).astype(np.int32)).cuda()
        fo = torch.from_numpy(rng.uniform(1, 40, n).astype(np.float32)).cuda()
        y = torch.from_numpy(rng.normal(size=(n, 2)).astype(np.float32)).cuda()
        print(f"case: fused training step, {n} rows, step {it}", flush=True)
        acts = ref._buffers(n)["h"]
        eng.shape_mlp_forward(fq, fl, mean, inv_std, ref.params, xb, acts[:3], acts[3], idx=mi,
                              qidx=qi, fo_cross=fo)
        l_ref = ref.loss_grad_after_forward(xb, y, lw).clone()
        ref.adam_step(1e-3)
        l_fus = fus.train_step(fq, fl, mean, inv_std, y, lw, 1e-3, idx=mi, qidx=qi, fo_cross=fo)
        torch.cuda.synchronize()
        assert torch.equal(l_fus, l_ref), (l_fus.item(), l_ref.item())
        assert torch.equal(fus.grad, ref.grad)
        assert torch.equal(fus.params, ref.params)
        assert torch.equal(fus.m, ref.m) and torch.equal(fus.v, ref.v)
        assert torch.equal(fus.step, ref.step)
    assert torch.equal(fus.packed, eng.shape_mlp_pack(ref.params))


def test_train_step_rejects_batches_off_its_grid(eng):
    net = MLP(eng, init_params(1))
    net.pack()
    fq = torch.zeros(1, 24, device="cuda")
    fl = torch.ones(100, 24, device="cuda")
    mean, inv_std = torch.zeros(96, device="cuda"), torch.ones(96, device="cuda")
    lw = torch.ones(2, device="cuda")
    for n in (100, 16):
        with pytest.raises(ShapeError) as e:
            net.train_step(fq, fl, mean, inv_std, torch.zeros(n, 2, device="cuda"), lw, 1e-3,
                           idx=torch.zeros(n, dtype=torch.int32, device="cuda"))
        assert e.value.code == -2
    assert int(net.step.item()) == 0


def test_training_resumes_from_checkpoint(eng, tmp_path):
    """Train a epochs, checkpoint to a file, load into a fresh triage object
    (other initial weights) and train b more from start_epoch = a: the
    parameters, Adam state and loss history equal those of a + b epochs in
    one run, bit for bit."""
    rng = np.random.default_rng(27)
    n_q, n_l, n = 3, 700, 5000
    f_q = rng.normal(size=(n_q, 24)).astype(np.float32)
    f_l = rng.normal(size=(n_l, 24)).astype(np.float32)
    f_q[:, 23] = rng.uniform(50, 100, n_q)
    f_l[:, 23] = rng.uniform(50, 100, n_l)
    fq, fl = torch.from_numpy(f_q).cuda(), torch.from_numpy(f_l).cuda()
    qi, mi = rng.integers(0, n_q, n), rng.integers(0, n_l, n)
    Y = rng.normal(size=(n, 2))
    FO = rng.uniform(1, 40, n)
    print("case: training, 3 epochs in one run", flush=True)
    ref = Triage(eng, seed=6)
    ref.fit_standardisation(fq, fl, qi, mi, fo=FO)
    h_ref = ref.train(fq, fl, qi, mi, Y, fo=FO, epochs=3, batch=1024, lr=1e-3)
    print("case: training, 2 epochs, checkpoint, 1 more", flush=True)
    a = Triage(eng, seed=6)
    a.fit_standardisation(fq, fl, qi, mi, fo=FO)
    h_a = a.train(fq, fl, qi, mi, Y, fo=FO, epochs=2, batch=1024, lr=1e-3)
    path = str(tmp_path / "triage.safetensors")
    a.save(path)
    b = Triage(eng, seed=7)
    b.load(path)
    h_b = b.train(fq, fl, qi, mi, Y, fo=FO, epochs=1, batch=1024, lr=1e-3, start_epoch=2)
    assert h_a + h_b == h_ref
    for x, y in ((b.mlp.params, ref.mlp.params), (b.mlp.m, ref.mlp.m), (b.mlp.v, ref.mlp.v),
                 (b.mlp.step, ref.mlp.step), (b.mean, ref.mean), (b.inv_std, ref.inv_std)):
        assert torch.equal(x, y)
    bad = b.state_dict()
    bad["params"] = bad["params"][:-1]
    with pytest.raises(ValueError):
        b.load_state_dict(bad)
