"""Work-granularity autotuning of the screening kernel (every tile variant
gives bit-identical results) and HIP-graph capture of library calls (replays
equal the direct calls, also after the inputs change in place)."""
import numpy as np
import pytest
import torch

from paper_2607_20766_amd import molgen
from paper_2607_20766_amd.engine import (SHAPE_E_UNSUPPORTED, SHAPE_SCREEN_ADAPTIVE,
                                         SHAPE_SCREEN_FIXED, SHAPE_SCREEN_VARIANTS, Engine,
                                         ShapeError, tune_cache_clear, tune_cache_file,
                                         tune_cache_size)
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu

QUERY_ID = 0xFFFFFF00
KEYS = ("T", "se_T", "O_ab", "O_aa", "O_bb", "n_used")


@pytest.fixture(scope="module")
def eng():
    require_gpu()
    e = Engine(0)
    yield e
    e.screen_variant(-1)


@pytest.fixture(scope="module")
def data(eng):
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(11, 203, 10, 50, workers=1)  # ragged count, uneven atoms
    return eng.molecules(q, mol_id=[QUERY_ID]), eng.molecules(L)


def _alloc(n, dev):
    out = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in KEYS[:5]}
    out["n_used"] = torch.empty(n, dtype=torch.int32, device=dev)
    return out


def _np(out):
    return {k: v.cpu().numpy().copy() for k, v in out.items()}


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("kw", [
    dict(mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=512, cap_per_pair=8192, tau=0.005),
    dict(mode=SHAPE_SCREEN_FIXED, n_per_side=4096),
    dict(mode=SHAPE_SCREEN_FIXED, n_per_side=320),   # 64-sample rounds: partial tiles
])
def test_all_variants_bit_identical(eng, data, kw):
    Q, lib = data
    print(f"case: tile variants, {kw}", flush=True)
    ref = None
    for v in range(SHAPE_SCREEN_VARIANTS):
        assert eng.screen_variant(v) == v
        got = _np(eng.shape_screen(Q, lib, seed=3, **kw))
        if ref is None:
            ref = got
        else:
            _same(ref, got)
    eng.screen_variant(-1)
    assert np.all(np.isfinite(ref["T"]))


def test_tuner_picks_a_variant(eng, data):
    Q, lib = data
    tune_cache_clear()
    before = _np(eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, seed=5))
    best, ms = eng.shape_screen_tune(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, seed=5)
    assert 0 <= best < SHAPE_SCREEN_VARIANTS
    assert eng.screen_variant() == best
    assert all(t > 0 for t in ms) and ms[best] == min(ms)
    _same(before, _np(eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_ADAPTIVE, seed=5)))
    with pytest.raises(ShapeError):
        eng.screen_variant(SHAPE_SCREEN_VARIANTS)
    eng.screen_variant(-1)


def test_graph_replays_match_direct_calls(eng, data):
    Q, lib = data
    dev = eng.torch_device
    n = lib.n_mols
    out = _alloc(n, dev)
    other = _alloc(n, dev)
    kw = dict(mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=512, cap_per_pair=8192, seed=7)

    def step():
        eng.shape_screen(Q, lib, out=out, **kw)

    direct = _np(eng.shape_screen(Q, lib, **kw))
    g = eng.capture(step)
    try:
        for rep in range(3):
            for v in out.values():
                v.fill_(-1)   # replays must rewrite every output
            print(f"case: graph replay {rep}", flush=True)
            g.replay()
            torch.cuda.synchronize()
            _same(direct, _np(out))
            # eager work of the program between replays
            eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_FIXED, n_per_side=256, seed=1, out=other)
            torch.cuda.synchronize()
        # inputs changed in place: rotate the query by a quarter turn about z
        xyz = Q.xyz.clone()
        Q.xyz[:, 0], Q.xyz[:, 1] = -xyz[:, 1], xyz[:, 0].clone()
        g.replay()
        torch.cuda.synchronize()
        moved = _np(out)
        _same(_np(eng.shape_screen(Q, lib, **kw)), moved)
        assert not np.array_equal(moved["T"], direct["T"])
        Q.xyz.copy_(xyz)
        g.replay()
        torch.cuda.synchronize()
        _same(direct, _np(out))
    finally:
        g.close()


def test_capture_refuses_sync_calls_and_growth(eng, data):
    Q, lib = data
    big = molgen.library(12, 2 * lib.n_mols + 500, 10, 50, workers=1)
    Lbig = eng.molecules(big)
    out = _alloc(Lbig.n_mols, eng.torch_device)

    def grows():
        eng.shape_screen(Q, Lbig, mode=SHAPE_SCREEN_FIXED, n_per_side=2 ** 20, seed=1, out=out)

    with pytest.raises(ShapeError) as ei:
        eng.capture(grows, warmup=False)
    assert ei.value.code == SHAPE_E_UNSUPPORTED

    def syncs():
        eng.shape_check_data()

    with pytest.raises(ShapeError) as ei:
        eng.capture(syncs, warmup=False)
    assert ei.value.code == SHAPE_E_UNSUPPORTED
    # the engine still works after a discarded capture
    got = _np(eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_FIXED, n_per_side=256, seed=1))
    assert np.all(np.isfinite(got["T"]))


def test_graph_survives_scratch_growth(eng, data):
    """An eager call that grows the context's scratch while a graph is alive
    retires the old buffers instead of freeing them, so the graph's replays
    still address live memory and give the captured calls' results; the
    retired buffers go with the last graph.  The replay below runs only once
    the context reports the retirement."""
    Q, lib = data
    n = lib.n_mols
    out = _alloc(n, eng.torch_device)
    kw = dict(mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=512, cap_per_pair=8192, seed=7)
    direct = _np(eng.shape_screen(Q, lib, **kw))
    g = eng.capture(lambda: eng.shape_screen(Q, lib, out=out, **kw))
    try:
        info = eng.memory_info()
        assert info["live_graphs"] == 1 and info["retired_bytes"] == 0
        big = molgen.library(13, 4 * n + 700, 10, 50, workers=1)
        Lbig = eng.molecules(big)
        print("case: eager screen growing scratch under a live graph", flush=True)
        eng.shape_screen(Q, Lbig, mode=SHAPE_SCREEN_FIXED, n_per_side=1 << 16, seed=1)
        torch.cuda.synchronize()
        info = eng.memory_info()
        assert info["retired_bytes"] > 0 and info["live_graphs"] == 1
        for v in out.values():
            v.fill_(-1)
        print("case: replay after growth", flush=True)
        g.replay()
        torch.cuda.synchronize()
        _same(direct, _np(out))
        # a graph launches only with the context that captured it
        other = Engine(0)
        with pytest.raises(ShapeError) as ei:
            load_library_graph_launch(other, g)
        assert ei.value.code == -1
        other.close()
    finally:
        g.close()
    info = eng.memory_info()
    assert info["live_graphs"] == 0 and info["retired_bytes"] == 0


def load_library_graph_launch(e, g):
    from paper_2607_20766_amd.engine import _stream, load_library
    e._check(load_library().shape_graph_launch(e._ctx, g._handle, _stream(None)))


def test_triage_screen_as_graph(eng, data):
    """The whole surrogate-triaged screen (features, first-order overlaps,
    fused network, top-k, seeded budgets, adaptive IS) replays as one graph."""
    from paper_2607_20766_amd.surrogate import Triage
    Q, lib = data
    tr = Triage(eng, seed=0)
    n = lib.n_mols
    dev = eng.torch_device
    f_q = torch.empty(1, 24, dtype=torch.float32, device=dev)
    f_l = torch.empty(n, 24, dtype=torch.float32, device=dev)
    bufs = tr.screen_buffers(n, frac=0.1)

    def step():
        eng.prepare_cache(True)   # each set is prepared once per screen
        eng.shape_features(Q, out=f_q)
        eng.shape_features(lib, out=f_l)
        tr.screen(Q, lib, f_q, f_l, frac=0.1, bufs=bufs)
        eng.prepare_cache(False)

    top, out, raw = tr.screen(Q, lib, eng.shape_features(Q), eng.shape_features(lib), frac=0.1)
    ref = (top.cpu().numpy(), _np(out), raw.cpu().numpy())
    g = eng.capture(step)
    try:
        for rep in range(3):
            bufs["top"].fill_(-1)
            bufs["raw"].fill_(0)
            for v in bufs["out"].values():
                v.fill_(-1)
            print(f"case: triage graph replay {rep}", flush=True)
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(bufs["top"].cpu().numpy(), ref[0])
            assert np.array_equal(bufs["raw"].cpu().numpy(), ref[2])
            _same(ref[1], _np(bufs["out"]))
            eng.shape_screen(Q, lib, mode=SHAPE_SCREEN_FIXED, n_per_side=256, seed=2)
            torch.cuda.synchronize()
    finally:
        g.close()


def test_prepare_cache_reuses_unchanged_sets(eng, data):
    from paper_2607_20766_amd.engine import SHAPE_SCREEN_ADAPTIVE as AD
    Q, lib = data
    kw = dict(mode=AD, round_per_pair=512, cap_per_pair=8192, seed=4)

    def run():
        f = eng.shape_features(lib).cpu().numpy()
        fo = eng.shape_fo_overlap(Q, lib).cpu().numpy()
        return f, fo, _np(eng.shape_screen(Q, lib, **kw))

    ref = run()
    eng.prepare_cache(True)
    try:
        got = run()
        assert np.array_equal(ref[0], got[0], equal_nan=True)
        assert np.array_equal(ref[1], got[1], equal_nan=True)
        _same(ref[2], got[2])
        # forgetting after an in-place change prepares the new data
        xyz = lib.xyz.clone()
        lib.xyz.mul_(1.1)
        eng.prepare_cache(True)
        moved = _np(eng.shape_screen(Q, lib, **kw))
        assert not np.array_equal(moved["T"], ref[2]["T"])
        lib.xyz.copy_(xyz)
        eng.prepare_cache(True)
        _same(ref[2], _np(eng.shape_screen(Q, lib, **kw)))
    finally:
        eng.prepare_cache(False)


def test_prepare_cache_still_reports_invalid_data(eng, data):
    Q, _ = data
    L = molgen.library(13, 20, 10, 50, workers=1)
    L.xyz[L.offsets[5] + 2, 1] = np.nan
    bad = eng.molecules(L)
    eng.prepare_cache(True)
    try:
        for rep in range(2):   # the second call reuses the preparation
            out = _np(eng.shape_screen(Q, bad, mode=SHAPE_SCREEN_FIXED, n_per_side=256, seed=1))
            assert np.isnan(out["T"][5]) and np.isfinite(np.delete(out["T"], 5)).all()
            with pytest.raises(ShapeError):
                eng.shape_check_data()
    finally:
        eng.prepare_cache(False)
    eng.shape_check_data()


def test_subset_screens_prepare_only_their_molecules(eng):
    """A screen of a small pair subset prepares only the listed molecules;
    its results equal the whole-library screen's for those pairs, with or
    without a reusable whole-set preparation, and a whole-library screen
    afterwards is not misled by the partial one."""
    from paper_2607_20766_amd.engine import SHAPE_SCREEN_ADAPTIVE as AD
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(19, 400, 10, 50, workers=1)
    Q = eng.molecules(q, mol_id=[QUERY_ID])
    lib = eng.molecules(L)
    kw = dict(mode=AD, round_per_pair=512, cap_per_pair=8192, seed=4)
    full = _np(eng.shape_screen(Q, lib, **kw))
    sub = np.array([399, 7, 7, 0, 123, 250], dtype=np.int32)
    pairs = torch.from_numpy(sub).cuda()
    part = _np(eng.shape_screen(Q, lib, pairs=pairs, **kw))
    for k in part:
        assert np.array_equal(part[k], full[k][sub]), k
    eng.prepare_cache(True)
    try:
        again = _np(eng.shape_screen(Q, lib, **kw))     # whole set, prepared for reuse
        part2 = _np(eng.shape_screen(Q, lib, pairs=pairs, **kw))  # reuses it
        part3 = _np(eng.shape_screen(Q, lib, pairs=pairs, **kw))
        eng.prepare_cache(True)                          # forget
        part4 = _np(eng.shape_screen(Q, lib, pairs=pairs, **kw))  # subset again
        whole = _np(eng.shape_screen(Q, lib, **kw))      # must prepare everything
    finally:
        eng.prepare_cache(False)
    _same(full, again)
    _same(full, whole)
    for p_ in (part2, part3, part4):
        for k in p_:
            assert np.array_equal(p_[k], full[k][sub]), k
    # indices outside the library: NaN and no samples, the rest unaffected
    odd = torch.tensor([5, 400, -3, 9], dtype=torch.int32, device="cuda")
    g = _np(eng.shape_screen(Q, lib, pairs=odd, **kw))
    assert np.isnan(g["T"][[1, 2]]).all() and (g["n_used"][[1, 2]] == 0).all()
    for k in g:
        assert np.array_equal(g[k][[0, 3]], full[k][[5, 9]]), k
    eng.shape_check_data()


def test_features_and_first_order_flag_invalid_data(eng):
    """Features and first-order overlaps read the caller's arrays directly:
    an invalid molecule gives NaN and raises the data-error flag."""
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(20, 30, 10, 50, workers=1)
    f_clean = eng.shape_features(eng.molecules(L)).cpu().numpy()
    L.xyz[L.offsets[4] + 1, 2] = np.inf
    Q = eng.molecules(q, mol_id=[QUERY_ID])
    lib = eng.molecules(L)
    lib.alpha[int(L.offsets[9])] = 0.0
    f = eng.shape_features(lib).cpu().numpy()
    assert np.isnan(f[4]).all() and np.isnan(f[9]).all()
    # molecules sharing a wave with a bad one keep their exact features
    assert np.array_equal(np.delete(f, [4, 9], 0), np.delete(f_clean, [4, 9], 0))
    with pytest.raises(ShapeError):
        eng.shape_check_data()
    eng.shape_check_data()
    fo = eng.shape_fo_overlap(Q, lib).cpu().numpy()
    assert np.isnan(fo[[4, 9]]).all() and np.isfinite(np.delete(fo, [4, 9])).all()
    with pytest.raises(ShapeError):
        eng.shape_check_data()
    eng.shape_check_data()
    # an index outside the library gives NaN without flagging the data
    bad_idx = torch.tensor([2, 30, -1], dtype=torch.int32, device="cuda")
    fo2 = eng.shape_fo_overlap(Q, lib, pairs=bad_idx).cpu().numpy()
    assert np.isfinite(fo2[0]) and np.isnan(fo2[1:]).all()
    eng.shape_check_data()


def test_tuner_cache_second_context_reuses_choice(eng, data):
    """A second context tuning the same kind of screen takes the first
    context's choice without timing anything, and screens to the same bits;
    another schedule is a different kind and is timed."""
    Q, lib = data
    kw = dict(mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=512, cap_per_pair=8192, seed=11)
    tune_cache_clear()
    best1, ms1 = eng.shape_screen_tune(Q, lib, **kw)
    assert all(t > 0 for t in ms1) and tune_cache_size() == 1
    out1 = _np(eng.shape_screen(Q, lib, **kw))
    e2 = Engine(0)
    print("case: tuning cache, second context", flush=True)
    best2, ms2 = e2.shape_screen_tune(Q, lib, **kw)
    assert best2 == best1 and e2.screen_variant() == best1
    assert all(t == -1 for t in ms2)
    _same(out1, _np(e2.shape_screen(Q, lib, **kw)))
    _, ms3 = e2.shape_screen_tune(Q, lib, **dict(kw, cap_per_pair=16384))
    assert all(t > 0 for t in ms3) and tune_cache_size() == 2
    eng.screen_variant(-1)


def test_tuner_cache_file_round_trip(eng, data, tmp_path):
    """Choices appended to the cache file are read back after the process
    table is cleared (as by a new process), and reused without timing."""
    Q, lib = data
    kw = dict(mode=SHAPE_SCREEN_FIXED, n_per_side=1024, seed=3)
    path = str(tmp_path / "tune.txt")
    tune_cache_clear()
    tune_cache_file(path)
    try:
        best, ms = eng.shape_screen_tune(Q, lib, **kw)
        assert all(t > 0 for t in ms)
        lines = open(path).read().splitlines()
        assert len(lines) == 1 and lines[0].startswith("shape-tune-v1 gfx950")
        assert lines[0].split()[-1] == str(best)
        tune_cache_clear()
        assert tune_cache_size() == 0
        tune_cache_file(path)
        assert tune_cache_size() == 1
        e2 = Engine(0)
        print("case: tuning cache read from a file", flush=True)
        best2, ms2 = e2.shape_screen_tune(Q, lib, **kw)
        assert best2 == best and all(t == -1 for t in ms2)
    finally:
        tune_cache_file(None)
        eng.screen_variant(-1)


def test_graph_of_long_screen_recomputes_its_order(eng):
    """A captured screen long enough to be launched in work order (seeded
    budgets) recomputes the order on every replay: replays equal direct calls,
    also after the budgets change in place and after eager long screens that
    reuse the context's order buffer for other pairs."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    n = 16 * n_cu + 77
    q = molgen.molecule(1, 0, 30)
    L = molgen.library(27, 3000, 1, 80, workers=4)
    Q, lib = eng.molecules(q, mol_id=[QUERY_ID]), eng.molecules(L)
    dev = eng.torch_device
    rng = np.random.default_rng(27)
    pairs = torch.from_numpy(rng.integers(0, L.n_mols, n).astype(np.int32)).to(dev)
    n_start = torch.from_numpy((rng.integers(0, 6, n) * 512).astype(np.int32)).to(dev)
    other_pairs = torch.flip(pairs, [0]).contiguous()
    kw = dict(mode=SHAPE_SCREEN_ADAPTIVE, round_per_pair=512, cap_per_pair=4096, tau=0.01,
              seed=4)
    out = _alloc(n, dev)
    scratch = _alloc(n, dev)

    def step():
        eng.shape_screen(Q, lib, pairs=pairs, n_start=n_start, out=out, **kw)

    step()
    torch.cuda.synchronize()
    g = eng.capture(step)
    try:
        for rep in range(4):
            if rep == 2:   # new budgets, written in place
                n_start.copy_(torch.flip(n_start, [0]))
            print(f"case: long-screen graph replay {rep}", flush=True)
            direct = _np(eng.shape_screen(Q, lib, pairs=pairs, n_start=n_start, **kw))
            for v in out.values():
                v.fill_(-1)
            g.replay()
            torch.cuda.synchronize()
            _same(direct, _np(out))
            # eager long screen of other pairs between replays
            eng.shape_screen(Q, lib, pairs=other_pairs, out=scratch, **kw)
            torch.cuda.synchronize()
    finally:
        g.close()
