"""GPU parity: the HIP library (through the C ABI) against the CPU oracle,
element by element, bit-exact for counts, accept flags and accepted ids.

Every case prints its name before it touches the GPU."""
import os

import numpy as np
import pytest

from oracle import reference as R
from paper_1810_11966_amd import synth
from tests import helpers

pytestmark = pytest.mark.gpu

TESTS = ("msd", "msd_basis", "window")
FORMS = ("plain", "persistent", "pruned", "persistent_pruned", "binned", "persistent_binned", "auto")


def forms_for(test):
    return list(FORMS)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_11966_amd import trig
    trig.load()
    return torch


def to_dev(torch, s):
    d = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(s.offsets)).to(d),
            torch.from_numpy(np.ascontiguousarray(s.x)).to(d),
            torch.from_numpy(np.ascontiguousarray(s.y)).to(d))


def run_gpu(torch, s, test="msd", form="plain", compact=True, **kw):
    from paper_1810_11966_amd import trig
    off, x, y = to_dev(torch, s)
    if getattr(s, "z", None) is not None:
        kw["hit_z"] = torch.from_numpy(np.ascontiguousarray(s.z)).to(off.device)
    r = trig.select(off, x, y, test=test, form=form, compact=compact, want_status=True, **kw)
    torch.cuda.synchronize()
    out = {"counts": r.counts.cpu().numpy(), "accept": r.accept.cpu().numpy(),
           "status": int(r.status.cpu().numpy()[0]) & 0xFFFFFFFF}
    if compact:
        n = int(r.n_accepted.cpu().numpy()[0])
        out["ids"] = r.ids.cpu().numpy()[:n]
    return out


def oracle_cfg(test, **kw):
    okw = {}
    for k_gpu, k_or in (("z", "z"), ("msd_max", "msd_max"), ("ndf", "ndf"),
                        ("slope_window", "window"), ("min_triplets", "min_triplets")):
        if k_gpu in kw:
            okw[k_or] = tuple(kw[k_gpu]) if isinstance(kw[k_gpu], (list, tuple)) else kw[k_gpu]
    return R.OracleConfig(test=test, **okw)


_ORACLE_CACHE = {}
THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_result(s, cfg):
    key = (s.sha256(), cfg)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = R.select_set(s, cfg, n_threads=THREADS)
    return _ORACLE_CACHE[key]


def assert_parity(torch, s, test, form, label, **kw):
    print(f"[parity] {label} test={test} form={form} events={s.n_events} hits={s.n_hits}", flush=True)
    got = run_gpu(torch, s, test, form, **kw)
    c, a, st, _ = oracle_result(s, oracle_cfg(test, **kw))
    bad = np.flatnonzero(got["counts"] != c)
    assert bad.size == 0, f"{label}: {bad.size} events differ, first {bad[:5]} gpu {got['counts'][bad[:5]]} cpu {c[bad[:5]]}"
    assert np.array_equal(got["accept"], a), label
    assert np.array_equal(got["ids"], R.accepted_ids(a)), label
    assert got["status"] == st, label
    return c


# ------------------------------------------------------------ hand-built ---

@pytest.mark.parametrize("form", FORMS)
def test_golden_cases(gpu, form):
    for case in helpers.golden_cases():
        s = helpers.golden_set(case)
        cfg = dict(case.get("cfg", {}))
        test = cfg.pop("test", "msd")
        kw = {}
        if "msd_max" in cfg:
            kw["msd_max"] = cfg["msd_max"]
        if "ndf" in cfg:
            kw["ndf"] = cfg["ndf"]
        if "window" in cfg:
            kw["slope_window"] = cfg["window"]
        for t in ([test] if test == "window" else ["msd", "msd_basis"]):
            print(f"[golden] {case['name']} {t} {form}", flush=True)
            got = run_gpu(gpu, s, t, form, **kw)
            assert got["counts"][0] == case["expected_count"], (case["name"], t, form)


# -------------------------------------------------------------- workloads ---

@pytest.mark.parametrize("test", TESTS)
def test_small_10k_all_forms(gpu, test):
    s = synth.make_event_set(synth.SMALL_10K)
    for form in forms_for(test):
        assert_parity(gpu, s, test, form, "small_10k")


@pytest.mark.parametrize("test", TESTS)
def test_near_threshold_stress(gpu, test):
    s = synth.concat([helpers.near_threshold_events(300, 8, seed=3, rel=1e-4),
                      helpers.near_threshold_events(100, 20, seed=4, rel=1e-6)])
    for form in forms_for(test):
        c = assert_parity(gpu, s, test, form, "near_threshold")
    assert c.sum() > 0


def test_pair_prune_boundary(gpu):
    """Triplets whose layer-0/1 residual part alone sits at the cut: the exact
    pair pruning of the batched form must keep every pair that can pass."""
    s = synth.concat([helpers.pair_boundary_events(300, 6, seed=1, rel=1e-6),
                      helpers.pair_boundary_events(300, 6, seed=2, rel=3e-8)])
    for test in ("msd", "msd_basis"):
        for form in FORMS:
            c = assert_parity(gpu, s, test, form, "pair boundary")
        assert c.sum() > 0
        for form in ("plain", "persistent_pruned"):
            assert_parity(gpu, s, test, form, "pair boundary ndf3", ndf=3, msd_max=(0.02, 0.016666668))


def test_block_shapes_and_large_events(gpu):
    """Batched form: events per block from 1 to 256 (sub-blocks when a block's
    hits exceed LDS), and events too large for LDS mixed into blocks."""
    base = synth.make_event_set(synth.SMALL_10K, n_events=3000)
    big = helpers.ragged_sizes_set([(1, 1, 5000), (2, 3, 4500), (70, 60, 4000), (3, 4100, 2)], seed=4)
    s = synth.concat([base.subset(0, 1000), big, base.subset(1000, 2000)])
    for test in ("msd", "window"):
        for form in ("pruned", "persistent_pruned"):
            for eb in (0, 1, 7, 64, 128):
                assert_parity(gpu, s, test, form, f"block_events={eb}", block_events=eb)
    dense = synth.make_event_set(synth.DENSE_100K, n_events=300)
    for eb in (1, 5, 40):
        assert_parity(gpu, dense, "msd", "persistent_pruned", f"dense block_events={eb}", block_events=eb)


def test_block_hit_range_edges(gpu):
    """Batched form at the edges of its whole-block staging: blocks of exactly
    the LDS capacity less one float4 group (1020 hits at 1024, 2044 at 2048)
    and one hit more, block ranges starting at every offset within a 16-byte
    group, and a last block whose hits all lie in the final partial float4
    group of the hit arrays (n_hits = 4k + 1, 2, 3).  Blocks of up to 52
    events at 2048 hits take the kernel with the small event table."""
    head = [(340, 340, 340), (340, 340, 341), (1, 2, 1), (339, 341, 340), (5, 6, 7)]
    n_head = sum(a + b + c for a, b, c in head)
    for tail, last in ((1, (1, 0, 0)), (2, (1, 1, 0)), (3, (1, 1, 1))):
        pad = (4 - (n_head + 3) % 4) % 4  # the hits before the last event: a multiple of 4
        s = helpers.ragged_sizes_set(head + [(1, 1, 1 + pad), last], seed=20 + tail)
        assert s.n_hits % 4 == tail and s.offsets[-4] == s.n_hits - tail
        for hb in (1024, 2048):  # at 2048 hits the first two events fill 2041 of 2044, three 2045
            for eb in (1, 2, 3):
                assert_parity(gpu, s, "msd", "pruned", f"hit range edges tail={tail} block_hits={hb} "
                              f"block_events={eb}", block_events=eb, block_hits=hb)
        assert_parity(gpu, s, "msd", "auto", f"hit range edges tail={tail}")


def test_misaligned_hit_arrays(gpu):
    """x and y starting 4 bytes past a 16-byte boundary: the batched form's
    staging takes its element-wise path; counts are unchanged."""
    from paper_1810_11966_amd import trig
    torch = gpu
    s = synth.make_event_set(synth.SMALL_10K, n_events=4000)
    c, a, st, _ = oracle_result(s, R.OracleConfig())
    off = torch.from_numpy(s.offsets).cuda()
    xf = torch.zeros(s.n_hits + 1, dtype=torch.float32, device="cuda")
    yf = torch.zeros(s.n_hits + 1, dtype=torch.float32, device="cuda")
    xf[1:] = torch.from_numpy(s.x).cuda()
    yf[1:] = torch.from_numpy(s.y).cuda()
    x, y = xf[1:], yf[1:]
    assert x.data_ptr() % 16 == 4
    for form in FORMS:
        print(f"[misaligned] {form}", flush=True)
        r = trig.select(off, x, y, form=form, compact=True)
        torch.cuda.synchronize()
        assert np.array_equal(r.counts.cpu().numpy(), c), form


def test_near_threshold_other_ndf_and_thresholds(gpu):
    s = helpers.near_threshold_events(200, 8, seed=9, rel=1e-4)
    for kw in ({"ndf": 3}, {"ndf": 1}, {"ndf": 7, "msd_max": (0.0085714, 0.0071428)},
               {"msd_max": (0.0300001, 0.0249999)}, {"min_triplets": 0}, {"min_triplets": 5}):
        for form in ("plain", "persistent_pruned"):
            assert_parity(gpu, s, "msd", form, f"ndf/threshold {kw}", **kw)
        assert_parity(gpu, s, "msd_basis", "persistent_pruned", f"ndf/threshold {kw}", **kw)


def test_other_geometry(gpu):
    s = synth.make_event_set(synth.EventSetSpec(n_events=3000, hits_mean=10, p_inject=0.3,
                                                sigma=0.05, z=(100.0, 300.0, 1000.0), salt=77))
    for test in TESTS:
        for form in forms_for(test):
            assert_parity(gpu, s, test, form, "geometry z=100/300/1000", z=(100.0, 300.0, 1000.0),
                          slope_window=(0.002, 0.003))


def test_ragged_layer_sizes(gpu):
    sizes = []
    for n in (0, 1, 2, 3, 31, 63, 64, 65, 127, 128, 129):
        sizes += [(n, 5, 7), (5, n, 7), (5, 7, n), (n, n, 3)]
    sizes += [(1, 1, 1), (64, 1, 64), (1, 64, 65), (9, 7, 513), (3, 2, 1025), (2, 3, 600)]
    s = helpers.ragged_sizes_set(sizes, seed=1)
    for test in TESTS:
        for form in forms_for(test):
            assert_parity(gpu, s, test, form, "ragged")
            for tp in (64, 128, 1024):
                if form == "persistent":
                    assert_parity(gpu, s, test, form, f"ragged tile_pairs={tp}", tile_pairs=tp)


def test_layer_orientation_grid(gpu):
    """Layer-0/1 size pairs on both sides of the lane-count boundaries (32,
    64) and of the per-wave buffer (48 or 64 entries): events that put layer 1
    into the lanes, events that put layer 0 there, and events of the general
    path; each has an exact track, so the exact pass of either orientation
    must find it."""
    ns = (1, 4, 7, 16, 21, 31, 32, 33, 40, 48, 49, 63, 64, 65, 80)
    sizes = [(a, b, 9) for a in ns for b in ns] + [(a, b, 70) for a in (5, 33, 65) for b in (5, 33, 65)]
    for seed in (2, 3):
        s = helpers.ragged_sizes_set(sizes, seed=seed)
        for test in ("msd", "window"):
            for form in ("pruned", "persistent_pruned", "auto"):
                c = assert_parity(gpu, s, test, form, f"orientation grid seed={seed}")
        assert (c > 0).all()


def test_dense_and_mixture_samples(gpu):
    dense = synth.make_event_set(synth.DENSE_100K, n_events=400)
    mix = synth.make_event_set(synth.MIXTURE_4M, n_events=4000)
    for s, label in ((dense, "dense_100k[:400]"), (mix, "mixture_4m[:4000]")):
        for form in ("plain", "pruned", "persistent_pruned", "binned", "persistent_binned"):
            assert_parity(gpu, s, "msd", form, label)
        for form in ("persistent", "binned"):
            assert_parity(gpu, s, "window", form, label)


def test_injected_exact_tracks_accept(gpu):
    """sigma = 0 pairs: every injected event is accepted (exercises accept and
    compaction with many accepted events)."""
    s = synth.make_event_set(synth.EventSetSpec(n_events=20000, hits_mean=8, p_inject=0.3, sigma=0.0,
                                                salt=55))
    for form in FORMS:
        c = assert_parity(gpu, s, "msd", form, "exact pairs")
    assert (c[s.n_tracks > 0] >= 2).all()


# ---------------------------------------------------- binning edge cases ---

def test_binned_key_interval_edges(gpu):
    """Pairs at the edge of the layer-1 key interval (|a| at beta), triplets
    at the edge of the layer-2 interval (|b| at beta), slopes at the window
    edge: the binned form keeps every candidate that can pass."""
    pair = synth.concat([helpers.pair_boundary_events(200, 6, seed=5, rel=1e-6),
                         helpers.pair_boundary_events(200, 6, seed=6, rel=3e-8)])
    kb = synth.concat([helpers.k_boundary_events(200, 6, seed=7, rel=1e-6),
                       helpers.k_boundary_events(200, 6, seed=8, rel=3e-8)])
    win = synth.concat([helpers.window_boundary_events(200, 6, seed=9, rel=1e-6),
                        helpers.window_boundary_events(200, 6, seed=10, rel=3e-8)])
    for form in ("plain", "binned", "persistent_binned", "pruned"):
        for test in ("msd", "msd_basis"):
            c1 = assert_parity(gpu, pair, test, form, "layer-1 key edge")
            c2 = assert_parity(gpu, kb, test, form, "layer-2 key edge")
        c3 = assert_parity(gpu, win, "window", form, "window edge")
    assert c1.sum() > 0 and c2.sum() > 0 and c3.sum() > 0
    for form in ("plain", "binned"):
        for test in ("msd", "msd_basis"):
            assert_parity(gpu, kb, test, form, "layer-2 key edge ndf3", ndf=3, msd_max=(0.02, 0.016666668))
        assert_parity(gpu, win, "window", form, "window edge W=0.0049999", slope_window=(0.0049999, 0.0050001))


def test_written_out_fit_far_from_axis(gpu):
    """Tracks with slopes up to 25 and 1000 (coordinates up to ~1e4 and
    ~4e5 cm) displaced near the cut: there the written-out fit's own rounding
    moves Q by up to ~1e-3 of the cut, its decisions differ from the basis
    form's for hundreds of triplets, and the pruned and binned forms' bounds
    on a and b (which grow with the coordinates) must still keep every
    triplet that passes."""
    sets = []
    for k, sm in enumerate((25.0, 1000.0)):
        sets += [helpers.near_threshold_events(150, 8, seed=40 + k, rel=1e-3, slope_max=sm),
                 helpers.pair_boundary_events(150, 6, seed=50 + k, rel=1e-3, slope_max=sm),
                 helpers.k_boundary_events(150, 6, seed=60 + k, rel=1e-3, slope_max=sm)]
    s = synth.concat(sets)
    for test in ("msd", "msd_basis"):
        for form in FORMS:
            c = assert_parity(gpu, s, test, form, "far from the axis")
        assert c.sum() > 0
    for form in ("pruned", "binned"):
        assert_parity(gpu, s, "msd", form, "far from the axis ndf3", ndf=3, msd_max=(0.02, 0.016666668))


def test_special_coordinate_values(gpu):
    """NaN, +-inf, huge, subnormal and zero coordinates, zero-width key ranges
    and events past the binned form's LDS capacity, in every form."""
    s = helpers.special_values_events(seed=3)
    for test in TESTS:
        for form in forms_for(test):
            assert_parity(gpu, s, test, form, "special values")


# ------------------------------------------------------------ error paths ---

def test_malformed_and_overflow_events(gpu):
    good = synth.make_event_set(synth.SMALL_10K, n_events=50)
    off = good.offsets.copy()
    off[3 * 10 + 1] = off[3 * 10 + 2] + 1      # event 10: layer 0 end past layer 1 end
    off[3 * 20 + 3] = good.n_hits + 5           # event 20 (and 21 start): beyond n_hits
    bad = synth.EventSet(off, good.x, good.y, good.n_tracks)
    for test in TESTS:
        for form in forms_for(test):
            assert_parity(gpu, bad, test, form, "malformed")
    n = 1291
    big = synth.EventSet(np.array([0, n, 2 * n, 3 * n, 3 * n + 1, 3 * n + 2, 3 * n + 3], np.int32),
                         np.zeros(3 * n + 3, np.float32), np.zeros(3 * n + 3, np.float32),
                         np.zeros(2, np.int8))
    for form in FORMS:
        got = run_gpu(gpu, big, "msd", form)
        assert got["counts"][0] == -2 and got["accept"][0] == 0 and got["status"] == 2
        assert got["counts"][1] == 1 and list(got["ids"]) == []


def test_empty_batch(gpu):
    from paper_1810_11966_amd import trig
    s = synth.EventSet(np.zeros(1, np.int32), np.zeros(0, np.float32), np.zeros(0, np.float32),
                       np.zeros(0, np.int8))
    torch = gpu
    off = torch.zeros(1, dtype=torch.int32, device="cuda")
    x = torch.zeros(0, dtype=torch.float32, device="cuda")
    for form in FORMS:
        r = trig.select(off, x, x, form=form, compact=True)
        torch.cuda.synchronize()
        assert int(r.n_accepted.cpu()[0]) == 0 and r.counts.numel() == 0


# ------------------------------------------------ determinism / composition ---

def test_repeatable_and_batch_composition(gpu):
    s = synth.make_event_set(synth.MIXTURE_4M, n_events=6000)
    base = run_gpu(gpu, s, "msd", "persistent")["counts"]
    for _ in range(3):
        assert np.array_equal(run_gpu(gpu, s, "msd", "persistent")["counts"], base)
    parts = [s.subset(0, 1000), s.subset(1000, 3000), s.subset(4000, 2000)]
    got = np.concatenate([run_gpu(gpu, p, "msd", "plain")["counts"] for p in parts])
    assert np.array_equal(got, base)


# ----------------------------------------------------------- full sizes ---

def test_medium_1m_full_size_sampled(gpu):
    """The 1M-event workload at full size in the benchmark's launch
    configuration: every form agrees with every other on all events, and the
    oracle checks a sample of 20k events (three ranges) one by one."""
    s = synth.make_event_set(synth.MEDIUM_1M)
    print("[full] medium_1m generated", flush=True)
    results = {}
    for form in FORMS:
        print(f"[full] medium_1m form={form}", flush=True)
        results[form] = run_gpu(gpu, s, "msd", form)
    base = results["plain"]
    for form, r in results.items():
        assert np.array_equal(r["counts"], base["counts"]), form
        assert np.array_equal(r["ids"], np.flatnonzero(base["accept"])), form
    for first in (0, 500_000, s.n_events - 7000):
        sub = s.subset(first, 7000 if first else 6000)
        c, a, st, _ = R.select_set(sub, n_threads=THREADS)
        assert np.array_equal(base["counts"][first:first + sub.n_events], c), first
    # the window test accepts the injected pairs
    w = run_gpu(gpu, s, "window", "persistent_pruned")
    sub = s.subset(0, 6000)
    c, _, _, _ = R.select_set(sub, R.OracleConfig(test="window"), n_threads=THREADS)
    assert np.array_equal(w["counts"][:6000], c)


_FULL = {}
# Oracle ranges of the full-size checks: every event of the 100k-event
# high-multiplicity workload (four ranges of 25k) and 250k events of the
# 4M-event mixture (five ranges of 50k spread over the batch).
FULL_RANGES = [("dense_100k", k * 25_000, 25_000) for k in range(4)] + \
              [("mixture_4m", first, 50_000) for first in (0, 1_000_000, 2_000_000, 3_000_000, 3_950_000)]


def full_size_results(torch, name):
    """The 100k-event high-multiplicity or the 4M-event mixture workload at
    full size: autotuned as the benchmark runs it (trig_autotune on the batch,
    then TRIG_EXEC_AUTOTUNE calls), and every other form, brute force
    included, on the same device buffers.  Computed once per module."""
    if name in _FULL:
        return _FULL[name]
    from paper_1810_11966_amd import trig
    s = synth.make_event_set(synth.WORKLOADS[name])
    print(f"[full] {name} generated events={s.n_events} hits={s.n_hits}", flush=True)
    off, x, y = to_dev(torch, s)
    trig.trig_autotune_reset()
    r, info = trig.autotune(off, x, y, test="msd", reps=1, compact=True, want_status=True)
    torch.cuda.synchronize()
    print(f"[full] {name} autotuned binned={info.binned} persistent={info.persistent} "
          f"shape={info.block_hits},{info.block_waves},{info.block_events}", flush=True)
    tuned = r.counts.cpu().numpy()
    del r
    res = {}
    for form in FORMS:
        print(f"[full] {name} form={form}", flush=True)
        g = trig.select(off, x, y, test="msd", form=form, compact=True, want_status=True)
        torch.cuda.synchronize()
        n = int(g.n_accepted.cpu().numpy()[0])
        res[form] = {"counts": g.counts.cpu().numpy(), "accept": g.accept.cpu().numpy(),
                     "ids": g.ids.cpu().numpy()[:n], "status": int(g.status.cpu().numpy()[0])}
        del g
    del off, x, y
    torch.cuda.empty_cache()
    trig.trig_autotune_reset()
    _FULL[name] = (s, tuned, res)
    return _FULL[name]


@pytest.mark.parametrize("name", ["dense_100k", "mixture_4m"])
def test_dense_and_mixture_full_size_all_forms(gpu, name):
    """At full size, every form equals GPU brute force (the plain one-wave-
    per-event kernel) on every event: counts, flags and accepted ids; the
    autotuned record's result too."""
    s, tuned, res = full_size_results(gpu, name)
    base = res["plain"]
    assert base["status"] == 0 and base["ids"].size > 0
    assert np.array_equal(base["ids"], np.flatnonzero(base["accept"]))
    assert np.array_equal(tuned, base["counts"])
    for form, r in res.items():
        assert np.array_equal(r["counts"], base["counts"]), form
        assert np.array_equal(r["accept"], base["accept"]), form
        assert np.array_equal(r["ids"], base["ids"]), form


@pytest.mark.parametrize("name,first,size", FULL_RANGES)
def test_dense_and_mixture_full_size_oracle(gpu, name, first, size):
    """The full-size GPU results against the oracle, event by event, over
    the ranges above (all 100k high-multiplicity events; 250k mixture events)."""
    s, tuned, res = full_size_results(gpu, name)
    sub = s.subset(first, size)
    print(f"[full] {name} oracle events [{first}, {first + size})", flush=True)
    c, a, _, _ = R.select_set(sub, n_threads=THREADS)
    for form in ("auto", "plain"):
        assert np.array_equal(res[form]["counts"][first:first + size], c), (name, form, first)
        assert np.array_equal(res[form]["accept"][first:first + size], a), (name, form, first)


def test_compaction_both_launch_paths(gpu):
    """Accepted-id lists on both sides of the compaction's launch split (4096
    blocks of 1024 events): below it each block sums the counts before it,
    above it a scan kernel runs.  Small events with many injected exact
    pairs, so that thousands of events are accepted; ids must be the ascending
    accepted events, and the oracle checks the counts of three ranges."""
    spec = synth.EventSetSpec(n_events=4_194_304 + 3000, hits_mean=1.0, p_inject=0.01, sigma=0.0, salt=77)
    s = synth.make_event_set(spec)
    for n in (4_194_304, s.n_events):
        sub = s.subset(0, n)
        print(f"[compact] events={n}", flush=True)
        r = run_gpu(gpu, sub, "msd", "pruned")
        assert r["ids"].size > 1000
        assert np.array_equal(r["ids"], np.flatnonzero(r["accept"]))
        for first in (0, n - 5000):
            part = sub.subset(first, 5000)
            c, a, _, _ = R.select_set(part, n_threads=THREADS)
            assert np.array_equal(r["counts"][first:first + 5000], c), (n, first)
            assert np.array_equal(r["accept"][first:first + 5000], a), (n, first)


# -------------------------------------------------------------- autotuner ---

@pytest.mark.parametrize("test", TESTS)
def test_autotune_records_and_matches_oracle(gpu, test):
    from paper_1810_11966_amd import trig
    trig.trig_autotune_reset()
    s = synth.concat([synth.make_event_set(synth.SMALL_10K),
                      synth.make_event_set(synth.DENSE_100K, n_events=300)])
    c, a, st, _ = oracle_result(s, oracle_cfg(test))
    off, x, y = to_dev(gpu, s)
    print(f"[autotune] {test} events={s.n_events} hits={s.n_hits}", flush=True)
    r, info = trig.autotune(off, x, y, test=test, reps=1, compact=True, want_status=True)
    gpu.cuda.synchronize()
    assert np.array_equal(r.counts.cpu().numpy(), c)
    assert np.array_equal(r.accept.cpu().numpy(), a)
    n = int(r.n_accepted.cpu().numpy()[0])
    assert np.array_equal(r.ids.cpu().numpy()[:n], R.accepted_ids(a))
    assert info.n_candidates == 1 + 3 * 2 * 4 * 2 + 2
    assert 0 < info.ms_best <= info.ms_rule
    if info.binned:
        assert info.block_hits == 0
    else:
        assert info.block_hits in (1024, 2048, 4096) and info.block_waves in (1, 2, 4)
        assert 1 <= info.block_events <= 128
    # later autotuned calls use the record; explicit block fields still win
    assert_parity(gpu, s, test, "auto", "autotuned")
    assert_parity(gpu, s, test, "auto", "autotuned+explicit", block_hits=1024, block_waves=1,
                  block_events=3)
    trig.trig_autotune_reset()
    assert_parity(gpu, s, test, "auto", "rule after reset")


def test_autotune_cache_file_round_trip(gpu, tmp_path):
    """A record made by trig_autotune survives trig_autotune_save, a reset
    and trig_autotune_load: the same shape is recorded again for this
    device, and autotuned calls with it match the oracle."""
    from paper_1810_11966_amd import trig
    trig.trig_autotune_reset()
    s = synth.make_event_set(synth.SMALL_10K, n_events=4000)
    off, x, y = to_dev(gpu, s)
    print(f"[autotune cache] events={s.n_events}", flush=True)
    _, info = trig.autotune(off, x, y, test="msd", reps=1)
    gpu.cuda.synchronize()
    rec = trig.autotune_lookup("msd", info.mult_class)
    assert rec is not None and rec["binned"] == info.binned and rec["persistent"] == info.persistent
    if not info.binned:
        assert (rec["block_hits"], rec["block_waves"]) == (info.block_hits, info.block_waves)
    path = tmp_path / "autotune.txt"
    trig.autotune_save(str(path))
    lines = path.read_text().splitlines()
    assert lines[0] == "trig-autotune-cache 1" and len(lines) == 2
    trig.trig_autotune_reset()
    assert trig.autotune_lookup("msd", info.mult_class) is None
    assert trig.autotune_load(str(path)) >= 1
    assert trig.autotune_lookup("msd", info.mult_class) == rec
    assert_parity(gpu, s, "msd", "auto", "autotuned from the cache file")
    trig.trig_autotune_reset()


# ---------------------------------------- two particles, decision only ---

def two_particle_oracle(s, test, **kw):
    cfg = oracle_cfg(test, **kw)
    c, _, st, _ = oracle_result(s, cfg)
    d = R.disjoint_accept(s.offsets, s.x, s.y, cfg, n_threads=THREADS)
    return c, d, st


def test_two_particle_acceptance_all_forms(gpu):
    """TRIG_ACCEPT_TWO_PARTICLES (two passing triplets with no hit in
    common, Sec. 3.1) in every form and test: flags and ids equal the
    oracle's pairwise comparison of the listed passing triplets, counts stay
    exact.  Events with duplicated hits and hits near the tracks give
    hundreds of events with two or more passing triplets that all share a
    hit."""
    from paper_1810_11966_amd import trig
    s = synth.concat([helpers.two_particle_events(3000, seed=5),
                      synth.make_event_set(synth.SMALL_10K, n_events=3000),
                      helpers.ragged_sizes_set([(70, 60, 90), (1, 300, 2), (40, 40, 600)], seed=3)])
    for test in TESTS:
        c, d, st = two_particle_oracle(s, test)
        assert d.sum() > 500 and ((c >= 2) & (d == 0)).sum() > 200
        for form in FORMS:
            print(f"[two particles] test={test} form={form}", flush=True)
            got = run_gpu(gpu, s, test, form, extra_flags=trig.TRIG_ACCEPT_TWO_PARTICLES)
            assert np.array_equal(got["counts"], c), (test, form)
            assert np.array_equal(got["accept"], d), (test, form, np.flatnonzero(got["accept"] != d)[:5])
            assert np.array_equal(got["ids"], R.accepted_ids(d)), (test, form)
            assert got["status"] == st


def test_two_particle_acceptance_dense_and_edges(gpu):
    """High multiplicity (events of the 100k-event workload, pairs injected)
    and the near-threshold and far-from-axis sets, two-particle mode."""
    from paper_1810_11966_amd import trig
    sets = {"dense": synth.make_event_set(synth.DENSE_100K, n_events=300),
            "near": helpers.near_threshold_events(200, 8, seed=31, rel=1e-6),
            "far": helpers.near_threshold_events(150, 8, seed=40, rel=1e-3, slope_max=25.0)}
    for name, s in sets.items():
        c, d, _ = two_particle_oracle(s, "msd")
        for form in ("plain", "pruned", "binned", "auto"):
            print(f"[two particles] {name} form={form}", flush=True)
            got = run_gpu(gpu, s, "msd", form, extra_flags=trig.TRIG_ACCEPT_TWO_PARTICLES)
            assert np.array_equal(got["counts"], c), (name, form)
            assert np.array_equal(got["accept"], d), (name, form)


def test_decision_only(gpu):
    """TRIG_DECISION_ONLY: counts are min(count, K) (K = min_triplets, or 2
    with two-particle acceptance), errors unchanged, flags those of the full
    count; forms may stop an event's search early."""
    from paper_1810_11966_amd import trig
    s = synth.concat([helpers.two_particle_events(1500, seed=8),
                      synth.make_event_set(synth.DENSE_100K, n_events=200),
                      synth.make_event_set(synth.SMALL_10K, n_events=2000)])
    for test in ("msd", "window"):
        for k in (0, 1, 2, 5):
            c, a, st, _ = oracle_result(s, oracle_cfg(test, min_triplets=k))
            for form in FORMS:
                print(f"[decision only] test={test} K={k} form={form}", flush=True)
                got = run_gpu(gpu, s, test, form, min_triplets=k, extra_flags=trig.TRIG_DECISION_ONLY)
                assert np.array_equal(got["counts"], np.where(c < 0, c, np.minimum(c, k))), (test, k, form)
                assert np.array_equal(got["accept"], a), (test, k, form)
                assert np.array_equal(got["ids"], R.accepted_ids(a)), (test, k, form)
        c, d, _ = two_particle_oracle(s, test)
        for form in ("plain", "persistent", "pruned", "binned"):
            got = run_gpu(gpu, s, test, form,
                          extra_flags=trig.TRIG_DECISION_ONLY | trig.TRIG_ACCEPT_TWO_PARTICLES)
            assert np.array_equal(got["counts"], np.where(c < 0, c, np.minimum(c, 2))), (test, form)
            assert np.array_equal(got["accept"], d), (test, form)


# ------------------------------------------------------------- per-hit z ---

def test_per_hit_z_all_forms(gpu):
    """Hits on staggered modules, each with its own z (trig_hits.z): every
    form against the oracle's per-triplet fit (Szz and its reciprocal per
    triplet) and slope window, on the 10k workload, near-threshold tracks on
    all stagger combinations, events with many passing triplets, ragged layer
    sizes on both sides of the one-pass limits (either layer in the lanes, or
    several passes), and events whose z no slope bound covers (0, negative,
    NaN, infinite, tiny z under huge coordinates: the every-triplet path)."""
    sets = {"small_10k": synth.staggered(synth.make_event_set(synth.SMALL_10K, n_events=4000)),
            "near": helpers.near_threshold_events_z(300, 6, seed=3, rel=1e-4),
            "near 1e-6": helpers.near_threshold_events_z(200, 6, seed=4, rel=1e-6),
            "two particles": synth.staggered(helpers.two_particle_events(1500, seed=6)),
            "ragged": synth.staggered(helpers.ragged_sizes_set(
                [sz for n in (1, 2, 31, 33, 63, 64, 65, 129) for sz in ((n, 5, 7), (5, n, 7), (n, n, 3))], seed=11)),
            "odd z": helpers.odd_z_events(5)}
    for name, s in sets.items():
        for test in ("msd", "window"):
            with np.errstate(all="ignore"):
                c = oracle_result(s, oracle_cfg(test))[0]
            assert c.sum() > 0, (name, test)
            for form in FORMS:
                print(f"[per-hit z] {name} test={test} form={form}", flush=True)
                with np.errstate(all="ignore"):
                    assert_parity(gpu, s, test, form, f"per-hit z {name}")


def test_per_hit_z_at_layer_positions_and_refusals(gpu):
    """Per-hit z equal to the layer positions gives the layer path's counts
    (the reciprocal of Szz is the same binary32 number at this geometry);
    the basis form with per-hit z is refused before any launch."""
    from paper_1810_11966_amd import trig
    s = synth.make_event_set(synth.SMALL_10K, n_events=3000)
    n = np.diff(s.offsets.astype(np.int64))
    zl = np.asarray(synth.Z_LAYERS, np.float32)[np.repeat(np.tile(np.arange(3), s.n_events), n)]
    sz = synth.EventSet(s.offsets, s.x, s.y, s.n_tracks, z=zl)
    for form in ("plain", "pruned", "binned"):
        assert np.array_equal(run_gpu(gpu, sz, "msd", form)["counts"], run_gpu(gpu, s, "msd", form)["counts"])
    with pytest.raises(trig.TrigError) as err:
        run_gpu(gpu, sz, "msd_basis", "plain")
    assert err.value.code == trig.TRIG_EUNSUPPORTED


def test_per_hit_z_two_particles_and_decision_only(gpu):
    from paper_1810_11966_amd import trig
    s = synth.concat([synth.staggered(helpers.two_particle_events(1500, seed=9)), helpers.odd_z_events(7)])
    for test in ("msd", "window"):
        cfg = oracle_cfg(test)
        with np.errstate(all="ignore"):
            c = oracle_result(s, cfg)[0]
            d = R.disjoint_accept(s.offsets, s.x, s.y, cfg, n_threads=THREADS, z=s.z)
        assert d.sum() > 100 and ((c >= 2) & (d == 0)).sum() > 50
        for form in ("plain", "persistent", "pruned", "auto"):
            print(f"[per-hit z] two particles test={test} form={form}", flush=True)
            got = run_gpu(gpu, s, test, form, extra_flags=trig.TRIG_ACCEPT_TWO_PARTICLES)
            assert np.array_equal(got["counts"], c), (test, form)
            assert np.array_equal(got["accept"], d), (test, form)
            got = run_gpu(gpu, s, test, form, extra_flags=trig.TRIG_DECISION_ONLY, min_triplets=3)
            assert np.array_equal(got["counts"], np.where(c < 0, c, np.minimum(c, 3))), (test, form)
