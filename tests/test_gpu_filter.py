"""GPU parity of the trigger-station filter (include/trig_filter.h) against
the oracle, bit-exact: offsets, x, y and the status word; edge cases; the
filtered output feeding the selection.  Every case prints its name first."""
import numpy as np
import pytest

from oracle import reference as R
from paper_1810_11966_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_11966_amd import trig
    trig.load()
    return torch


def run_filter(torch, off, st, x, y, layers, capacity=None, misalign=False):
    from paper_1810_11966_amd import filter as F
    d = torch.device("cuda:0")
    t_off = torch.from_numpy(np.asarray(off, np.int64)).to(d)
    st = np.asarray(st, np.uint8)
    if misalign:
        # station numbers one byte past a 4-byte boundary: the byte-load path
        buf = torch.zeros(len(st) + 1, dtype=torch.uint8, device=d)
        buf[1:] = torch.from_numpy(st).to(d)
        t_st = buf[1:]
    else:
        t_st = torch.from_numpy(st).to(d)
    t_x = torch.from_numpy(np.asarray(x, np.float32)).to(d)
    t_y = torch.from_numpy(np.asarray(y, np.float32)).to(d)
    if capacity is None:
        capacity = int(np.isin(st, layers).sum())
    r = F.filter_stations(t_off, t_st, t_x, t_y, layers, capacity)
    torch.cuda.synchronize()
    lo = r.layer_offsets.cpu().numpy()
    n = int(lo[-1])  # hits written (the total, or the capacity when it is smaller)
    return lo, r.x.cpu().numpy()[:n], r.y.cpu().numpy()[:n], int(r.status.cpu().numpy()[0])


def assert_filter_parity(torch, label, off, st, x, y, layers=synth.TRIGGER_STATIONS, **kw):
    print(f"[filter] {label} events={len(off) - 1} hits={len(st)}", flush=True)
    lo, fx, fy, status = run_filter(torch, off, st, x, y, layers, **kw)
    elo, ex, ey, est = R.filter_stations(off, st, x, y, layers)
    assert np.array_equal(lo, elo), label
    assert np.array_equal(fx, ex) and np.array_equal(fy, ey), label
    assert status == est, label
    return lo, fx, fy


def test_small_sets_both_orders(gpu):
    base = synth.make_event_set(synth.SMALL_10K)
    for shuffle in (True, False):
        raw = synth.embed_raw(base, other_mean=25.0, shuffle=shuffle, seed=1)
        lo, fx, fy = assert_filter_parity(gpu, f"small_10k shuffle={shuffle}", raw.offsets, raw.station,
                                          raw.x, raw.y)
        assert np.array_equal(lo, base.offsets) and np.array_equal(fx, base.x)
        assert_filter_parity(gpu, f"small_10k misaligned shuffle={shuffle}", raw.offsets, raw.station, raw.x,
                             raw.y, misalign=True)


def test_event_sizes_and_layers(gpu):
    rng = np.random.default_rng(5)
    sizes = [0, 1, 2, 3, 4, 5, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 5000, 9001]
    lens = rng.choice(sizes, 700)
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    st = rng.integers(0, 16, int(off[-1])).astype(np.uint8)
    st[: int(off[-1]) // 7] = 255  # also station 255
    x = rng.standard_normal(int(off[-1])).astype(np.float32)
    y = rng.standard_normal(int(off[-1])).astype(np.float32)
    for layers in ((13, 14, 15), (0, 255, 7), (15, 0, 3)):
        assert_filter_parity(gpu, f"sizes layers={layers}", off, st, x, y, layers)
        assert_filter_parity(gpu, f"sizes misaligned layers={layers}", off, st, x, y, layers, misalign=True)
    # every hit a trigger hit; no trigger hit at all
    st_all = np.resize(np.array([13, 14, 15], np.uint8), int(off[-1]))
    assert_filter_parity(gpu, "all trigger hits", off, st_all, x, y)
    assert_filter_parity(gpu, "no trigger hit", off, np.full(int(off[-1]), 3, np.uint8), x, y)


def test_malformed_empty_and_capacity(gpu):
    base = synth.make_event_set(synth.SMALL_10K, n_events=500)
    raw = synth.embed_raw(base, other_mean=10.0, seed=2)
    off = raw.offsets.copy()
    off[10] = off[11] + 1          # event 9 ends before it starts (and event 10 starts after it ends)
    off[200] = -3                  # negative start of event 200 (and end of event 199)
    assert_filter_parity(gpu, "malformed", off, raw.station, raw.x, raw.y)
    # an empty batch writes the single offset 0
    lo, fx, _, status = run_filter(gpu, np.zeros(1, np.int64), np.zeros(0, np.uint8), np.zeros(0, np.float32),
                                   np.zeros(0, np.float32), (13, 14, 15), capacity=0)
    assert lo.tolist() == [0] and status == 0
    # too small an output: the status bit, and nothing written past it
    total = int(base.offsets[-1])
    cap = total // 2
    print(f"[filter] capacity {cap} of {total}", flush=True)
    lo, fx, fy, status = run_filter(gpu, raw.offsets, raw.station, raw.x, raw.y, (13, 14, 15), capacity=cap)
    assert status & 4
    assert np.array_equal(fx, base.x[:cap]) and np.array_equal(fy, base.y[:cap])
    assert lo[-1] == cap
    ok = base.offsets <= cap
    assert np.array_equal(lo[ok], base.offsets[ok])


def test_filtered_events_feed_the_selection(gpu):
    """The filter's output, passed as it is to trig_select, gives the same
    counts as the selection on the original trigger-layer events (100k
    events of the 1M-event workload's recipe, hits in detector order, about
    470 hits per event)."""
    from paper_1810_11966_amd import trig
    base = synth.make_event_set(synth.MEDIUM_1M, n_events=100_000)
    raw = synth.embed_raw(base, other_mean=30.0, shuffle=False, square=True, seed=4)
    print(f"[filter] pipeline events={raw.n_events} hits={raw.n_hits}", flush=True)
    from paper_1810_11966_amd import filter as F
    d = gpu.device("cuda:0")
    t = [gpu.from_numpy(a).to(d) for a in (raw.offsets, raw.station, raw.x, raw.y)]
    r = F.filter_stations(*t, raw.layers, base.n_hits)
    sel = trig.select(r.layer_offsets, r.x[:base.n_hits], r.y[:base.n_hits], form="auto", compact=True)
    ref = trig.select(*[gpu.from_numpy(a).to(d) for a in (base.offsets, base.x, base.y)], form="auto")
    gpu.cuda.synchronize()
    assert int(r.status.cpu()[0]) == 0
    assert np.array_equal(r.layer_offsets.cpu().numpy(), base.offsets)
    assert np.array_equal(sel.counts.cpu().numpy(), ref.counts.cpu().numpy())
    sub = base.subset(0, 5000)
    c, _, _, _ = R.select_set(sub, n_threads=8)
    assert np.array_equal(sel.counts.cpu().numpy()[:5000], c)


def window_records(off, st, layers):
    """Per event, the lane windows the count kernel records: windows of 32
    hits from the event's first hit rounded down to a multiple of 16, each
    counted when it holds a trigger hit of the event."""
    trig = np.isin(st, np.asarray(layers, np.uint8))
    recs = np.zeros(len(off) - 1, np.int64)
    for e in range(len(off) - 1):
        a, b = int(off[e]), int(off[e + 1])
        base = a & ~15
        while base < b:
            recs[e] += bool(trig[max(a, base):min(b, base + 32)].any())
            base += 32
    return recs


def test_trigger_hit_lists_at_capacity(gpu):
    """The count kernel keeps, per group of 4 events (events w, w+4, w+8,
    w+12 of a block of 16), up to 128 records of 32-hit windows with trigger
    hits for the scatter; a group that needs more is scattered from a second
    pass over its station numbers.  Groups at 127, 128 and 129 records, in
    both paths, bit-exact against the oracle."""
    rng = np.random.default_rng(9)
    n_ev = 32
    lens = np.full(n_ev, 1024)             # multiples of 16: every event's windows start at its first hit
    lens[1 + 4 * 3] = 1024 + 16            # group 1 of block 0: 129 records
    lens[16 + 2 + 4 * 2] = 1024 - 32       # group 2 of block 1: 127 records
    lens[n_ev - 1] = 1001                  # a ragged last event
    off = np.zeros(n_ev + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    layers = (13, 14, 15)
    st = rng.choice(np.array(layers, np.uint8), int(off[-1]))
    # event 16 + 3 (group 3 of block 1): every other window without a trigger
    # hit, and the rest a mix of trigger and other stations
    a = int(off[19])
    for k in range(32):
        w = st[a + 32 * k:a + 32 * k + 32]
        w[:] = rng.integers(0, 12, 32) if k % 2 else np.where(rng.random(32) < 0.5, w, 3)
    recs = window_records(off, st, layers)
    groups = recs.reshape(2, 4, 4).sum(axis=1)  # [block, w]
    assert groups[0, 0] == 128 and groups[0, 1] == 129 and groups[1, 2] == 127 and groups[1, 3] == 112
    x = rng.standard_normal(len(st)).astype(np.float32)
    y = rng.standard_normal(len(st)).astype(np.float32)
    assert_filter_parity(gpu, "lists at capacity", off, st, x, y, layers)
    assert_filter_parity(gpu, "lists at capacity misaligned", off, st, x, y, layers, misalign=True)
