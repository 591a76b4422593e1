"""Event building from a time-ordered hit stream, on the CPU: the oracle
against hand-worked cases, its whole-array form against its hit-by-hit
form, and the free-stream generator against the events it was made from."""
import numpy as np

from oracle import reference as R
from paper_1810_11966_amd import synth

I64_MIN, I64_MAX = -(2**63), 2**63 - 1


def test_build_events_hand_cases():
    cases = [
        ([], 5, [0], 0),
        ([7], 0, [0, 1], 0),
        ([0, 10, 20], 10, [0, 3], 0),              # a difference equal to the gap stays in the event
        ([0, 10, 20], 9, [0, 1, 2, 3], 0),
        ([5, 5, 5], 0, [0, 3], 0),                  # equal times never start an event
        ([0, 100, 50, 200], 10, [0, 1, 3, 4], 1),   # a decrease: status, and no start at 50
        ([I64_MIN, I64_MAX], I64_MAX, [0, 1, 2], 0),  # difference 2^64 - 1, taken exactly
        ([I64_MIN, I64_MAX], 0, [0, 1, 2], 0),
        ([-5, -3], 1, [0, 1, 2], 0),
        ([-5, -3], 2, [0, 2], 0),
        ([1, 2, 4, 8, 16, 32], 3, [0, 3, 4, 5, 6], 0),
    ]
    for t, gap, want, st in cases:
        got, status = R.build_events(np.asarray(t, dtype=np.int64), gap)
        assert got.tolist() == want and status == st, (t, gap)
        got2, status2 = R.build_events_numpy(np.asarray(t, dtype=np.int64), gap)
        assert got2.tolist() == want and status2 == st, (t, gap)


def test_build_events_numpy_matches_hit_by_hit():
    rng = np.random.default_rng(3)
    for trial in range(60):
        n = int(rng.integers(0, 3000))
        steps = rng.choice([0, 1, 2, 5, 30, 1000], n)
        t = np.cumsum(steps).astype(np.int64) + int(rng.integers(-(2**40), 2**40))
        if trial % 3 == 1 and n > 10:
            t[rng.integers(0, n, 5)] -= 50                       # a few decreases
        if trial % 5 == 2 and n > 2:
            t[: n // 2] = I64_MIN + np.arange(n // 2)            # extremes
            t[n // 2:] = I64_MAX - np.arange(n - n // 2)[::-1]
        gap = int(rng.choice([0, 1, 4, 29, 2**62]))
        a, sa = R.build_events(t, gap)
        b, sb = R.build_events_numpy(t, gap)
        assert np.array_equal(a, b) and sa == sb, trial


def test_free_stream_recovers_separated_events():
    """Interactions at least spread + gap + 1 ns apart: building events with
    that gap gives back the generating events' offsets, each event with its
    own hits."""
    base = synth.make_event_set(synth.SMALL_10K, n_events=400)
    raw = synth.embed_raw(base, other_mean=20.0, shuffle=False, seed=2, square=True)
    s = synth.free_stream(raw, rate_hz=1e7, spread_ns=10, min_spacing_ns=10 + 25 + 1, seed=4)
    assert np.all(np.diff(s.t) >= 0)
    off, st = R.build_events_numpy(s.t, 25)
    assert st == 0
    assert np.array_equal(off, raw.offsets)
    # each built event holds its generating event's hits (in time order)
    assert np.array_equal(s.event, np.repeat(np.arange(raw.n_events), np.diff(raw.offsets)))


def test_free_stream_pile_up_merges_events():
    """Poisson interactions at 10 MHz with 10 ns of time spread: events that
    start within 10 + gap ns of the previous one's last hit merge; every
    built event is a run of whole generating events."""
    base = synth.make_event_set(synth.SMALL_10K, n_events=2000)
    raw = synth.embed_raw(base, other_mean=5.0, shuffle=False, seed=3, square=True)
    s = synth.free_stream(raw, rate_hz=1e7, spread_ns=10, seed=5)
    assert np.all(np.diff(s.t) >= 0)
    off, st = R.build_events_numpy(s.t, 5)
    assert st == 0 and 1 < len(off) - 1 < raw.n_events
    for e in range(len(off) - 1):
        ev = s.event[off[e]:off[e + 1]]
        # a built event holds every hit of each generating event it touches
        for g in np.unique(ev):
            assert (s.event == g).sum() == (ev == g).sum()
