"""GPU tests of the serving runtime: each slice's result equals trig_select's
(and the oracle's) alone and in a mix; slices overlap on the device;
admission by HBM footprint; backpressure; a malformed slice does not affect
the others."""
import numpy as np
import pytest

from oracle import reference as R
from paper_1810_11966_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srv_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_11966_amd import serve, trig
    trig.load()
    return serve


def make_slices(n, seed, lo=2000, hi=60000):
    rng = np.random.default_rng(seed)
    pool = synth.make_event_set(synth.MEDIUM_1M, n_events=hi * 3)
    out = []
    for _ in range(n):
        size = int(rng.integers(lo, hi + 1))
        first = int(rng.integers(0, pool.n_events - size))
        out.append(pool.subset(first, size))
    return out


def direct_counts(s):
    import torch
    from paper_1810_11966_amd import trig
    dev = [torch.from_numpy(a).cuda() for a in (s.offsets, s.x, s.y)]
    r = trig.select(*dev, form="pruned", compact=True)
    torch.cuda.synchronize()
    return r.counts.cpu().numpy()


def test_alone_equals_mix_equals_oracle(srv_mod):
    slices = make_slices(12, seed=1)
    print("[serve] alone", flush=True)
    alone = []
    with srv_mod.Server(1 << 30, 1 << 30, n_streams=4) as srv:
        for s in slices:
            t = srv.submit(s.offsets, s.x, s.y)
            f = srv.poll(60000)
            assert f is not None and f.ticket == t and f.status == 0
            alone.append(f)
    print("[serve] mix", flush=True)
    with srv_mod.Server(1 << 30, 1 << 30, n_streams=4) as srv:
        # stage every slice first, then release them together: up to four
        # are on the device at once
        srv.pause(True)
        tickets = {i: srv.submit(s.offsets, s.x, s.y) for i, s in enumerate(slices)}
        assert all(t is not None for t in tickets.values())
        assert srv.stats().in_flight == 0
        srv.pause(False)
        done = {}
        while len(done) < len(slices):
            f = srv.poll(60000)
            assert f is not None
            done[f.ticket] = f
        st = srv.stats()
    assert st.completed == len(slices) and st.max_in_flight >= 2
    for i, s in enumerate(slices):
        mix = done[tickets[i]]
        assert np.array_equal(mix.counts, alone[i].counts), i
        assert np.array_equal(mix.ids, alone[i].ids), i
        assert np.array_equal(mix.counts, direct_counts(s)), i
    for i in (0, 5):
        c, a, _, _ = R.select_set(slices[i], n_threads=8)
        assert np.array_equal(alone[i].counts, c)
        assert np.array_equal(alone[i].ids, R.accepted_ids(a))
    # overlap: some slice was admitted before the previous one finished
    fin = sorted(done.values(), key=lambda f: f.t_admit)
    assert any(fin[k + 1].t_admit < fin[k].t_done for k in range(len(fin) - 1))


def test_admission_by_footprint_and_backpressure(srv_mod):
    slices = make_slices(8, seed=2, lo=30000, hi=60000)
    big = max(s.n_hits for s in slices)
    # HBM for about one slice: at most one in flight however many streams
    hbm = int(big * 8 * 1.6) + (4 << 20)
    with srv_mod.Server(hbm, 1 << 30, n_streams=4) as srv:
        done, tickets, _ = srv_mod.run_stream(srv, slices, np.zeros(len(slices)), pace=False)
        st = srv.stats()
        assert st.completed == len(slices)
        assert st.hbm_peak <= hbm
        for i, s in enumerate(slices):
            assert np.array_equal(done[tickets[i]].counts, direct_counts(s))
        # a slice larger than the whole arena is refused, not queued forever
        huge = synth.make_event_set(synth.MEDIUM_1M, n_events=200000)
        with pytest.raises(Exception):
            srv.submit(huge.offsets, huge.x, huge.y)
    # tiny pinned staging: submit reports busy until results are polled
    with srv_mod.Server(1 << 30, int(big * 8 * 1.5) + (2 << 20), n_streams=2, max_pending=2) as srv:
        done, tickets, _ = srv_mod.run_stream(srv, slices, np.zeros(len(slices)), pace=False)
        st = srv.stats()
        assert st.completed == len(slices) and st.rejected_busy > 0
        for i, s in enumerate(slices):
            assert np.array_equal(done[tickets[i]].counts, direct_counts(s))


def test_malformed_slice_is_isolated(srv_mod):
    slices = make_slices(4, seed=3, lo=3000, hi=8000)
    bad = slices[1]
    off = bad.offsets.copy()
    off[3 * 7 + 1] = off[3 * 7 + 2] + 1
    bad = synth.EventSet(off, bad.x, bad.y, bad.n_tracks)
    mixed = [slices[0], bad, slices[2], slices[3]]
    with srv_mod.Server(1 << 28, 1 << 28, n_streams=3) as srv:
        done, tickets, _ = srv_mod.run_stream(srv, mixed, np.zeros(4), pace=False)
    fb = done[tickets[1]]
    assert fb.status == 0 and fb.counts[7] == -1 and (fb.event_status & 1)
    for i in (0, 2, 3):
        assert np.array_equal(done[tickets[i]].counts, direct_counts(mixed[i]))
        assert done[tickets[i]].event_status == 0


def test_paced_stream_latency(srv_mod):
    """A short Poisson stream at a fixed offered load: all slices finish,
    latencies are positive and ordered as timestamps should be."""
    slices = make_slices(10, seed=4, lo=10000, hi=100000)
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(0.004, len(slices)))
    with srv_mod.Server(1 << 31, 1 << 31, n_streams=4) as srv:
        done, tickets, wall = srv_mod.run_stream(srv, slices, arrivals, pace=True)
    lat = np.array([f.t_done - f.t_submit for f in done.values()])
    assert len(done) == len(slices) and (lat > 0).all()
    assert all(f.t_submit <= f.t_admit <= f.t_done for f in done.values())
