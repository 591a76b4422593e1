"""Seeded synthetic trigger-station events.

This module only draws hit coordinates; it holds none of the selection
arithmetic.  Both the CPU oracle (through the tests and the benchmark) and the
GPU library consume exactly the bytes it produces.

Geometry follows the paper's description of the MUCH trigger station (Sec. 2
and Sec. 3.1): three detector layers 10 cm apart behind the last absorber, hits
carrying (x, y) per layer, an uninstrumented hole around the beam pipe and an
outer edge.  Multiplicities are per-layer Poisson draws.  A fraction of events
receives muon pairs: straight tracks from the target at the origin, seen once
per layer and Gaussian-smeared.

Layout (the library's input format): ``offsets`` is int32[3*E+1], event-major
then layer, so the hits of event e in layer l are
``[offsets[3e+l], offsets[3e+l+1])``; ``x`` and ``y`` are float32[H] in cm.

Determinism: events are generated in fixed chunks of ``CHUNK`` events; chunk c
of a set draws from ``numpy.random.default_rng([seed, salt, c])``.  The result
depends only on (spec, seed), never on how many processes generate it.
"""
from __future__ import annotations

import hashlib
import os
import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

CHUNK = 1 << 16
Z_LAYERS = (400.0, 410.0, 420.0)


@dataclass(frozen=True)
class EventSetSpec:
    """Recipe for one synthetic event set.

    hits_mean: Poisson mean of noise hits per layer (constant over events), or
      None to use the minimum-bias-like mixture
      ``mean_e = mixture_peak * (1 - b**2)`` with ``b ~ U[0, 1]``.
    p_inject: probability that an event receives muon pairs.
    pairs: inclusive range of the number of pairs given to an injected event.
    sigma: Gaussian smearing of each injected hit coordinate (cm).
    r_min, r_max: annulus of noise hits (cm); also bounds the track acceptance.
    z: layer positions (cm); only used to place injected hits.
    salt: distinguishes sets that share a seed.
    """

    n_events: int
    hits_mean: Optional[float] = 8.0
    mixture_peak: float = 0.0
    p_inject: float = 0.05
    pairs: tuple = (1, 1)
    sigma: float = 0.3
    r_min: float = 20.0
    r_max: float = 200.0
    z: tuple = Z_LAYERS
    salt: int = 0


# The five workloads: small oracle-checkable set, the plain-vs-batched set,
# the uneven mixture, the serving stream's per-slice recipe and the
# high-multiplicity stress set.
SMALL_10K = EventSetSpec(n_events=10_000, hits_mean=8.0, p_inject=0.05, salt=1)
MEDIUM_1M = EventSetSpec(n_events=1_000_000, hits_mean=30.0, p_inject=0.01, salt=2)
MIXTURE_4M = EventSetSpec(n_events=4_000_000, hits_mean=None, mixture_peak=120.0,
                          p_inject=0.01, salt=3)
SLICE_RECIPE = EventSetSpec(n_events=0, hits_mean=30.0, p_inject=0.01, salt=4)
DENSE_100K = EventSetSpec(n_events=100_000, hits_mean=200.0, p_inject=0.10,
                          pairs=(1, 3), salt=5)

WORKLOADS = {
    "small_10k": SMALL_10K,
    "medium_1m": MEDIUM_1M,
    "mixture_4m": MIXTURE_4M,
    "dense_100k": DENSE_100K,
}


@dataclass
class EventSet:
    offsets: np.ndarray          # int32[3E+1]
    x: np.ndarray                # float32[H]
    y: np.ndarray                # float32[H]
    n_tracks: np.ndarray         # int8[E], injected tracks per event
    spec: Optional[EventSetSpec] = None
    seed: int = 0
    meta: dict = field(default_factory=dict)
    z: Optional[np.ndarray] = None  # float32[H]: per-hit z (cm), or None for the layer positions

    @property
    def n_events(self) -> int:
        return (len(self.offsets) - 1) // 3

    @property
    def n_hits(self) -> int:
        return int(len(self.x))

    def layer_counts(self) -> np.ndarray:
        """int64[E, 3] hits per event and layer."""
        return np.diff(self.offsets.astype(np.int64)).reshape(-1, 3)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.offsets, self.x, self.y) + ((self.z,) if self.z is not None else ()):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def subset(self, first: int, count: int) -> "EventSet":
        """Events [first, first+count) as a self-contained set (offsets rebased)."""
        lo = int(self.offsets[3 * first])
        hi = int(self.offsets[3 * (first + count)])
        off = (self.offsets[3 * first: 3 * (first + count) + 1].astype(np.int64) - lo)
        return EventSet(off.astype(np.int32), self.x[lo:hi].copy(), self.y[lo:hi].copy(),
                        self.n_tracks[first:first + count].copy(), self.spec, self.seed,
                        z=None if self.z is None else self.z[lo:hi].copy())


def _track_tan_range(spec: EventSetSpec):
    # Unsmeared track radius r_l = tan(theta) * z_l must stay inside the
    # annulus at every layer: the nearest layer bounds it from below, the
    # farthest from above.
    zmin, zmax = min(spec.z), max(spec.z)
    return spec.r_min / zmin, spec.r_max / zmax


def _gen_chunk(spec: EventSetSpec, seed: int, chunk: int, n_ev: int):
    rng = np.random.default_rng([seed, spec.salt, chunk])
    if spec.hits_mean is None:
        b = rng.random(n_ev)
        lam = spec.mixture_peak * (1.0 - b * b)
        noise = rng.poisson(np.repeat(lam, 3).reshape(n_ev, 3))
    else:
        noise = rng.poisson(spec.hits_mean, size=(n_ev, 3))
    inj = rng.random(n_ev) < spec.p_inject
    lo, hi = spec.pairs
    npairs = np.where(inj, rng.integers(lo, hi + 1, size=n_ev), 0)
    ntr = (2 * npairs).astype(np.int64)
    counts = noise + ntr[:, None]
    seg_len = counts.reshape(-1)
    seg_end = np.cumsum(seg_len)
    seg_start = seg_end - seg_len
    n_hits = int(seg_end[-1]) if len(seg_end) else 0

    x = np.empty(n_hits, dtype=np.float64)
    y = np.empty(n_hits, dtype=np.float64)

    # Noise hits: uniform in area over the annulus.
    is_track = np.zeros(n_hits, dtype=bool)
    seg_tr = np.repeat(ntr, 3)
    if n_hits:
        # mark the last seg_tr positions of each segment as track slots
        tr_total = int(seg_tr.sum())
        if tr_total:
            seg_of_tr = np.repeat(np.arange(len(seg_len)), seg_tr)
            rank = np.arange(tr_total) - np.repeat(np.cumsum(seg_tr) - seg_tr, seg_tr)
            pos = seg_end[seg_of_tr] - seg_tr[seg_of_tr] + rank
            is_track[pos] = True
        n_noise = n_hits - int(is_track.sum())
        r = np.sqrt(rng.uniform(spec.r_min ** 2, spec.r_max ** 2, size=n_noise))
        phi = rng.uniform(0.0, 2.0 * np.pi, size=n_noise)
        noise_idx = np.flatnonzero(~is_track)
        x[noise_idx] = r * np.cos(phi)
        y[noise_idx] = r * np.sin(phi)

        if tr_total:
            # Tracks: isotropic in solid angle inside the acceptance cone.
            n_trk = int(ntr.sum())
            tmin, tmax = _track_tan_range(spec)
            cmax, cmin = 1.0 / math.sqrt(1 + tmin * tmin), 1.0 / math.sqrt(1 + tmax * tmax)
            cos_t = rng.uniform(cmin, cmax, size=n_trk)
            tan_t = np.sqrt(1.0 - cos_t * cos_t) / cos_t
            phi_t = rng.uniform(0.0, 2.0 * np.pi, size=n_trk)
            ev_of_trk = np.repeat(np.arange(n_ev), ntr)
            rank_in_ev = np.arange(n_trk) - np.repeat(np.cumsum(ntr) - ntr, ntr)
            for layer in range(3):
                zl = spec.z[layer]
                seg = 3 * ev_of_trk + layer
                pos = seg_end[seg] - ntr[ev_of_trk] + rank_in_ev
                x[pos] = tan_t * np.cos(phi_t) * zl + rng.normal(0.0, 1.0, n_trk) * spec.sigma
                y[pos] = tan_t * np.sin(phi_t) * zl + rng.normal(0.0, 1.0, n_trk) * spec.sigma

            # Move the appended track hits to uniformly random slots of their
            # layer segment (the tail steps of a Fisher-Yates shuffle).
            for k in range(int(seg_tr.max())):
                segs = np.flatnonzero(seg_tr > k)
                m = seg_end[segs] - seg_tr[segs] + k
                q = seg_start[segs] + np.floor(rng.random(len(segs)) * (m - seg_start[segs] + 1)).astype(np.int64)
                xm, ym = x[m].copy(), y[m].copy()
                x[m], y[m] = x[q], y[q]
                x[q], y[q] = xm, ym

    return (seg_len, x.astype(np.float32), y.astype(np.float32), ntr.astype(np.int8))


def make_event_set(spec: EventSetSpec, seed: int = 0, n_events: Optional[int] = None) -> EventSet:
    """Generate ``spec`` (optionally only its first ``n_events`` events)."""
    n = spec.n_events if n_events is None else int(n_events)
    n_chunks = (n + CHUNK - 1) // CHUNK
    jobs = [(c, min(CHUNK, n - c * CHUNK)) for c in range(n_chunks)]
    # Chunks draw from independent streams, so threads give the same bytes.
    workers = max(1, min(8, len(os.sched_getaffinity(0)), n_chunks))
    if workers > 1:
        with ThreadPoolExecutor(workers) as pool:
            parts = list(pool.map(lambda job: _gen_chunk(spec, seed, job[0], job[1]), jobs))
    else:
        parts = [_gen_chunk(spec, seed, c, n_ev) for c, n_ev in jobs]
    seg_lens = [q[0] for q in parts]
    xs = [q[1] for q in parts]
    ys = [q[2] for q in parts]
    ntrs = [q[3] for q in parts]
    if n == 0:
        return EventSet(np.zeros(1, np.int32), np.zeros(0, np.float32), np.zeros(0, np.float32),
                        np.zeros(0, np.int8), spec, seed)
    seg = np.concatenate(seg_lens)
    off = np.zeros(len(seg) + 1, dtype=np.int64)
    np.cumsum(seg, out=off[1:])
    if off[-1] > np.iinfo(np.int32).max:
        raise ValueError("event set exceeds int32 hit offsets")
    return EventSet(off.astype(np.int32), np.concatenate(xs), np.concatenate(ys),
                    np.concatenate(ntrs), spec, seed)


def from_layers(events) -> EventSet:
    """Build a set from explicit hits: ``events`` is a list of events, each a
    list of three sequences of (x, y) pairs (layer 0, 1, 2)."""
    off = [0]
    xs, ys = [], []
    for ev in events:
        if len(ev) != 3:
            raise ValueError("each event needs exactly three layers")
        for layer in ev:
            for (hx, hy) in layer:
                xs.append(hx); ys.append(hy)
            off.append(len(xs))
    return EventSet(np.asarray(off, np.int32), np.asarray(xs, np.float32).reshape(-1),
                    np.asarray(ys, np.float32).reshape(-1), np.zeros(len(events), np.int8))


def concat(sets) -> EventSet:
    """Concatenate event sets into one batch (offsets rebased).  Per-hit z
    is kept if every set has it."""
    sets = list(sets)
    offs, xs, ys, nts = [np.zeros(1, np.int64)], [], [], []
    base = 0
    for s in sets:
        offs.append(s.offsets[1:].astype(np.int64) + base)
        base += s.n_hits
        xs.append(s.x); ys.append(s.y); nts.append(s.n_tracks)
    z = None
    if sets and all(s.z is not None for s in sets):
        z = np.concatenate([s.z for s in sets])
    return EventSet(np.concatenate(offs).astype(np.int32),
                    np.concatenate(xs) if xs else np.zeros(0, np.float32),
                    np.concatenate(ys) if ys else np.zeros(0, np.float32),
                    np.concatenate(nts) if nts else np.zeros(0, np.int8), z=z)


def staggered(s: EventSet, z=Z_LAYERS, dz: float = 0.75, n_sectors: int = 16) -> EventSet:
    """The events of ``s`` (generated at the layer positions ``z``) on
    staggered modules: a hit in azimuthal sector k of 2 pi / n_sectors sits at
    z_l - dz for even k and z_l + dz for odd k (overlapping module rows, as
    each hit carries its own position, Sec. 3.2 last paragraph), and is moved
    along its line of sight from the target to that z, so that a straight
    track from the target stays one.  Returns a set with per-hit z."""
    n = np.diff(s.offsets.astype(np.int64))
    layer = np.repeat(np.tile(np.arange(3), s.n_events), n)
    x = s.x.astype(np.float64)
    y = s.y.astype(np.float64)
    sector = np.floor((np.arctan2(y, x) + np.pi) / (2 * np.pi / n_sectors)).astype(np.int64) % n_sectors
    zl = np.asarray(z, np.float64)[layer]
    zh = zl + np.where(sector % 2 == 0, -dz, dz)
    f = zh / zl
    return EventSet(s.offsets.copy(), (x * f).astype(np.float32), (y * f).astype(np.float32), s.n_tracks.copy(),
                    s.spec, s.seed, z=zh.astype(np.float32))


def slice_stream(n_slices: int, seed: int = 0, offered_rate: float = 1e7,
                 min_events: int = 10_000, max_events: int = 1_000_000,
                 recipe: EventSetSpec = SLICE_RECIPE):
    """Serving workload: slice sizes U{min..max} events and Poisson arrival
    times whose rate makes the offered load ``offered_rate`` events/s.

    Returns (sizes int64[n], arrival_s float64[n], per-slice seeds int64[n]);
    slice i is ``make_event_set(replace(recipe, n_events=sizes[i]), seeds[i])``.
    """
    rng = np.random.default_rng([seed, recipe.salt, 0x5E7])
    sizes = rng.integers(min_events, max_events + 1, size=n_slices)
    mean_size = 0.5 * (min_events + max_events)
    rate = offered_rate / mean_size
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_slices))
    seeds = rng.integers(0, 2 ** 31 - 1, size=n_slices)
    return sizes.astype(np.int64), arrivals, seeds.astype(np.int64)


def make_slice(size: int, seed: int, recipe: EventSetSpec = SLICE_RECIPE) -> EventSet:
    return make_event_set(replace(recipe, n_events=int(size)), int(seed))


# ------------------------------------------------------ all-station events ---

TRIGGER_STATIONS = (13, 14, 15)  # station numbers of trigger layers 0, 1, 2
N_STATIONS = 16


@dataclass
class RawEventSet:
    """Events with the hits of every station (input of the station filter):
    int64 offsets[E+1], uint8 station[H], fp32 x[H], y[H]."""
    offsets: np.ndarray
    station: np.ndarray
    x: np.ndarray
    y: np.ndarray
    layers: tuple = TRIGGER_STATIONS

    @property
    def n_events(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_hits(self) -> int:
        return int(len(self.station))


def embed_raw(base: EventSet, other_mean: float = 30.0, shuffle: bool = True, seed: int = 0,
              layers=TRIGGER_STATIONS, n_stations: int = N_STATIONS, square: bool = False) -> RawEventSet:
    """The events of ``base`` with hits on every station: the base set's hits
    of layer l on station ``layers[l]``, and Poisson(other_mean) hits (uniform
    in the annulus) on each other station.  ``shuffle``: the hits of an event
    in random order (each trigger layer keeping its hits' order); otherwise
    in detector order (grouped by station, ascending).  ``square``: the other
    stations' hits uniform in the square [-200, 200]^2 instead (cheaper; the
    filter never reads their coordinates).  Filtering the result on
    ``layers`` gives back ``base`` exactly."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5157]))
    n = base.n_events
    lc = np.diff(base.offsets.astype(np.int64)).reshape(n, 3)
    counts = rng.poisson(other_mean, (n, n_stations)).astype(np.int64)
    for l, s in enumerate(layers):
        counts[:, s] = lc[:, l]
    per_event = counts.sum(axis=1)
    offsets = np.zeros(n + 1, np.int64)
    np.cumsum(per_event, out=offsets[1:])
    station = np.repeat(np.tile(np.arange(n_stations, dtype=np.uint8), n), counts.ravel())
    total = int(offsets[-1])
    if square:
        x = rng.random(total, dtype=np.float32) * np.float32(400.0) - np.float32(200.0)
        y = rng.random(total, dtype=np.float32) * np.float32(400.0) - np.float32(200.0)
    else:
        r = np.sqrt(rng.uniform(20.0 ** 2, 200.0 ** 2, total))
        phi = rng.uniform(0.0, 2 * np.pi, total)
        x = (r * np.cos(phi)).astype(np.float32)
        y = (r * np.sin(phi)).astype(np.float32)
    if shuffle:
        ev = np.repeat(np.arange(n, dtype=np.int64), per_event)
        perm = np.lexsort((rng.random(total), ev))
        station = station[perm]
    base_layer = np.repeat(np.tile(np.arange(3), n), lc.ravel())
    for l, s in enumerate(layers):
        sel = station == s
        x[sel] = base.x[base_layer == l]
        y[sel] = base.y[base_layer == l]
    return RawEventSet(offsets, station, x, y, tuple(layers))


@dataclass
class HitStream:
    """A free-streaming timeslice (input of event building): int64 times t[H]
    in non-decreasing order, with each hit's station number and x, y, and the
    generating event of each hit (int64 event[H], for tests)."""
    t: np.ndarray
    station: np.ndarray
    x: np.ndarray
    y: np.ndarray
    event: np.ndarray

    @property
    def n_hits(self) -> int:
        return int(len(self.t))


def free_stream(raw: RawEventSet, rate_hz: float = 1e7, spread_ns: int = 10, min_spacing_ns: int = 0,
                seed: int = 0, t0: int = 0) -> HitStream:
    """The events of ``raw`` as a free-streaming timeslice: interactions at
    Poisson times (rate ``rate_hz``, integer nanoseconds from ``t0``, each
    at least ``min_spacing_ns`` after the previous one), every hit at its
    interaction's time plus U{0..spread_ns} ns, and the whole stream ordered
    by time (a stable sort, so hits of one event at the same time keep their
    order).  With min_spacing_ns > spread_ns + gap the events do not mix,
    and building events with that gap gives back ``raw``'s events."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x7153]))
    n = raw.n_events
    dt = np.rint(rng.exponential(1e9 / rate_hz, n)).astype(np.int64) + int(min_spacing_ns)
    dt[0] = 0
    t_event = int(t0) + np.cumsum(dt)
    per = np.diff(raw.offsets.astype(np.int64))
    event = np.repeat(np.arange(n, dtype=np.int64), per)
    t = t_event[event] + rng.integers(0, int(spread_ns) + 1, raw.n_hits, dtype=np.int64)
    if min_spacing_ns > spread_ns:
        # events do not overlap: ordering each event's hits is enough
        order = np.lexsort((t, event))
    else:
        order = np.argsort(t, kind="stable")
    return HitStream(t[order], raw.station[order], raw.x[order], raw.y[order], event[order])
