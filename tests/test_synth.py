"""The seeded synthetic event generator: determinism and shape statistics."""
from dataclasses import replace

import numpy as np

from paper_1810_11966_amd import synth


def test_deterministic_and_seed_sensitive():
    a = synth.make_event_set(synth.SMALL_10K)
    b = synth.make_event_set(synth.SMALL_10K)
    c = synth.make_event_set(synth.SMALL_10K, seed=1)
    assert a.sha256() == b.sha256() != c.sha256()


def test_prefix_generation_matches_full_set():
    spec = replace(synth.MEDIUM_1M, n_events=3 * synth.CHUNK // 2)
    full = synth.make_event_set(spec)
    part = synth.make_event_set(spec, n_events=synth.CHUNK)
    assert np.array_equal(full.offsets[: len(part.offsets)], part.offsets)
    assert np.array_equal(full.x[: part.n_hits], part.x)


def test_csr_well_formed_and_marginals():
    s = synth.make_event_set(synth.SMALL_10K)
    off = s.offsets.astype(np.int64)
    assert off[0] == 0 and off[-1] == s.n_hits and (np.diff(off) >= 0).all()
    assert s.x.dtype == np.float32 and s.y.dtype == np.float32 and s.offsets.dtype == np.int32
    n = s.layer_counts()
    ntr = s.n_tracks.astype(np.int64)
    noise = n - ntr[:, None]
    assert abs(noise.mean() - 8.0) < 0.1
    assert abs(noise.var() - 8.0) < 0.4  # Poisson
    inj = (ntr > 0).mean()
    assert abs(inj - 0.05) < 0.01 and set(np.unique(ntr)) <= {0, 2}
    r = np.hypot(s.x.astype(np.float64), s.y.astype(np.float64))
    # noise is uniform in area: fraction inside radius R is (R^2-20^2)/(200^2-20^2)
    frac = (r < 110.0).mean()
    assert abs(frac - (110 ** 2 - 20 ** 2) / (200 ** 2 - 20 ** 2)) < 0.01


def test_injected_tracks_point_to_vertex():
    spec = replace(synth.SMALL_10K, n_events=2000, p_inject=1.0, sigma=0.0, hits_mean=0.0)
    s = synth.make_event_set(spec)
    n = s.layer_counts()
    assert (n == 2).all()
    for l in range(3):
        sl = s.offsets[3 * np.arange(s.n_events) + l]
        # slopes of the two tracks agree across layers to fp32 precision
        for t in range(2):
            xs = s.x[sl + t].astype(np.float64) / synth.Z_LAYERS[l]
            r = np.hypot(s.x[sl + t], s.y[sl + t])
            assert (r >= 20 - 1e-3).all() and (r <= 200 + 1e-3).all()
            if l == 0:
                base = np.sort(np.stack([s.x[sl] / 400.0, s.x[sl + 1] / 400.0]), axis=0)
    for l in (1, 2):
        sl = s.offsets[3 * np.arange(s.n_events) + l]
        other = np.sort(np.stack([s.x[sl] / synth.Z_LAYERS[l], s.x[sl + 1] / synth.Z_LAYERS[l]]), axis=0)
        assert np.allclose(other, base, atol=1e-5)


def test_mixture_and_dense_shapes():
    mix = synth.make_event_set(synth.MIXTURE_4M, n_events=20000)
    lam = mix.layer_counts().mean()
    assert abs(lam - 120 * (1 - 1 / 3)) < 2.0  # E[120(1-b^2)] = 80
    dense = synth.make_event_set(synth.DENSE_100K, n_events=3000)
    ntr = dense.n_tracks
    assert abs((ntr > 0).mean() - 0.10) < 0.02 and set(np.unique(ntr)) <= {0, 2, 4, 6}


def test_slice_stream_rate():
    sizes, arr, seeds = synth.slice_stream(4000, seed=0)
    assert sizes.min() >= 10_000 and sizes.max() <= 1_000_000
    rate = len(arr) / arr[-1]
    assert abs(rate - 1e7 / 505_000) / (1e7 / 505_000) < 0.05


def test_subset_and_concat_roundtrip():
    s = synth.make_event_set(synth.SMALL_10K, n_events=500)
    parts = [s.subset(0, 100), s.subset(100, 250), s.subset(350, 150)]
    t = synth.concat(parts)
    assert t.sha256() == s.sha256()
