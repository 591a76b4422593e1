"""Shared test helpers: golden fixtures, event-set builders for edge cases."""
import json
import os

import numpy as np

from paper_1810_11966_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_cases():
    with open(os.path.join(GOLDEN, "handbuilt.json")) as f:
        return json.load(f)["cases"]


def golden_set(case):
    return synth.from_layers([case["layers"]])


def near_threshold_triplets(n, seed, plane_T=0.03, ndf=2, rel=1e-3, z=(400.0, 410.0, 420.0),
                            slope_max=0.45):
    """n triplets (ci, cj, ck) float32 whose fit residual sum of squares lies
    within a relative ``rel`` of ndf*T: a vertex-pointing line plus a
    displacement of the right length in the plane orthogonal to z."""
    rng = np.random.default_rng(seed)
    z = np.asarray(z, np.float64)
    zh = z / np.linalg.norm(z)
    # any orthonormal pair orthogonal to z (built here, independently of the oracle)
    e = np.array([1.0, 0.0, 0.0])
    p = e - zh * (e @ zh)
    p /= np.linalg.norm(p)
    q = np.cross(zh, p)
    m = rng.uniform(-slope_max, slope_max, n)
    target = ndf * plane_T * (1.0 + rng.uniform(-rel, rel, n))
    ang = rng.uniform(0, 2 * np.pi, n)
    r = np.sqrt(target)
    c = m[:, None] * z[None, :] + (r * np.cos(ang))[:, None] * p[None, :] + \
        (r * np.sin(ang))[:, None] * q[None, :]
    c = c.astype(np.float32)
    return c[:, 0], c[:, 1], c[:, 2]


def near_threshold_events(n_events, per_layer, seed, z=(400.0, 410.0, 420.0), rel=2e-3):
    """Events whose hits form many triplets near the MSD threshold in both
    planes: each event holds ``per_layer`` near-threshold tracks, hits of the
    same track in the same slot of each layer."""
    rng = np.random.default_rng(seed + 17)
    xs, ys, off = [], [], [0]
    for e in range(n_events):
        n = per_layer
        xi, xj, xk = near_threshold_triplets(n, seed * 1000 + 2 * e, 0.03, 2, rel, z)
        yi, yj, yk = near_threshold_triplets(n, seed * 1000 + 2 * e + 1, 0.025, 2, rel, z)
        for cx, cy in ((xi, yi), (xj, yj), (xk, yk)):
            perm = rng.permutation(n)
            xs.append(cx[perm]); ys.append(cy[perm])
            off.append(off[-1] + n)
    return synth.EventSet(np.asarray(off, np.int32), np.concatenate(xs), np.concatenate(ys),
                          np.zeros(n_events, np.int8))


def ragged_sizes_set(sizes, seed, with_tracks=True, spread=200.0):
    """One event per (n0, n1, n2) in ``sizes`` with random hits; events with
    all layers non-empty also get an exact vertex-pointing track so that some
    triplets pass."""
    rng = np.random.default_rng(seed)
    events = []
    for (n0, n1, n2) in sizes:
        layers = []
        m = rng.uniform(-0.4, 0.4, 2)
        for l, n in enumerate((n0, n1, n2)):
            pts = rng.uniform(-spread, spread, (n, 2)).astype(np.float32)
            if with_tracks and min(n0, n1, n2) > 0:
                zl = (400.0, 410.0, 420.0)[l]
                pts[rng.integers(0, n)] = (m[0] * zl, m[1] * zl)
            layers.append([tuple(map(float, p)) for p in pts])
        events.append(layers)
    return synth.from_layers(events)


def pair_boundary_events(n_events, per_layer, seed, rel=1e-6, z=(400.0, 410.0, 420.0)):
    """Events whose tracks are displaced along u = (z1, -z0, 0)/|(z0, z1)|,
    the direction that changes only the layer-0/1 part a of the residual, by
    |a| within a relative ``rel`` of sqrt(ndf*T) (ndf 2): triplets sit right at
    the boundary where f32(a*a) crosses Qmax."""
    rng = np.random.default_rng(seed)
    z = np.asarray(z, np.float64)
    u = np.array([z[1], -z[0], 0.0]) / np.hypot(z[0], z[1])
    xs, ys, off = [], [], [0]
    for e in range(n_events):
        n = per_layer
        cx, cy = [], []
        for T, store in ((0.03, cx), (0.025, cy)):
            m = rng.uniform(-0.4, 0.4, n)
            r = np.sqrt(2 * T) * (1.0 + rng.uniform(-rel, rel, n)) * rng.choice([-1.0, 1.0], n)
            c = m[:, None] * z[None, :] + r[:, None] * u[None, :]
            store.append(c.astype(np.float32))
        cx, cy = cx[0], cy[0]
        for l in range(3):
            perm = rng.permutation(n)
            xs.append(cx[perm, l]); ys.append(cy[perm, l])
            off.append(off[-1] + n)
    return synth.EventSet(np.asarray(off, np.int32), np.concatenate(xs), np.concatenate(ys),
                          np.zeros(n_events, np.int8))
