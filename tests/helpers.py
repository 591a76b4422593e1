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


def near_threshold_events(n_events, per_layer, seed, z=(400.0, 410.0, 420.0), rel=2e-3, slope_max=0.45):
    """Events whose hits form many triplets near the MSD threshold in both
    planes: each event holds ``per_layer`` near-threshold tracks, hits of the
    same track in the same slot of each layer."""
    rng = np.random.default_rng(seed + 17)
    xs, ys, off = [], [], [0]
    for e in range(n_events):
        n = per_layer
        xi, xj, xk = near_threshold_triplets(n, seed * 1000 + 2 * e, 0.03, 2, rel, z, slope_max)
        yi, yj, yk = near_threshold_triplets(n, seed * 1000 + 2 * e + 1, 0.025, 2, rel, z, slope_max)
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


def pair_boundary_events(n_events, per_layer, seed, rel=1e-6, z=(400.0, 410.0, 420.0), slope_max=0.4):
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
            m = rng.uniform(-slope_max, slope_max, n)
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


def k_boundary_events(n_events, per_layer, seed, rel=1e-6, z=(400.0, 410.0, 420.0), slope_max=0.4):
    """Events whose tracks are displaced along the unit vector orthogonal to
    z and to (z1, -z0, 0): only the layer-2 part b of the residual changes, by
    |b| within a relative ``rel`` of sqrt(ndf*T) (ndf 2), so triplets sit
    where f32(b*b) crosses Qmax (the edge of the binned form's layer-2 key
    interval)."""
    rng = np.random.default_rng(seed)
    z = np.asarray(z, np.float64)
    zh = z / np.linalg.norm(z)
    u = np.array([z[1], -z[0], 0.0]) / np.hypot(z[0], z[1])
    v = np.cross(zh, u)
    xs, ys, off = [], [], [0]
    for e in range(n_events):
        n = per_layer
        cs = []
        for T in (0.03, 0.025):
            m = rng.uniform(-slope_max, slope_max, n)
            r = np.sqrt(2 * T) * (1.0 + rng.uniform(-rel, rel, n)) * rng.choice([-1.0, 1.0], n)
            cs.append((m[:, None] * z[None, :] + r[:, None] * v[None, :]).astype(np.float32))
        for l in range(3):
            perm = rng.permutation(n)
            xs.append(cs[0][perm, l]); ys.append(cs[1][perm, l])
            off.append(off[-1] + n)
    return synth.EventSet(np.asarray(off, np.int32), np.concatenate(xs), np.concatenate(ys),
                          np.zeros(n_events, np.int8))


def window_boundary_events(n_events, per_layer, seed, w=(0.005, 0.005), rel=1e-6, z=(400.0, 410.0, 420.0)):
    """Slope-window edge cases: layer-1 and layer-2 slopes differ from the
    layer-0 slope by the window within a relative ``rel`` (either sign)."""
    rng = np.random.default_rng(seed)
    xs, ys, off = [], [], [0]
    for e in range(n_events):
        n = per_layer
        layers = []
        base = rng.uniform(-0.4, 0.4, (n, 2))
        for l in range(3):
            s = base.copy()
            if l > 0:
                for p in range(2):
                    s[:, p] += w[p] * (1.0 + rng.uniform(-rel, rel, n)) * rng.choice([-1.0, 1.0], n)
            layers.append((s * z[l]).astype(np.float32))
        for l in range(3):
            perm = rng.permutation(n)
            xs.append(layers[l][perm, 0]); ys.append(layers[l][perm, 1])
            off.append(off[-1] + n)
    return synth.EventSet(np.asarray(off, np.int32), np.concatenate(xs), np.concatenate(ys),
                          np.zeros(n_events, np.int8))


def special_values_events(seed):
    """Hits with NaN, +-inf, huge, subnormal and zero coordinates, mixed with
    vertex tracks; events whose keys are all equal; events past the binned
    form's LDS capacity."""
    rng = np.random.default_rng(seed)
    z = (400.0, 410.0, 420.0)
    events = []

    def track(m):
        return [(m[0] * zl, m[1] * zl) for zl in z]

    def noisy(n):
        return [tuple(map(float, p)) for p in rng.uniform(-200, 200, (n, 2)).astype(np.float32)]

    nan, inf = float("nan"), float("inf")
    specials = [(nan, 1.0), (1.0, nan), (inf, 0.0), (-inf, 5.0), (0.0, inf), (1e30, 1e30),
                (-3e38, 2e38), (1e-40, -1e-40), (0.0, 0.0), (-0.0, 0.0)]
    for k in range(len(specials)):
        layers = [noisy(6) for _ in range(3)]
        for l in range(3):
            layers[l].append(specials[(k + l) % len(specials)])
            layers[l].append(specials[(k + 3 * l + 1) % len(specials)])
            layers[l].append(track((0.1 * k - 0.3, 0.05))[l])
        events.append(layers)
    # every hit special
    events.append([[specials[(l + i) % len(specials)] for i in range(7)] for l in range(3)])
    # all hits identical (zero key width): every triplet passes
    events.append([[track((0.2, -0.1))[l]] * 9 for l in range(3)])
    # subnormal vertex tracks: every triplet passes
    events.append([[(1e-41 * (i + 1), -2e-41 * (i + 1)) for i in range(5)] for l in range(3)])
    # a vertex track among hits at the origin
    events.append([[(0.0, 0.0)] * 4 + [track((0.3, 0.3))[l]] for l in range(3)])
    # more hits than the binned form keeps in LDS (layer 1, layer 2)
    for sizes in ((20, 700, 20), (20, 20, 700), (5, 513, 512), (20, 256, 256), (20, 257, 30), (30, 40, 257)):
        layers = [noisy(n) for n in sizes]
        for l in range(3):
            layers[l][0] = track((0.05, -0.2))[l]
        layers[1][-1] = (nan, nan)
        events.append(layers)
    return synth.from_layers(events)


def two_particle_events(n_events, seed, z=(400.0, 410.0, 420.0), noise=6):
    """Events whose passing triplets share hits in many ways: 1-3 exact
    vertex tracks, each hit duplicated with probability 0.3 and joined by a
    hit within 0.05 cm of it with probability 0.3 (per layer), plus uniform
    noise hits.  One track with near hits gives several passing triplets
    that all share a hit; duplicates and second tracks give triplets with no
    hit in common."""
    rng = np.random.default_rng(seed)
    events = []
    for _ in range(n_events):
        layers = [[], [], []]
        for _t in range(int(rng.integers(1, 4)) if rng.random() < 0.9 else 0):
            m = rng.uniform(-0.4, 0.4, 2)
            for l, zl in enumerate(z):
                h = (float(np.float32(m[0] * zl)), float(np.float32(m[1] * zl)))
                layers[l].append(h)
                if rng.random() < 0.3:
                    layers[l].append(h)
                if rng.random() < 0.3:
                    d = rng.uniform(-0.05, 0.05, 2)
                    layers[l].append((float(np.float32(h[0] + d[0])), float(np.float32(h[1] + d[1]))))
        for l in range(3):
            pts = rng.uniform(-200, 200, (int(rng.integers(0, noise + 1)), 2)).astype(np.float32)
            layers[l] += [tuple(map(float, p)) for p in pts]
            rng.shuffle(layers[l])
        events.append(layers)
    return synth.from_layers(events)


def near_threshold_events_z(n_events, per_layer, seed, rel=1e-4, dz=0.75, z=(400.0, 410.0, 420.0), slope_max=0.45):
    """Events on staggered modules whose tracks sit near the MSD cut: each
    track's three hits at z_l -/+ dz (chosen per hit), displaced orthogonally
    to its own (zi, zj, zk) so that its residual sum of squares lies within a
    relative ``rel`` of ndf*T in both planes.  Returns a set with per-hit z."""
    rng = np.random.default_rng(seed + 91)
    xs, ys, zs, off = [], [], [], [0]
    for e in range(n_events):
        cx, cy, cz = [], [], []
        for t in range(per_layer):
            zt = tuple(zl + dz * rng.choice([-1.0, 1.0]) for zl in z)
            xi, xj, xk = near_threshold_triplets(1, seed * 100000 + 2 * (e * per_layer + t), 0.03, 2, rel, zt,
                                                 slope_max)
            yi, yj, yk = near_threshold_triplets(1, seed * 100000 + 2 * (e * per_layer + t) + 1, 0.025, 2, rel, zt,
                                                 slope_max)
            cx.append((xi[0], xj[0], xk[0]))
            cy.append((yi[0], yj[0], yk[0]))
            cz.append(zt)
        cx, cy, cz = np.asarray(cx, np.float32), np.asarray(cy, np.float32), np.asarray(cz, np.float32)
        for l in range(3):
            perm = rng.permutation(per_layer)
            xs.append(cx[perm, l]); ys.append(cy[perm, l]); zs.append(cz[perm, l])
            off.append(off[-1] + per_layer)
    return synth.EventSet(np.asarray(off, np.int32), np.concatenate(xs), np.concatenate(ys),
                          np.zeros(n_events, np.int8), z=np.concatenate(zs))


def odd_z_events(seed):
    """Per-hit z that no slope bound covers, among exact tracks: z = 0,
    negative, NaN and infinite z in each layer, and huge coordinates over tiny
    z (slopes near overflow)."""
    rng = np.random.default_rng(seed)
    base = two_particle_events(40, seed=seed + 1, noise=4)
    s = synth.staggered(base)
    z = s.z.copy()
    x, y = s.x.copy(), s.y.copy()
    for e in range(0, base.n_events, 4):
        l = e % 3
        lo, hi = s.offsets[3 * e + l], s.offsets[3 * e + l + 1]
        if hi > lo:
            z[lo] = (0.0, -405.0, np.nan, np.inf)[(e // 4) % 4]
    for e in range(2, base.n_events, 8):
        lo, hi = s.offsets[3 * e], s.offsets[3 * e + 3]
        z[lo:hi] = np.float32(1e-3)
        x[lo:hi] = (rng.uniform(-1, 1, hi - lo) * 3e37).astype(np.float32)
    return synth.EventSet(s.offsets, x, y, s.n_tracks, z=z)
