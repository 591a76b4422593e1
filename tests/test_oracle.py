"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these tests needs a GPU.  Each check is chosen so that a plausible
mistake in the oracle (a dropped term, a wrong sign or layer index, a
transposed operand, the wrong degrees of freedom or threshold) fails it.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import reference as R
from paper_1810_11966_amd import synth
from tests import helpers

Z = (400.0, 410.0, 420.0)
MODES = ("msd", "msd_basis", "window")


def cfg_for(case):
    kw = dict(case.get("cfg", {}))
    return R.OracleConfig(**kw)


# ---------------------------------------------------------------- golden ---

@pytest.mark.parametrize("case", helpers.golden_cases(), ids=lambda c: c["name"])
def test_golden_handbuilt_counts(oracle_lib, case):
    """Closed-form counts of hand-built events (tests/golden/handbuilt.json)."""
    s = helpers.golden_set(case)
    cfg = cfg_for(case)
    modes = [cfg.test] if cfg.test == "window" else ["msd", "msd_basis"]
    for mode in modes:
        c = R.OracleConfig(**{**cfg.__dict__, "test": mode})
        counts, accept, status, _ = R.select_set(s, c)
        assert status == 0
        assert counts[0] == case["expected_count"], (mode, case["why"])
        assert accept[0] == int(case["expected_count"] >= 2)
        n_counts, n_accept, _ = R.select_numpy(s.offsets, s.x, s.y, c)
        assert n_counts[0] == case["expected_count"]


# -------------------------------------------------- the fit, exact forms ---

def test_basis_is_orthonormal_complement_of_z(oracle_lib):
    """(u, v) must span the plane orthogonal to z: u.z = v.z = u.v = 0,
    |u| = |v| = 1, u has no layer-2 component (fp32 constants, 1e-7 level)."""
    for z in [Z, (1.0, 2.0, 2.0), (100.0, 300.0, 1000.0)]:
        b = R.basis_c(R.OracleConfig(z=z)).astype(np.float64)
        u = np.array([b[0], b[1], 0.0])
        v = b[2:5]
        zz = np.asarray(z, np.float64) / np.linalg.norm(z)
        assert abs(u @ zz) < 3e-7 and abs(v @ zz) < 3e-7 and abs(u @ v) < 3e-7
        assert abs(u @ u - 1) < 3e-7 and abs(v @ v - 1) < 3e-7
        # C and NumPy constants agree bit for bit
        assert np.array_equal(np.asarray(R.basis_f32(z), np.float32), R.basis_c(R.OracleConfig(z=z)))


def test_exact_fit_closed_form():
    """The exact fit's Q equals |c|^2 - (c.z)^2/|z|^2 (Lagrange identity form,
    sum over layer pairs of (c_l z_m - c_m z_l)^2 / |z|^2)."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        c = rng.uniform(-200, 200, 3).astype(np.float32)
        q = R.fit_msd_exact(*c, Z, 1)
        cf = [Fraction(float(v)) for v in c]
        zf = [Fraction(v) for v in Z]
        lag = sum((cf[l] * zf[m] - cf[m] * zf[l]) ** 2 for l in range(3) for m in range(l + 1, 3))
        assert q == lag / sum(v * v for v in zf)


def test_exact_fit_equality_passes():
    """Equality at the threshold passes ("rejected if above", Sec. 3.2 step
    2b): with z = (1, 2, 2) and c = (3, 0, 0), Q = 9 - 9/9 = 8 exactly."""
    q = R.fit_msd_exact(3.0, 0.0, 0.0, (1.0, 2.0, 2.0), 2)
    assert q == 4
    cfg = R.OracleConfig(z=(1.0, 2.0, 2.0), msd_max=(4.0, 4.0), ndf=2)
    s = synth.from_layers([[[(3.0, 3.0)], [(0.0, 0.0)], [(0.0, 0.0)]]])
    for mode in ("msd", "msd_basis"):
        c = R.OracleConfig(**{**cfg.__dict__, "test": mode})
        # the fp32 evaluation of this triplet is within a few ulp of 8; the
        # comparison is "<=" so a threshold of 4(1+2^-20) passes, 4(1-2^-20) fails
        up = R.OracleConfig(**{**c.__dict__, "msd_max": (4.0 * (1 + 2 ** -20),) * 2})
        dn = R.OracleConfig(**{**c.__dict__, "msd_max": (4.0 * (1 - 2 ** -20),) * 2})
        assert R.select_set(s, up)[0][0] == 1
        assert R.select_set(s, dn)[0][0] == 0


@pytest.mark.parametrize("mode", ["msd", "msd_basis"])
@pytest.mark.parametrize("plane_T", [0.03, 0.025])
def test_fp32_msd_within_bound_of_exact_fit(oracle_lib, mode, plane_T):
    """The oracle's fp32 MSD of random and near-threshold triplets stays within
    a rigorous error bound of the exact fit (the bound of its own evaluation
    order), and its decision equals the exact decision outside that band."""
    ci, cj, ck = helpers.near_threshold_triplets(600, seed=11, plane_T=plane_T, rel=3e-3)
    rng = np.random.default_rng(12)
    r = rng.uniform(-200, 200, (200, 3)).astype(np.float32)
    ci, cj, ck = (np.concatenate([a, r[:, i]]) for i, a in enumerate((ci, cj, ck)))
    cfg = R.OracleConfig(test=mode, msd_max=(plane_T, plane_T))
    bound = (R.fp32_fit_error_bound if mode == "msd" else R.fp32_error_bound)(ci, cj, ck, Z)
    T32 = Fraction(float(np.float32(plane_T)))
    decided = 0
    for t in range(len(ci)):
        exact = R.fit_msd_exact(ci[t], cj[t], ck[t], Z, 2)
        got = R.triplet_msd_c(cfg, ci[t], cj[t], ck[t])
        # fl(Q / 2) = Q / 2 exactly or within one rounding of it
        assert abs(Fraction(got) * 2 - exact * 2) <= Fraction(float(bound[t])) * (1 + Fraction(1, 10 ** 6)) \
            + Fraction(got) * 2 * Fraction(1, 2 ** 23)
        margin = Fraction(float(bound[t])) / 2 + T32 * Fraction(1, 2 ** 21)
        if abs(exact - T32) > margin:
            decided += 1
            assert (got <= float(T32)) == (exact <= T32)
    assert decided > 600  # most near-threshold cases are outside the band


def test_fit_error_bound_is_not_slack_free(oracle_lib):
    """The default evaluation's bound must hold on triplets built to round
    badly (large coordinates, steep tracks) and must not be trivially large:
    on near-threshold triplets it stays below 1e-3 of the cut."""
    ci, cj, ck = helpers.near_threshold_triplets(400, seed=13, plane_T=0.03, rel=1e-3, slope_max=0.48)
    b = R.fp32_fit_error_bound(ci, cj, ck, Z)
    assert (b < 0.06 * 1e-3).all()
    cfg = R.OracleConfig(test="msd", msd_max=(0.03, 0.03), ndf=1)
    worst = 0.0
    for t in range(len(ci)):
        exact = R.fit_msd_exact(ci[t], cj[t], ck[t], Z, 1)
        got = Fraction(R.triplet_msd_c(cfg, ci[t], cj[t], ck[t]))
        err = abs(got - exact)
        assert err <= Fraction(float(b[t]))
        worst = max(worst, float(err / Fraction(float(b[t]))))
    assert worst > 1e-3  # the bound is not off by orders of magnitude


def test_fp32_decisions_agree_with_float64_fit(oracle_lib):
    """C oracle counts == counts from the float64 fit, on events built from
    near-threshold tracks, wherever every triplet is clear of the band."""
    s = helpers.near_threshold_events(40, 6, seed=5, rel=5e-2)
    counts, _, _, _ = R.select_set(s)
    off = s.offsets
    checked = 0
    for e in range(s.n_events):
        sl = [slice(off[3 * e + l], off[3 * e + l + 1]) for l in range(3)]
        I, J, K = np.meshgrid(np.arange(sl[0].start, sl[0].stop), np.arange(sl[1].start, sl[1].stop),
                              np.arange(sl[2].start, sl[2].stop), indexing="ij")
        qx = R.fit_msd_f64(s.x[I], s.x[J], s.x[K], Z, 2)
        qy = R.fit_msd_f64(s.y[I], s.y[J], s.y[K], Z, 2)
        bx = R.fp32_fit_error_bound(s.x[I], s.x[J], s.x[K], Z) / 2 + 1e-9
        by = R.fp32_fit_error_bound(s.y[I], s.y[J], s.y[K], Z) / 2 + 1e-9
        Tx, Ty = float(np.float32(0.03)), float(np.float32(0.025))
        if (np.abs(qx - Tx) <= bx).any() or (np.abs(qy - Ty) <= by).any():
            continue
        assert counts[e] == int(np.count_nonzero((qx <= Tx) & (qy <= Ty)))
        checked += 1
    assert checked >= 30


def test_tiny_bruteforce_exact(oracle_lib):
    """Tiny random events: the oracle's count equals the count decided in
    exact rational arithmetic (events with a triplet inside the rounding band
    are skipped)."""
    rng = np.random.default_rng(21)
    checked = 0
    for trial in range(60):
        n = rng.integers(0, 4, 3)
        layers = []
        m = rng.uniform(-0.4, 0.4, 2)
        for l in range(3):
            pts = []
            for _ in range(n[l]):
                if rng.random() < 0.6:  # near a vertex-pointing line
                    pts.append((m[0] * Z[l] + rng.normal(0, 0.25), m[1] * Z[l] + rng.normal(0, 0.25)))
                else:
                    pts.append(tuple(rng.uniform(-200, 200, 2)))
            layers.append(pts)
        s = synth.from_layers([layers])
        got = R.select_set(s)[0][0]
        o = s.offsets
        exact, ambiguous = 0, False
        Tx, Ty = Fraction(float(np.float32(0.03))), Fraction(float(np.float32(0.025)))
        for i in range(o[0], o[1]):
            for j in range(o[1], o[2]):
                for k in range(o[2], o[3]):
                    qx = R.fit_msd_exact(s.x[i], s.x[j], s.x[k], Z, 2)
                    qy = R.fit_msd_exact(s.y[i], s.y[j], s.y[k], Z, 2)
                    bx = Fraction(float(R.fp32_fit_error_bound(s.x[i], s.x[j], s.x[k], Z))) / 2
                    by = Fraction(float(R.fp32_fit_error_bound(s.y[i], s.y[j], s.y[k], Z))) / 2
                    if abs(qx - Tx) <= bx + Tx / 2 ** 21 or abs(qy - Ty) <= by + Ty / 2 ** 21:
                        ambiguous = True
                    exact += int(qx <= Tx and qy <= Ty)
        if not ambiguous:
            assert got == exact
            checked += 1
    assert checked > 50


# ---------------------------------------------------------- invariants ---

def _fuzz_set(seed, n_events=40, lam=6, near=True):
    s = synth.make_event_set(synth.EventSetSpec(n_events=n_events, hits_mean=lam, p_inject=0.5,
                                                pairs=(1, 2), sigma=0.15, salt=99), seed)
    if near:
        s = synth.concat([s, helpers.near_threshold_events(10, 4, seed=seed, rel=1e-2)])
    return s


@pytest.mark.parametrize("mode", MODES)
def test_invariant_permutation_within_layer(oracle_lib, mode):
    s = _fuzz_set(1)
    cfg = R.OracleConfig(test=mode)
    base = R.select_set(s, cfg)[0]
    rng = np.random.default_rng(2)
    perm = np.arange(s.n_hits)
    for seg in range(3 * s.n_events):
        lo, hi = s.offsets[seg], s.offsets[seg + 1]
        perm[lo:hi] = lo + rng.permutation(hi - lo)
    p = synth.EventSet(s.offsets, s.x[perm], s.y[perm], s.n_tracks)
    assert np.array_equal(R.select_set(p, cfg)[0], base)


@pytest.mark.parametrize("mode", MODES)
def test_invariant_sign_flip_and_xy_swap(oracle_lib, mode):
    s = _fuzz_set(3)
    cfg = R.OracleConfig(test=mode)
    base = R.select_set(s, cfg)[0]
    assert base.sum() > 0
    for fx, fy in ((-1, 1), (1, -1), (-1, -1)):
        f = synth.EventSet(s.offsets, (fx * s.x).astype(np.float32), (fy * s.y).astype(np.float32), s.n_tracks)
        assert np.array_equal(R.select_set(f, cfg)[0], base)
    sw = synth.EventSet(s.offsets, s.y, s.x, s.n_tracks)
    cfg_sw = R.OracleConfig(test=mode, msd_max=cfg.msd_max[::-1], window=cfg.window[::-1])
    assert np.array_equal(R.select_set(sw, cfg_sw)[0], base)


@pytest.mark.parametrize("mode", ["msd", "msd_basis"])
def test_invariant_power_of_two_scaling(oracle_lib, mode):
    """Coordinates x 2^k with thresholds x 4^k: every fp32 product and sum
    scales exactly, so every decision is unchanged."""
    s = _fuzz_set(4)
    cfg = R.OracleConfig(test=mode)
    base = R.select_set(s, cfg)[0]
    for k in (-3, 2):
        f = synth.EventSet(s.offsets, (s.x * 2.0 ** k).astype(np.float32),
                           (s.y * 2.0 ** k).astype(np.float32), s.n_tracks)
        c2 = R.OracleConfig(test=mode, msd_max=tuple(float(np.float32(t)) * 4.0 ** k for t in cfg.msd_max))
        assert np.array_equal(R.select_set(f, c2)[0], base)


def test_invariant_adding_vertex_point_does_not_change_fit():
    """The fit goes through the vertex, so adding (z=0, c=0) to the exact
    least-squares problem leaves Q unchanged."""
    rng = np.random.default_rng(8)
    for _ in range(50):
        c = rng.uniform(-200, 200, 3)
        cf = [Fraction(float(np.float32(v))) for v in c] + [Fraction(0)]
        zf = [Fraction(v) for v in Z] + [Fraction(0)]
        m = sum(a * b for a, b in zip(cf, zf)) / sum(b * b for b in zf)
        q4 = sum((a - m * b) ** 2 for a, b in zip(cf, zf))
        assert q4 == R.fit_msd_exact(*c, Z, 1)


@pytest.mark.parametrize("mode", MODES)
def test_batch_composition_does_not_matter(oracle_lib, mode):
    s = _fuzz_set(6)
    cfg = R.OracleConfig(test=mode)
    base = R.select_set(s, cfg)[0]
    parts = [s.subset(0, 17), s.subset(17, 13), s.subset(30, s.n_events - 30)]
    got = np.concatenate([R.select_set(p, cfg)[0] for p in parts])
    assert np.array_equal(got, base)
    assert np.array_equal(R.select_set(s, cfg, n_threads=5)[0], base)


# ------------------------------------------------- window factorisation ---

def test_window_count_factorises(oracle_lib):
    """Window mode: a triplet passes iff (i, j) and (i, k) pass separately, so
    count = sum_i a_i b_i with a_i = #{j ok with i}, b_i = #{k ok with i}."""
    s = _fuzz_set(7, lam=10)
    counts = R.select_set(s, R.OracleConfig(test="window"))[0]
    W = np.float32(0.005)
    zs = [np.float32(v) for v in Z]
    for e in range(s.n_events):
        o = s.offsets[3 * e: 3 * e + 4]
        sx = [s.x[o[l]:o[l + 1]] / zs[l] for l in range(3)]
        sy = [s.y[o[l]:o[l + 1]] / zs[l] for l in range(3)]
        okj = (np.abs(sx[1][None, :] - sx[0][:, None]) < W) & (np.abs(sy[1][None, :] - sy[0][:, None]) < W)
        okk = (np.abs(sx[2][None, :] - sx[0][:, None]) < W) & (np.abs(sy[2][None, :] - sy[0][:, None]) < W)
        assert counts[e] == int((okj.sum(1) * okk.sum(1)).sum())


# ----------------------------------------------------------- two oracles ---

@pytest.mark.parametrize("mode", MODES)
def test_c_and_numpy_oracles_agree(oracle_lib, mode):
    for seed in range(3):
        s = _fuzz_set(10 + seed, n_events=60, lam=7)
        cfg = R.OracleConfig(test=mode, ndf=2 + (seed == 2))
        c, a, st, _ = R.select_set(s, cfg)
        n, na, nst = R.select_numpy(s.offsets, s.x, s.y, cfg)
        assert np.array_equal(c, n) and np.array_equal(a, na) and st == nst


# --------------------------------------------------------- error cases ---

def test_malformed_ranges_and_overflow(oracle_lib):
    good = helpers.golden_set(helpers.golden_cases()[1])  # two tracks, 6 hits
    off = np.concatenate([good.offsets, good.offsets[1:] + good.n_hits]).astype(np.int32)
    x = np.concatenate([good.x, good.x]); y = np.concatenate([good.y, good.y])
    # event 1: layer range reversed
    bad = off.copy(); bad[4] = bad[5] + 1
    c, a, st, _ = R.select(bad, x, y)
    assert c[0] == 2 and c[1] == -1 and a[1] == 0 and st == 1
    # event 1: end beyond n_hits
    bad = off.copy(); bad[6] = len(x) + 1
    c, a, st, _ = R.select(bad, x, y)
    assert c[1] == -1 and st == 1
    # negative start
    bad = off.copy(); bad[0] = -1
    c, a, st, _ = R.select(bad, x, y)
    assert c[0] == -1
    # 1291^3 > INT32_MAX: count not representable
    n = 1291
    offo = np.array([0, n, 2 * n, 3 * n], np.int32)
    xo = np.zeros(3 * n, np.float32)
    c, a, st, _ = R.select(offo, xo, xo)
    assert c[0] == -2 and a[0] == 0 and st == 2
    # min_triplets = 0 accepts every well-formed event, never a malformed one
    bad = off.copy(); bad[4] = bad[5] + 1
    c, a, st, _ = R.select(bad, x, y, R.OracleConfig(min_triplets=0))
    assert a[0] == 1 and a[1] == 0


def test_empty_batch(oracle_lib):
    c, a, st, _ = R.select(np.zeros(1, np.int32), np.zeros(0, np.float32), np.zeros(0, np.float32))
    assert len(c) == 0 and st == 0


# ------------------------------------------------------- special values ---

@pytest.mark.parametrize("mode", MODES)
def test_special_coordinate_values(oracle_lib, mode):
    """NaN and infinite coordinates never pass (every comparison with NaN is
    false and an infinite residual exceeds any threshold); the two oracles
    agree on them, and the events with closed-form counts get them."""
    s = helpers.special_values_events(seed=3)
    cfg = R.OracleConfig(test=mode)
    c, a, st, _ = R.select_set(s, cfg)
    with np.errstate(all="ignore"):
        n, na, nst = R.select_numpy(s.offsets, s.x, s.y, cfg)
    assert np.array_equal(c, n) and np.array_equal(a, na) and st == nst == 0
    # all hits identical on one vertex track: 9^3 triplets; five subnormal
    # vertex tracks: every one of the 5^3 triplets lies within 1e-40 cm of a
    # line through the vertex; four hits at the origin plus one track: 4^3 + 1
    assert c[11] == 9 ** 3 and c[12] == 5 ** 3 and c[13] == 4 ** 3 + 1
    # special values only: no layer-0 hit has two finite coordinates below
    # 1e30 in magnitude, so no triplet can pass
    assert c[10] == 0


# ------------------------------------------- the two evaluation orders ---

@pytest.mark.parametrize("name,n_events", [("small_10k", None), ("medium_1m", 100_000),
                                           ("mixture_4m", 5_000), ("dense_100k", 300)])
def test_evaluation_orders_agree_on_workloads(oracle_lib, name, n_events):
    """The fit written out (default) and its basis-form evaluation round
    differently, but on the benchmark workloads no triplet's decision differs:
    every triplet of the 10k-event workload, the first 100k events of the
    1M-event workload and samples of the mixture and dense workloads (each
    triplet decided both ways, both planes)."""
    spec = synth.WORKLOADS[name]
    s = synth.make_event_set(spec, n_events=n_events) if n_events else synth.make_event_set(spec)
    threads = max(1, min(8, len(__import__("os").sched_getaffinity(0))))
    d = R.msd_disagreements(s.offsets, s.x, s.y, n_threads=threads)
    assert int(d.sum()) == 0, (name, int((d > 0).sum()))


def test_evaluation_orders_can_disagree(oracle_lib):
    """The disagreement counter itself: near-threshold triplets within a few
    ulps of the cut are decided differently by the two orders for some
    triplets (so a zero above is a measurement, not a tautology)."""
    s = helpers.near_threshold_events(400, 8, seed=21, rel=1e-7)
    d = R.msd_disagreements(s.offsets, s.x, s.y, n_threads=4)
    c_fit = R.select_set(s, R.OracleConfig(test="msd"))[0]
    c_basis = R.select_set(s, R.OracleConfig(test="msd_basis"))[0]
    assert d.sum() > 0
    # an event whose counts differ has disagreeing triplets
    assert ((c_fit != c_basis) <= (d > 0)).all()
    assert (np.abs(c_fit.astype(np.int64) - c_basis) <= d).all()


def test_evaluation_orders_disagree_far_from_axis(oracle_lib):
    """Far from the axis (slopes up to 25 and 1000, coordinates up to ~4e5 cm)
    the written-out fit's rounding moves Q by up to ~1e-3 of the cut: hundreds
    of near-cut triplets are decided differently by the two orders, so the GPU
    parity sets built this way tell the two tests apart."""
    for k, sm in enumerate((25.0, 1000.0)):
        s = helpers.near_threshold_events(150, 8, seed=40 + k, rel=1e-3, slope_max=sm)
        d = R.msd_disagreements(s.offsets, s.x, s.y, n_threads=4)
        assert d.sum() > 100, (sm, int(d.sum()))


# ------------------------------------------ two-particle (disjoint) acceptance ---

def _track(m, z=(400.0, 410.0, 420.0), dx=(0.0, 0.0, 0.0)):
    """Hits of a straight line through the vertex with slopes m = (mx, my),
    one per layer, x displaced by dx per layer (cm)."""
    return [(float(np.float32(m[0] * zl + d)), float(np.float32(m[1] * zl))) for zl, d in zip(z, dx)]


def test_disjoint_pair_definition_on_index_lists(oracle_lib):
    """Hand-built triplet lists (hit indices per layer): two triplets count as
    two particles only if they differ in every layer's hit."""
    cases = [
        ([], False),
        ([(0, 0, 0)], False),
        ([(0, 0, 0), (1, 1, 1)], True),
        ([(0, 0, 0), (0, 1, 1)], False),                       # shared layer-0 hit
        ([(0, 0, 0), (1, 0, 1)], False),                       # shared layer-1 hit
        ([(0, 0, 0), (1, 1, 0)], False),                       # shared layer-2 hit
        ([(0, 0, 0), (0, 1, 1), (1, 0, 1)], False),            # pairwise sharing, no common hit
        ([(0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 0)], False),
        ([(0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 0), (1, 1, 1)], True),
        ([(5, 7, 9)] * 3 + [(6, 8, 10)], True),
    ]
    for trips, want in cases:
        assert R.has_disjoint_pair(trips) == want, trips


def test_disjoint_acceptance_hand_built_events(oracle_lib):
    """Events with known passing triplets (exact vertex tracks, cross
    combinations far off any line): the count mode and the two-particle mode
    differ exactly where the passing triplets share a hit."""
    a, b = (0.1, 0.05), (-0.2, 0.15)
    ta, tb = _track(a), _track(b)
    near = _track(a, dx=(0.0, 0.0, 0.05))  # 0.05 cm off the line in layer 2: still passes
    events = {
        "one track": ([[ta[0]], [ta[1]], [ta[2]]], 1, 0),
        "two tracks": ([[ta[0], tb[0]], [tb[1], ta[1]], [ta[2], tb[2]]], 2, 1),
        "track and a near layer-2 hit": ([[ta[0]], [ta[1]], [ta[2], near[2]]], 2, 0),
        "track, hits duplicated": ([[ta[0]] * 2, [ta[1]] * 2, [ta[2]] * 2], 8, 1),
        "track, layer 0 duplicated": ([[ta[0]] * 2, [ta[1]], [ta[2]]], 2, 0),
        "two near hits in layers 0 and 2 around one layer-1 hit":
            ([[ta[0], _track(a, dx=(0.04, 0, 0))[0]], [ta[1]], [ta[2], near[2]]], 4, 0),
        "two tracks, one duplicated": ([[ta[0], tb[0], tb[0]], [tb[1], ta[1], tb[1]], [ta[2], tb[2]]], 5, 1),
    }
    s = synth.from_layers([v[0] for v in events.values()])
    c, acc, _, _ = R.select_set(s)
    d = R.disjoint_accept(s.offsets, s.x, s.y)
    for k, (name, (_, want_c, want_d)) in enumerate(events.items()):
        assert c[k] == want_c, (name, c[k])
        assert d[k] == want_d, (name, d[k])
    assert (d <= acc).all()  # two particles need at least two triplets


@pytest.mark.parametrize("test", ["msd", "msd_basis", "window"])
def test_disjoint_acceptance_invariants(oracle_lib, test):
    """On events with many passing triplets (sigma = 0 pairs, hits
    duplicated): two-particle acceptance implies two passing triplets, does
    not depend on the order of the hits within a layer, and equals the count
    mode on events whose passing triplets are two exact tracks."""
    base = synth.make_event_set(synth.EventSetSpec(n_events=3000, hits_mean=6, p_inject=0.5, sigma=0.0, salt=91))
    cfg = R.OracleConfig(test=test)
    c, _, _, _ = R.select_set(base, cfg)
    d = R.disjoint_accept(base.offsets, base.x, base.y, cfg)
    assert ((d == 1) <= (c >= 2)).all()
    assert d.sum() > 100
    rng = np.random.default_rng(3)
    perm = np.arange(base.n_hits)
    for q in range(3 * base.n_events):
        lo, hi = base.offsets[q], base.offsets[q + 1]
        perm[lo:hi] = lo + rng.permutation(hi - lo)
    assert np.array_equal(R.disjoint_accept(base.offsets, base.x[perm], base.y[perm], cfg), d)


# --------------------------------------------------------------- per-hit z ---

def _with_z(s, z):
    return synth.EventSet(s.offsets, s.x, s.y, s.n_tracks, z=np.asarray(z, np.float32))


def test_per_hit_z_at_layer_positions_equals_layer_path(oracle_lib):
    """Per-hit z equal to the layer positions gives the layer path's counts
    for the fit and the window test: at the default geometry the binary32
    division 1 / Szz and the rounded binary64 reciprocal are the same number,
    so both paths take the same slope."""
    z32 = [np.float32(v) for v in Z]
    szz = (z32[0] * z32[0] + z32[1] * z32[1]) + z32[2] * z32[2]
    assert np.float32(1.0) / szz == np.float32(1.0 / float(szz))
    s = synth.make_event_set(synth.SMALL_10K, n_events=3000)
    n = np.diff(s.offsets.astype(np.int64))
    zh = np.asarray(Z, np.float32)[np.repeat(np.tile(np.arange(3), s.n_events), n)]
    for test in ("msd", "window"):
        cfg = R.OracleConfig(test=test)
        assert np.array_equal(R.select_set(_with_z(s, zh), cfg)[0], R.select_set(s, cfg)[0])


def test_per_hit_z_near_threshold_against_exact_fit(oracle_lib):
    """Staggered z per hit (z_l -/+ 0.75 cm, all eight combinations): the
    fp32 MSD of near-threshold triplets stays within the rigorous bound of its
    own evaluation order (binary32 reciprocal of the triplet's Szz) from the
    exact rational fit, and the decision equals the exact decision outside
    that band."""
    rng = np.random.default_rng(21)
    T = 0.03
    T32 = Fraction(float(np.float32(T)))
    decided = 0
    for combo in range(8):
        zt = tuple(Z[l] + (0.75 if (combo >> l) & 1 else -0.75) for l in range(3))
        ci, cj, ck = helpers.near_threshold_triplets(80, seed=100 + combo, plane_T=T, rel=3e-3, z=zt)
        bound = R.fp32_fit_error_bound(ci, cj, ck, zt, w_division=True)
        # one event per triplet: (x, y) = (c, 0) passes the y plane
        s = synth.from_layers([[[(float(ci[t]), 0.0)], [(float(cj[t]), 0.0)], [(float(ck[t]), 0.0)]]
                               for t in range(len(ci))])
        zh = np.tile(np.asarray(zt, np.float32), len(ci))
        got = R.select_set(_with_z(s, zh), R.OracleConfig(msd_max=(T, T)))[0]
        for t in range(len(ci)):
            exact = R.fit_msd_exact(ci[t], cj[t], ck[t], zt, 2)
            if abs(exact - T32) > Fraction(float(bound[t])) / 2 + T32 * Fraction(1, 2 ** 21):
                decided += 1
                assert bool(got[t]) == (exact <= T32), (combo, t)
    assert decided > 500


def test_per_hit_z_invariants(oracle_lib):
    """Staggered events: doubling every z leaves every decision bit-exact
    (the slope halves exactly and m z is unchanged), and so does permuting the
    hits of a layer together with their z; exact tracks on staggered modules
    still pass."""
    base = synth.make_event_set(synth.EventSetSpec(n_events=2000, hits_mean=6, p_inject=0.5, sigma=0.0, salt=33))
    s = synth.staggered(base)
    assert len(np.unique(s.z)) == 6
    for test in ("msd", "window"):
        cfg = R.OracleConfig(test=test)
        c = R.select_set(s, cfg)[0]
        assert (c[base.n_tracks > 0] >= 2).all()
        if test == "msd":
            assert np.array_equal(R.select_set(_with_z(s, 2 * s.z), cfg)[0], c)
        rng = np.random.default_rng(4)
        perm = np.arange(s.n_hits)
        for q in range(3 * s.n_events):
            lo, hi = s.offsets[q], s.offsets[q + 1]
            perm[lo:hi] = lo + rng.permutation(hi - lo)
        p = synth.EventSet(s.offsets, s.x[perm], s.y[perm], s.n_tracks, z=s.z[perm])
        assert np.array_equal(R.select_set(p, cfg)[0], c)
    with pytest.raises(ValueError):
        R.select_set(s, R.OracleConfig(test="msd_basis"))
