"""Writes handbuilt.json: hand-built trigger-station events whose passing
triplet counts follow from closed forms, not from any implementation.

Run from the repository root:  python tests/golden/make_golden.py

Closed forms used (layers at z = (400, 410, 420) cm, Sz2 = 504500 cm^2):
  * A track through the vertex, c_l = m z_l, has zero fit residual: it passes
    any non-negative threshold (paper Sec. 3.2 step 2: the fit is c = m z).
  * Moving one hit of such a track by delta along x in layer j leaves the y
    plane untouched and gives the x-z fit a residual sum of squares
    Q = delta^2 (1 - z_j^2 / Sz2): the squared length of the part of
    delta*e_j orthogonal to z.  The triplet passes the x plane iff
    Q / ndf <= 0.03 (paper Sec. 3.2 step 2b; ndf the degrees of freedom).
      layer 0: 1 - z0^2/Sz2 = 0.682854;  layer 1: 0.666799;  layer 2: 0.650347
  * Triplets mixing hits of tracks with clearly different slopes have a
    residual of order (slope difference) x (10 cm), far above the cut.
  * Every passing triplet is counted (step 3 counts triplets), so duplicating
    each hit of a track d times multiplies its triplets by d^3.
No number in the output is computed by the oracle or by the GPU library.
"""
import json
import os

Z = (400.0, 410.0, 420.0)
SZ2 = sum(z * z for z in Z)


def track(mx, my, dx=(0.0, 0.0, 0.0), dy=(0.0, 0.0, 0.0)):
    """Per-layer hits of a vertex-pointing track with optional displacements."""
    return [[(mx * Z[l] + dx[l], my * Z[l] + dy[l])] for l in range(3)]


def merge(*events):
    out = [[], [], []]
    for ev in events:
        for l in range(3):
            out[l].extend(ev[l])
    return out


def dup(ev, d):
    return [[h for h in layer for _ in range(d)] for layer in ev]


def factor(j):
    return 1.0 - Z[j] * Z[j] / SZ2


CASES = []


def case(name, layers, expected, why, cite, cfg=None):
    CASES.append({"name": name, "layers": [[list(h) for h in layer] for layer in layers],
                  "expected_count": expected, "why": why, "cite": cite,
                  "cfg": cfg or {}})


STEP2 = "paper Sec. 3.2, Algorithm, step 2 (fit through the vertex, MSD cut 0.03 / 0.025)"
STEP13 = "paper Sec. 3.2, Algorithm, steps 1 and 3 (all one-hit-per-layer triplets, count)"

case("one_track", track(0.25, 0.125), 1,
     "single vertex-pointing track: zero residual, one triplet", STEP2)
case("two_tracks", merge(track(0.25, 0.125), track(-0.3, 0.2)), 2,
     "two vertex-pointing tracks; the six mixed triplets have slope differences "
     "of 0.55/0.075 and residuals of metres", STEP13)
case("three_tracks", merge(track(0.25, 0.125), track(-0.3, 0.2), track(0.1, -0.35)), 3,
     "three well separated tracks", STEP13)
case("duplicated_hits_d2", dup(merge(track(0.25, 0.125), track(-0.3, 0.2)), 2), 16,
     "each hit of two tracks duplicated twice: 2 * 2^3 passing triplets", STEP13)
case("duplicated_hits_d3", dup(track(-0.2, -0.2), 3), 27,
     "each hit of one track three times: 3^3 passing triplets", STEP13)
empty = merge(track(0.25, 0.125), track(-0.3, 0.2))
empty[2] = []
case("empty_layer", empty, 0, "no hit in layer 2: no triplet exists", STEP13)
off_axis = [[(100.0, 0.0), (0.0, 100.0), (-100.0, 0.0), (0.0, -100.0)],
            [(160.0, 0.0), (0.0, 160.0), (-160.0, 0.0), (0.0, -160.0)],
            [(40.0, 0.0), (0.0, 40.0), (-40.0, 0.0), (0.0, -40.0)]]
case("off_axis_noise", off_axis, 0,
     "hits at radii 100/160/40 cm: no triplet points back to the vertex", STEP2)

# Single displaced hit: Q = delta^2 * factor(j); cut Q/ndf <= T.
for j, delta, ndf in [(1, 0.29, 2), (1, 0.31, 2), (1, 0.36, 3), (1, 0.38, 3), (1, 0.36, 2),
                      (0, 0.30, 2), (2, 0.30, 2), (0, 0.29, 2), (2, 0.31, 2)]:
    dx = [0.0, 0.0, 0.0]
    dx[j] = delta
    q = delta * delta * factor(j)
    passes = q / ndf <= 0.03
    case(f"displaced_x_layer{j}_d{delta}_ndf{ndf}", track(0.25, 0.125, dx=tuple(dx)),
         int(passes),
         f"x displaced by {delta} cm in layer {j}: Q = {q:.6f}, Q/ndf = {q / ndf:.6f} "
         f"{'<=' if passes else '>'} 0.03", STEP2, {"ndf": ndf})
for j, delta in [(1, 0.27), (1, 0.28)]:
    dy = [0.0, 0.0, 0.0]
    dy[j] = delta
    q = delta * delta * factor(j)
    passes = q / 2 <= 0.025
    case(f"displaced_y_layer{j}_d{delta}", track(0.25, 0.125, dy=tuple(dy)), int(passes),
         f"y displaced by {delta} cm in layer {j}: Q/2 = {q / 2:.6f} "
         f"{'<=' if passes else '>'} 0.025 (the y-z threshold)", STEP2)
# the same 0.28 cm displacement in x passes the looser x-z threshold
case("displaced_x_layer1_d0.28", track(0.25, 0.125, dx=(0.0, 0.28, 0.0)), 1,
     f"x displaced by 0.28 cm in layer 1: Q/2 = {0.28 ** 2 * factor(1) / 2:.6f} <= 0.03", STEP2)

# Slope-window test: |c_l/z_l - c_0/z_0| < W for l = 1, 2.
for delta, expect in [(2.0, 1), (2.2, 0)]:
    case(f"window_layer2_dx{delta}", track(0.25, 0.125, dx=(0.0, 0.0, delta)), expect,
         f"slope change {delta}/420 = {delta / 420:.5f} vs window 0.005",
         "slope window 0.005 on layers 2 and 3 relative to layer 1", {"test": "window"})

# Equality at the threshold passes (a triplet is rejected only if its MSD is
# above the cut): hits on the beam line give Q = 0 exactly in any evaluation
# order, and a zero threshold must still accept them.
case("beam_line_zero_threshold", [[(0.0, 0.0)], [(0.0, 0.0)], [(0.0, 0.0)]], 1,
     "Q = 0 exactly and the cut is Q/ndf <= 0: equality passes", STEP2,
     {"msd_max": [0.0, 0.0]})
# The slope window compares layers 2 and 3 with layer 1 (not with each other).
case("window_vs_layer1_chain", [[(0.0, 0.0)], [(1.64, 0.0)], [(3.36, 0.0)]], 0,
     "slopes 0, 0.004, 0.008: layer 3 is 0.008 from layer 1 (0.004 from layer 2)",
     "slope window 0.005 on layers 2 and 3 relative to layer 1", {"test": "window"})
case("window_vs_layer1_fan", [[(0.0, 0.0)], [(1.64, 0.0)], [(-1.68, 0.0)]], 1,
     "slopes 0, 0.004, -0.004: both within 0.005 of layer 1 (0.008 apart)",
     "slope window 0.005 on layers 2 and 3 relative to layer 1", {"test": "window"})
# The window inequality is strict: 102.5/410 = 0.25 exactly.
case("window_equality_fails", [[(0.0, 0.0)], [(102.5, 0.0)], [(0.0, 0.0)]], 0,
     "slope difference exactly 0.25 with window 0.25: strict '<' rejects",
     "slope window |dx/z| < W", {"test": "window", "window": [0.25, 0.25]})
case("window_just_inside", [[(0.0, 0.0)], [(102.4, 0.0)], [(0.0, 0.0)]], 1,
     "slope difference 0.24976 < 0.25", "slope window |dx/z| < W",
     {"test": "window", "window": [0.25, 0.25]})

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "handbuilt.json")
    with open(out, "w") as f:
        json.dump({"z": Z, "cases": CASES}, f, indent=1)
    print(f"wrote {len(CASES)} cases to {out}")
