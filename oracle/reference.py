"""CPU oracle for the trigger-station triplet selection (paper Sec. 3.2).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product library, which shares no
code with it.

Contents
  * ``OracleConfig``             the parameters of the selection.
  * ``select``                   the plain C oracle (trig_oracle.c,
                                 ``trig_select_ref``) over a batch of events:
                                 per-event passing-triplet counts, accept
                                 flags, error bits; fp32 decisions.
  * ``select_numpy``             an independent NumPy float32 implementation of
                                 the same fp32 decisions (vectorised per event).
  * ``msd_disagreements``        per event, the triplets whose decision differs
                                 between the two evaluation orders of the fit.
  * ``fit_msd_exact``            the paper's fit through the vertex in exact
                                 rational arithmetic (``fractions.Fraction``).
  * ``fit_msd_f64``              the same fit in float64 (vectorised).
  * ``fp32_fit_error_bound``     a rigorous bound on |Q_fp32 - Q_exact| for the
                                 default (fit written out) evaluation.
  * ``fp32_error_bound``         the same for the basis-form evaluation.
  * ``disjoint_accept``          two-particle acceptance: two passing triplets
                                 with no hit in common (Sec. 3.1).
  * ``accepted_ids``             ascending ids of accepted events.
  * ``filter_stations``          trigger-station filtering, the step before the
                                 selection: per event the hits of the three
                                 trigger layers, in input order.
  * ``build_events``             event building from a time-ordered stream
                                 (time-gap clustering), the step before the
                                 filter; ``build_events_numpy`` the same over
                                 whole arrays.

The fp32 decision contract, MSD test (default): the fit of Sec. 3.2 step 2
written out, per plane c in {x, y} with the hits c_i, c_j, c_k of layers 0, 1,
2 (every line one rounding to binary32 per operation, left to right):
    Szz = (z0*z0 + z1*z1) + z2*z2,   w = f32(1 / f64(Szz))
    m   = ((c_i*z0 + c_j*z1) + c_k*z2) * w       slope of c = m z
    r_l = c_l - m*z_l                             residuals, l = 0, 1, 2
    Q   = (r0*r0 + r1*r1) + r2*r2
    pass_c  <=>  Q / ndf <= T_c                  (fp32 division, equality passes)

MSD_BASIS test: the same Q evaluated in an orthonormal basis (u, v) of the
plane orthogonal to (z0, z1, z2):
    a   = U0*c_i + U1*c_j                      (two products, then one sum)
    b   = (V0*c_i + V1*c_j) + V2*c_k
    Q   = a*a + b*b
with U0 = f32(z1/n01), U1 = f32(-z0/n01), V0 = f32(z0 z2/d), V1 = f32(z1 z2/d),
V2 = f32(-s01/d), s01 = z0^2 + z1^2, n01 = sqrt(s01), d = n01 * sqrt(s01 + z2^2),
all of it in float64 before the final rounding.  In exact arithmetic
a^2 + b^2 equals the residual sum of squares of the least-squares line
c = m z through the vertex.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "trig_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

TESTS = {"msd": 0, "window": 1, "msd_basis": 2}
INT32_MAX = 2 ** 31 - 1


@dataclass(frozen=True)
class OracleConfig:
    """Selection parameters.  Defaults: the paper's thresholds (0.03 in x-z,
    0.025 in y-z, per degree of freedom), two degrees of freedom, accept at two
    or more passing triplets; layers at 400/410/420 cm."""

    test: str = "msd"
    z: tuple = (400.0, 410.0, 420.0)
    msd_max: tuple = (0.03, 0.025)
    ndf: int = 2
    window: tuple = (0.005, 0.005)
    min_triplets: int = 2


class _Cfg(ctypes.Structure):
    _fields_ = [("test", ctypes.c_int32), ("z", ctypes.c_float * 3),
                ("msd_max", ctypes.c_float * 2), ("ndf", ctypes.c_int32),
                ("window", ctypes.c_float * 2), ("min_triplets", ctypes.c_int32)]


def _to_c(cfg: OracleConfig) -> _Cfg:
    c = _Cfg()
    c.test = TESTS[cfg.test]
    for i in range(3):
        c.z[i] = cfg.z[i]
    c.msd_max[0], c.msd_max[1] = cfg.msd_max
    c.ndf = cfg.ndf
    c.window[0], c.window[1] = cfg.window
    c.min_triplets = cfg.min_triplets
    return c


GCC_FLAGS = ["-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared", "-pthread", "-std=c11", "-Wall"]


def build(force: bool = False) -> str:
    """Compile trig_oracle.c into liboracle.so (plain gcc, contraction off)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *GCC_FLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        lib.trig_select_ref_z.restype = ctypes.c_double
        lib.trig_select_ref_z.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Cfg),
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                          ctypes.c_int32]
        lib.trig_select_ref.restype = ctypes.c_double
        lib.trig_select_ref.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Cfg),
                                      ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_uint32), ctypes.c_int32]
        lib.trig_ref_msd_disagreements.restype = ctypes.c_int64
        lib.trig_ref_msd_disagreements.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.POINTER(_Cfg), ctypes.c_void_p]
        lib.trig_ref_disjoint.restype = ctypes.c_int64
        lib.trig_ref_disjoint.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Cfg),
                                          ctypes.c_void_p]
        lib.oracle_has_disjoint_pair.restype = ctypes.c_int32
        lib.oracle_has_disjoint_pair.argtypes = [ctypes.c_int64, ctypes.c_void_p]
        lib.oracle_triplet_msd.restype = ctypes.c_float
        lib.oracle_triplet_msd.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_float,
                                           ctypes.c_float, ctypes.c_float]
        lib.oracle_basis.restype = None
        lib.oracle_basis.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def select(offsets, x, y, cfg: OracleConfig = OracleConfig(), n_threads: int = 1, z=None):
    """C oracle over a CSR batch (z: per-hit z positions, or None for the
    configured layer positions).

    Returns (counts int32[E], accept uint8[E], status uint32, seconds).
    counts[e] is the number of passing triplets, -1 for a malformed layer
    range, -2 if n0*n1*n2 exceeds INT32_MAX; accept[e] = counts[e] >= min."""
    lib = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    xs = np.ascontiguousarray(x, dtype=np.float32)
    ys = np.ascontiguousarray(y, dtype=np.float32)
    zs = None if z is None else np.ascontiguousarray(z, dtype=np.float32)
    n_ev = (len(off) - 1) // 3
    counts = np.zeros(n_ev, np.int32)
    accept = np.zeros(n_ev, np.uint8)
    st = ctypes.c_uint32(0)
    c = _to_c(cfg)
    dt = lib.trig_select_ref_z(n_ev, _ptr(off), len(xs), _ptr(xs), _ptr(ys), None if zs is None else _ptr(zs),
                               ctypes.byref(c), _ptr(counts), _ptr(accept), ctypes.byref(st), int(n_threads))
    if dt < 0:
        raise ValueError("trig_select_ref rejected its arguments")
    return counts, accept, int(st.value), float(dt)


def select_set(evset, cfg: OracleConfig = OracleConfig(), n_threads: int = 1):
    return select(evset.offsets, evset.x, evset.y, cfg, n_threads, z=getattr(evset, "z", None))


def msd_disagreements(offsets, x, y, cfg: OracleConfig = OracleConfig(), n_threads: int = 1):
    """Per event, the number of triplets whose decision differs between the
    MSD (fit written out) and MSD_BASIS evaluations of the fit, both planes
    (cfg.test is ignored).  int32[E]; malformed events count 0."""
    from concurrent.futures import ThreadPoolExecutor
    lib = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    xs = np.ascontiguousarray(x, dtype=np.float32)
    ys = np.ascontiguousarray(y, dtype=np.float32)
    n_ev = (len(off) - 1) // 3
    out = np.zeros(n_ev, np.int32)
    c = _to_c(cfg)
    n_threads = max(1, int(n_threads))
    bounds = np.linspace(0, n_ev, 4 * n_threads + 1).astype(np.int64)

    def run(k):
        e0, e1 = int(bounds[k]), int(bounds[k + 1])
        if e1 > e0:
            part = out[e0:e1]
            r = lib.trig_ref_msd_disagreements(e0, e1, _ptr(off), len(xs), _ptr(xs), _ptr(ys), ctypes.byref(c),
                                               part.ctypes.data_as(ctypes.c_void_p))
            if r < 0:
                raise ValueError("trig_ref_msd_disagreements rejected its arguments")

    with ThreadPoolExecutor(n_threads) as ex:
        list(ex.map(run, range(len(bounds) - 1)))
    return out


def disjoint_accept(offsets, x, y, cfg: OracleConfig = OracleConfig(), n_threads: int = 1, z=None):
    """Two-particle acceptance per event (uint8[E]): 1 if two of the event's
    passing triplets have no hit in common (the trigger signature of Sec. 3.1,
    two particles pointing back to the target), else 0.  The passing triplets
    are listed and every pair compared (trig_ref_disjoint)."""
    from concurrent.futures import ThreadPoolExecutor
    lib = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    xs = np.ascontiguousarray(x, dtype=np.float32)
    ys = np.ascontiguousarray(y, dtype=np.float32)
    zs = None if z is None else np.ascontiguousarray(z, dtype=np.float32)
    n_ev = (len(off) - 1) // 3
    out = np.zeros(n_ev, np.uint8)
    c = _to_c(cfg)
    n_threads = max(1, int(n_threads))
    bounds = np.linspace(0, n_ev, 4 * n_threads + 1).astype(np.int64)

    def run(k):
        e0, e1 = int(bounds[k]), int(bounds[k + 1])
        if e1 > e0:
            part = out[e0:e1]
            r = lib.trig_ref_disjoint(e0, e1, _ptr(off), len(xs), _ptr(xs), _ptr(ys),
                                      None if zs is None else _ptr(zs), ctypes.byref(c),
                                      part.ctypes.data_as(ctypes.c_void_p))
            if r < 0:
                raise ValueError("trig_ref_disjoint rejected its arguments")

    with ThreadPoolExecutor(n_threads) as ex:
        list(ex.map(run, range(len(bounds) - 1)))
    return out


def has_disjoint_pair(triplets) -> bool:
    """Whether a list of (i, j, k) hit-index triplets holds two with no hit
    in common (the oracle's pair comparison)."""
    t = np.ascontiguousarray(np.asarray(triplets, dtype=np.int64).reshape(-1, 3))
    return bool(_load().oracle_has_disjoint_pair(len(t), t.ctypes.data_as(ctypes.c_void_p)))


def triplet_msd_c(cfg: OracleConfig, ci: float, cj: float, ck: float) -> float:
    """fl(Q/ndf) of one triplet in one plane as the C oracle computes it."""
    c = _to_c(cfg)
    return float(_load().oracle_triplet_msd(ctypes.byref(c), ci, cj, ck))


def basis_c(cfg: OracleConfig) -> np.ndarray:
    out = np.zeros(5, np.float32)
    c = _to_c(cfg)
    _load().oracle_basis(ctypes.byref(c), _ptr(out))
    return out


def accepted_ids(accept: np.ndarray) -> np.ndarray:
    """Ascending ids of accepted events (the list of selected events that the
    paper transfers back to the host, Sec. 5.3 step 6)."""
    return np.flatnonzero(np.asarray(accept) != 0).astype(np.int32)


# --------------------------------------------------------------------------
# Independent NumPy float32 implementation of the same decisions
# --------------------------------------------------------------------------

def basis_f32(z):
    """(U0, U1, V0, V1, V2) as float32, from the float64 formulas above."""
    z0, z1, z2 = (float(np.float32(v)) for v in z)
    s01 = z0 * z0 + z1 * z1
    n01 = math.sqrt(s01)
    d = n01 * math.sqrt(s01 + z2 * z2)
    return tuple(np.float32(v) for v in (z1 / n01, -z0 / n01, (z0 * z2) / d,
                                          (z1 * z2) / d, -s01 / d))


def _plane_pass_np(ci, cj, ck, cfg: OracleConfig, plane: int):
    """Boolean [n0, n1, n2] array of plane decisions for one event."""
    f32 = np.float32
    T = f32(cfg.msd_max[plane]) if cfg.test != "window" else None
    if cfg.test == "msd_basis":
        U0, U1, V0, V1, V2 = basis_f32(cfg.z)
        a = (U0 * ci)[:, None] + (U1 * cj)[None, :]
        b = ((V0 * ci)[:, None] + (V1 * cj)[None, :])[:, :, None] + (V2 * ck)[None, None, :]
        q = (a * a)[:, :, None] + b * b
        return (q / f32(cfg.ndf)) <= T
    if cfg.test == "msd":
        z = [f32(v) for v in cfg.z]
        szz = (z[0] * z[0] + z[1] * z[1]) + z[2] * z[2]
        w = f32(1.0 / float(szz))
        p0, p1, p2 = ci * z[0], cj * z[1], ck * z[2]
        s = (p0[:, None] + p1[None, :])[:, :, None] + p2[None, None, :]
        m = s * w
        r0 = ci[:, None, None] - m * z[0]
        r1 = cj[None, :, None] - m * z[1]
        r2 = ck[None, None, :] - m * z[2]
        q = (r0 * r0 + r1 * r1) + r2 * r2
        return (q / f32(cfg.ndf)) <= T
    W = f32(cfg.window[plane])
    z = [f32(v) for v in cfg.z]
    si, sj, sk = ci / z[0], cj / z[1], ck / z[2]
    ok_j = np.abs(sj[None, :] - si[:, None]) < W
    ok_k = np.abs(sk[None, :] - si[:, None]) < W
    return ok_j[:, :, None] & ok_k[:, None, :]


def select_numpy(offsets, x, y, cfg: OracleConfig = OracleConfig()):
    """Same outputs as ``select`` (without timing), event by event in NumPy."""
    off = np.asarray(offsets, dtype=np.int64)
    xs = np.asarray(x, dtype=np.float32)
    ys = np.asarray(y, dtype=np.float32)
    n_ev = (len(off) - 1) // 3
    counts = np.zeros(n_ev, np.int32)
    status = 0
    with np.errstate(all="ignore"):
        for e in range(n_ev):
            o = off[3 * e: 3 * e + 4]
            if not (0 <= o[0] <= o[1] <= o[2] <= o[3] <= len(xs)):
                counts[e] = -1
                status |= 1
                continue
            n = np.diff(o)
            if int(n[0]) * int(n[1]) * int(n[2]) > INT32_MAX:
                counts[e] = -2
                status |= 2
                continue
            if n.min() == 0:
                continue
            seg = [slice(o[l], o[l + 1]) for l in range(3)]
            px = _plane_pass_np(xs[seg[0]], xs[seg[1]], xs[seg[2]], cfg, 0)
            py = _plane_pass_np(ys[seg[0]], ys[seg[1]], ys[seg[2]], cfg, 1)
            counts[e] = int(np.count_nonzero(px & py))
    accept = ((counts >= 0) & (counts >= cfg.min_triplets)).astype(np.uint8)
    return counts, accept, status


# --------------------------------------------------------------------------
# The fit as the paper states it, in exact and in float64 arithmetic
# --------------------------------------------------------------------------

def fit_msd_exact(ci, cj, ck, z, ndf) -> Fraction:
    """MSD per degree of freedom of the least-squares line c = m z through
    the vertex, fitted to the three hits of one plane (paper Sec. 3.2, step
    2a/2b), in exact rational arithmetic on the binary32 input values."""
    c = [Fraction(float(np.float32(v))) for v in (ci, cj, ck)]
    zz = [Fraction(float(np.float32(v))) for v in z]
    m = sum(cl * zl for cl, zl in zip(c, zz)) / sum(zl * zl for zl in zz)
    q = sum((cl - m * zl) ** 2 for cl, zl in zip(c, zz))
    return q / ndf


def fit_msd_f64(ci, cj, ck, z, ndf):
    """Same fit in float64, vectorised over arrays of triplets."""
    ci, cj, ck = (np.asarray(v, dtype=np.float32).astype(np.float64) for v in (ci, cj, ck))
    z0, z1, z2 = (float(np.float32(v)) for v in z)
    m = (ci * z0 + cj * z1 + ck * z2) / (z0 * z0 + z1 * z1 + z2 * z2)
    q = (ci - m * z0) ** 2 + (cj - m * z1) ** 2 + (ck - m * z2) ** 2
    return q / ndf


def fp32_fit_error_bound(ci, cj, ck, z, w_division=False):
    """Upper bound on |Q_fp32 - Q_exact| for the default evaluation (the fit
    written out), before the division by ndf, vectorised over triplets of
    finite binary32 inputs whose intermediate results stay finite.

    Standard model: every operation returns x(1 + d), |d| <= u = 2^-24 (an
    intermediate that falls into the subnormal range adds at most 2^-150
    absolute; the result carries a slack far above that).  With
    P = sum c_l z_l, A = sum |c_l| z_l, S = sum z_l^2 (exact, on the binary32
    z), g3 = 3u / (1 - 3u):
      s = (c_i z0 + c_j z1) + c_k z2:   |s - P| <= g3 A
      w = (1/S)(1 + e_w), e_w measured on the binary32 w of the contract
      m = s w (1 + d):                   |m - m*| <= dm =
            [g3 A (1 + e_w)(1 + u) + |P| (e_w + u + e_w u)] / S
      t_l = m z_l (1 + d), r_l = (c_l - t_l)(1 + d):
            |r_l - r*_l| <= dl = dm z_l + u |m| z_l + u |c_l - t_l|,
            |m| <= |m*| + dm,  |c_l - t_l| <= |r*_l| + dm z_l + u |m| z_l
      Q = (r0^2 + r1^2) + r2^2, three roundings on each term:
            |Q - sum r_l^2| <= g3 sum r_l^2
    hence |Q - Q*| <= sum_l (2 |r*_l| dl + dl^2) + g3 sum_l (|r*_l| + dl)^2,
    with r*_l = c_l - m* z_l the exact residuals.  Evaluated in float64 with
    a relative slack of 1e-6 and an absolute one of 1e-30."""
    u = 2.0 ** -24
    g3 = 3 * u / (1 - 3 * u)
    zf = [float(np.float32(v)) for v in z]
    z32 = [np.float32(v) for v in z]
    szz32 = (z32[0] * z32[0] + z32[1] * z32[1]) + z32[2] * z32[2]
    # w as the evaluation takes it: f32(1 / f64(Szz)) for layer positions, a
    # binary32 division for per-hit z (w_division)
    w32 = np.float32(1.0) / szz32 if w_division else np.float32(1.0 / float(szz32))
    S_exact = sum(Fraction(v) ** 2 for v in zf)
    e_w = float(abs(Fraction(float(w32)) * S_exact - 1))
    S = float(S_exact)
    c = [np.asarray(v, dtype=np.float32).astype(np.float64) for v in (ci, cj, ck)]
    P = sum(cl * zl for cl, zl in zip(c, zf))
    A = sum(np.abs(cl) * zl for cl, zl in zip(c, zf))
    mstar = P / S
    dm = (g3 * A * (1 + e_w) * (1 + u) + np.abs(P) * (e_w + u + e_w * u)) / S
    mabs = np.abs(mstar) + dm
    total = 0.0
    sq = 0.0
    for cl, zl in zip(c, zf):
        rstar = cl - mstar * zl
        ct = np.abs(rstar) + dm * zl + u * mabs * zl
        dl = dm * zl + u * mabs * zl + u * ct
        total = total + 2 * np.abs(rstar) * dl + dl * dl
        sq = sq + (np.abs(rstar) + dl) ** 2
    return (total + g3 * sq) * (1 + 1e-6) + 1e-30


def fp32_error_bound(ci, cj, ck, z):
    """Upper bound on |Q_fp32 - Q_exact| for the basis-form evaluation
    (before the division by ndf), vectorised.

    With u = 2^-24 and exact basis (u0, u1, v0, v1, v2): each fp32 constant
    carries a relative error <= u(1 + 2^-28) (float64 evaluation, then one
    rounding); a is a two-term dot product with two roundings on top, b a
    three-term one with three; so |a_fp - a| <= 4u (|u0 ci| + |u1 cj|) and
    |b_fp - b| <= 5u (|v0 ci| + |v1 cj| + |v2 ck|) (generous).  Squaring and
    the final sum add at most 3u |Q| (+ O(u^2)).  The bound returned is
    2|a|da + da^2 + 2|b|db + db^2 + 4u(a^2 + b^2 + da^2 + db^2) with a, b
    taken from the float64 evaluation plus their own error."""
    u = 2.0 ** -24
    z0, z1, z2 = (float(np.float32(v)) for v in z)
    s01 = z0 * z0 + z1 * z1
    n01 = math.sqrt(s01)
    d = n01 * math.sqrt(s01 + z2 * z2)
    bu = (z1 / n01, -z0 / n01)
    bv = ((z0 * z2) / d, (z1 * z2) / d, -s01 / d)
    ci, cj, ck = (np.asarray(v, dtype=np.float32).astype(np.float64) for v in (ci, cj, ck))
    a = bu[0] * ci + bu[1] * cj
    b = bv[0] * ci + bv[1] * cj + bv[2] * ck
    da = 4 * u * (abs(bu[0] * ci) + abs(bu[1] * cj)) * (1 + 1e-6)
    db = 5 * u * (abs(bv[0] * ci) + abs(bv[1] * cj) + abs(bv[2] * ck)) * (1 + 1e-6)
    aa = np.abs(a) + da
    bb = np.abs(b) + db
    return 2 * aa * da + da * da + 2 * bb * db + db * db + 4 * u * (aa * aa + bb * bb)


def filter_stations(offsets, station, x, y, layers):
    """Trigger-station filtering, the step before the selection (the paper
    keeps only the trigger station's hits before the transfer to the GPU,
    Sec. 5.3, implementation i3).  Written from its definition, event by
    event: the hits of trigger layer l of event e are the hits h in
    [offsets[e], offsets[e+1]) with station[h] == layers[l], in input order.
    An event whose range is not within [0, n_hits], is decreasing or holds
    more than 2^31 - 1 hits keeps no hit and sets status bit 1.

    Returns (layer_offsets int32[3E+1], x fp32[total], y fp32[total], status)
    in the selection's input layout (event, then layer)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    station = np.asarray(station, dtype=np.uint8)
    n_events, n_hits = len(offsets) - 1, len(station)
    starts, xs, ys, status, at = [], [], [], 0, 0
    for e in range(n_events):
        a, b = int(offsets[e]), int(offsets[e + 1])
        ok = 0 <= a <= b <= n_hits and b - a <= 2**31 - 1
        if not ok:
            status |= 1
        for layer in layers:
            starts.append(at)
            if ok:
                idx = a + np.flatnonzero(station[a:b] == layer)
                xs.append(np.asarray(x)[idx])
                ys.append(np.asarray(y)[idx])
                at += len(idx)
    starts.append(at)
    cat = (lambda parts: np.concatenate(parts).astype(np.float32) if parts else np.zeros(0, np.float32))
    return np.asarray(starts, dtype=np.int64).astype(np.int32), cat(xs), cat(ys), status


def build_events(t, gap):
    """Event building from a time-ordered hit stream (the paper's outlook,
    Sec. 8: free-streaming data, hits with times and no hardware trigger; it
    gives no algorithm).  Reading: time-gap clustering.  Written from its
    definition, hit by hit: a new event starts at the first hit and at every
    hit whose time exceeds the previous hit's by more than gap (times are
    Python integers here, so the difference is exact); a hit whose time is
    below the previous hit's sets status bit 1 and starts no event.

    Returns (offsets int64[E+1] over the stream's order, status)."""
    t = [int(v) for v in np.asarray(t, dtype=np.int64)]
    gap = int(gap)
    starts, status = [], 0
    for h, th in enumerate(t):
        if h == 0:
            starts.append(0)
            continue
        if th < t[h - 1]:
            status |= 1
        elif th - t[h - 1] > gap:
            starts.append(h)
    offsets = starts + [len(t)] if t else [0]
    return np.asarray(offsets, dtype=np.int64), status


def build_events_numpy(t, gap):
    """build_events with numpy over whole arrays (same definition; for the
    full-size checks): the unsigned 64-bit difference of two int64 times is
    the true difference whenever the later time is the larger one."""
    t = np.asarray(t, dtype=np.int64)
    if len(t) == 0:
        return np.zeros(1, np.int64), 0
    up = t[1:] > t[:-1]
    diff = t[1:].view(np.uint64) - t[:-1].view(np.uint64)
    new = up & (diff > np.uint64(gap))
    status = 1 if bool((t[1:] < t[:-1]).any()) else 0
    offsets = np.concatenate([[0], np.flatnonzero(new) + 1, [len(t)]]).astype(np.int64)
    return offsets, status
