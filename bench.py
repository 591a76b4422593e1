#!/usr/bin/env python3
"""Throughput of the trigger-station triplet selection on one MI355X.

One step = one trig_select call over the whole resident batch (validation,
triplet counting, accept flags and the ordered accepted-id list) in the
production form: the batched form (workgroups staging event blocks in LDS,
exact pair pruning) with the launch shape the library's autotuner picks on
this batch during the warm-up.  The plain one-wave-per-event brute-force form is timed beside it on
the same input, and both must produce identical counts.  A serving leg then
streams timeslices cut from the same events through the serving runtime at a
fixed offered load and reports p50/p99 slice latency.  Inputs are generated on the host
(seeded, synthetic), copied to HBM before the timed region, and outputs stay
in HBM.

Prints ONE JSON line (stdout).  Progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload medium_1m]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published HBM peak, and the fp32 vector-ALU op peak derived from the
# unit counts: 256 CUs x 128 fp32 lanes per clock (the rate behind the
# published 157.3 TFLOP/s, which counts an FMA as two) x 2.4 GHz, one
# non-fused, non-packed fp32 operation per lane per clock.
HBM_PEAK_GBS = 8000.0
VALU_F32_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12  # 78.64
OPS_PER_TRIPLET = {"msd": 28, "msd_basis": 8, "window": 4}

WORKLOAD_TEXT = {
    "medium_1m": "1,000,000 events; Poisson(30) noise hits per layer in r=[20,200] cm; "
                 "muon pair injected with p=0.01, sigma 0.3 cm; z=400/410/420 cm; MSD cut "
                 "0.03/0.025 per dof, ndf 2; accept at >=2 triplets",
    "small_10k": "10,000 events; Poisson(8) hits per layer; pair injection p=0.05",
    "mixture_4m": "4,000,000 events; Poisson(120(1-b^2)) hits per layer, b~U[0,1]; p=0.01",
    "dense_100k": "100,000 events; Poisson(200) hits per layer; 10% events with 1-3 pairs",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="medium_1m", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--test", default="msd", choices=["msd", "msd_basis", "window"])
    ap.add_argument("--form", default="auto",
                    help="form of the timed step (auto: trig_autotune picks the shape in the warm-up)")
    ap.add_argument("--compare", default="plain,pruned,persistent_pruned,binned",
                    help="other forms timed on the same input (comma separated)")
    ap.add_argument("--compare-steps", type=int, default=5, help="timed steps of each compared form")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="target wall time of the CPU-oracle baseline sample (all threads; the one-thread "
                         "sample takes about as long again)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-form", action="store_true", help="time only --form (profiling runs)")
    ap.add_argument("--shape", default="", metavar="HB,NW,EB",
                    help="explicit block_hits,block_waves,block_events for --form (profiling runs)")
    ap.add_argument("--serve-slices", type=int, default=1000,
                    help="timeslices of the serving leg (0 = skip it)")
    ap.add_argument("--serve-load", type=float, default=1e7, help="offered load of the serving leg, events/s")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--no-extra-legs", action="store_true", help="skip the two-particle and per-hit z legs")
    ap.add_argument("--filter-events", type=int, default=100_000,
                    help="events of the station-filter leg (0: skip it)")
    return ap.parse_args()


def algorithmic(sets_counts, n_events):
    """Per-launch algorithmic quantities from the layer counts."""
    n = sets_counts.astype(np.int64)
    triplets = int((n[:, 0] * n[:, 1] * n[:, 2]).sum())
    hits = int(n.sum())
    # dominant kernel: reads 3 offsets + 8 B per hit, writes the 4-byte count
    # (+1-byte flag in the plain kernel)
    return triplets, hits


def kernel_source_hash():
    h = hashlib.sha256()
    for p in ("paper_1810_11966_amd/csrc/trig.hip", "paper_1810_11966_amd/csrc/trig_device.hpp",
              "paper_1810_11966_amd/csrc/trig_block.hpp", "paper_1810_11966_amd/csrc/trig_binned.hpp"):
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, form: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f).get("records", {}).get(f"{kernel}/{workload}/{form}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return float(rec["bytes_per_launch"])


WARM_SECONDS = 0.5


def warm_gpu(torch, call, seconds=None):
    """Repeat `call` (untimed) until `seconds` of wall time have passed: the
    GPU raises its clock over the first fraction of a second of sustained
    work (a kernel timed right after three short warm-up calls ran 0.304 ms
    against 0.236 ms after 0.5 s of work, same box), and the legs measure the
    sustained rate."""
    seconds = WARM_SECONDS if seconds is None else seconds
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end:
        for _ in range(8):
            call()
        torch.cuda.synchronize()


def time_form(torch, trig, hip_events, dev_in, n_events, form, test, steps, warmup, compact=True, shape=None):
    off, x, y = dev_in
    stream = torch.cuda.current_stream().cuda_stream
    counts = torch.empty(n_events, dtype=torch.int32, device="cuda")
    accept = torch.empty(n_events, dtype=torch.uint8, device="cuda")
    ids = torch.empty(n_events, dtype=torch.int32, device="cuda")
    n_acc = torch.zeros(1, dtype=torch.int32, device="cuda")
    kw = {}
    if shape:
        kw = dict(zip(("block_hits", "block_waves", "block_events"), shape))
    p = trig.make_params(test=test, flags=trig.FORMS[form] | (trig.TRIG_OUT_COMPACT if compact else 0), **kw)
    p.out_accepted_ids = ids.data_ptr()
    p.out_n_accepted = n_acc.data_ptr()
    ws_bytes = trig.trig_workspace_bytes(n_events, p)
    ws = torch.empty(max(ws_bytes, 1) + 256, dtype=torch.uint8, device="cuda")
    addr = (ws.data_ptr() + 255) & ~255
    p.workspace = addr if ws_bytes else None
    p.workspace_bytes = ws_bytes
    ev = trig.TrigEventsCsr(n_events, off.data_ptr())
    hits = trig.TrigHits(x.numel(), x.data_ptr(), y.data_ptr())

    def call():
        rc = trig.trig_select(ev, hits, p, counts.data_ptr(), accept.data_ptr(), stream)
        if rc:
            raise trig.TrigError(rc, trig.trig_last_error_detail())

    tuned = None
    if p.flags & trig.TRIG_EXEC_AUTOTUNE:
        # the library's autotuner picks the launch shape on this batch
        # (untimed, part of the warm-up)
        rc, info = trig.trig_autotune(ev, hits, p, counts.data_ptr(), accept.data_ptr(), 3, stream)
        if rc:
            raise trig.TrigError(rc, trig.trig_last_error_detail())
        tuned = {"n_candidates": info.n_candidates, "mult_class": info.mult_class,
                 "form": "binned" if info.binned else "batched", "block_hits": info.block_hits,
                 "block_waves": info.block_waves, "block_events": info.block_events,
                 "persistent": bool(info.persistent), "ms_best": info.ms_best, "ms_rule": info.ms_rule}
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    warm_gpu(torch, call)
    starts = [hip_events.HipEvent() for _ in range(steps)]
    stops = [hip_events.HipEvent() for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        trig.trig_set_kernel_events(starts[k].handle, stops[k].handle)
        call()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    trig.trig_set_kernel_events(0, 0)
    kern_ms = [starts[k].elapsed_ms(stops[k]) for k in range(steps)]
    return {
        "elapsed_s": t1 - t0,
        "kernel_ms_mean": float(np.mean(kern_ms)),
        "kernel_ms_min": float(np.min(kern_ms)),
        "counts": counts,
        "accept": accept,
        "ids": ids[: int(n_acc.item())],
        "n_accepted": int(n_acc.item()),
        "autotuned": tuned,
    }


class SliceView:
    """Events [first, first+count) of a set: rebased offsets, x and y views."""

    def __init__(self, s, first, count):
        lo = int(s.offsets[3 * first])
        self.offsets = (s.offsets[3 * first: 3 * (first + count) + 1] - lo).astype(np.int32)
        hi = lo + int(self.offsets[-1])
        self.x, self.y = s.x[lo:hi], s.y[lo:hi]
        self.first, self.n_events = first, count


def serving_leg(s, full_counts, test, n_slices, load, n_streams, seed=11):
    """Timeslices of U[1e4, 1e6] events cut from the resident workload at
    random positions arrive as a Poisson stream with the given offered load
    (events/s); the server admits them by HBM footprint and overlaps their
    copies and kernels.  Every slice's counts must equal the full-batch
    result on the same events.  Latency = result on the host - scheduled
    arrival (so a late submit counts against it)."""
    from paper_1810_11966_amd import serve, trig
    rng = np.random.default_rng(seed)
    sizes = rng.integers(10_000, min(1_000_000, s.n_events) + 1, n_slices)
    firsts = [int(rng.integers(0, s.n_events - n + 1)) for n in sizes]
    slices = [SliceView(s, f, int(n)) for f, n in zip(firsts, sizes)]
    rate = load / float(np.mean(sizes))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_slices))
    arrivals -= arrivals[0]
    big = max(sl.x.size for sl in slices)
    dev_slice = 16 * big + 32 * int(max(sizes)) + (8 << 20)   # generous device footprint
    host_slice = 8 * big + 32 * int(max(sizes)) + (8 << 20)   # staging: inputs and results
    # the autotuned form: the record trig_autotune made on the full batch
    # covers the slices' multiplicity class
    params = trig.make_params(test=test, flags=trig.TRIG_EXEC_AUTOTUNE)
    with serve.Server(hbm_budget_bytes=(n_streams + 1) * dev_slice,
                      pinned_budget_bytes=(n_streams + 4) * host_slice,
                      n_streams=n_streams, max_pending=64, params=params) as srv:
        # one small slice first: code objects and pinned pages are warm
        srv.submit(slices[0].offsets, slices[0].x, slices[0].y)
        srv.poll(60000)
        origin = srv.now()
        trace = {}
        done, tickets, wall = serve.run_stream(srv, slices, arrivals, pace=True, poll_ms=1, deadline_s=240,
                                               submit_threads=4, trace=trace)
        st = srv.stats()
    lat, qwait, ev_done, rows = [], [], 0, []
    for i, sl in enumerate(slices):
        f = done[tickets[i]]
        if f.status != 0 or not np.array_equal(f.counts, full_counts[sl.first: sl.first + sl.n_events]):
            print(f"bench.py: served slice {i} differs from the full-batch result", file=sys.stderr)
            sys.exit(1)
        arrive = origin + arrivals[i]
        lat.append(f.t_done - arrive)
        qwait.append(f.t_admit - f.t_submit)
        ev_done += sl.n_events
        tr = trace.get(i, {})
        rows.append({"latency_ms": 1e3 * (f.t_done - arrive), "events": sl.n_events,
                     "input_mb": (sl.x.size * 8 + sl.offsets.size * 4) / 1e6,
                     "submit_delay_ms": 1e3 * (f.t_submit - arrive), "admit_ms": 1e3 * (f.t_admit - f.t_submit),
                     "admit_to_done_ms": 1e3 * (f.t_done - f.t_admit),
                     "submitter_wake_late_ms": 1e3 * tr.get("wake_late_s", float("nan")),
                     "busy_retries": tr.get("busy_retries", -1),
                     "staging_ms": 1e3 * tr.get("submit_call_s", float("nan"))})
    lat = np.array(lat) * 1e3
    mb = np.array([r["input_mb"] for r in rows])
    fit = np.linalg.lstsq(np.vstack([np.ones_like(mb), mb]).T, lat, rcond=None)[0]
    return {"slices": n_slices, "slice_events": "U[10000, 1000000]", "offered_events_per_s": load,
            "arrival_rate_per_s": rate, "events_per_s": ev_done / wall, "wall_s": wall,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "mean_admission_wait_ms": 1e3 * float(np.mean(qwait)),
            "streams": n_streams, "submit_threads": 4, "max_in_flight": int(st.max_in_flight),
            "latency": "scheduled arrival to result on the host (includes the copy into pinned staging, "
                       "H2D, kernels, D2H)",
            "latency_fit_ms": {"intercept": float(fit[0]), "per_mb": float(fit[1])},
            "submit_delay_ms": {"p50": float(np.percentile([r["submit_delay_ms"] for r in rows], 50)),
                                "p99": float(np.percentile([r["submit_delay_ms"] for r in rows], 99)),
                                "max": float(max(r["submit_delay_ms"] for r in rows))},
            "busy_rejections": int(st.rejected_busy),
            "form": "autotuned (the record of the full batch's multiplicity class)",
            "graph_capture": "none: each slice issues its copies and five launches directly on its stream",
            "slowest": sorted(rows, key=lambda r: -r["latency_ms"])[:3],
            "counts_identical_to_full_batch": True}


def cpu_baseline(s, test, target_s):
    """The oracle on the host: all threads of the affinity mask over a prefix
    sized to about target_s, and one thread over a prefix sized to about
    target_s as well."""
    from oracle import reference as R
    threads = max(1, len(os.sched_getaffinity(0)))
    cfg = R.OracleConfig(test=test)

    def sized(n_threads, budget):
        probe = min(s.n_events, 2000 if n_threads == 1 else 5000)
        _, _, _, dt = R.select_set(s.subset(0, probe), cfg, n_threads=n_threads)
        per_event = max(dt, 1e-6) / probe
        n = int(min(s.n_events, max(probe, budget / per_event)))
        counts, _, _, dt = R.select_set(s.subset(0, n), cfg, n_threads=n_threads)
        return n, dt, counts

    n, dt, counts = sized(threads, target_s)
    n1, dt1, counts1 = sized(1, target_s)
    if not np.array_equal(counts1, counts[:n1] if n1 <= n else counts1):
        print("bench.py: the oracle's counts depend on its thread count", file=sys.stderr)
        sys.exit(1)
    import platform
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": n / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} events of the workload, plain C oracle (gcc -O2, fp contraction "
                      f"off), {threads} threads, compute only, {dt:.2f} s",
            "host_cpu": cpu,
            "one_thread": {"value": n1 / dt1, "unit": "events/s", "cores": 1,
                           "sample": f"first {n1} events, 1 thread, compute only, {dt1:.2f} s"}}, counts


def _timed_calls(torch, trig, dev_in, n_ev, form, test, steps, extra_flags=0, hit_z=None):
    """Mean ms of one trig_select call (steps after one call and the GPU's
    warm-up) and its outputs."""
    off, x, y = dev_in
    r = trig.select(off, x, y, hit_z=hit_z, test=test, form=form, compact=True, extra_flags=extra_flags)

    def again():
        trig.select(off, x, y, hit_z=hit_z, test=test, form=form, compact=True, extra_flags=extra_flags,
                    workspace=r.workspace, out=(r.counts, r.accept))
    torch.cuda.synchronize()
    warm_gpu(torch, again)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        again()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps, r


def two_particle_leg(torch, trig, dev_in, n_ev, test, steps=10):
    """Two-particle acceptance (two passing triplets with no common hit) in
    the autotuned form on the resident batch: time per call and accepted
    events, beside the count mode."""
    ms, r = _timed_calls(torch, trig, dev_in, n_ev, "auto", test, steps, trig.TRIG_ACCEPT_TWO_PARTICLES)
    ms_c, rc = _timed_calls(torch, trig, dev_in, n_ev, "auto", test, steps)
    if not torch.equal(r.counts, rc.counts):
        print("bench.py: two-particle mode changed the counts", file=sys.stderr)
        sys.exit(1)
    return {"ms": ms, "events_per_s": n_ev / (ms * 1e-3), "accepted": int(r.n_accepted.item()),
            "count_mode_ms": ms_c, "count_mode_accepted": int(rc.n_accepted.item()),
            "form": "autotuned counting form, then the two-particle kernel on events with two or more passing triplets"}


def per_hit_z_leg(torch, trig, s, test, steps=5, oracle_events=5000):
    """The same events on staggered modules (each hit at z_l -/+ 0.75 cm by
    azimuthal sector, its own z per hit): the per-event slope-pruned form and
    the every-triplet form, identical counts, and the oracle on the first
    events."""
    from paper_1810_11966_amd import synth
    sz = synth.staggered(s)
    d = torch.device("cuda:0")
    dev_in = tuple(torch.from_numpy(a).to(d) for a in (sz.offsets, sz.x, sz.y))
    zt = torch.from_numpy(sz.z).to(d)
    out = {"workload": "the medium workload's events on staggered modules: z_l -/+ 0.75 cm by azimuthal "
                       "sector (16 sectors), hits moved along their line of sight"}
    ref = None
    for form in ("pruned", "plain"):
        ms, r = _timed_calls(torch, trig, dev_in, sz.n_events, form, test, steps, hit_z=zt)
        out[form] = {"ms": ms, "events_per_s": sz.n_events / (ms * 1e-3)}
        if ref is None:
            ref = r.counts.clone()
        elif not torch.equal(ref, r.counts):
            print("bench.py: per-hit z forms disagree", file=sys.stderr)
            sys.exit(1)
    from oracle import reference as R
    sub = sz.subset(0, oracle_events)
    c = R.select_set(sub, R.OracleConfig(test=test), n_threads=max(1, len(os.sched_getaffinity(0))))[0]
    if not np.array_equal(ref[:oracle_events].cpu().numpy(), c):
        print("bench.py: per-hit z counts differ from the oracle", file=sys.stderr)
        sys.exit(1)
    out["oracle_sample_bit_exact"] = f"first {oracle_events} events"
    out["pruned_vs_plain"] = out["plain"]["ms"] / out["pruned"]["ms"]
    del dev_in, zt
    torch.cuda.empty_cache()
    return out


def filter_leg(n_events, reps=20, seed=0):
    """Trigger-station filtering (include/trig_filter.h) on events with about
    5000 hits on 16 stations in detector order (the trigger layers are three
    of them, with the 1M-event workload's Poisson(30) hits each): the time of
    one call (three kernels) on the current stream, bit-exact against the
    embedded trigger-layer events, and HBM bytes per call against 8 TB/s."""
    import torch
    from paper_1810_11966_amd import filter as F
    from paper_1810_11966_amd import synth
    base = synth.make_event_set(synth.MEDIUM_1M, n_events=n_events)
    raw = synth.embed_raw(base, other_mean=378.0, shuffle=False, square=True, seed=seed)
    d = torch.device("cuda:0")
    t = [torch.from_numpy(a).to(d) for a in (raw.offsets, raw.station, raw.x, raw.y)]
    ws = torch.empty(F.workspace_bytes(raw.n_events), dtype=torch.uint8, device=d)
    r = None
    for _ in range(3):
        r = F.filter_stations(*t, raw.layers, base.n_hits, workspace=ws)
    torch.cuda.synchronize()
    if not (np.array_equal(r.layer_offsets.cpu().numpy(), base.offsets)
            and np.array_equal(r.x.cpu().numpy(), base.x) and np.array_equal(r.y.cpu().numpy(), base.y)
            and int(r.status.cpu()[0]) == 0):
        print("bench.py: the station filter's output differs from the embedded events", file=sys.stderr)
        sys.exit(1)
    warm_gpu(torch, lambda: F.repeat(r))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        F.repeat(r)  # the same call, arguments marshalled once: the library's kernels only
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    # offsets in (8 B/event), station numbers (1 B/hit), x and y of trigger hits in and out (16 B/hit),
    # offsets out (12 B/event)
    nbytes = 20 * raw.n_events + raw.n_hits + 16 * base.n_hits
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": f"{raw.n_events} events, {raw.n_hits} hits on 16 stations in detector order "
                        f"({raw.n_hits / raw.n_events:.0f} per event), {base.n_hits} of them on the trigger layers",
            "ms": ms, "events_per_s": raw.n_events / (ms * 1e-3), "bit_exact": True,
            "roofline": {"kernel": "k_filter_count + k_scan_i64 + k_filter_scatter", "bound": "hbm",
                         "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                         "algorithmic_bytes": nbytes}}


def events_leg(n_events, reps=20, seed=0, gap_ns=5):
    """Event building (include/trig_events.h) on a free-streaming timeslice:
    the filter leg's kind of events (about 5000 hits on 16 stations) as
    interactions at Poisson times of 10 MHz, each hit at its interaction's
    time plus U{0..10} ns, ordered by time; built with a 5 ns gap (pile up
    merges some interactions).  The time of one call (three kernels),
    bit-exact against the oracle's whole-array definition, and HBM bytes
    per call (8 B per hit of times, 8 B per event of offsets) against 8 TB/s."""
    import torch
    from oracle import reference as R
    from paper_1810_11966_amd import events as EB
    from paper_1810_11966_amd import synth
    base = synth.make_event_set(synth.MEDIUM_1M, n_events=n_events)
    raw = synth.embed_raw(base, other_mean=378.0, shuffle=False, square=True, seed=seed)
    s = synth.free_stream(raw, rate_hz=1e7, spread_ns=10, seed=seed)
    want, wst = R.build_events_numpy(s.t, gap_ns)
    d = torch.device("cuda:0")
    t = torch.from_numpy(s.t).to(d)
    ws = torch.empty(EB.workspace_bytes(s.n_hits) + 256, dtype=torch.uint8, device=d)
    r = None
    for _ in range(3):
        r = EB.build_events(t, gap_ns, workspace=ws)
    torch.cuda.synchronize()
    n_ev = int(r.n_events.cpu().numpy()[0])
    if not (n_ev == len(want) - 1 and np.array_equal(r.offsets[:n_ev + 1].cpu().numpy(), want)
            and int(r.status.cpu()[0]) == wst):
        print("bench.py: event building differs from the oracle", file=sys.stderr)
        sys.exit(1)
    warm_gpu(torch, lambda: EB.repeat(r))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        EB.repeat(r)  # the same call, arguments marshalled once: the library's kernels only
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    nbytes = 8 * s.n_hits + 8 * (n_ev + 1) + 8
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": f"{raw.n_events} interactions at 10 MHz, {s.n_hits} hits ({s.n_hits / raw.n_events:.0f} "
                        f"per interaction, 10 ns time spread), gap {gap_ns} ns: {n_ev} events built",
            "ms": ms, "hits_per_s": s.n_hits / (ms * 1e-3), "events_per_s": n_ev / (ms * 1e-3), "bit_exact": True,
            "roofline": {"kernel": "k_eb_count + k_scan_i64 + k_eb_scatter", "bound": "hbm", "achieved": gbs,
                         "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0, "algorithmic_bytes": nbytes}}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the selection is per event and shards trivially by "
              "event range, and the library has no multi-GPU path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1810_11966_amd import hip_events, synth, trig
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    trig.load()

    spec = synth.WORKLOADS[args.workload]
    log(f"[bench] generating {args.workload}")
    t = time.perf_counter()
    s = synth.make_event_set(spec)
    log(f"[bench] generated {s.n_events} events, {s.n_hits} hits in {time.perf_counter() - t:.1f}s")
    n_ev = s.n_events
    layer_n = s.layer_counts()
    triplets, hits = algorithmic(layer_n, n_ev)

    dev_in = tuple(torch.from_numpy(a).to("cuda") for a in (s.offsets, s.x, s.y))
    torch.cuda.synchronize()

    log(f"[bench] timing form={args.form} steps={args.steps} warmup={args.warmup}")
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    main_r = time_form(torch, trig, hip_events, dev_in, n_ev, args.form, args.test, args.steps, args.warmup,
                       shape=shape)
    ms_per_step = 1e3 * main_r["elapsed_s"] / args.steps
    value = n_ev * args.steps / main_r["elapsed_s"]
    log(f"[bench] {args.form}: {ms_per_step:.3f} ms/step, {value:.4g} events/s, "
        f"dominant kernel {main_r['kernel_ms_mean']:.3f} ms")

    # algorithmic bytes of the dominant kernel: 12 B of offsets per event,
    # 8 B per hit, 4 B count and 1 B flag per event
    kern_bytes = 12 * n_ev + 8 * hits + 5 * n_ev
    kern_s = main_r["kernel_ms_mean"] / 1e3
    tuned = main_r["autotuned"]
    if tuned:
        dominant = "k_binned" if tuned["form"] == "binned" else (
            "k_block_pipe" if tuned["persistent"] else "k_block")
    elif "binned" in args.form:
        dominant = "k_binned"
    elif "pruned" in args.form:
        dominant = "k_block_pipe" if "persistent" in args.form else "k_block"
    else:
        dominant = "k_persistent" if "persistent" in args.form else "k_plain"
    traffic = load_traffic(dominant, args.workload, args.form)
    if dominant in ("k_plain", "k_persistent"):
        # brute force: bound by the fp32 vector ALU (ops per triplet x triplets)
        ops = OPS_PER_TRIPLET[args.test] * triplets
        roofline = {"kernel": dominant, "bound": "alu", "achieved": ops / kern_s / 1e12,
                    "peak": VALU_F32_PEAK_TOPS, "unit": "TFLOP/s", "frac": ops / kern_s / 1e12 / VALU_F32_PEAK_TOPS,
                    "traffic": traffic, "ops_per_triplet": OPS_PER_TRIPLET[args.test]}
    else:
        roofline = {"kernel": dominant, "bound": "hbm", "achieved": kern_bytes / kern_s / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": kern_bytes / kern_s / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
                    "algorithmic_bytes": kern_bytes}

    extra = {}
    plain_info = None
    forms = {}
    compare = [f for f in args.compare.split(",") if f and f != args.form] if not args.only_form else []
    for form in compare:
        log(f"[bench] timing form={form} steps={args.compare_steps}")
        r = time_form(torch, trig, hip_events, dev_in, n_ev, form, args.test, args.compare_steps, 1)
        same = bool(torch.equal(r["counts"], main_r["counts"]) and torch.equal(r["ids"], main_r["ids"]))
        if not same:
            print(f"bench.py: form {form} and form {args.form} disagree", file=sys.stderr)
            sys.exit(1)
        forms[form] = {"events_per_s": n_ev * args.compare_steps / r["elapsed_s"],
                       "ms_per_step": 1e3 * r["elapsed_s"] / args.compare_steps,
                       "kernel_ms": r["kernel_ms_mean"], "counts_identical": same}
        log(f"[bench] {form}: {forms[form]['ms_per_step']:.3f} ms/step, kernel {r['kernel_ms_mean']:.3f} ms")
        if form == "plain":
            pk_s = r["kernel_ms_mean"] / 1e3
            ops = OPS_PER_TRIPLET[args.test] * triplets
            plain_info = dict(forms[form])
            plain_info["roofline"] = {"kernel": "k_plain", "bound": "alu", "achieved": ops / pk_s / 1e12,
                                      "peak": VALU_F32_PEAK_TOPS, "unit": "TFLOP/s",
                                      "frac": ops / pk_s / 1e12 / VALU_F32_PEAK_TOPS,
                                      "traffic": load_traffic("k_plain", args.workload, "plain"),
                                      "ops_per_triplet": OPS_PER_TRIPLET[args.test]}
    if plain_info:
        extra["batched_vs_plain"] = value / plain_info["events_per_s"]

    serving = None
    if args.serve_slices > 0 and not args.only_form:
        log(f"[bench] serving leg: {args.serve_slices} slices at {args.serve_load:.3g} events/s offered")
        serving = serving_leg(s, main_r["counts"].cpu().numpy(), args.test, args.serve_slices,
                              args.serve_load, args.serve_streams)
        log(f"[bench] serving: p50 {serving['p50_ms']:.2f} ms, p99 {serving['p99_ms']:.2f} ms, "
            f"{serving['events_per_s']:.4g} events/s")

    two = hz = None
    if not args.only_form and not args.no_extra_legs:
        log("[bench] two-particle leg")
        two = two_particle_leg(torch, trig, dev_in, n_ev, args.test)
        log(f"[bench] two particles: {two['ms']:.3f} ms, {two['accepted']} accepted "
            f"(count mode {two['count_mode_ms']:.3f} ms, {two['count_mode_accepted']})")
        if args.test != "msd_basis":
            log("[bench] per-hit z leg")
            hz = per_hit_z_leg(torch, trig, s, args.test)
            log(f"[bench] per-hit z: pruned {hz['pruned']['ms']:.3f} ms, plain {hz['plain']['ms']:.3f} ms")

    filt = None
    if args.filter_events > 0 and not args.only_form:
        log(f"[bench] station filter leg: {args.filter_events} events")
        filt = filter_leg(args.filter_events)
        log(f"[bench] filter: {filt['ms']:.3f} ms, {filt['events_per_s']:.4g} events/s, "
            f"{filt['roofline']['achieved']:.0f} GB/s")

    building = None
    if args.filter_events > 0 and not args.only_form:
        log(f"[bench] event building leg: {args.filter_events // 5} interactions")
        building = events_leg(args.filter_events // 5)
        log(f"[bench] event building: {building['ms']:.3f} ms, {building['hits_per_s']:.4g} hits/s, "
            f"{building['roofline']['achieved']:.0f} GB/s")

    probes = None
    if not args.only_form:
        from paper_1810_11966_amd import probe
        log("[bench] device probes: fp32 VALU rate, copy bandwidth")
        probes = {"valu_f32_tops": probe.measure_valu(torch) / 1e12,
                  "copy_gbs": probe.measure_copy(torch) / 1e9,
                  "valu_note": "non-fused, non-packed fp32 mul/add, 16 independent ops per thread and iteration",
                  "copy_note": "1 GiB float4 copy, read + write bytes per second"}
        log(f"[bench] probes: {probes['valu_f32_tops']:.1f} T fp32 ops/s, {probes['copy_gbs']:.0f} GB/s copy")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu, cpu_counts = cpu_baseline(s, args.test, args.cpu_seconds)
        got = main_r["counts"][: len(cpu_counts)].cpu().numpy()
        if not np.array_equal(got, cpu_counts):
            print("bench.py: GPU counts differ from the oracle on the baseline sample", file=sys.stderr)
            sys.exit(1)
        extra["oracle_sample_bit_exact"] = True

    out = {
        "metric": "events/s (batched vs plain, bit-exact decisions); p99 timeslice latency",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator; stands in for the paper's simulated CBM events)",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}", "n_events": n_ev,
                   "n_hits": hits, "test": args.test, "form": args.form, "seed": 0,
                   "shape": list(shape) if shape else None},
        "autotuned": tuned,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "triplet_tests_per_s_effective": triplets * args.steps / main_r["elapsed_s"],
        "n_accepted": main_r["n_accepted"],
        "plain": plain_info,
        "forms": forms,
        "p99_slice_latency_ms": serving["p99_ms"] if serving else None,
        "serving": serving,
        "station_filter": filt,
        "event_building": building,
        "two_particles": two,
        "per_hit_z": hz,
        "device_probes": probes,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
