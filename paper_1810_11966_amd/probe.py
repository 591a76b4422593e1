"""Measured ceilings of the device: fp32 VALU op rate and HBM copy bandwidth
(kernels in csrc/probe.hip, declared in include/trig_probe.h)."""
from __future__ import annotations

from . import hip_events, trig


def measure_valu(torch, n_blocks: int = 256 * 32, iters: int = 4096, reps: int = 3) -> float:
    """Best fp32 VALU rate (ops/s) over ``reps`` launches."""
    lib = trig.load()
    out = torch.empty(n_blocks * 256, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    a, b = hip_events.HipEvent(), hip_events.HipEvent()
    best = 0.0
    for r in range(reps + 1):
        a.record(stream)
        if lib.trig_probe_valu(n_blocks, iters, 0.5, out.data_ptr(), stream):
            raise RuntimeError("trig_probe_valu failed")
        b.record(stream)
        b.synchronize()
        if r:
            best = max(best, n_blocks * 256.0 * iters * 16 / (a.elapsed_ms(b) * 1e-3))
    return best


def measure_copy(torch, nbytes: int = 1 << 30, reps: int = 5, n_blocks: int = 256 * 16) -> float:
    """Best copy bandwidth (read + write bytes per second)."""
    lib = trig.load()
    n_vec4 = nbytes // 16
    src = torch.empty(n_vec4 * 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    a, b = hip_events.HipEvent(), hip_events.HipEvent()
    best = 0.0
    for r in range(reps + 1):
        a.record(stream)
        if lib.trig_probe_copy(src.data_ptr(), dst.data_ptr(), n_vec4, n_blocks, stream):
            raise RuntimeError("trig_probe_copy failed")
        b.record(stream)
        b.synchronize()
        if r:
            best = max(best, 32.0 * n_vec4 / (a.elapsed_ms(b) * 1e-3))
    return best


def main(argv=None):
    import argparse
    import sys
    import torch
    ap = argparse.ArgumentParser(description="device ceilings: fp32 VALU rate, copy bandwidth")
    ap.add_argument("--valu", action="store_true")
    ap.add_argument("--copy", type=int, default=0, metavar="BYTES", help="copy probe over BYTES of input")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    trig.load()
    if a.valu:
        print(f"valu {measure_valu(torch, reps=a.reps) / 1e12:.2f} T fp32 ops/s", flush=True)
    if a.copy:
        print(f"copy {a.copy} B: {measure_copy(torch, nbytes=a.copy, reps=a.reps) / 1e9:.0f} GB/s (read+write)",
              flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
