"""The C ABI library on the host: it loads, exports what include/trig.h
declares, and rejects bad arguments before touching the GPU.  Also checks
the gfx950 instructions of the MSD kernels (no fused multiply-add, no packed
fp32, fp32 subnormals kept).  No test here needs a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1810_11966_amd import build, trig

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h)
           for h in ("trig.h", "trig_probe.h", "trig_serve.h", "trig_filter.h", "trig_events.h")]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(trig.LIB_PATH):
        build.build()
    return trig.load()


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trig_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(names) == set(trig.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", trig.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_params_struct_layout_matches_header(lib, tmp_path):
    """ctypes mirrors of the structs agree with a C compiler's layout."""
    fields = [f for f, _ in trig.TrigParams._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "trig.h"', "int main(void) {",
           'printf("%zu %zu %zu\\n", sizeof(trig_params), sizeof(trig_events_csr), sizeof(trig_hits));']
    for f in fields:
        src.append(f'printf("%zu\\n", offsetof(trig_params, {f}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(v) for v in out[:3]]
    assert sizes == [ctypes.sizeof(trig.TrigParams), ctypes.sizeof(trig.TrigEventsCsr),
                     ctypes.sizeof(trig.TrigHits)]
    for f, off in zip(fields, out[3:]):
        assert getattr(trig.TrigParams, f).offset == int(off), f


def test_params_defaults(lib):
    p = trig.trig_params_init()
    assert p.abi_version == trig.TRIG_ABI_VERSION and p.test == trig.TRIG_TEST_MSD
    assert list(p.z) == [400.0, 410.0, 420.0]
    assert abs(p.msd_max[0] - 0.03) < 1e-9 and abs(p.msd_max[1] - 0.025) < 1e-9
    assert p.ndf == 2 and p.min_triplets == 2 and p.flags == 0


def test_workspace_sizes(lib):
    p = trig.make_params()
    assert trig.trig_workspace_bytes(1000, p) == 0
    p.flags = trig.TRIG_OUT_COMPACT
    assert trig.trig_workspace_bytes(1000, p) > 0
    p.flags = trig.TRIG_EXEC_PERSISTENT
    ws = trig.trig_workspace_bytes(10 ** 6, p)
    assert ws >= 8 * 10 ** 6 and ws % 256 == 0


def _call(p, n_events=4, n_hits=12, offsets=0x1000, x=0x2000, y=0x3000, counts=0x4000, accept=0x5000):
    ev = trig.TrigEventsCsr(n_events, offsets)
    hits = trig.TrigHits(n_hits, x, y)
    return trig.trig_select(ev, hits, p, counts, accept, 0)


@pytest.mark.parametrize("mutate,code", [
    (lambda p: setattr(p, "abi_version", 1), trig.TRIG_EINVAL),
    (lambda p: setattr(p, "test", 7), trig.TRIG_EINVAL),
    (lambda p: p.z.__setitem__(1, 0.0), trig.TRIG_EINVAL),
    (lambda p: p.z.__setitem__(2, float("inf")), trig.TRIG_EINVAL),
    (lambda p: p.msd_max.__setitem__(0, -1.0), trig.TRIG_EINVAL),
    (lambda p: p.msd_max.__setitem__(1, float("nan")), trig.TRIG_EINVAL),
    (lambda p: p.msd_max.__setitem__(0, float("inf")), trig.TRIG_EINVAL),
    (lambda p: p.slope_window.__setitem__(1, float("inf")), trig.TRIG_EINVAL),
    (lambda p: p.slope_window.__setitem__(0, -0.1), trig.TRIG_EINVAL),
    (lambda p: setattr(p, "ndf", 0), trig.TRIG_EINVAL),
    (lambda p: setattr(p, "min_triplets", -1), trig.TRIG_EINVAL),
    (lambda p: setattr(p, "tile_pairs", 65), trig.TRIG_EINVAL),
    (lambda p: p.reserved.__setitem__(3, 1), trig.TRIG_EINVAL),
    (lambda p: setattr(p, "flags", 1 << 20), trig.TRIG_EINVAL),
    (lambda p: setattr(p, "flags", trig.TRIG_OUT_COMPACT), trig.TRIG_EINVAL),  # no id buffers
    (lambda p: setattr(p, "flags", trig.TRIG_EXEC_PERSISTENT), trig.TRIG_EWORKSPACE),
    (lambda p: setattr(p, "flags", trig.TRIG_EXEC_BINNED | trig.TRIG_EXEC_PRUNED), trig.TRIG_EUNSUPPORTED),
    (lambda p: setattr(p, "flags", trig.TRIG_EXEC_BINNED | trig.TRIG_EXEC_AUTOTUNE), trig.TRIG_EUNSUPPORTED),
    (lambda p: setattr(p, "flags", trig.TRIG_EXEC_BINNED | trig.TRIG_EXEC_PERSISTENT), trig.TRIG_EWORKSPACE),
])
def test_rejects_bad_params_before_any_launch(lib, mutate, code):
    p = trig.make_params()
    mutate(p)
    assert _call(p) == code
    assert trig.trig_last_error_detail() != ""


def test_rejects_null_and_negative_sizes(lib):
    p = trig.make_params()
    assert _call(p, n_events=-1) == trig.TRIG_EINVAL
    assert _call(p, n_hits=-1) == trig.TRIG_EINVAL
    assert _call(p, offsets=0) == trig.TRIG_EINVAL
    assert _call(p, x=0) == trig.TRIG_EINVAL
    assert _call(p, counts=0) == trig.TRIG_EINVAL
    assert lib.trig_select(None, None, None, None, None, None) == trig.TRIG_EINVAL
    p.flags = trig.TRIG_EXEC_PERSISTENT
    p.workspace = 0x10010  # misaligned
    p.workspace_bytes = 1 << 30
    assert _call(p) == trig.TRIG_EWORKSPACE


def test_params_check(lib):
    from paper_1810_11966_amd import serve
    serve._lib()
    p = trig.make_params()
    assert lib.trig_params_check(p) == trig.TRIG_OK
    p.flags = trig.TRIG_OUT_COMPACT  # output pointers are not required here
    assert lib.trig_params_check(p) == trig.TRIG_OK
    p.ndf = 0
    assert lib.trig_params_check(p) == trig.TRIG_EINVAL


def test_server_rejects_bad_config_without_gpu(lib):
    from paper_1810_11966_amd import serve
    import ctypes
    serve._lib()
    cfg = serve.ServerConfig()
    cfg.params = trig.make_params()
    h = ctypes.c_void_p()
    cfg.hbm_budget_bytes, cfg.pinned_budget_bytes, cfg.n_streams, cfg.max_pending = 0, 1 << 20, 2, 4
    assert lib.trig_server_create(ctypes.byref(cfg), ctypes.byref(h)) == trig.TRIG_EINVAL
    cfg.hbm_budget_bytes, cfg.n_streams = 1 << 20, 0
    assert lib.trig_server_create(ctypes.byref(cfg), ctypes.byref(h)) == trig.TRIG_EINVAL
    cfg.n_streams = 2
    cfg.params.ndf = 0
    assert lib.trig_server_create(ctypes.byref(cfg), ctypes.byref(h)) == trig.TRIG_EINVAL
    assert not h.value


def test_strerror_and_event_hook(lib):
    for code in (0, -1, -2, -3, -4):
        assert trig.trig_strerror(code)
    assert trig.trig_strerror(-99) == "unknown error code"
    assert trig.trig_set_kernel_events(0x10, 0) == trig.TRIG_EINVAL
    assert trig.trig_set_kernel_events(0, 0) == trig.TRIG_OK


# ------------------------------------------------------------------- ISA ---

@pytest.fixture(scope="module")
def isa():
    return open(build.build_isa()).read()


def kernel_bodies(isa_text):
    bodies, name, cur = {}, None, []
    for line in isa_text.splitlines():
        m = re.match(r"^(_Z\w+):", line)
        if m:
            if name:
                bodies[name] = "\n".join(cur)
            name, cur = m.group(1), []
        elif name:
            cur.append(line)
            if line.strip().startswith(".Lfunc_end"):
                bodies[name] = "\n".join(cur)
                name = None
    return bodies


def test_msd_kernels_have_no_fma_or_packed_fp32(isa):
    bodies = kernel_bodies(isa)
    msd = {k: v for k, v in bodies.items() if re.search(r"Msd(BasisTest|FitTest|BasisPrune|FitPrune|BasisBin|FitBin)", k)}
    assert len(msd) >= 16
    for name, body in msd.items():
        bad = re.findall(r"\b(v_fma\w*|v_fmac\w*|v_mac_f32\w*|v_mad_f32\w*|v_mad_legacy\w*|"
                         r"v_pk_(?:add|mul|fma)_f32\w*)", body)
        assert not bad, (name, bad[:5])


def kernel_descriptors(isa_text):
    """{kernel: {field: int}} from the .amdhsa_kernel blocks."""
    out, name = {}, None
    for line in isa_text.splitlines():
        t = line.strip()
        if t.startswith(".amdhsa_kernel "):
            name = t.split()[1]
            out[name] = {}
        elif t.startswith(".end_amdhsa_kernel"):
            name = None
        elif name and t.startswith(".amdhsa_"):
            parts = t.split()
            if len(parts) == 2 and parts[1].lstrip("-").isdigit():
                out[name][parts[0][len(".amdhsa_"):]] = int(parts[1])
    return out


def test_kernel_resources(isa):
    """No kernel spills to scratch; the binned kernels fit six waves per SIMD
    (their LDS allows six 4-wave workgroups per CU): at most 80 VGPRs plus
    AGPRs out of the 512 per SIMD lane."""
    desc = kernel_descriptors(isa)
    assert len(desc) >= 10
    for name, d in desc.items():
        assert d["private_segment_fixed_size"] == 0, name
    binned = {k: v for k, v in desc.items() if "k_binned" in k}
    assert len(binned) == 3
    for name, d in binned.items():
        assert d["next_free_vgpr"] <= 80, (name, d["next_free_vgpr"])


def test_fp32_subnormals_enabled(isa):
    modes = re.findall(r"\.amdhsa_float_denorm_mode_32\s+(\d+)", isa)
    assert modes and all(m == "3" for m in modes)


def test_autotune_argument_checks(lib):
    p = trig.make_params(flags=trig.TRIG_EXEC_AUTOTUNE)
    assert trig.trig_workspace_bytes(100, p) >= 256  # block counter for stealing
    assert _call(p) == trig.TRIG_EWORKSPACE
    fit = trig.make_params(test="msd_basis", flags=trig.TRIG_EXEC_AUTOTUNE)
    assert trig.trig_workspace_bytes(100, fit) >= 256
    ev = trig.TrigEventsCsr(1, 0x1000)
    hits = trig.TrigHits(0, None, None)
    plain = trig.make_params()
    rc, _ = trig.trig_autotune(ev, hits, plain, 0x2000, 0x3000, 1, 0)
    assert rc == trig.TRIG_EINVAL  # flag not set
    rc, _ = trig.trig_autotune(ev, hits, fit, 0x2000, 0x3000, 0, 0)
    assert rc == trig.TRIG_EINVAL  # reps out of range
    rc, _ = trig.trig_autotune(ev, hits, fit, 0x2000, 0x3000, 101, 0)
    assert rc == trig.TRIG_EINVAL
    trig.trig_autotune_reset()


def test_autotune_cache_file_errors_and_round_trip(tmp_path):
    """trig_autotune_save / _load without a GPU: an empty table saves as the
    header alone and loads back with nothing recorded; a well-formed record
    for some device is read (and recorded only for a matching device, of
    which there is none here); missing files, bad headers and malformed
    lines are refused with TRIG_EINVAL before anything is recorded."""
    trig.trig_autotune_reset()
    f = tmp_path / "cache.txt"
    trig.autotune_save(str(f))
    assert f.read_text() == "trig-autotune-cache 1\n"
    assert trig.autotune_load(str(f)) == 0
    good = ("trig-autotune-cache 1\n"
            "gfx950:sramecc+:xnack-/256cu 0 6 batched 2048 4 0.84999999999999998 0\n"
            "gfx950:sramecc+:xnack-/256cu 0 9 binned 0 0 0 1\n\n")
    f.write_text(good)
    assert trig.autotune_load(str(f)) == 0  # no device of this process matches
    bad_files = [
        "",                                                           # empty
        "trig-autotune-cache 2\n",                                    # header
        good + "gfx950/256cu 0 6 batched 2048 4 0.85\n",              # missing field
        good + "gfx950/256cu 3 6 batched 2048 4 0.85 0\n",            # test
        good + "gfx950/256cu 0 32 batched 2048 4 0.85 0\n",           # class
        good + "gfx950/256cu 0 6 batched 3000 4 0.85 0\n",            # block_hits
        good + "gfx950/256cu 0 6 batched 2048 3 0.85 0\n",            # block_waves
        good + "gfx950/256cu 0 6 batched 2048 4 1.5 0\n",             # fill
        good + "gfx950/256cu 0 6 binned 2048 0 0 0\n",                # binned with a shape
        good + "gfx950/256cu 0 6 batched 2048 4 0.85 2\n",            # stealing flag
        good + "gfx950/256cu 0 6 batched 2048 4 0.85 0 extra\n",      # trailing field
    ]
    for text in bad_files:
        f.write_text(text)
        with pytest.raises(trig.TrigError) as e:
            trig.autotune_load(str(f))
        assert e.value.code == trig.TRIG_EINVAL, text
    with pytest.raises(trig.TrigError):
        trig.autotune_load(str(tmp_path / "missing.txt"))
    with pytest.raises(trig.TrigError):
        trig.autotune_save(str(tmp_path / "no_such_dir" / "c.txt"))
    lib = trig.load()
    assert lib.trig_autotune_save(None) == trig.TRIG_EINVAL
    assert lib.trig_autotune_load(None, None) == trig.TRIG_EINVAL
    found = ctypes.c_int32(7)
    res = trig.TrigAutotuneResult()
    assert lib.trig_autotune_lookup(0, 6, None, ctypes.byref(res)) == trig.TRIG_EINVAL
    assert lib.trig_autotune_lookup(3, 6, ctypes.byref(found), ctypes.byref(res)) == trig.TRIG_EINVAL
    assert lib.trig_autotune_lookup(0, 32, ctypes.byref(found), ctypes.byref(res)) == trig.TRIG_EINVAL
    assert lib.trig_autotune_lookup(0, 6, ctypes.byref(found), ctypes.byref(res)) == trig.TRIG_OK
    assert found.value == 0


def test_lane_division_identity():
    """The batched kernel's lane division: floor(lane / n) = (lane *
    ceil(2^16 / n)) >> 16 for every lane < 64 and 1 <= n <= 64, with the
    product inside 24 bits (a 24-bit multiply)."""
    for n in range(1, 65):
        r = (65536 + n - 1) // n
        for lane in range(64):
            assert lane * r < (1 << 24)
            assert (lane * r) >> 16 == lane // n, (n, lane)


def test_binned_interval_widening_covers_one_step():
    """The binned form widens each key-interval end by |f| 2^-22 + 2^-126
    (binary32 multiply, add, subtract: the kernel's operation order).  The
    result must lie at or beyond the next binary32 value in that direction
    for every finite f, so that the cell range covers the exact interval."""
    import numpy as np
    f32 = np.float32
    rng = np.random.default_rng(7)
    vals = np.concatenate([
        rng.uniform(-1, 1, 20000).astype(f32) * f32(2.0) ** rng.integers(-149, 128, 20000).astype(f32),
        np.array([0.0, -0.0, 1e-45, -1e-45, 1.17549435e-38, -1.17549435e-38, 3.4028235e38, -3.4028235e38,
                  1.0, -1.0, 0.24494897, -0.24494897], dtype=f32)])
    vals = vals[np.isfinite(vals)]
    with np.errstate(over="ignore"):
        d = (np.abs(vals) * f32(2.0 ** -22)).astype(f32) + f32(2.0 ** -126)
        down = (vals - d).astype(f32)
        up = (vals + d).astype(f32)
    assert (down <= np.nextafter(vals, f32(-np.inf))).all()
    assert (up >= np.nextafter(vals, f32(np.inf))).all()


def test_noalloc_rejects_before_any_launch(lib):
    """trig_select_noalloc takes no workspace, and refuses a batch whose
    scratch need exceeds its static array before touching the device."""
    p = trig.make_params(flags=trig.TRIG_EXEC_PERSISTENT)
    ev = trig.TrigEventsCsr(1_000_000, 0x1000)
    hits = trig.TrigHits(12, 0x2000, 0x3000)
    assert trig.trig_workspace_bytes(1_000_000, p) > trig.TRIG_NOALLOC_SCRATCH_BYTES
    assert trig.trig_select_noalloc(ev, hits, p, 0x4000, 0x5000, 0) == trig.TRIG_EWORKSPACE
    assert "scratch" in trig.trig_last_error_detail()
    p.workspace = 0x10000
    p.workspace_bytes = 1 << 30
    assert trig.trig_select_noalloc(ev, hits, p, 0x4000, 0x5000, 0) == trig.TRIG_EINVAL
    assert lib.trig_select_noalloc(None, None, None, None, None, None) == trig.TRIG_EINVAL
