"""trig_select_noalloc (include/trig.h) through the C ABI: the same counts,
flags and accepted ids as trig_select with a caller workspace, for the forms
that use scratch memory, on two calls in a row (the second with a smaller
batch, so that state left in the static scratch by the first would show).
Every case prints its name before it touches the GPU."""
import numpy as np
import pytest

from paper_1810_11966_amd import synth

pytestmark = pytest.mark.gpu

FORMS = ("persistent", "persistent_pruned", "persistent_binned", "auto", "pruned")


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_11966_amd import trig
    trig.load()
    return torch


def run(torch, s, form, noalloc):
    from paper_1810_11966_amd import trig
    d = torch.device("cuda:0")
    off, x, y = (torch.from_numpy(np.ascontiguousarray(a)).to(d) for a in (s.offsets, s.x, s.y))
    n = s.n_events
    counts = torch.full((n,), -7, dtype=torch.int32, device=d)
    accept = torch.full((n,), 9, dtype=torch.uint8, device=d)
    ids = torch.full((max(n, 1),), -1, dtype=torch.int32, device=d)
    n_acc = torch.full((1,), -1, dtype=torch.int32, device=d)
    status = torch.zeros(1, dtype=torch.int32, device=d)
    p = trig.make_params(flags=trig.FORMS[form] | trig.TRIG_OUT_COMPACT)
    p.out_accepted_ids = ids.data_ptr()
    p.out_n_accepted = n_acc.data_ptr()
    p.out_status = status.data_ptr()
    ev = trig.TrigEventsCsr(n, off.data_ptr())
    hits = trig.TrigHits(x.numel(), x.data_ptr(), y.data_ptr())
    stream = torch.cuda.current_stream(d).cuda_stream
    ws = None
    if noalloc:
        rc = trig.trig_select_noalloc(ev, hits, p, counts.data_ptr(), accept.data_ptr(), stream)
    else:
        nbytes = trig.trig_workspace_bytes(n, p)
        if nbytes:
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=d)
            p.workspace = (ws.data_ptr() + 255) & ~255
            p.workspace_bytes = nbytes
        rc = trig.trig_select(ev, hits, p, counts.data_ptr(), accept.data_ptr(), stream)
    assert rc == 0, trig.trig_last_error_detail()
    torch.cuda.synchronize()
    k = int(n_acc.cpu()[0])
    return counts.cpu().numpy(), accept.cpu().numpy(), ids.cpu().numpy()[:k], int(status.cpu()[0])


def test_noalloc_matches_workspace_calls(gpu):
    big = synth.concat([synth.make_event_set(synth.MEDIUM_1M, n_events=200_000),
                        synth.make_event_set(synth.EventSetSpec(n_events=20_000, hits_mean=8, p_inject=0.3,
                                                                sigma=0.0, salt=55))])
    small = synth.make_event_set(synth.EventSetSpec(n_events=30_000, hits_mean=8, p_inject=0.3, sigma=0.0,
                                                    salt=56))
    for form in FORMS:
        for label, s in (("first call, 220k events", big), ("second call, 30k events", small)):
            print(f"[noalloc] {form} {label}", flush=True)
            want = run(gpu, s, form, noalloc=False)
            got = run(gpu, s, form, noalloc=True)
            for a, b, what in zip(got, want, ("counts", "accept", "ids", "status")):
                assert np.array_equal(a, b), (form, label, what)
            assert want[2].size > 100, (form, label)
