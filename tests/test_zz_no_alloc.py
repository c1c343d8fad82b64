"""cwt_execute_noalloc (static device scratch, no allocation) against cwt_execute.

Each case calls the allocation-free entry point through the C ABI twice in a
row, the second time with fewer channels, and requires the outputs to equal
cwt_execute's bit for bit (the two entry points run the same kernels on the
same inputs; only where the workspace lives differs).  A request whose
workspace exceeds the static scratch is refused before anything is launched.
"""
import ctypes

import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _reference(plan, x):
    """cwt_execute with its own workspace (the existing entry point)."""
    return plan.execute(x)


def _noalloc(lib, plan, x, out):
    from paper_2506_07793_amd import _lib
    stream = torch.cuda.current_stream()
    rc = lib.cwt_execute_noalloc(plan.handle, _vp(x), int(x.shape[0]), _vp(out),
                                 ctypes.c_void_p(stream.cuda_stream))
    _lib.check(rc)
    return out


CASES = [
    # (label, n, sfreq, n_freqs, out mode, precision, C first, C second)
    ("register-resident L=4096 complex64", 4096, 1000.0, 100, "complex64", "fp32", 64, 5),
    ("mixed-radix register-resident L=2000 power", 2000, 1000.0, 40, "power", "fp32", 24, 3),
    ("runtime radices L=3000 power", 3000, 1000.0, 40, "power", "fp32", 24, 3),
    ("band power L=4096", 4096, 1000.0, 40, "bandpower", "fp32", 16, 1),
    ("split FP16 L=4096 complex64", 4096, 1000.0, 30, "complex64", "split_f16", 8, 2),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_execute_twice(case):
    import paper_2506_07793_amd as cwt
    from paper_2506_07793_amd import _lib
    label, n, sfreq, F, out_mode, prec, C1, C2 = case
    print("case:", label, flush=True)
    lib = _lib.load()
    freqs = synth.log_freqs(1.0, 100.0, F)
    plan = cwt.Plan(n, sfreq, freqs, n_cycles=synth.eeg_cycles(freqs), out=out_mode,
                    precision=prec)
    x1 = torch.from_numpy(synth.eeg(C1, n, sfreq, 11)).cuda()
    x2 = torch.from_numpy(synth.eeg(C2, n, sfreq, 12)).cuda()
    ref1 = _reference(plan, x1).clone()
    ref2 = _reference(plan, x2).clone()
    o1 = plan.alloc_output(C1)
    o2 = plan.alloc_output(C2)
    o1.view(torch.uint8).fill_(0xFF)  # NaN pattern: every element must be rewritten
    o2.view(torch.uint8).fill_(0xFF)
    _noalloc(lib, plan, x1, o1)
    _noalloc(lib, plan, x2, o2)  # second call, fewer channels, same scratch
    torch.cuda.synchronize()
    assert torch.equal(o1.view(torch.uint8), ref1.view(torch.uint8)), label
    assert torch.equal(o2.view(torch.uint8), ref2.view(torch.uint8)), label
    plan.close()


def test_noalloc_binding_and_stream_order():
    """Through the binding, on a side stream: consecutive calls on one stream
    reuse the scratch in order and each output equals cwt_execute's."""
    import paper_2506_07793_amd as cwt
    freqs = synth.log_freqs(1.0, 100.0, 50)
    plan = cwt.Plan(4096, 1000.0, freqs, n_cycles=synth.eeg_cycles(freqs))
    xs = [torch.from_numpy(synth.eeg(C, 4096, 1000.0, 20 + C)).cuda() for C in (32, 7, 32)]
    refs = [plan.execute(x).clone() for x in xs]
    s = torch.cuda.Stream()
    outs = [plan.alloc_output(x.shape[0]) for x in xs]
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        for x, o in zip(xs, outs):
            plan.execute_noalloc(x, o, stream=s)
    s.synchronize()
    for r, o in zip(refs, outs):
        assert torch.equal(r, o)
    plan.close()


def test_noalloc_refuses_more_than_the_scratch():
    """A workspace above CWT_NOALLOC_SCRATCH_BYTES is refused before any
    launch: CWT_E_UNSUPPORTED, the output untouched."""
    import paper_2506_07793_amd as cwt
    from paper_2506_07793_amd import _lib
    lib = _lib.load()
    freqs = synth.log_freqs(1.0, 100.0, 10)
    plan = cwt.Plan(4096, 1000.0, freqs, n_cycles=synth.eeg_cycles(freqs))
    per_channel = (plan.L // 2 + 1) * 8  # one half spectrum
    C = _lib.CWT_NOALLOC_SCRATCH_BYTES // per_channel + 1
    assert plan.workspace_size(C) > _lib.CWT_NOALLOC_SCRATCH_BYTES
    x = torch.zeros(C, 4096, device="cuda")
    sentinel = torch.full((1024,), 7.0, device="cuda")
    rc = lib.cwt_execute_noalloc(plan.handle, _vp(x), C, _vp(sentinel), None)
    assert rc == _lib.CWT_E_UNSUPPORTED
    assert b"scratch" in lib.cwt_last_error()
    torch.cuda.synchronize()
    assert bool((sentinel == 7.0).all())
    # the largest C that fits runs, and equals cwt_execute
    Cmax = C - 1
    assert plan.workspace_size(Cmax) <= _lib.CWT_NOALLOC_SCRATCH_BYTES
    xm = torch.from_numpy(synth.eeg(Cmax, 4096, 1000.0, 31)).cuda()
    ref = plan.execute(xm)
    o = plan.alloc_output(Cmax)
    _noalloc(lib, plan, xm, o)
    torch.cuda.synchronize()
    assert torch.equal(o, ref)
    plan.close()
