"""Device memory and ordering contract of the ABI on the GPU.

* Every byte the library takes through the caller's allocator callbacks comes
  back (plans, a plan's own workspace, autotuning, sampled-wavelet plans,
  stream servers), counted by the binding's torch-backed callbacks.
* Frees are stream-ordered: a plan destroyed on a stream while its launches
  there are still queued yields correct outputs, even when the memory is
  handed out again at once (torch's allocator, or HIP's pool).
* The stream server and the batch entry point wait for plan tables that are
  still being written on another stream.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_07793_amd as cwt
from paper_2506_07793_amd import _lib
from paper_2506_07793_amd.stream import Server
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def _busy(stream, n=40, size=4096):
    """Queue some tens of ms of unrelated work on `stream`."""
    with torch.cuda.stream(stream):
        a = torch.randn(size, size, device="cuda")
        b = torch.randn(size, size, device="cuda")
        for _ in range(n):
            a = torch.mm(a, b) * (1.0 / size)
    return a


def _eeg_plan(memory="torch", **kw):
    freqs = synth.log_freqs(1.0, 100.0, kw.pop("F", 100))
    return cwt.Plan(kw.pop("n", 4096), 1000.0, freqs, n_cycles=synth.eeg_cycles(freqs),
                    memory=memory, **kw), freqs


def test_every_byte_comes_back():
    mem = cwt.TorchDeviceMemory()
    plan, freqs = _eeg_plan(memory=mem, max_channels=8)
    assert mem.bytes_out > 0 and mem.outstanding == mem.bytes_out
    assert plan.desc.device_bytes == mem.bytes_out
    assert plan.desc.max_channels == 8
    x = torch.from_numpy(synth.eeg(8, 4096, 1000.0, 3)).cuda()
    a = plan.execute(x)            # the plan's own workspace
    b = plan.execute(x, ws=plan.alloc_workspace(8))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(cwt.CwtError) as ei:  # more channels than max_channels, no ws
        lib = _lib.load()
        x9 = torch.zeros(9, 4096, device="cuda")
        o9 = plan.alloc_output(9)
        import ctypes
        _lib.check(lib.cwt_execute(plan.handle, ctypes.c_void_p(x9.data_ptr()), 9,
                                   ctypes.c_void_p(o9.data_ptr()), None, 0, None))
    assert ei.value.code == _lib.CWT_E_INVALID
    before = mem.outstanding
    plan.autotune(4)  # temporaries through the same callbacks, all returned
    torch.cuda.synchronize()
    assert mem.outstanding == before
    plan.close()
    torch.cuda.synchronize()
    assert mem.outstanding == 0 and mem.bytes_back == mem.bytes_out

    # sampled-wavelet plan: temporaries and tables
    mem2 = cwt.TorchDeviceMemory()
    t = (np.arange(301) - 150) / 1000.0
    wv = np.stack([np.exp(-0.5 * (t / 0.05) ** 2) * np.exp(2j * np.pi * f * t) for f in (10, 20)])
    pu = cwt.Plan.from_wavelets(1000, 1000.0, [10.0, 20.0], wv, memory=mem2)
    assert mem2.outstanding > 0
    pu.close()
    assert mem2.outstanding == 0

    # stream server: rings and batch buffers
    mem3 = cwt.TorchDeviceMemory()
    bp_plan, f3 = _eeg_plan(n=2000, F=40, out="bandpower")
    srv = Server(1 << 30, max_batch=8, memory=mem3)
    sess = [srv.open(bp_plan, 4, 50) for _ in range(3)]
    assert mem3.outstanding > 0
    assert srv.stats()["hbm_bytes_used"] <= mem3.outstanding
    x = synth.eeg(4, 2100, 1000.0, 5)
    for s in sess:
        assert s.push(x)
    srv.flush()
    sess[0].close()
    srv.close()
    torch.cuda.synchronize()
    assert mem3.outstanding == 0 and mem3.bytes_out > 0
    bp_plan.close()


@pytest.mark.parametrize("memory", ["torch", None], ids=["torch-allocator", "hip-pool"])
def test_destroy_while_work_in_flight(memory):
    """cwt_plan_destroy on a stream whose queued launches still use the plan:
    the call returns at once, a new plan made right away (whose tables could
    take the freed memory) does not disturb them, and the outputs equal those
    of a run that finished before."""
    plan, freqs = _eeg_plan(memory=memory)
    C = 64
    x = torch.from_numpy(synth.eeg(C, 4096, 1000.0, 21)).cuda()
    ref = plan.execute(x).clone()
    torch.cuda.synchronize()
    s2 = torch.cuda.Stream()
    outs = [plan.alloc_output(C) for _ in range(3)]
    wss = [plan.alloc_workspace(C) for _ in range(3)]
    keep = _busy(s2)  # the launches below wait behind this on s2
    for o, w in zip(outs, wss):
        plan.execute(x, out=o, ws=w, stream=s2)
    plan.close(stream=s2)  # frees ordered behind the launches on s2
    assert not s2.query(), "the work on s2 finished before the plan was destroyed"
    # a new plan on the current stream, other frequencies, made at once
    plan2, _ = _eeg_plan(memory=memory, F=60)
    junk = [torch.full((1 << 20,), float("nan"), device="cuda") for _ in range(8)]
    s2.synchronize()
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o, ref)
    del keep, junk
    plan2.close()


def test_server_waits_for_plan_tables():
    """A band-power plan whose tables are still being generated behind other
    work on its creation stream is used by a server at once: the server's
    stream waits for them, and the results match the oracle."""
    sA = torch.cuda.Stream()
    keep = _busy(sA, n=60)
    freqs = synth.log_freqs(1.0, 100.0, 40)
    cyc = synth.eeg_cycles(freqs)
    plan = cwt.Plan(2000, 1000.0, freqs, n_cycles=cyc, out="bandpower", stream=sA)
    srv = Server(1 << 30, max_batch=4, deadline_us=100)
    s = srv.open(plan, 3, 50)
    x = synth.eeg(3, 2050, 1000.0, 8)
    assert s.push(x)
    srv.flush()
    res = []
    while True:
        r = s.poll()
        if r is None:
            break
        res.append(r)
    assert [r[1] for r in res] == [39, 40]
    for bp, h, _, _ in res:
        end = (h + 1) * 50
        ref = oracle.stream_band_power(x[:, end - 2000:end].astype(np.float64), 1000.0, freqs,
                                       cyc, 50)
        assert np.max(np.abs(bp - ref) / ref.max(axis=0, keepdims=True)) <= 1e-5
    srv.close()
    del keep
    plan.close()


def test_batch_waits_for_plan_tables():
    """Same for cwt_execute_batch: plans created behind busy work on another
    stream, the batch launched at once on the current stream."""
    sA = torch.cuda.Stream()
    keep = _busy(sA, n=60)
    items, refs = [], []
    for i, (n, F) in enumerate(((3000, 30), (4096, 20))):
        freqs = synth.log_freqs(1.0, 100.0, F)
        p = cwt.Plan(n, 1000.0, freqs, n_cycles=synth.eeg_cycles(freqs), out="power", stream=sA)
        x = torch.from_numpy(synth.eeg(2, n, 1000.0, 30 + i)).cuda()
        items.append((p, x, p.alloc_output(2)))
    b = cwt.Batch(items)
    ws = b.alloc_workspace()
    b.execute(ws)
    torch.cuda.synchronize()
    for p, x, o in items:
        # the batch runs the runtime-radix kernel for every length, so it
        # rounds differently from cwt_execute's register-resident kernel at
        # L = 4096; unwritten tables would give garbage, not ~1e-7 differences
        r = p.execute(x)
        torch.cuda.synchronize()
        assert torch.isfinite(o).all()
        assert float((o - r).abs().max() / r.abs().max()) <= 1e-5
    del keep
    for p, _, _ in items:
        p.close()
