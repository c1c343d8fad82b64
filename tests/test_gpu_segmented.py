"""Padded lengths above 20480 (long recordings): segmented plans against the
oracle's direct cyclic convolution over the whole padded length.

The oracle evaluates each output as a cyclic sum over the full period L, so
the checks sample windows of outputs: the first samples (whose inputs wrap
to the end of the padded signal), the samples on either side of every
segment boundary, and the last samples.  Bar: the FP32 path's, max |P - P_ref|
over the largest reference power of the row <= 1e-5 (complex W also checked
by the oracle's relative error measure)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_07793_amd as cwt
from paper_2506_07793_amd import _lib
import synth

pytestmark = pytest.mark.gpu
BAR = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def _windows(plan, n, width=64):
    """Start of each checked output window: both ends and both sides of every
    segment boundary."""
    B = int(plan.desc.segment_outputs)
    starts = {0, n - width}
    for s in range(1, int(plan.desc.n_segments)):
        b = s * B
        starts.update({max(0, b - width), min(n - width, b)})
    return sorted(starts)


def _ref_excerpt(x, n, sfreq, freqs, cyc, rows, L, margin, t0, width):
    """Oracle outputs of rows at [t0, t0 + width) from a circular excerpt of
    the zero-padded signal reaching M = margin + 64 samples beyond the window
    on either side (every output depends only on the samples within the
    wavelets' support, the margin, to below 1e-8 of the envelope's peak)."""
    M = int(margin) + 64
    idx = (t0 - M + np.arange(2 * M + width)) % L
    xpad = np.where(idx < n, x[:, np.minimum(idx, n - 1)], 0.0)
    return oracle.cwt(np.ascontiguousarray(xpad), sfreq, freqs, cyc, pad="none", rows=rows,
                      t0=M, nt=width)


def _ref_rows(x, sfreq, freqs, cyc, rows, L, starts, width):
    """Oracle outputs of (channel, freq) rows over the windows: [rows, windows, width]."""
    return np.stack([oracle.cwt(x, sfreq, freqs, cyc, L=L, rows=rows, t0=t0, nt=width)
                     for t0 in starts], axis=1)


@pytest.mark.parametrize("n,pad,sfreq", [(50000, "smooth7", 1000.0), (40009, "none", 500.0),
                                         (30000, "linear", 2048.0)],
                         ids=["smooth7-50000", "none-prime-40009", "linear-30000"])
def test_segmented_complex_matches_oracle(n, pad, sfreq):
    freqs = synth.log_freqs(2.0, min(100.0, 0.4 * sfreq), 24)
    cyc = synth.eeg_cycles(freqs)
    C = 3
    x = synth.eeg(C, n, sfreq, 41)
    plan = cwt.Plan(n, sfreq, freqs, n_cycles=cyc, pad=pad)
    assert plan.n_segments >= 2 and plan.L >= n
    print("n=%d pad=%s: L=%d, %d segments of %d (outputs %d, margin %d)" % (
        n, pad, plan.L, plan.n_segments, plan.desc.segment_len, plan.desc.segment_outputs,
        plan.desc.segment_margin))
    W = plan.execute(torch.from_numpy(x).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    assert np.isfinite(W).all()
    width = 64
    starts = _windows(plan, n, width)
    rows = np.array([(c, f) for c in range(C) for f in (0, len(freqs) // 2, len(freqs) - 1)])
    ref = _ref_rows(x.astype(np.float64), sfreq, freqs, cyc, rows, plan.L, starts, width)
    got = np.stack([np.stack([W[c, f, t0:t0 + width] for t0 in starts]) for c, f in rows])
    for r, (c, f) in enumerate(rows):
        # the row's largest power over the windows, or over the whole row
        # computed by the library, whichever is larger, sets the scale
        Pg, Pr = np.abs(got[r]) ** 2, np.abs(ref[r]) ** 2
        scale = max(Pr.max(), (np.abs(W[c, f]) ** 2).max())
        e = float(np.abs(Pg - Pr).max() / scale)
        assert e <= BAR, (c, f, e)
    e_P, e_W = oracle.parity_errors(got.reshape(len(rows), -1), ref.reshape(len(rows), -1))
    print("  e_P=%.3e e_W=%.3e over %d windows x %d rows" % (e_P, e_W, len(starts), len(rows)))
    plan.close()


def test_segmented_power_and_bandpower():
    n, sfreq = 45000, 1000.0
    freqs = synth.log_freqs(1.0, 100.0, 40)
    cyc = synth.eeg_cycles(freqs)
    C = 2
    x = synth.eeg(C, n, sfreq, 42)
    xt = torch.from_numpy(x).cuda()
    pw = cwt.Plan(n, sfreq, freqs, n_cycles=cyc, out="power")
    bp = cwt.Plan(n, sfreq, freqs, n_cycles=cyc, out="bandpower")
    cx = cwt.Plan(n, sfreq, freqs, n_cycles=cyc)
    P = pw.execute(xt).cpu().numpy()
    Bp = bp.execute(xt).cpu().numpy()
    W = cx.execute(xt)
    torch.cuda.synchronize()
    # power equals |W|^2 of the complex plan (same kernel, same rounding of W)
    Pw = (W.abs() ** 2).cpu().numpy()
    assert float(np.abs(P - Pw).max() / Pw.max()) <= 1e-6
    width = 48
    starts = _windows(pw, n, width)
    groups = oracle.band_groups(freqs)
    x64 = x.astype(np.float64)
    margin = pw.desc.segment_margin
    for c in range(C):
        rows = np.array([(c, f) for f in range(len(freqs))])
        ref = np.stack([_ref_excerpt(x64, n, sfreq, freqs, cyc, rows, pw.L, margin, t0, width)
                        for t0 in starts], axis=1)
        Pr = np.abs(ref) ** 2  # [F, windows, width]
        Pg = np.stack([P[c, :, t0:t0 + width] for t0 in starts], axis=1)
        e = float(np.abs(Pg - Pr).max() / Pr.max())
        assert e <= BAR, ("power", c, e)
        Br = oracle.band_power(Pr.reshape(1, len(freqs), -1), groups)[0]
        Bg = np.stack([Bp[c, :, t0:t0 + width] for t0 in starts], axis=1).reshape(len(groups), -1)
        eb = float(np.abs(Bg - Br).max() / Br.max())
        print("channel %d: power e=%.3e, band power e=%.3e" % (c, e, eb))
        assert eb <= BAR, ("bandpower", c, eb)
    for p in (pw, bp, cx):
        p.close()


def test_segmented_two_stages_equal_execute():
    n, sfreq = 33000, 1000.0
    freqs = synth.log_freqs(3.0, 80.0, 12)
    cyc = synth.eeg_cycles(freqs)
    C = 5
    xt = torch.from_numpy(synth.eeg(C, n, sfreq, 43)).cuda()
    plan = cwt.Plan(n, sfreq, freqs, n_cycles=cyc, out="power")
    a = plan.execute(xt)
    ws = plan.alloc_workspace(C)
    plan.forward_spectra(xt, ws)
    b = plan.alloc_output(C)
    plan.transform_spectra(C, b, ws)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_segmented_entry_points_that_refuse():
    from paper_2506_07793_amd.stream import Server
    n, sfreq = 30000, 1000.0
    freqs = synth.log_freqs(1.0, 40.0, 8)  # every EEG band owns a frequency
    cyc = synth.eeg_cycles(freqs)
    plan = cwt.Plan(n, sfreq, freqs, n_cycles=cyc, out="bandpower")
    assert plan.n_segments >= 2
    x = torch.from_numpy(synth.eeg(2, n, sfreq, 44)).cuda()
    with pytest.raises(cwt.CwtError) as e:
        plan.execute_noalloc(x, plan.alloc_output(2))
    assert e.value.code == _lib.CWT_E_UNSUPPORTED
    with pytest.raises(cwt.CwtError) as e:
        out = torch.empty(2 * plan.output_bytes(2), dtype=torch.uint8, device="cuda")
        plan.execute_batches(x, 2, out, plan.alloc_batches_workspace(2), 2, x_batch_stride=0,
                             out_batch_stride=plan.output_bytes(2))
    assert e.value.code == _lib.CWT_E_UNSUPPORTED
    b = cwt.Batch([(plan, x, plan.alloc_output(2))])
    with pytest.raises(cwt.CwtError) as e:
        b.execute(b.alloc_workspace())
    assert e.value.code == _lib.CWT_E_UNSUPPORTED
    srv = Server(1 << 30)
    with pytest.raises(cwt.CwtError) as e:
        srv.open(plan, 2, 50)
    assert e.value.code == _lib.CWT_E_UNSUPPORTED
    srv.close()
    torch.cuda.synchronize()
    plan.close()


def test_long_recording_full_size():
    """Five minutes of 64-channel EEG at 1000 Hz, 100 frequencies, power out
    (7.7 GB), and its time; windows checked against oracle excerpts (the
    full-length oracle costs O(L^2) in the wavelet's evaluation here)."""
    n, sfreq, C = 300000, 1000.0, 64
    d = synth.eeg_64ch(C=1, N=16)  # the workload's frequency grid
    freqs, cyc = d["freqs"], d["n_cycles"]
    x = synth.eeg(C, n, sfreq, 45)
    xt = torch.from_numpy(x).cuda()
    plan = cwt.Plan(n, sfreq, freqs, n_cycles=cyc, out="power")
    out = plan.alloc_output(C)
    ws = plan.alloc_workspace(C)
    plan.execute(xt, out=out, ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        plan.execute(xt, out=out, ws=ws)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 3
    print("64 ch x %d samples x 100 freqs, power: %d segments of %d, %.2f ms per call "
          "(%.2e samples x freqs / s)" % (n, plan.n_segments, plan.desc.segment_len, ms,
                                          C * n * 100 / (ms * 1e-3)))
    rng = np.random.default_rng(46)
    rows = np.stack([rng.integers(0, C, 6), rng.integers(0, 100, 6)], axis=1)
    width = 32
    worst = 0.0
    x64 = x.astype(np.float64)
    for t0 in _windows(plan, n, width):
        ref = _ref_excerpt(x64, n, sfreq, freqs, cyc, rows, plan.L, plan.desc.segment_margin, t0,
                           width)
        for r, (c, f) in enumerate(rows):
            Pg = out[c, f, t0:t0 + width].cpu().numpy()
            Pr = np.abs(ref[r]) ** 2
            scale = float(out[c, f].max())
            worst = max(worst, float(np.abs(Pg - Pr).max() / scale))
    print("  max |P - P_ref| / row peak over %d windows x %d rows: %.3e" % (
        len(_windows(plan, n, width)), len(rows), worst))
    assert worst <= BAR
    plan.close()
