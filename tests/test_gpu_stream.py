"""Streaming server on the GPU: trailing-hop band power vs the FP64 oracle,
batching across sessions, HBM-budget admission and backpressure."""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_07793_amd as cwt
from paper_2506_07793_amd import _lib
from paper_2506_07793_amd.stream import Server, now_ns
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def _plan(W, sfreq, F, fmax):
    freqs = synth.log_freqs(1.0, fmax, F)
    cyc = synth.eeg_cycles(freqs)
    return cwt.Plan(W, sfreq, freqs, n_cycles=cyc, out="bandpower"), freqs, cyc


def _check(results, x, W, hop, sfreq, freqs, cyc, label, max_checks=None):
    """results: list of (bp, hop_idx); x: the full pushed signal [C, T]."""
    assert results, "no results"
    worst = 0.0
    checked = 0
    for bp, h in results:
        end = (h + 1) * hop
        assert end >= W
        win = x[:, end - W:end].astype(np.float64)
        ref = oracle.stream_band_power(win, sfreq, freqs, cyc, hop)
        scale = np.maximum(ref.max(axis=0, keepdims=True), 1e-30)
        e = float(np.max(np.abs(bp - ref) / scale))
        worst = max(worst, e)
        checked += 1
        if max_checks and checked >= max_checks:
            break
    print("%s: %d windows, worst per-band relative error %.3e" % (label, checked, worst))
    assert worst <= TOL


def test_single_session_matches_oracle():
    W, hop, sfreq, C = 500, 25, 250.0, 3
    plan, freqs, cyc = _plan(W, sfreq, 12, 100.0)
    srv = Server(1 << 30, max_batch=8, deadline_us=200)
    s = srv.open(plan, C, hop)
    x = synth.eeg(C, 1500, sfreq, seed=7)
    rng = np.random.default_rng(0)
    pos = 0
    while pos < x.shape[1]:  # ragged pushes: partial hops and several hops at once
        m = int(rng.integers(1, 60))
        m = min(m, x.shape[1] - pos)
        assert s.push(x[:, pos:pos + m])
        pos += m
        if rng.random() < 0.3:
            srv.flush()
    srv.flush()
    res = []
    while True:
        r = s.poll()
        if r is None:
            break
        res.append((r[0], r[1]))
    # one result per hop once the window is full: hops 19 .. 59
    assert [h for _, h in res] == list(range(W // hop - 1, x.shape[1] // hop))
    _check(res, x, W, hop, sfreq, freqs, cyc, "single session")
    st = srv.stats()
    assert st["results"] == len(res) and st["hops"] == x.shape[1] // hop
    srv.close()
    plan.close()


def test_many_sessions_batched():
    W, hop, sfreq, C = 1000, 50, 500.0, 4
    plan, freqs, cyc = _plan(W, sfreq, 16, 120.0)
    srv = Server(1 << 31, max_batch=16, deadline_us=2000)
    sess = [srv.open(plan, C, hop) for _ in range(10)]
    xs = [synth.eeg(C, 2000, sfreq, seed=100 + i) for i in range(10)]
    for k in range(0, 2000, hop):  # interleaved pushes of one hop each
        for s, x in zip(sess, xs):
            assert s.push(x[:, k:k + hop])
    srv.flush()
    for i, (s, x) in enumerate(zip(sess, xs)):
        res = []
        while True:
            r = s.poll()
            if r is None:
                break
            res.append((r[0], r[1]))
        assert len(res) == 2000 // hop - W // hop + 1
        _check(res, x, W, hop, sfreq, freqs, cyc, "session %d" % i, max_checks=6)
    st = srv.stats()
    assert st["batches"] < st["hops"]  # hops of different sessions shared launches
    srv.close()
    plan.close()


@pytest.mark.parametrize("W,hop,sfreq,C,F", [(2000, 50, 1000.0, 64, 40), (4096, 102, 2048.0, 256, 40)])
def test_serving_shapes(W, hop, sfreq, C, F):
    """Serving shapes: 64 ch x 2 s at 1000 Hz (hop 50) and 256 ch x 2 s at 2048 Hz (hop 102)."""
    plan, freqs, cyc = _plan(W, sfreq, F, 100.0)
    srv = Server(8 << 30, max_batch=4, deadline_us=500)
    s = srv.open(plan, C, hop)
    x = synth.eeg(C, W + 2 * hop, sfreq, seed=9)
    assert s.push(x)
    srv.flush()
    res = []
    while True:
        r = s.poll()
        if r is None:
            break
        res.append((r[0], r[1]))
    n_hops = (W + 2 * hop) // hop
    assert [h for _, h in res] == [h for h in range(n_hops) if (h + 1) * hop >= W]
    _check(res, x, W, hop, sfreq, freqs, cyc, "W=%d C=%d" % (W, C), max_checks=1)
    srv.close()
    plan.close()


def test_budget_backpressure_and_close():
    W, hop, sfreq, C = 500, 25, 250.0, 2
    plan, freqs, cyc = _plan(W, sfreq, 12, 100.0)
    srv = Server(1 << 20, max_batch=4, max_pending=3)
    opened = []
    with pytest.raises(cwt.CwtError) as ei:
        for _ in range(1000):
            opened.append(srv.open(plan, C, hop))
    assert ei.value.code == _lib.CWT_E_BUDGET
    assert 1 <= len(opened) < 1000
    st = srv.stats()
    assert st["hbm_bytes_used"] <= st["hbm_budget_bytes"]
    s = opened[0]
    # the history before the first full window fills the ring and is not
    # held against max_pending
    assert s.push(np.zeros((C, W - hop), np.float32))
    # a push that would complete more than max_pending window hops is refused whole
    assert not s.push(np.zeros((C, 4 * hop), np.float32))
    assert srv.stats()["rejected"] == 1
    assert s.push(np.zeros((C, 2 * hop), np.float32))
    # closing a session releases its ring: one more session fits again
    opened[-1].close()
    opened.append(srv.open(plan, C, hop))
    t0 = now_ns()
    srv.flush()
    assert now_ns() >= t0
    srv.close()  # closes the remaining sessions
    plan.close()


def test_open_rejects_bad_arguments():
    plan_c = cwt.Plan(500, 250.0, [10.0, 20.0], n_cycles=5.0)  # complex output
    plan_b, _, _ = _plan(500, 250.0, 12, 100.0)
    srv = Server(1 << 30)
    for args, code in (((plan_c, 2, 25), _lib.CWT_E_INVALID), ((plan_b, 0, 25), _lib.CWT_E_INVALID),
                       ((plan_b, 2, 0), _lib.CWT_E_INVALID), ((plan_b, 2, 501), _lib.CWT_E_INVALID)):
        with pytest.raises(cwt.CwtError) as ei:
            srv.open(*args)
        assert ei.value.code == code
    srv.close()
    plan_c.close()
    plan_b.close()


@pytest.mark.parametrize("n_s,C,sfreq,W,hop", [(512, 64, 1000.0, 2000, 50), (64, 256, 2048.0, 4096, 102)])
def test_serving_full_size(n_s, C, sfreq, W, hop):
    """The benchmarked serving shapes: 512 sessions of 64 channels at 1000 Hz
    and 64 sessions of 256 channels at 2048 Hz (2 s window, 50 ms hop, 40
    frequencies 1-100 Hz, band power), hops pushed interleaved across
    sessions.  Every session yields exactly its full-window results in hop
    order, all finite and non-negative; four channels of the last window of
    three sessions are checked against the oracle."""
    plan, freqs, cyc = _plan(W, sfreq, 40, 100.0)
    srv = Server(8 << 30, max_batch=512, deadline_us=1000)
    sess = [srv.open(plan, C, hop) for _ in range(n_s)]
    T = W + 2 * hop
    expect = [h for h in range(T // hop) if (h + 1) * hop >= W]  # full-window hops
    xs = [synth.eeg(C, T, sfreq, seed=1000 + i) for i in range(n_s)]
    for k in range(0, T, hop):
        for s, x in zip(sess, xs):
            assert s.push(x[:, k:k + hop])
    srv.flush()
    for i, (s, x) in enumerate(zip(sess, xs)):
        res = []
        while True:
            r = s.poll()
            if r is None:
                break
            res.append((r[0], r[1]))
        assert [h for _, h in res] == expect, i
        for bp, _ in res:
            assert np.all(np.isfinite(bp)) and float(bp.min()) >= 0.0
        if i in (0, n_s // 2 - 1, n_s - 1):
            bp, h = res[-1]
            _check([(bp[:4], h)], x[:4], W, hop, sfreq, freqs, cyc, "session %d" % i)
    st = srv.stats()
    assert st["results"] == len(expect) * n_s and st["hops"] == n_s * (T // hop)
    srv.close()
    plan.close()


@pytest.mark.parametrize("K", [1, 4, 9])
def test_several_windows_of_a_session_per_launch(K):
    """A session's whole recording pushed at once: the history before the
    first full window and many window hops share launches (at most K windows
    of the session per launch, rings of W + (K - 1) hop samples).  Every
    window hop yields its result in order, matching the oracle, and the
    results do not depend on K beyond rounding (the forward FFT packs two
    window rows per complex transform, and with an odd channel count a row's
    partner depends on how the hops were batched)."""
    W, hop, sfreq, C = 1000, 50, 1000.0, 3
    plan, freqs, cyc = _plan(W, sfreq, 24, 100.0)
    x = synth.eeg(C, 2200, sfreq, seed=17)
    out = {}
    for k in (1, K):
        srv = Server(1 << 30, max_batch=64, deadline_us=300, max_pending=64,
                     max_session_windows=k)
        s = srv.open(plan, C, hop)
        assert s.push(x)
        srv.flush()
        res = []
        while True:
            r = s.poll()
            if r is None:
                break
            res.append((r[0], r[1]))
        st = srv.stats()
        srv.close()
        n_win = x.shape[1] // hop - (W // hop - 1)
        assert [h for _, h in res] == list(range(W // hop - 1, x.shape[1] // hop))
        assert st["results"] == n_win and st["hops"] == x.shape[1] // hop
        # windows per launch bounded by k (plus one launch holding the history)
        assert st["batches"] >= -(-n_win // k)
        out[k] = res
    _check(out[K], x, W, hop, sfreq, freqs, cyc, "K=%d" % K, max_checks=8)
    for (a, ha), (b, hb) in zip(out[1], out[K]):
        assert ha == hb
        assert np.max(np.abs(a - b) / np.max(np.abs(b), axis=0, keepdims=True)) <= 2e-6
    plan.close()


def test_server_on_caller_stream():
    """The server enqueues everything on the stream it is given; results
    match the oracle and the caller's stream is left usable."""
    W, hop, sfreq, C = 500, 25, 250.0, 2
    plan, freqs, cyc = _plan(W, sfreq, 12, 100.0)
    st = torch.cuda.Stream()
    srv = Server(1 << 30, max_batch=8, deadline_us=200, stream=st)
    assert srv.stream is st
    s = srv.open(plan, C, hop)
    x = synth.eeg(C, 700, sfreq, seed=23)
    assert s.push(x)
    srv.flush()
    res = []
    while True:
        r = s.poll()
        if r is None:
            break
        res.append((r[0], r[1]))
    _check(res, x, W, hop, sfreq, freqs, cyc, "caller stream", max_checks=3)
    srv.close()
    st.synchronize()
    plan.close()


def test_linear_padded_serving_matches_oracle():
    """Serving with a linear-edge plan (zero padding to L >= W + the widest
    wavelet's support, so no cyclic wrap of the window's oldest samples
    reaches its trailing hop): 64 channels, 2 s at 1000 Hz, hop 50, 40
    frequencies; every result matches the oracle's linear-padded
    trailing-hop band power."""
    W, hop, sfreq, C = 2000, 50, 1000.0, 64
    freqs = synth.log_freqs(1.0, 100.0, 40)
    cyc = synth.eeg_cycles(freqs)
    plan = cwt.Plan(W, sfreq, freqs, n_cycles=cyc, out="bandpower", pad="linear")
    assert plan.L > W
    srv = Server(1 << 31, max_batch=16, deadline_us=300)
    s = srv.open(plan, C, hop)
    x = synth.eeg(C, W + 3 * hop, sfreq, seed=41)
    assert s.push(x)
    srv.flush()
    res = []
    while True:
        r = s.poll()
        if r is None:
            break
        res.append((r[0], r[1]))
    assert [h for _, h in res] == [h for h in range(x.shape[1] // hop) if (h + 1) * hop >= W]
    worst = 0.0
    for bp, h in res:
        end = (h + 1) * hop
        ref = oracle.stream_band_power(x[:8, end - W:end].astype(np.float64), sfreq, freqs, cyc,
                                       hop, pad="linear")
        worst = max(worst, float(np.max(np.abs(bp[:8] - ref) / ref.max(axis=0, keepdims=True))))
    print("linear-padded serving (L=%d): worst per-band relative error %.3e" % (plan.L, worst))
    assert worst <= TOL
    srv.close()
    plan.close()
