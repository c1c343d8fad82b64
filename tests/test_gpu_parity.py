"""GPU parity of the plain FP32 path against the FP64 oracle (through the C ABI).

Gate (the workload's stated tolerance): e_P = max|P_gpu - P_orc| / max P_orc
<= 1e-5 per recording, with P = |W|^2; e_W = max|dW| / max|W| is reported.
The oracle gets the same float32 input samples promoted to float64.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_07793_amd as cwt
import synth

pytestmark = pytest.mark.gpu

TOL_P = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _run(x32, sfreq, freqs, cyc, **kw):
    plan = cwt.Plan(x32.shape[-1], sfreq, freqs, n_cycles=cyc, **kw)
    out = plan.execute(torch.from_numpy(np.ascontiguousarray(x32)).cuda())
    torch.cuda.synchronize()
    return plan, out.cpu().numpy()


def _parity(Wg, Wr, label):
    e_P, e_W = oracle.parity_errors(Wg, Wr)
    print("%s: e_P=%.3e e_W=%.3e" % (label, e_P, e_W), flush=True)
    assert e_P <= TOL_P, "%s: e_P=%g" % (label, e_P)
    return e_P, e_W


# ------------------------------------------------------------------ tables --

@pytest.mark.parametrize("n,sfreq,F,wavelet", [(4096, 1000.0, 100, "morlet"), (1000, 1000.0, 50, "morlet"),
                                              (2000, 1000.0, 40, "gabor"), (4116, 2048.0, 30, "morlet"),
                                              (4096, 1000.0, 60, "gmw"), (1000, 1000.0, 40, "gmw")])
def test_tables_within_one_ulp_of_fp64(n, sfreq, F, wavelet):
    """FP64 GPU generators: each stored spectrum bin (1/L folded in) and each
    twiddle is within one FP32 ulp of the FP64 value."""
    gmw = wavelet == "gmw"
    freqs = synth.log_freqs(1.0, (0.45 if gmw else min(100.0 / sfreq, 0.45)) * sfreq, F)
    cyc = synth.eeg_cycles(freqs)
    plan = cwt.Plan(n, sfreq, freqs, n_cycles=None if gmw else cyc, wavelet=wavelet)
    H, band, tw = plan.tables()
    L = plan.L
    kind = {"gabor": oracle.GABOR, "gmw": oracle.GMW}.get(wavelet, oracle.MORLET)
    for i, (f, s) in enumerate(zip(freqs, cyc)):
        lo, K, off = band[i]
        Hf = oracle.wavelet_spectrum(L, sfreq, f, s, kind) / L
        idx = (lo + np.arange(K)) % L
        ref = Hf[idx]
        got = H[off:off + K].astype(np.float64)
        ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got - ref) <= ulp + 1e-45), (i, np.max(np.abs(got - ref) / ulp))
        # bins outside the stored band are below 1e-12 of the peak
        mask = np.ones(L, bool)
        mask[idx] = False
        assert np.all(np.abs(Hf[mask]) <= 1e-12 * np.abs(Hf).max())
    m = np.arange(L)
    ref = np.exp(2j * np.pi * m / L)
    d = np.abs(tw.astype(np.complex128) - ref)
    assert np.max(d) <= 1.2e-7
    plan.close()


# ------------------------------------------- two tones, 1 ch x 1000 --

@pytest.mark.parametrize("pad,L", [("smooth7", 1000), ("pow2", 1024)])
def test_two_tone_single_channel(pad, L):
    """1 ch x 1000 samples at 1000 Hz, Morlet sigma 7, 50 freqs 1-50 Hz."""
    x = synth.two_tone_signal().astype(np.float32)
    freqs = np.arange(1.0, 51.0)
    plan, W = _run(x, 1000.0, freqs, 7.0, pad=pad)
    assert plan.L == L
    ref = oracle.cwt(x.astype(np.float64), 1000.0, freqs, 7.0, L=L)
    _parity(W, ref, "two-tone " + pad)
    plan.close()


# ----------------------------------------- EEG 64 ch x 4096, 100 freqs --

def _eeg(C):
    d = synth.eeg_64ch(C=C)
    return d["x"], d["sfreq"], d["freqs"], d["n_cycles"]


def test_eeg_full_oracle_two_channels():
    x, sfreq, freqs, cyc = _eeg(2)
    plan, W = _run(x, sfreq, freqs, cyc)
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc)
    _parity(W, ref, "eeg C=2 full")
    # per-row worst (each (c, f) row relative to its own peak power)
    Pg, Pr = oracle.power(W), oracle.power(ref)
    row = np.max(np.abs(Pg - Pr), axis=2) / np.max(Pr, axis=2)
    print("worst per-row e_P %.3e" % row.max())
    assert row.max() <= 1e-4
    plan.close()


def test_eeg_full_size_sampled_rows():
    """64 ch x 4096 x 100 freqs (the benchmarked shape), oracle on sampled rows."""
    x, sfreq, freqs, cyc = _eeg(64)
    plan, W = _run(x, sfreq, freqs, cyc)
    assert W.shape == (64, 100, 4096)
    rng = np.random.default_rng(11)
    rows = np.stack([rng.integers(0, 64, 24), rng.integers(0, 100, 24)], axis=1)
    rows[0] = (0, 0)
    rows[1] = (63, 99)
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc, rows=rows)
    got = W[rows[:, 0], rows[:, 1]]
    _parity(got, ref, "eeg 64ch sampled")
    plan.close()


def test_eeg_full_size_pipelined_batches():
    """The benchmarked launch form: cwt_execute_batches over three distinct
    64 ch x 4096 x 100-freq batches (each launch the transform of one batch
    and the forward FFT of the next), oracle on sampled rows of every batch,
    and the middle batch equal bit for bit to a plain cwt_execute."""
    nb, C = 3, 64
    ds = [synth.eeg_64ch(seed=20 + i) for i in range(nb)]
    sfreq, freqs, cyc = ds[0]["sfreq"], ds[0]["freqs"], ds[0]["n_cycles"]
    xs = np.stack([d["x"] for d in ds]).astype(np.float32)
    plan = cwt.Plan(4096, sfreq, freqs, n_cycles=cyc)
    assert plan.desc.kernel == 1
    x = torch.from_numpy(xs).cuda()
    out = torch.empty((nb,) + tuple(plan.output_shape(C)), dtype=torch.complex64, device="cuda")
    ws = plan.alloc_batches_workspace(C)
    plan.execute_batches(x, nb, out, ws, C)
    single = plan.execute(x[1])
    torch.cuda.synchronize()
    assert torch.equal(out[1], single)
    rng = np.random.default_rng(12)
    for i in range(nb):
        rows = np.stack([rng.integers(0, C, 6), rng.integers(0, 100, 6)], axis=1)
        rows[0] = (i, 99 - i)
        ref = oracle.cwt(xs[i].astype(np.float64), sfreq, freqs, cyc, rows=rows)
        got = out[i][torch.from_numpy(rows[:, 0]).cuda(), torch.from_numpy(rows[:, 1]).cuda()]
        _parity(got.cpu().numpy(), ref, "pipelined batch %d sampled" % i)
    plan.close()


def test_eeg_power_and_bandpower():
    x, sfreq, freqs, cyc = _eeg(3)
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc)
    Pr = oracle.power(ref)
    plan, P = _run(x, sfreq, freqs, cyc, out="power")
    assert P.dtype == np.float32
    e = np.max(np.abs(P - Pr)) / Pr.max()
    print("power e_P %.3e" % e)
    assert e <= TOL_P
    plan.close()
    plan, BP = _run(x, sfreq, freqs, cyc, out="bandpower")
    g = oracle.band_groups(freqs)
    BPr = oracle.band_power(Pr, g)
    assert BP.shape == BPr.shape == (3, 5, 4096)
    for b in range(5):
        e = np.max(np.abs(BP[:, b] - BPr[:, b])) / BPr[:, b].max()
        print("band %d e=%.3e" % (b, e))
        assert e <= TOL_P
    assert np.array_equal(plan.band_of_freq(),
                          np.concatenate([np.full(len(gi), i) for i, gi in enumerate(g)]))
    plan.close()


# ------------------------------------------------------- shapes and edges --

@pytest.mark.parametrize("C,N,sfreq,pad,expl", [
    (3, 105, 250.0, "none", 0),        # odd L = 3*5*7
    (1, 4097, 1000.0, "smooth7", 0),   # ragged: L = 4116 = 4*3*7^3
    (2, 777, 500.0, "smooth7", 0),     # L = 784 = 16*7^2
    (5, 300, 300.0, "explicit", 512),
    (1, 1, 100.0, "smooth7", 0),       # L = 1 (Morlet: exactly zero output)
    (2, 3, 100.0, "smooth7", 0),       # L = 3
    (1, 16384, 2048.0, "smooth7", 0),
    (4, 999, 1000.0, "smooth7", 0),    # L = 1000 with a 1-sample crop
    (3, 1000, 1000.0, "pow2", 0),      # L = 1024 register-resident kernel
    (2, 2000, 1000.0, "pow2", 0),      # L = 2048 register-resident kernel
    (1, 7000, 2048.0, "pow2", 0),      # L = 8192 register-resident kernel
    (65, 4096, 1000.0, "smooth7", 0),  # odd channel count, L = 4096
])
def test_shapes_and_edges(C, N, sfreq, pad, expl):
    rng = np.random.default_rng(N)
    x = rng.normal(0, 20, size=(C, N)).astype(np.float32)
    freqs = synth.log_freqs(max(0.5, sfreq / 400), 0.45 * sfreq, 12)
    cyc = synth.eeg_cycles(freqs)
    plan, W = _run(x, sfreq, freqs, cyc, pad=pad, explicit_len=expl)
    if C * N * plan.L * 12 <= 3e9:
        ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc, L=plan.L)
        Wg = W
    else:
        rows = [(c, f) for c in range(C) for f in (0, 5, 11)]
        ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc, L=plan.L, rows=rows)
        Wg = np.stack([W[c, f] for c, f in rows])
    _parity(Wg, ref, "C=%d N=%d L=%d radices=%s kernel=%d" % (C, N, plan.L, plan.radices,
                                                              plan.desc.kernel))
    plan.close()


@pytest.mark.parametrize("n", [1, 2])
def test_tiny_lengths_gabor(n):
    """N = L = 1 and 2 with Gabor (non-zero at zero frequency)."""
    x = np.array([[3.5, -1.25][:n]], dtype=np.float32)
    freqs = np.array([10.0, 40.0])
    cyc = np.array([2.0, 2.0])
    plan, W = _run(x, 100.0, freqs, cyc, wavelet="gabor")
    ref = oracle.cwt(x.astype(np.float64), 100.0, freqs, cyc, kind="gabor")
    assert np.abs(ref).max() > 1e-3
    _parity(W, ref, "N=%d gabor" % n)
    plan.close()


def test_stages_equal_execute():
    """cwt_forward_spectra + cwt_transform_spectra == cwt_execute, bitwise."""
    x, sfreq, freqs, cyc = _eeg(5)
    plan = cwt.Plan(4096, sfreq, freqs, n_cycles=cyc)
    xt = torch.from_numpy(x).cuda()
    a = plan.execute(xt)
    ws = plan.alloc_workspace(5)
    b = plan.alloc_output(5)
    plan.forward_spectra(xt, ws)
    plan.transform_spectra(5, b, ws)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_paper_workload_20480_sampled():
    """The paper's own throughput workload at its full size (64 channels x 10 s
    at 2048 Hz = 20 480 samples, the largest padded length one workgroup
    transforms; Morlet sigma 7 at 30-90 Hz in 1 Hz steps), as the bench
    times it: sampled rows against the oracle over windows at both ends and
    the middle (each output a full cyclic sum over L)."""
    C, n, sfreq = 64, 20480, 2048.0
    freqs = np.arange(30.0, 91.0)
    x = synth.eeg(C, n, sfreq, 46)
    plan, W = _run(x, sfreq, freqs, 7.0)
    assert plan.L == 20480 and plan.n_segments == 0
    rng = np.random.default_rng(47)
    rows = [(int(c), int(f)) for c, f in zip(rng.integers(0, C, 8), rng.integers(0, 61, 8))]
    got, ref = [], []
    for t0 in (0, n // 2 - 32, n - 64):
        ref.append(oracle.cwt(x.astype(np.float64), sfreq, freqs, 7.0, rows=rows, t0=t0, nt=64))
        got.append(np.stack([W[c, f, t0:t0 + 64] for c, f in rows]))
    got, ref = np.concatenate(got, axis=1), np.concatenate(ref, axis=1)
    # scale each row by its largest power over the whole row (the library's)
    for r, (c, f) in enumerate(rows):
        scale = float((np.abs(W[c, f]) ** 2).max())
        e = float(np.abs(np.abs(got[r]) ** 2 - np.abs(ref[r]) ** 2).max() / scale)
        assert e <= TOL_P, (c, f, e)
    _parity(got, ref, "paper workload L=20480 radices=%s" % plan.radices)
    plan.close()


def test_max_length_20000_sampled():
    """Largest supported padded length (160 KB of LDS), oracle on sampled rows."""
    x = synth.eeg(2, 20000, 2048.0, seed=3)
    freqs = synth.log_freqs(0.5, 200.0, 30)
    cyc = synth.eeg_cycles(freqs)
    plan, W = _run(x, 2048.0, freqs, cyc)
    assert plan.L == 20000
    rows = [(0, 0), (1, 14), (0, 29), (1, 3)]
    ref = oracle.cwt(x.astype(np.float64), 2048.0, freqs, cyc, rows=rows)
    _parity(np.stack([W[c, f] for c, f in rows]), ref, "L=20000 radices=%s" % plan.radices)
    plan.close()


def test_gabor_and_near_nyquist():
    """Gabor (kappa = 0) and a small-sigma frequency whose spectrum reaches Nyquist."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=(2, 640)).astype(np.float32)
    freqs = np.array([3.0, 40.0, 110.0, 124.0])
    cyc = np.array([3.0, 6.0, 2.0, 1.5])
    for wavelet in ("morlet", "gabor"):
        plan, W = _run(x, 250.0, freqs, cyc, wavelet=wavelet)
        kind = oracle.GABOR if wavelet == "gabor" else oracle.MORLET
        ref = oracle.cwt(x.astype(np.float64), 250.0, freqs, cyc, kind=kind)
        _parity(W, ref, wavelet + " near Nyquist")
        plan.close()


def test_zero_channels_is_noop_and_determinism():
    x, sfreq, freqs, cyc = _eeg(4)
    plan = cwt.Plan(4096, sfreq, freqs, n_cycles=cyc)
    xt = torch.from_numpy(x).cuda()
    out = plan.alloc_output(4)
    ws = plan.alloc_workspace(4)
    from paper_2506_07793_amd import _lib
    lib = _lib.load()
    import ctypes
    rc = lib.cwt_execute(plan.handle, ctypes.c_void_p(xt.data_ptr()), 0,
                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                         ws.numel(), None)
    assert rc == 0
    a = plan.execute(xt).cpu()
    b = plan.execute(xt).cpu()
    assert torch.equal(a, b), "two runs differ bitwise"
    # workspace too small is rejected before launch
    rc = lib.cwt_execute(plan.handle, ctypes.c_void_p(xt.data_ptr()), 4,
                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), 16, None)
    assert rc == _lib.CWT_E_INVALID
    plan.close()


def test_two_streams_concurrently():
    x, sfreq, freqs, cyc = _eeg(8)
    plan = cwt.Plan(4096, sfreq, freqs, n_cycles=cyc, out="power")
    xt = torch.from_numpy(x).cuda()
    ref = plan.execute(xt).clone()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    o1 = plan.alloc_output(8)
    o2 = plan.alloc_output(8)
    w1, w2 = plan.alloc_workspace(8), plan.alloc_workspace(8)
    plan.execute(xt, out=o1, ws=w1, stream=s1)
    plan.execute(xt, out=o2, ws=w2, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(o1, ref) and torch.equal(o2, ref)
    plan.close()


@pytest.mark.parametrize("out", ["complex64", "power", "bandpower"])
def test_fixed_and_generic_kernels_agree(out, monkeypatch):
    """The register-resident kernel (L = 4096) and the generic kernel both
    match the oracle, and each other to FP32 rounding."""
    x, sfreq, freqs, cyc = _eeg(2)
    xt = torch.from_numpy(x).cuda()
    monkeypatch.setenv("CWT_GENERIC_ONLY", "1")
    pg = cwt.Plan(4096, sfreq, freqs, n_cycles=cyc, out=out)
    monkeypatch.delenv("CWT_GENERIC_ONLY")
    pf = cwt.Plan(4096, sfreq, freqs, n_cycles=cyc, out=out)
    assert pg.desc.kernel == 0 and pf.desc.kernel == 1
    a = pg.execute(xt).cpu().numpy()
    b = pf.execute(xt).cpu().numpy()
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc)
    if out == "complex64":
        _parity(a, ref, "generic")
        _parity(b, ref, "fixed")
    else:
        Pr = oracle.power(ref)
        if out == "bandpower":
            Pr = oracle.band_power(Pr, oracle.band_groups(freqs))
        for name, got in (("generic", a), ("fixed", b)):
            e = np.max(np.abs(got - Pr)) / Pr.max()
            print("%s %s e=%.3e" % (out, name, e))
            assert e <= TOL_P
    pg.close()
    pf.close()


@pytest.mark.parametrize("generic", [False, True])
def test_dispatch_timing_records_each_launch(generic, monkeypatch):
    """cwt_plan_timing_start/stop: one positive duration per timed transform
    launch (later launches untimed), results unchanged by timing, bad
    arguments rejected, and a stop without a start records nothing."""
    x, sfreq, freqs, cyc = _eeg(4)
    if generic:
        monkeypatch.setenv("CWT_GENERIC_ONLY", "1")
    plan = cwt.Plan(4096, sfreq, freqs, n_cycles=cyc)
    assert plan.desc.kernel == (0 if generic else 1)
    xt = torch.from_numpy(x).cuda()
    ref = plan.execute(xt).clone()
    assert len(plan.timing_stop()) == 0
    plan.timing_start(3)
    outs = [plan.execute(xt) for _ in range(5)]
    ms = plan.timing_stop()
    assert len(ms) == 3, ms
    assert np.all(ms > 0) and np.all(ms < 1000), ms
    for o in outs:
        assert torch.equal(o, ref)
    # a second start reuses the events; the stage call is timed as well
    ws = plan.alloc_workspace(4)
    out = plan.alloc_output(4)
    plan.forward_spectra(xt, ws)
    plan.timing_start(2)
    plan.transform_spectra(4, out, ws)
    ms2 = plan.timing_stop()
    assert len(ms2) == 1 and ms2[0] > 0
    assert torch.equal(out, ref)
    from paper_2506_07793_amd import _lib
    lib = _lib.load()
    assert lib.cwt_plan_timing_start(plan.handle, -1) == _lib.CWT_E_INVALID
    assert lib.cwt_plan_timing_start(plan.handle, 70000) == _lib.CWT_E_INVALID
    assert lib.cwt_plan_timing_stop(plan.handle, None, 2, None) == _lib.CWT_E_INVALID
    plan.close()


@pytest.mark.parametrize("L", [1024, 2048, 4096, 8192])
@pytest.mark.parametrize("out", ["complex64", "power"])
def test_band_path_edges(L, out):
    """Register-resident lengths: rows whose spectrum band has at most 256
    bins take the band path, wider ones the full passes.  The grid is chosen
    so that both kinds occur, including bands that wrap past bin 0, bands that
    end at the last positive bin and bands of 1 to 256 bins; every row is
    checked against the oracle."""
    sfreq = 1000.0
    N = L - 37  # ragged crop
    # 20 log-spaced frequencies alternating 3 and 12 cycles, one 3-cycle wavelet
    # at 499 Hz (band = whole spectrum) and a long wavelet at 495 Hz whose
    # narrow band runs up to the last positive bin
    freqs = np.concatenate([synth.log_freqs(0.3, 480.0, 20), [499.0, 495.0]])
    cyc = np.concatenate([np.where(np.arange(20) % 2 == 0, 3.0, 12.0), [3.0, 60.0 * L / 1024]])
    rng = np.random.default_rng(L)
    x = rng.normal(0, 20, size=(2, N)).astype(np.float32)
    plan, W = _run(x, sfreq, freqs, cyc, pad="pow2", out=out)
    assert plan.L == L and plan.desc.kernel == 1
    _, band, _ = plan.tables()
    lo, K = band[:, 0], band[:, 1]
    assert (K <= 256).any() and (K > 256).any(), K
    narrow = K <= 256
    assert (lo[narrow] < 0).any(), "no narrow band wrapping past bin 0"
    # (the spectrum vanishes at negative frequencies, so a band ends at the
    # last positive bin at the latest; bands wrapping past bin 0 read the
    # conjugated upper half)
    assert ((lo + K == L // 2) & narrow).any(), "no narrow band up to the last positive bin"
    assert (K == L).any(), "no whole-spectrum band"
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc, L=L)
    if out == "complex64":
        _parity(W, ref, "band path L=%d" % L)
    else:
        Pr = oracle.power(ref)
        e = np.max(np.abs(W - Pr)) / Pr.max()
        print("band path L=%d power e=%.3e" % (L, e))
        assert e <= TOL_P
    plan.close()



@pytest.mark.parametrize("n,precision,out", [(4096, "fp32", "complex64"), (4096, "fp32", "bandpower"),
                                             (1000, "fp32", "power"), (4096, "split_bf16", "complex64"),
                                             (1000, "fp32", "complex64"), (2000, "fp32", "bandpower"),
                                             (1200, "fp32", "power"), (1200, "fp32", "complex64"),
                                             (1600, "fp32", "complex64"), (800, "fp32", "bandpower"),
                                             (400, "fp32", "power"), (200, "fp32", "complex64"),
                                             (4000, "fp32", "complex64"), (8000, "fp32", "bandpower"),
                                             (5000, "fp32", "power"), (10000, "fp32", "complex64"),
                                             (2500, "fp32", "bandpower")])
def test_execute_batches_matches_execute(n, precision, out):
    """cwt_execute_batches gives, batch for batch, exactly cwt_execute's
    output: with the register-resident kernels (L = 4096 and the mixed-radix
    L = 200 to 10000; transform of one batch and forward FFT of the next in
    one launch), with the runtime-radix kernel (L = 1200) and with the
    split-precision path; a zero stride reuses one buffer; n_batches = 0 is a
    no-op; bad arguments are rejected."""
    C, nb = 3, 5
    d = synth.eeg_64ch(C=C * nb, N=n, F=40)
    x = torch.from_numpy(d["x"]).cuda().view(nb, C, -1)
    plan = cwt.Plan(n, d["sfreq"], d["freqs"], n_cycles=d["n_cycles"], precision=precision,
                    out=out)
    assert plan.desc.kernel == (1 if n in (200, 400, 800, 1000, 1600, 2000, 2500, 4000, 4096,
                                           5000, 8000, 10000) else 0)
    refs = [plan.execute(x[i]).clone() for i in range(nb)]
    outb = torch.stack([torch.empty_like(refs[0]) for _ in range(nb)])
    ws = plan.alloc_batches_workspace(C)
    s = torch.cuda.Stream()
    # the references, and the allocator blocks that ws and outb may reuse,
    # belong to the current stream: let them finish before s starts
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.execute_batches(x, nb, outb, ws, C, stream=s)
    torch.cuda.synchronize()
    for i in range(nb):
        assert torch.equal(outb[i], refs[i]), "batch %d differs" % i
    one = torch.empty_like(refs[0])
    plan.execute_batches(x[0], 4, one, ws, C, x_batch_stride=0, out_batch_stride=0)
    torch.cuda.synchronize()
    assert torch.equal(one, refs[0])
    one.zero_()
    plan.execute_batches(x, 0, one, ws, C)
    torch.cuda.synchronize()
    assert not one.abs().any()
    from paper_2506_07793_amd import _lib
    lib = _lib.load()
    import ctypes
    vp = ctypes.c_void_p
    args = (vp(x.data_ptr()), C * n, 2, C, vp(outb.data_ptr()))
    assert lib.cwt_execute_batches(plan.handle, *args, 12, vp(ws.data_ptr()), ws.numel(),
                                   None) == _lib.CWT_E_INVALID  # stride not a multiple of 8
    assert lib.cwt_execute_batches(plan.handle, *args, plan.output_bytes(C), vp(ws.data_ptr()),
                                   ws.numel() // 2, None) == _lib.CWT_E_INVALID  # one half only
    assert lib.cwt_execute_batches(plan.handle, vp(x.data_ptr()), -1, 2, C, vp(outb.data_ptr()),
                                   0, vp(ws.data_ptr()), ws.numel(), None) == _lib.CWT_E_INVALID
    plan.close()



# ------------------------------------------------ generalized Morse wavelet --

@pytest.mark.parametrize("n,pad,out", [(4096, "smooth7", "complex64"), (4096, "smooth7", "power"),
                                       (4096, "smooth7", "bandpower"), (1000, "smooth7", "complex64"),
                                       (3000, "pow2", "complex64"), (777, "smooth7", "power")])
def test_gmw_parity(n, pad, out):
    """GMW plans (beta 17.5, gamma 3, the paper's values) against the oracle:
    register-resident (band and wide rows), runtime-radix and power-of-two
    lengths, every output mode."""
    d = synth.eeg_64ch(C=2, N=n, F=40)
    x, sfreq, freqs = d["x"], d["sfreq"], d["freqs"]
    plan, W = _run(x, sfreq, freqs, None, wavelet="gmw", pad=pad, out=out)
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, None, kind="gmw", L=plan.L)
    if out == "complex64":
        _parity(W, ref, "gmw n=%d L=%d kernel=%d" % (n, plan.L, plan.desc.kernel))
    else:
        Pr = oracle.power(ref)
        if out == "bandpower":
            Pr = oracle.band_power(Pr, oracle.band_groups(freqs))
        e = np.max(np.abs(W - Pr)) / Pr.max()
        print("gmw %s n=%d e=%.3e" % (out, n, e))
        assert e <= TOL_P
    plan.close()


@pytest.mark.parametrize("beta,gamma", [(17.5, 3.0), (3.0, 1.0), (8.0, 2.0)])
def test_gmw_tone_amplitude(beta, gamma):
    """A tone A sin(w0 t) at an exact bin: at f0 the GMW transform is
    -i A sqrt(u_p sfreq / f0) exp(i w0 t) (closed form; the oracle's own pin)."""
    N, sfreq, b0, A = 4096, 1000.0, 164, 20.0
    f0 = b0 * sfreq / N
    x = (A * np.sin(2 * np.pi * b0 * np.arange(N) / N)).astype(np.float32)
    plan = cwt.Plan(N, sfreq, [f0], wavelet="gmw", gmw_beta=beta, gmw_gamma=gamma)
    W = plan.execute(torch.from_numpy(x[None, :]).cuda()).cpu().numpy()[0, 0]
    up = (beta / gamma) ** (1.0 / gamma)
    amp = A * np.sqrt(up * sfreq / f0)
    ref = -1j * amp * np.exp(2j * np.pi * b0 * np.arange(N) / N)
    e = np.max(np.abs(W - ref)) / amp
    print("gmw tone beta=%g gamma=%g e=%.3e" % (beta, gamma, e))
    assert e <= 1e-5
    plan.close()


@pytest.mark.parametrize("N", [101, 127, 128, 499, 997, 1024, 1999, 2048, 2477, 2500])
def test_length_sweep_lengths(N):
    """Lengths of the length sweep (primes, powers of two, round numbers;
    Morlet sigma 7, 61 frequencies 30-90 Hz at 1000 Hz) against the oracle."""
    sfreq, freqs = 1000.0, np.arange(30.0, 91.0)
    x = synth.eeg(2, N, sfreq, N)
    plan, W = _run(x, sfreq, freqs, 7.0)
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, 7.0, L=plan.L)
    _parity(W, ref, "sweep N=%d L=%d kernel=%d" % (N, plan.L, plan.desc.kernel))
    plan.close()


@pytest.mark.parametrize("n,sfreq", [(2000, 1000.0), (1000, 250.0)])
def test_linear_edge_mode_parity(n, sfreq):
    """pad="linear" (no cyclic wrap at the edges) against the oracle."""
    freqs = synth.log_freqs(1.0, min(100.0, 0.45 * sfreq), 30)
    cyc = synth.eeg_cycles(freqs)
    x = synth.eeg(2, n, sfreq, 21)
    plan, W = _run(x, sfreq, freqs, cyc, pad="linear")
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc, pad="linear")
    assert plan.L == oracle.pad_length(n, "linear", support=oracle.linear_support(sfreq, freqs, cyc))
    _parity(W, ref, "linear n=%d L=%d" % (n, plan.L))
    plan.close()


# ------------------------------------------------- sampled (user) wavelets --

def _chirp_wavelets(F, w, sfreq, seed):
    """Arbitrary complex wavelets: Gaussian-windowed linear chirps with random
    centre frequency, sweep, width and phase (complex spectra, not symmetric)."""
    rng = np.random.default_rng(seed)
    t = (np.arange(w) - w // 2) / sfreq
    out = np.empty((F, w), np.complex128)
    for i in range(F):
        f0 = rng.uniform(3.0, 0.3 * sfreq)
        sd = rng.uniform(0.2, 0.45) * (w / 2) / sfreq
        sweep = rng.uniform(-0.5, 0.5) * f0 / (4 * sd)
        out[i] = np.exp(-0.5 * (t / sd) ** 2) * np.exp(
            2j * np.pi * (f0 * t + sweep * t * t) + 1j * rng.uniform(0, 2 * np.pi)) / np.sqrt(sfreq)
    return out.astype(np.complex64)


@pytest.mark.parametrize("n,w,pad,out", [(4096, 301, "smooth7", "complex64"), (4096, 1024, "pow2", "power"),
                                         (1000, 251, "smooth7", "complex64"), (1000, 64, "smooth7", "bandpower"),
                                         (2000, 401, "linear", "complex64")])
def test_sampled_wavelet_parity(n, w, pad, out):
    """Plans from sampled wavelets (complex spectra; register-resident and
    runtime-radix kernels, every output mode, linear padding) against the
    oracle's direct cyclic convolution with the placed wavelets."""
    sfreq = 1000.0
    F = 12
    freqs = synth.log_freqs(2.0, 100.0, F)
    wv = _chirp_wavelets(F, w, sfreq, n + w)
    x = synth.eeg(2, n, sfreq, w)
    plan = cwt.Plan.from_wavelets(n, sfreq, freqs, wv, pad=pad, out=out)
    assert plan.desc.spectrum_complex == 1
    W = plan.execute(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = oracle.cwt_user(x.astype(np.float64), wv.astype(np.complex128), pad=pad,
                          L=plan.L if pad != "linear" else None)
    assert ref.shape[-1] == n
    if out == "complex64":
        _parity(W, ref, "user n=%d w=%d L=%d kernel=%d" % (n, w, plan.L, plan.desc.kernel))
    else:
        Pr = oracle.power(ref)
        if out == "bandpower":
            Pr = oracle.band_power(Pr, oracle.band_groups(freqs))
        e = np.max(np.abs(W - Pr)) / Pr.max()
        print("user %s n=%d e=%.3e" % (out, n, e))
        assert e <= TOL_P
    plan.close()


def test_sampled_wavelet_tables_and_paths():
    """Spectra within FP32 rounding of the FP64 DFT of the placed wavelets;
    the sampled textbook Morlet reproduces the closed-form plan; batches of
    one plan (fused launches) equal single calls; stream sessions refuse the
    plan."""
    n, sfreq = 4096, 1000.0
    freqs = np.array([8.0, 20.0, 45.0])
    sig = 7.0
    rng = np.random.default_rng(3)
    # spectra against the FP64 DFT of the placed wavelets
    wv = _chirp_wavelets(3, 333, sfreq, 9)
    plan = cwt.Plan.from_wavelets(n, sfreq, freqs, wv)
    H, band, _ = plan.tables()
    ref = np.fft.fft(oracle.user_wavelet_time(wv.astype(np.complex128), plan.L), axis=1) / plan.L
    for i in range(3):
        lo, K, off = band[i]
        idx = (lo + np.arange(K)) % plan.L
        d = np.abs(H[off:off + K].astype(np.complex128) - ref[i, idx])
        assert np.max(d) <= 2e-7 * np.abs(ref[i]).max() + 1e-30
        mask = np.ones(plan.L, bool)
        mask[idx] = False
        assert np.all(np.abs(ref[i, mask]) <= 1e-12 * np.abs(ref[i]).max() * 1.01)
    # batches through the fused launches
    x = torch.from_numpy(synth.eeg(6, n, sfreq, 5)).cuda().view(3, 2, n)
    refs = [plan.execute(x[i]).clone() for i in range(3)]
    outb = torch.stack([torch.empty_like(refs[0]) for _ in range(3)])
    plan.execute_batches(x, 3, outb, plan.alloc_batches_workspace(2), 2)
    torch.cuda.synchronize()
    for i in range(3):
        assert torch.equal(outb[i], refs[i])
    plan.close()
    # sampled Morlet (periodised onto L) against the closed-form plan
    t = np.arange(n)
    rows = []
    for f in freqs:
        s = sig / (2 * np.pi * f)
        half = int(np.ceil(8 * s * sfreq))
        m = np.arange(-half, half + 1)
        kappa = np.exp(-sig * sig / 2)
        c = (1 + np.exp(-sig * sig) - 2 * np.exp(-0.75 * sig * sig)) ** -0.5
        u = m / sfreq / s
        wm = np.sqrt(1 / sfreq) * s ** -0.5 * c * np.pi ** -0.25 * np.exp(-0.5 * u * u) * (
            np.exp(1j * sig * u) - kappa)
        circ = np.zeros(n, complex)
        np.add.at(circ, m % n, wm)
        rows.append(circ[(t - n // 2) % n])
    xs = synth.eeg(2, n, sfreq, 8)
    pu = cwt.Plan.from_wavelets(n, sfreq, freqs, np.array(rows))
    pc = cwt.Plan(n, sfreq, freqs, n_cycles=sig)
    assert pu.L == pc.L == n
    Wu = pu.execute(torch.from_numpy(xs).cuda()).cpu().numpy()
    Wc = pc.execute(torch.from_numpy(xs).cuda()).cpu().numpy()
    refc = oracle.cwt(xs.astype(np.float64), sfreq, freqs, sig)
    _parity(Wu, refc, "sampled Morlet")
    _parity(Wc, refc, "closed-form Morlet")
    # streams need closed-form spectra
    from paper_2506_07793_amd import stream as cstream
    pb = cwt.Plan.from_wavelets(2000, sfreq, synth.log_freqs(1.0, 100.0, 40),
                                _chirp_wavelets(40, 101, sfreq, 4), out="bandpower")
    srv = cstream.Server(1 << 30)
    with pytest.raises(cwt.CwtError) as e:
        srv.open(pb, 4, 50)
    assert e.value.code == _lib_codes().CWT_E_UNSUPPORTED
    srv.close()
    for p in (pu, pc, pb):
        p.close()


def _lib_codes():
    from paper_2506_07793_amd import _lib
    return _lib


def _skipped_passes(K, L, radices):
    """Leading passes a band of K bins lets the runtime-radix kernel replace
    by its prologue: while K <= L / (product of the radices so far)."""
    p0, ns = 0, 1
    while p0 < len(radices) - 1 and K * ns * radices[p0] <= L:
        ns *= radices[p0]
        p0 += 1
    return p0


@pytest.mark.parametrize("L", [98, 1000, 1680, 2187, 4116, 10000])
@pytest.mark.parametrize("out", ["complex64", "power", "bandpower"])
def test_generic_band_prologue(L, out, monkeypatch):
    """Runtime-radix kernel: rows whose band fits in L / Ns consecutive bins
    replace the first passes (radix product Ns) by one complex product per
    element.  The grid mixes 3-, 12- and 80-cycle wavelets from 0.3 Hz to
    near Nyquist plus a whole-spectrum row, so that every number of replaced
    passes from none to all but the last occurs (even and odd first radices,
    bands wrapping past bin 0, a ragged crop); every row against the oracle."""
    sfreq = 1000.0
    N = L - 5
    # 2000- and 1000-cycle rows: bands of one to three bins at every L here
    freqs = np.concatenate([synth.log_freqs(0.3, 480.0, 24), [499.0, 20.0, 7.7]])
    cyc = np.concatenate([np.tile([3.0, 12.0, 80.0], 8), [3.0, 2000.0, 1000.0]])
    rng = np.random.default_rng(L + 7)
    x = rng.normal(0, 20, size=(2, N)).astype(np.float32)
    monkeypatch.setenv("CWT_GENERIC_ONLY", "1")  # L = 1000 has a register-resident kernel
    plan, W = _run(x, sfreq, freqs, cyc, pad="explicit", explicit_len=L, out=out)
    monkeypatch.delenv("CWT_GENERIC_ONLY")
    assert plan.L == L and plan.desc.kernel == 0
    rad = plan.radices
    _, band, _ = plan.tables()
    p0 = np.array([_skipped_passes(int(K), L, rad) for K in band[:, 1]])
    print("L=%d radices %s skipped passes per row %s" % (L, rad, p0.tolist()))
    assert (p0 == 0).any() and (p0 >= 1).any()
    if L in (98, 1000, 10000):  # every pass but the storing one replaced
        assert (p0 == len(rad) - 1).any()
    if len(rad) >= 3:
        assert ((p0 >= 1) & (p0 < len(rad) - 1)).any()
    assert (band[p0 > 0, 0] < 0).any(), "no wrapped band among the replaced rows"
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc, L=L)
    if out == "complex64":
        # per row as well, for the rows that carry signal (a wavelet far
        # longer than the record can leave a row at 1e-60 of the peak)
        pw = np.abs(ref) ** 2
        for i in range(len(freqs)):
            if pw[:, i].max() < 1e-6 * pw.max():
                continue
            e_P, _ = oracle.parity_errors(W[:, i], ref[:, i])
            assert e_P <= TOL_P, (i, p0[i], e_P)
        _parity(W, ref, "generic band prologue L=%d" % L)
    else:
        Pr = oracle.power(ref)
        if out == "bandpower":
            Pr = oracle.band_power(Pr, oracle.band_groups(freqs))
        e = np.max(np.abs(W - Pr)) / Pr.max()
        print("generic band prologue L=%d %s e=%.3e" % (L, out, e))
        assert e <= TOL_P
    plan.close()


@pytest.mark.parametrize("L,generic", [(1000, True), (4116, True), (4096, False), (2048, False),
                                       (1000, False), (2000, False)])
def test_generic_band_prologue_sampled_wavelets(L, generic, monkeypatch):
    """Narrow bands with complex spectra (plans from sampled wavelets): the
    runtime-radix prologue (L 1000, 4116), the register-resident band path
    (L 4096, 2048) and the mixed-radix register-resident first-pass
    prologue (L 1000, 2000).  A float32 wavelet's rounding noise reaches every bin, so
    only wavelets with exactly representable single-bin spectra have narrow
    bands: i^j (bin L/4) and (-1)^j (bin L/2), one bin each, beside two
    Gaussian-windowed tones whose bands cover the spectrum."""
    sfreq = 1000.0
    N = L - 3
    j = np.arange(L)
    t = (j - L // 2) / sfreq
    wv = np.stack([1j ** (j % 4), (-1.0) ** j,
                   np.exp(-0.5 * (t / 0.05) ** 2) * np.exp(2j * np.pi * 30.0 * t),
                   np.exp(-0.5 * (t / 0.02) ** 2) * np.exp(2j * np.pi * 90.0 * t)]) / 50.0
    freqs = np.array([250.0, 499.0, 30.0, 90.0])
    x = synth.eeg(2, N, sfreq, 11)
    if generic:
        monkeypatch.setenv("CWT_GENERIC_ONLY", "1")
    plan = cwt.Plan.from_wavelets(N, sfreq, freqs, wv, pad="explicit", explicit_len=L)
    monkeypatch.delenv("CWT_GENERIC_ONLY", raising=False)
    fixed = not generic
    assert plan.L == L and plan.desc.kernel == (1 if fixed else 0)
    assert plan.desc.spectrum_complex == 1
    _, band, _ = plan.tables()
    p0 = [_skipped_passes(int(K), L, plan.radices) for K in band[:, 1]]
    print("sampled L=%d bands %s skipped passes %s" % (L, band[:, :2].tolist(), p0))
    assert band[0, 1] == 1 and band[1, 1] == 1
    assert fixed or p0[0] == len(plan.radices) - 1
    W = plan.execute(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = oracle.cwt_user(x.astype(np.float64), wv.astype(np.complex64).astype(np.complex128),
                          pad="explicit", L=L)
    for i in range(4):
        _parity(W[:, i], ref[:, i], "sampled generic band prologue L=%d row %d" % (L, i))
    plan.close()


def test_launch_work_item_limit():
    """One workgroup per output row: a call whose launch would hold 2^32
    work-items or more is refused before any launch (here 4096 rows of
    1024-thread workgroups per channel: 1024 channels and up), and the largest
    channel count below the limit still runs."""
    from paper_2506_07793_amd import _lib
    L = 16384
    freqs = synth.log_freqs(0.5, 400.0, 4096)
    plan = cwt.Plan(L, 1000.0, freqs, n_cycles=7.0)
    assert plan.L == L and plan.desc.kernel == 0 and plan.desc.threads == 1024
    C = 1100
    x = torch.zeros(C, L, device="cuda")
    ws = plan.alloc_workspace(C)
    with pytest.raises(_lib.CwtError) as e:
        plan.forward_spectra(x, ws)
    assert e.value.code == _lib.CWT_E_UNSUPPORTED and "split C" in str(e.value)
    plan.forward_spectra(x[:1000], ws)  # 1000 x 4096 x 1024 < 2^32
    torch.cuda.synchronize()
    plan.close()


@pytest.mark.parametrize("L", [200, 400, 800, 1000, 1600, 2000, 2500, 4000, 5000, 8000, 10000])
@pytest.mark.parametrize("out", ["complex64", "power", "bandpower"])
def test_mixed_radix_register_kernel(L, out, monkeypatch):
    """Mixed-radix register-resident kernels (L = 200 = 10*20, 400 = 20*20,
    800 = 4*10*20, 1000 = 5*20*10, 1600 = 4*20*20, 2000 = 5*20*20, 2500 =
    5*5*20*5, 4000 = 10*20*20, 5000 = 5*20*10*5, 8000 = 20*20*20, 10000 =
    5*20*20*5; 20 values per thread, 32, 16, 8, 5, 4, 3, 2 or 1 transforms
    per workgroup, two to four passes): rows whose band fits in S = L / R0
    bins (R0 the first radix) replace the first pass by one product per
    element, wider rows stage their band and run every pass.  The grid
    mixes both kinds (and bands wrapping past bin 0), 5 channels (a forward
    pair past the last channel), a row count that is not a multiple of the
    transforms per workgroup and a ragged crop; every row against the oracle,
    and the whole output against the runtime-radix kernel's."""
    sfreq = 1000.0
    N = L - 7
    freqs = np.concatenate([synth.log_freqs(0.4, 470.0, 20), [499.0, 12.0, 60.0]])
    cyc = np.concatenate([np.tile([3.0, 7.0, 40.0, 9.0], 5), [3.0, 300.0, 2.5]])
    C = 5
    x = synth.eeg(C, N, sfreq, L + 3)
    plan, W = _run(x, sfreq, freqs, cyc, pad="explicit", explicit_len=L, out=out)
    assert plan.L == L and plan.desc.kernel == 1
    S = L // plan.radices[0]
    _, band, _ = plan.tables()
    narrow = band[:, 1] <= S
    print("L=%d: %d narrow rows (K <= %d), %d wide; K = %s" % (
        L, narrow.sum(), S, (~narrow).sum(), band[:, 1].tolist()))
    assert narrow.any() and (~narrow).any()
    assert (band[narrow, 0] < 0).any(), "no wrapped band among the narrow rows"
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc, L=L)
    if out == "complex64":
        pw = np.abs(ref) ** 2
        for i in range(len(freqs)):
            if pw[:, i].max() < 1e-6 * pw.max():
                continue
            e_P, _ = oracle.parity_errors(W[:, i], ref[:, i])
            assert e_P <= TOL_P, (i, bool(narrow[i]), e_P)
        _parity(W, ref, "mixed radix L=%d" % L)
    else:
        Pr = oracle.power(ref)
        if out == "bandpower":
            Pr = oracle.band_power(Pr, oracle.band_groups(freqs))
        e = np.max(np.abs(W - Pr)) / Pr.max()
        print("mixed radix L=%d %s e=%.3e" % (L, out, e))
        assert e <= TOL_P
    monkeypatch.setenv("CWT_GENERIC_ONLY", "1")
    gplan, Wg = _run(x, sfreq, freqs, cyc, pad="explicit", explicit_len=L, out=out)
    monkeypatch.delenv("CWT_GENERIC_ONLY")
    assert gplan.desc.kernel == 0
    scale = np.abs(Wg).max()
    d = np.abs(W - Wg).max() / scale
    print("  against the runtime-radix kernel: max |diff| / max = %.2e" % d)
    assert d <= 2e-6
    plan.close()
    gplan.close()


@pytest.mark.parametrize("L,variant", [(1000, 0), (2000, 0), (1000, 1), (800, 0), (800, 1),
                                       (1600, 0), (1600, 1), (200, 0), (200, 1), (400, 0),
                                       (400, 1), (4000, 0), (4000, 1), (8000, 0), (8000, 1),
                                       (5000, 0), (5000, 1), (10000, 0), (10000, 1),
                                       (2500, 0), (2500, 1)])
def test_mixed_radix_twiddle_variants_and_sizes(L, variant, monkeypatch):
    """Both twiddle methods of the mixed-radix kernels (table, powers), one
    channel (the forward's second channel absent) and 64 channels (many
    workgroups; the last partly filled), against the oracle on sampled rows."""
    monkeypatch.setenv("CWT_FIXED_VARIANT", str(variant))
    d = synth.eeg_64ch(C=64, N=L, F=37)
    for C in (1, 64):
        x = d["x"][:C]
        plan, W = _run(x, d["sfreq"], d["freqs"], d["n_cycles"])
        assert plan.L == L and plan.desc.kernel == 1
        rows = np.array([(c, f) for c in sorted({0, C // 2, C - 1}) for f in (0, 11, 23, 36)])
        ref = oracle.cwt(x.astype(np.float64), d["sfreq"], d["freqs"], d["n_cycles"], rows=rows)
        got = np.stack([W[c, f] for c, f in rows])
        e_P, e_W = oracle.parity_errors(got, ref)
        print("L=%d variant %d C=%d: e_P=%.3e e_W=%.3e" % (L, variant, C, e_P, e_W))
        assert e_P <= TOL_P
        plan.close()


@pytest.mark.parametrize("L,radix", [(19683, [9, 9, 9, 9, 3]), (19440, [16, 15, 9, 9]),
                                     (20480, [16, 16, 16, 5]), (16875, [15, 15, 15, 5]),
                                     (14406, [21, 14, 7, 7]), (18432, [16, 12, 12, 8]),
                                     (16800, [15, 14, 10, 8]), (17496, [24, 9, 9, 9])])
@pytest.mark.parametrize("out", ["complex64", "bandpower"])
def test_runtime_radix_32_value_plans(L, radix, out):
    """Runtime-radix plans of the 32-value class (at most 768 threads, up to
    32 values per thread in a pass), which the planner takes where they save
    a pass (19683: 5 passes instead of 9; 19440: 4 instead of 6) and, above
    16 384 points, before the 24-value class at equal passes (18432, 16800):
    sampled rows over windows at both ends and the middle of a ragged crop
    against the oracle, complex and band power."""
    sfreq = 1000.0
    N = L - 3
    C = 3
    freqs = synth.log_freqs(1.0, 100.0, 20)
    cyc = synth.eeg_cycles(freqs)
    x = synth.eeg(C, N, sfreq, L % 1000 + 5)
    plan, W = _run(x, sfreq, freqs, cyc, pad="explicit", explicit_len=L, out=out)
    assert plan.L == L and plan.desc.kernel == 0
    assert plan.radices == radix and plan.desc.threads <= 768, (plan.radices, plan.desc.threads)
    starts = (0, N // 2 - 32, N - 64)
    x64 = x.astype(np.float64)
    if out == "complex64":
        rows = [(c, f) for c in range(C) for f in (0, 9, 19)]
        ref = np.concatenate([oracle.cwt(x64, sfreq, freqs, cyc, L=L, rows=rows, t0=t0, nt=64)
                              for t0 in starts], axis=1)
        got = np.concatenate([np.stack([W[c, f, t0:t0 + 64] for c, f in rows]) for t0 in starts],
                             axis=1)
        _parity(got, ref, "32-value plan L=%d %s" % (L, radix))
    else:
        groups = oracle.band_groups(freqs)
        rows = [(c, f) for c in range(C) for f in range(len(freqs))]
        for t0 in (starts[0], starts[2]):
            ref = oracle.cwt(x64, sfreq, freqs, cyc, L=L, rows=rows, t0=t0, nt=64)
            P = (np.abs(ref) ** 2).reshape(C, len(freqs), 64)
            Br = oracle.band_power(P, groups)
            e = float(np.abs(W[:, :, t0:t0 + 64] - Br).max() / Br.max())
            print("32-value plan L=%d band power window %d: e=%.3e" % (L, t0, e))
            assert e <= TOL_P
    plan.close()
