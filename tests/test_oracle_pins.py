"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a closed form evaluated here in
high precision (mpmath), quadrature, a brute-force computation by an
independent route (numpy's FFT for the cyclic-convolution identity), or an
invariant of the mathematics.  Together they are chosen so that a dropped term,
a wrong sign or index, or a transposed operand in the oracle fails at least
one of them (``test_oracle_mutants.py`` plants such mistakes to show it).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import synth

mp.mp.dps = 40


# ---------------------------------------------------------------- constants --

def _mp_psi_hat(sigma, u, c, kappa):
    return c * mp.pi ** (-0.25) * (mp.exp(-(sigma - u) ** 2 / 2) - kappa * mp.exp(-u ** 2 / 2))


@pytest.mark.parametrize("sigma", [3.0, 5.0, 7.0, 10.0])
def test_morlet_constants_unit_energy_and_admissible(orc, sigma):
    """Morlet equation: c and kappa make int |Psi_hat|^2 du = 1 and Psi_hat(0) = 0."""
    c, kappa = orc.wavelet_constants(sigma, orc.MORLET)
    # Admissibility: the Fourier transform vanishes at zero frequency.
    assert abs(orc.mother_spectrum(sigma, 0.0)[0]) < 1e-15
    # Unit L2 energy by adaptive quadrature in 40-digit arithmetic.
    E = mp.quad(lambda u: _mp_psi_hat(mp.mpf(sigma), u, mp.mpf(c), mp.mpf(kappa)) ** 2,
                [-mp.inf, 0, sigma, mp.inf])
    assert abs(float(E) - 1.0) < 1e-15
    # kappa is exactly the value that zeroes Psi_hat(0).
    assert abs(kappa - math.exp(-sigma * sigma / 2)) <= 1e-17 + 1e-15 * kappa


def test_gabor_constants(orc):
    """Gabor equation: kappa = 0; unit energy then needs c = 1."""
    c, kappa = orc.wavelet_constants(7.0, orc.GABOR)
    assert kappa == 0.0 and c == 1.0
    E = mp.quad(lambda u: _mp_psi_hat(mp.mpf(7), u, 1, 0) ** 2, [-mp.inf, 7, mp.inf])
    assert abs(float(E) - 1.0) < 1e-15


def test_mother_spectrum_matches_closed_form(orc):
    for sigma in (3.0, 6.5, 10.0):
        c, kappa = orc.wavelet_constants(sigma)
        u = np.linspace(-4, 20, 97)
        got = orc.mother_spectrum(sigma, u)
        ref = np.array([float(_mp_psi_hat(mp.mpf(sigma), mp.mpf(v), mp.mpf(c), mp.mpf(kappa)))
                        for v in u])
        assert np.max(np.abs(got - ref)) < 1e-15


# ------------------------------------------------------------------ padding --

def _smooth7_sieve(limit):
    vals = set()
    p2 = 1
    while p2 <= limit:
        p3 = p2
        while p3 <= limit:
            p5 = p3
            while p5 <= limit:
                p7 = p5
                while p7 <= limit:
                    vals.add(p7)
                    p7 *= 7
                p5 *= 5
            p3 *= 3
        p2 *= 2
    return np.array(sorted(vals))


def test_pad_smooth7_against_sieve(orc):
    """Section "Fast Fourier transform": smallest 2,3,5,7-smooth length >= N."""
    s = _smooth7_sieve(120000)
    for n in list(range(1, 3000)) + list(range(3000, 100001, 37)) + [4097, 10007, 16385, 19999]:
        expect = int(s[np.searchsorted(s, n)])
        assert orc.pad_length(n) == expect, n
    assert orc.pad_length(4097) == 4116
    assert orc.pad_length(10007) == 10080
    assert orc.pad_length(102) == 105
    assert orc.pad_length(1000) == 1000 and orc.pad_length(2000) == 2000


def test_pad_pow2_and_explicit(orc):
    for n in (1, 2, 3, 1000, 1024, 1025, 4096, 20000):
        m = orc.pad_length(n, "pow2")
        assert m >= n and m & (m - 1) == 0 and (m // 2 < n or m == 1)
    assert orc.pad_length(1000, "none") == 1000
    assert orc.pad_length(1000, "explicit", 1500) == 1500
    with pytest.raises(ValueError):
        orc.pad_length(1000, "explicit", 999)


# ------------------------------------------------- spectrum <-> time domain --

def _periodised_time_morlet(L, sfreq, f, sigma, kind=0):
    """sqrt(dt) * sum_m psi_s((j + m L) dt): the textbook time-domain Morlet.

    psi(t) = c pi^-1/4 exp(-t^2/2) (exp(i sigma t) - kappa), psi_s(t) = s^-1/2 psi(t/s),
    written here independently of the oracle (c and kappa from their closed forms).
    """
    if kind == 0:
        kappa = math.exp(-sigma * sigma / 2)
        c = (1 + math.exp(-sigma * sigma) - 2 * math.exp(-0.75 * sigma * sigma)) ** -0.5
    else:
        kappa, c = 0.0, 1.0
    s = sigma / (2 * math.pi * f)
    dt = 1.0 / sfreq
    j = np.arange(L)
    acc = np.zeros(L, dtype=np.complex128)
    for m in range(-40, 41):
        u = (j + m * L) * dt / s
        acc += np.exp(-0.5 * u * u) * (np.exp(1j * sigma * u) - kappa)
    return math.sqrt(dt) * s ** -0.5 * c * math.pi ** -0.25 * acc


@pytest.mark.parametrize("L,sfreq,f,sigma,kind", [
    (1000, 1000.0, 10.0, 7.0, 0), (1000, 1000.0, 40.0, 7.0, 0), (1000, 1000.0, 3.0, 3.0, 0),
    (4096, 1000.0, 1.0, 3.0, 0), (4096, 1000.0, 25.0, 10.0, 0), (4096, 1000.0, 100.0, 10.0, 0),
    (512, 250.0, 20.0, 5.0, 1), (2000, 1000.0, 60.0, 10.0, 1),
])
def test_idft_of_spectrum_is_periodised_time_wavelet(orc, L, sfreq, f, sigma, kind):
    """IDFT(H_f) equals the sampled, periodised time-domain wavelet.

    Holds whenever the wavelet spectrum is negligible above Nyquist (true for
    every case here); pins the prefactor sqrt(2 pi s sfreq), the scale map
    s = sigma / (2 pi f), the sign of the oscillation and the IDFT direction.
    """
    h = orc.wavelet_time(orc.wavelet_spectrum(L, sfreq, f, sigma, kind))
    ref = _periodised_time_morlet(L, sfreq, f, sigma, kind)
    assert np.max(np.abs(h - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("L,sfreq,f,sigma", [
    (4096, 1000.0, 20.0, 10.0), (4096, 1000.0, 50.0, 10.0), (1000, 1000.0, 10.0, 7.0),
    (1000, 1000.0, 30.0, 7.0), (2000, 1000.0, 12.0, 6.0), (4096, 1000.0, 2.0, 3.0),
])
def test_unit_energy_within_riemann_bound(orc, L, sfreq, f, sigma):
    """sum_j |h_f[j]|^2 = 1 up to the Riemann-sum error 2 exp(-pi^2 (f L / (sigma sfreq))^2)."""
    r = f * L / (sigma * sfreq)
    assert r >= 1.4  # resolved: the window holds enough of the wavelet's spectrum samples
    h = orc.wavelet_time(orc.wavelet_spectrum(L, sfreq, f, sigma))
    E = float(np.sum(np.abs(h) ** 2))
    assert abs(E - 1.0) <= 2 * math.exp(-math.pi ** 2 * r * r) + 2e-13


def test_unit_energy_fails_by_design_when_unresolved(orc):
    """f = 1 Hz, sigma 3, 1 s window: too few bins across the spectrum; energy is not 1."""
    h = orc.wavelet_time(orc.wavelet_spectrum(1000, 1000.0, 1.0, 3.0))
    assert abs(float(np.sum(np.abs(h) ** 2)) - 1.0) > 0.5


def test_nyquist_bin_is_negative_frequency(orc):
    """Reading: for even L the Nyquist bin carries omega = -pi sfreq (numpy fftfreq)."""
    L, sfreq, f, sigma = 16, 16.0, 6.0, 1.0
    H = orc.wavelet_spectrum(L, sfreq, f, sigma)
    c, kappa = orc.wavelet_constants(sigma)
    s = sigma / (2 * math.pi * f)
    u = s * (-math.pi * sfreq)
    ref = math.sqrt(2 * math.pi * s * sfreq) * float(
        _mp_psi_hat(mp.mpf(sigma), mp.mpf(u), mp.mpf(c), mp.mpf(kappa)))
    assert abs(H[L // 2] - ref) < 1e-15 * max(1.0, abs(ref))
    # the other reading (+pi sfreq) gives a clearly different value here
    alt = math.sqrt(2 * math.pi * s * sfreq) * float(
        _mp_psi_hat(mp.mpf(sigma), mp.mpf(-u), mp.mpf(c), mp.mpf(kappa)))
    assert abs(alt - ref) > 0.1 * abs(alt)


# ----------------------------------------------------------- full pipeline --

@pytest.mark.parametrize("n,pad,explicit,kind", [
    (5, "smooth7", None, 0), (16, "smooth7", None, 0), (37, "smooth7", None, 0),
    (37, "pow2", None, 0), (50, "explicit", 63, 0), (64, "none", None, 1),
    (61, "smooth7", None, 1), (1, "smooth7", None, 0),
])
def test_direct_matches_fft_cyclic_brute_force(orc, n, pad, explicit, kind):
    """Direct O(N L) cyclic convolution == IFFT(FFT(x_pad) * H) (numpy FFT), n <= 64."""
    rng = np.random.default_rng(n)
    sfreq = 100.0
    freqs = np.array([3.0, 11.5, 30.0, 47.0])  # 47 Hz, sigma 1.5: spectrum reaches Nyquist
    cyc = np.array([4.0, 6.0, 10.0, 1.5])
    x = rng.normal(size=(3, n))
    L = orc.pad_length(n, pad, explicit)
    W = orc.cwt(x, sfreq, freqs, cyc, kind=kind, L=L)
    H = orc.wavelet_bank(L, sfreq, freqs, cyc, kind)
    xp = np.zeros((3, L))
    xp[:, :n] = x
    Wf = np.fft.ifft(np.fft.fft(xp)[:, None, :] * H[None], axis=-1)[:, :, :n]
    assert np.max(np.abs(W - Wf)) <= 1e-12 * np.max(np.abs(Wf))


def test_two_tone_closed_form(orc):
    """Exact-bin tones, L = N: W[t] = (A/2i)(H[b0] e^{i w0 t} - H[L-b0] e^{-i w0 t})."""
    N, sfreq = 1000, 1000.0
    comps = [(10.0, 1.0), (40.0, 0.5)]
    x = synth.tones(N, sfreq, comps)[None, :]
    freqs = np.arange(1.0, 51.0)
    W = orc.cwt(x, sfreq, freqs, 7.0)[0]
    t = np.arange(N)
    ref = np.zeros_like(W)
    for fi, f in enumerate(freqs):
        H = orc.wavelet_spectrum(N, sfreq, f, 7.0)
        for f0, A in comps:
            b0 = int(round(f0 * N / sfreq))
            w0 = 2 * np.pi * b0 * t / N
            ref[fi] += A / 2j * (H[b0] * np.exp(1j * w0) - H[N - b0] * np.exp(-1j * w0))
    assert np.max(np.abs(W - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_sinusoid_peak_amplitude_and_argmax(orc):
    """A pure sinusoid peaks at its own frequency with its analytic amplitude.

    |W| at f = f0 is (A/2) sqrt(2 pi s sfreq) c pi^-1/4 (1 - e^{-sigma^2}), evaluated
    here in 40-digit arithmetic from the closed forms; the grid argmax of the
    time-averaged power is the tone frequency (noise-free).
    """
    N, sfreq, sigma = 1000, 1000.0, 7.0
    freqs = np.arange(1.0, 51.0)
    x = synth.tones(N, sfreq, [(10.0, 1.0), (40.0, 0.5)])[None, :]
    W = orc.cwt(x, sfreq, freqs, sigma)[0]
    sg = mp.mpf(sigma)
    c = (1 + mp.exp(-sg ** 2) - 2 * mp.exp(-3 * sg ** 2 / 4)) ** -0.5
    for f0, A, expect in ((10.0, 1.0, 9.936457), (40.0, 0.5, 2.484114)):
        s = sg / (2 * mp.pi * f0)
        amp = float(A / 2 * mp.sqrt(2 * mp.pi * s * sfreq) * c * mp.pi ** -0.25 * (1 - mp.exp(-sg ** 2)))
        assert abs(amp - expect) < 1e-6
        fi = int(f0) - 1
        # the other tone and the negative-frequency term perturb |W| by < 1e-5
        assert np.max(np.abs(np.abs(W[fi]) - amp)) < 1e-5 * amp
    P = (np.abs(W) ** 2).mean(axis=1)
    assert freqs[np.argmax(P[:25])] == 10.0
    assert freqs[29 + np.argmax(P[29:])] == 40.0


def test_two_tone_noisy_signal_peaks(orc):
    """Two tones (sin 10 + 0.5 sin 40 + noise 0.5, seeded): power peaks near the tones."""
    x = synth.two_tone_signal()
    freqs = np.arange(1.0, 51.0)
    P = orc.power(orc.cwt(x, 1000.0, freqs, 7.0)[0]).mean(axis=1)
    assert abs(freqs[np.argmax(P[:25])] - 10.0) <= 1.0
    assert abs(freqs[29 + np.argmax(P[29:])] - 40.0) <= 1.0


# --------------------------------------------------------------- invariants --

def _rand(seed, C, N):
    return np.random.default_rng(seed).normal(size=(C, N))


def test_linearity(orc):
    x, y = _rand(1, 2, 300), _rand(2, 2, 300)
    freqs, cyc = [4.0, 17.0, 60.0], [3.0, 7.0, 10.0]
    Wx = orc.cwt(x, 250.0, freqs, cyc)
    Wy = orc.cwt(y, 250.0, freqs, cyc)
    Wz = orc.cwt(2.5 * x - 0.75 * y, 250.0, freqs, cyc)
    assert np.max(np.abs(Wz - (2.5 * Wx - 0.75 * Wy))) <= 1e-13 * np.max(np.abs(Wz))


def test_cyclic_shift_equivariance(orc):
    """L = N: shifting the input cyclically shifts every output row the same way."""
    x = _rand(3, 1, 360)
    freqs, cyc = [5.0, 20.0, 45.0], 6.0
    W = orc.cwt(x, 360.0, freqs, cyc, pad="none")
    Ws = orc.cwt(np.roll(x, 37, axis=1), 360.0, freqs, cyc, pad="none")
    assert np.max(np.abs(Ws - np.roll(W, 37, axis=2))) <= 1e-13 * np.max(np.abs(W))


def test_dc_null_and_gabor_dc(orc):
    """L = N: sum_t W[t] = X[0] H[0]; zero for Morlet (Psi_hat(0) = 0), not for Gabor."""
    x = _rand(4, 1, 256) + 3.0
    W = orc.cwt(x, 256.0, [8.0], 3.0, pad="none")[0, 0]
    assert abs(W.sum()) <= 1e-12 * np.sum(np.abs(W))
    Wg = orc.cwt(x, 256.0, [8.0], 3.0, kind="gabor", pad="none")[0, 0]
    H0 = orc.wavelet_spectrum(256, 256.0, 8.0, 3.0, orc.GABOR)[0]
    assert abs(Wg.sum() - x.sum() * H0) <= 1e-12 * abs(x.sum() * H0)


def test_parseval(orc):
    """L = N: sum_t |W[t]|^2 = (1/L) sum_b |X[b] H[b]|^2 with X from numpy's FFT."""
    x = _rand(5, 1, 500)
    for f, cyc in ((7.0, 4.0), (33.0, 9.0)):
        W = orc.cwt(x, 500.0, [f], cyc)[0, 0]
        H = orc.wavelet_spectrum(500, 500.0, f, cyc)
        X = np.fft.fft(x[0])
        assert abs(np.sum(np.abs(W) ** 2) - np.sum(np.abs(X * H) ** 2) / 500) <= 1e-12 * np.sum(
            np.abs(W) ** 2)


def test_rows_and_window_selection(orc):
    """Row/t-window selection returns the same numbers as the full transform."""
    x = _rand(6, 3, 200)
    freqs, cyc = [3.0, 9.0, 27.0, 81.0], 5.0
    W = orc.cwt(x, 200.0, freqs, cyc)
    rows = [(2, 1), (0, 3), (1, 0)]
    Wr = orc.cwt(x, 200.0, freqs, cyc, rows=rows, t0=50, nt=120)
    for i, (c, f) in enumerate(rows):
        assert np.array_equal(Wr[i], W[c, f, 50:170])


# ------------------------------------------------------------ band reductions --

def test_band_groups_counts(orc):
    """Band edges reading: 40 log-spaced 1-100 Hz frequencies split 12/6/4/7/11."""
    freqs = synth.log_freqs(1.0, 100.0, 40)
    g = orc.band_groups(freqs)
    assert [len(a) for a in g] == [12, 6, 4, 7, 11]
    assert sorted(np.concatenate(g).tolist()) == list(range(40))


# Band power and the streaming trailing-hop value, pinned against the tone
# closed form.  For L = N and tones x = sum_k A_k sin(w_k t + phi_k) on exact
# DFT bins b_k, the cyclic convolution with h = IDFT(H_f) is
#   W_f[t] = sum_k (A_k / 2i) (e^{i phi_k} H_f[b_k] e^{i w_k t}
#                              - e^{-i phi_k} H_f[L - b_k] e^{-i w_k t}),
# evaluated here with no convolution.  Band membership of the grid is written
# out by hand (not computed by a rule) for the edge reading delta [1, 4),
# theta [4, 8), alpha [8, 13), beta [13, 30), gamma [30, 100], and the grid has
# a frequency on every edge.  Tones close in frequency beat, so |W|^2 changes
# within a 50-sample hop: a window shifted by one sample, a sum for a mean or a
# band closed at the wrong end each change the result far beyond the 1e-12
# bar.

BAND_GRID = np.array([1.0, 2.5, 3.999, 4.0, 6.0, 7.5, 8.0, 10.0, 12.5, 13.0, 21.0, 29.5,
                      30.0, 60.0, 100.0])
BAND_MEMBERS = [[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11], [12, 13, 14]]
# (frequency Hz, amplitude, phase) per channel; every frequency is a bin of
# L = 2000 at 1000 Hz (0.5 Hz spacing)
BAND_TONES = [
    [(2.5, 1.2, 0.3), (6.0, 0.7, 1.1), (9.5, 1.0, 0.0), (11.0, 0.8, 2.0), (17.5, 0.5, 0.4),
     (23.0, 0.45, 2.9), (41.0, 0.3, 1.7), (57.5, 0.25, 0.2)],
    [(3.5, 0.9, 2.2), (7.0, 0.6, 0.5), (10.5, 1.1, 1.3), (12.0, 0.4, 0.8), (26.0, 0.5, 1.9),
     (35.0, 0.35, 0.6), (58.5, 0.2, 2.4), (99.5, 0.15, 1.0)],
]


def _tone_signal(N, sfreq, tones):
    t = np.arange(N) / sfreq
    return np.stack([sum(A * np.sin(2 * np.pi * f0 * t + ph) for f0, A, ph in ch)
                     for ch in tones])


def _tone_closed_form(orc, N, sfreq, freqs, cycles, tones):
    """[C, F, N] complex W from the tone closed form (L = N, exact bins)."""
    t = np.arange(N)
    W = np.zeros((len(tones), len(freqs), N), dtype=np.complex128)
    for fi, (f, s) in enumerate(zip(freqs, cycles)):
        H = orc.wavelet_spectrum(N, sfreq, f, s)
        for c, ch in enumerate(tones):
            for f0, A, ph in ch:
                b0 = int(round(f0 * N / sfreq))
                assert abs(b0 * sfreq / N - f0) < 1e-12  # exact bin
                w0 = 2 * np.pi * b0 * t / N
                W[c, fi] += A / 2j * (np.exp(1j * ph) * H[b0] * np.exp(1j * w0)
                                      - np.exp(-1j * ph) * H[N - b0] * np.exp(-1j * w0))
    return W


def _hand_band_means(P):
    """[C, F, ...] power -> [C, 5, ...] by the hand-written membership."""
    return np.stack([sum(P[:, i] for i in m) / len(m) for m in BAND_MEMBERS], axis=1)


def test_band_groups_on_the_edges(orc):
    """Each grid frequency lands in the band written out by hand, edges included."""
    got = [list(g) for g in orc.band_groups(BAND_GRID)]
    assert got == BAND_MEMBERS


def test_band_power_tone_closed_form(orc):
    """Band power = mean over the band's grid frequencies of |W|^2, against the
    tone closed form (every output sample, both channels)."""
    N, sfreq = 2000, 1000.0
    cyc = synth.eeg_cycles(BAND_GRID)
    x = _tone_signal(N, sfreq, BAND_TONES)
    Wref = _tone_closed_form(orc, N, sfreq, BAND_GRID, cyc, BAND_TONES)
    ref = _hand_band_means(np.abs(Wref) ** 2)
    got = orc.band_power(orc.power(orc.cwt(x, sfreq, BAND_GRID, cyc)),
                         orc.band_groups(BAND_GRID))
    assert got.shape == ref.shape == (2, 5, N)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(ref)
    for b in range(5):  # every band, not just the strongest
        assert np.max(np.abs(got[:, b] - ref[:, b])) <= 1e-10 * np.max(ref[:, b])


def test_band_power_varies_within_a_hop(orc):
    """The pin below is sensitive to the window position: the closed-form band
    power changes by far more than 1e-12 when the 50-sample window moves by
    one sample."""
    N, sfreq, hop = 2000, 1000.0, 50
    cyc = synth.eeg_cycles(BAND_GRID)
    BP = _hand_band_means(np.abs(_tone_closed_form(orc, N, sfreq, BAND_GRID, cyc,
                                                   BAND_TONES)) ** 2)
    cur = BP[:, :, N - hop:].mean(axis=2)
    early = BP[:, :, N - hop - 1:N - 1].mean(axis=2)
    assert np.min(np.abs(cur - early) / cur) > 1e-7


def test_stream_band_power_tone_closed_form(orc):
    """Streaming value: band power averaged over the window's last `hop`
    samples (t in [W - hop, W)), against the tone closed form."""
    N, sfreq, hop = 2000, 1000.0, 50
    cyc = synth.eeg_cycles(BAND_GRID)
    x = _tone_signal(N, sfreq, BAND_TONES)
    Wref = _tone_closed_form(orc, N, sfreq, BAND_GRID, cyc, BAND_TONES)
    ref = np.zeros((2, 5))
    for c in range(2):
        for b, m in enumerate(BAND_MEMBERS):
            acc = 0.0
            for t in range(N - hop, N):
                acc += sum(abs(Wref[c, i, t]) ** 2 for i in m) / len(m)
            ref[c, b] = acc / hop
    got = orc.stream_band_power(x, sfreq, BAND_GRID, cyc, hop)
    assert got.shape == (2, 5)
    assert np.max(np.abs(got - ref) / ref) <= 1e-11


# --------------------------------------------------------------- fixtures --

def test_two_tone_golden_samples(orc):
    """Regression guard: the oracle reproduces the samples make_golden.py stored."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "two_tone_oracle_samples.txt")
    rows = np.loadtxt(path)
    W = orc.cwt(synth.two_tone_signal(), 1000.0, np.arange(1.0, 51.0), 7.0)[0]
    for fi, t, re, im in rows:
        w = W[int(fi), int(t)]
        assert abs(w.real - re) <= 1e-13 * max(1.0, abs(re))
        assert abs(w.imag - im) <= 1e-13 * max(1.0, abs(im))


# ------------------------------------------------- generalized Morse wavelet --
# The GMW equation of "Fourier transformed formula", read with the unit step
# and alpha = 2 (e gamma / beta)^(beta / gamma).  Its moments are Gamma
# functions, which fix alpha, both exponents and the step independently of the
# oracle's own expression.

GMW_PARAMS = [(17.5, 3.0), (3.0, 1.0), (8.0, 2.0), (5.0, 4.0)]


def _mp_gmw_alpha(beta, gamma):
    return 2 * (mp.e * gamma / beta) ** (beta / gamma)


@pytest.mark.parametrize("beta,gamma", GMW_PARAMS)
def test_gmw_peak_is_two_at_closed_form_location(orc, beta, gamma):
    """Peak value 2 at u_p = (beta / gamma)^(1 / gamma), zero slope there."""
    b, g = mp.mpf(beta), mp.mpf(gamma)
    up = float((b / g) ** (1 / g))
    assert abs(orc.gmw_peak(beta, gamma) - up) <= 1e-15 * up
    v = orc.gmw_spectrum([up, up * (1 - 1e-3), up * (1 + 1e-3)], beta, gamma)
    assert abs(v[0] - 2.0) < 1e-13
    assert v[1] < 2.0 and v[2] < 2.0
    h = 1e-5 * up
    d = orc.gmw_spectrum([up + h, up - h], beta, gamma)
    assert abs(d[0] - d[1]) / (2 * h) < 1e-6


@pytest.mark.parametrize("beta,gamma", GMW_PARAMS)
def test_gmw_moments_match_gamma_functions(orc, beta, gamma):
    """int_0^inf Psi_hat du = alpha Gamma((beta+1)/gamma) / gamma and
    int_0^inf Psi_hat^2 du = alpha^2 Gamma((2 beta+1)/gamma) / (gamma 2^((2 beta+1)/gamma)),
    by 40-digit quadrature of the oracle's values against mpmath's Gamma."""
    b, g = mp.mpf(beta), mp.mpf(gamma)
    a = _mp_gmw_alpha(b, g)
    up = float((b / g) ** (1 / g))
    f = lambda u: mp.mpf(orc.gmw_spectrum([float(u)], beta, gamma)[0])
    # the integrand is below exp(-800) beyond u^gamma = 800 (the tail is
    # negligible; the FP64 product alpha u^beta exp(-u^gamma) would overflow
    # long before infinity)
    umax = 800 ** (1 / gamma)
    pts = [0, up / 2, up, 2 * up, 4 * up, umax]
    m1 = mp.quad(f, pts)
    m2 = mp.quad(lambda u: f(u) ** 2, pts)
    e1 = a * mp.gamma((b + 1) / g) / g
    e2 = a ** 2 * mp.gamma((2 * b + 1) / g) / (g * 2 ** ((2 * b + 1) / g))
    assert abs(float(m1 / e1) - 1) < 1e-12
    assert abs(float(m2 / e2) - 1) < 1e-12


def test_gmw_vanishes_at_nonpositive_frequencies(orc):
    """The unit-step reading: the GMW is analytic (no negative frequencies)."""
    v = orc.gmw_spectrum([-5.0, -1.0, -1e-9, 0.0])
    assert np.all(v == 0.0)
    H = orc.wavelet_spectrum(1000, 1000.0, 40.0, None, "gmw")
    assert np.all(H[500:] == 0.0) and H[0] == 0.0 and H.max() > 0
    # near Nyquist: the Nyquist bin of an even length is a negative frequency
    # (numpy's fftfreq convention), so it stays zero although the band reaches it
    H = orc.wavelet_spectrum(1000, 1000.0, 450.0, None, "gmw")
    assert H[499] > 0.1 * H.max() and np.all(H[500:] == 0.0)


@pytest.mark.parametrize("beta,gamma", [(17.5, 3.0), (3.0, 1.0)])
def test_gmw_tone_closed_form(orc, beta, gamma):
    """A tone A sin(w0 t) at an exact bin b0: the analytic wavelet keeps only the
    positive-frequency term, so at f0 = b0 sfreq / N the transform is exactly
    W[t] = -i A sqrt(u_p sfreq / f0) exp(i w0 t) (peak value 2, s w0 = u_p)."""
    N, sfreq, b0, A = 1000, 1000.0, 40, 0.7
    f0 = b0 * sfreq / N
    x = A * np.sin(2 * np.pi * b0 * np.arange(N) / N)
    W = orc.cwt(x[None, :], sfreq, [f0, 2 * f0], None, kind="gmw", beta=beta, gamma=gamma)[0]
    up = (mp.mpf(beta) / gamma) ** (1 / mp.mpf(gamma))
    amp = float(A * mp.sqrt(up * sfreq / f0))
    ref = -1j * amp * np.exp(2j * np.pi * b0 * np.arange(N) / N)
    assert np.max(np.abs(W[0] - ref)) <= 1e-12 * amp
    # at 2 f0 the tone sits at half the scaled peak frequency: Psi_hat(u_p / 2)
    half = float(_mp_gmw_alpha(mp.mpf(beta), gamma) * (up / 2) ** beta * mp.exp(-(up / 2) ** gamma))
    amp2 = float(A / 2 * mp.sqrt(up * sfreq / (2 * f0))) * half
    assert np.max(np.abs(np.abs(W[1]) - amp2)) <= 1e-12 * amp


# ------------------------------------------------------- linear edge mode --

def _time_morlet(m, sfreq, f, sigma, kind=0):
    """sqrt(dt) psi_s(m dt), the textbook time-domain Morlet (not periodised)."""
    if kind == 0:
        kappa = math.exp(-sigma * sigma / 2)
        c = (1 + math.exp(-sigma * sigma) - 2 * math.exp(-0.75 * sigma * sigma)) ** -0.5
    else:
        kappa, c = 0.0, 1.0
    s = sigma / (2 * math.pi * f)
    dt = 1.0 / sfreq
    u = np.asarray(m, dtype=np.float64) * dt / s
    return math.sqrt(dt) * s ** -0.5 * c * math.pi ** -0.25 * np.exp(-0.5 * u * u) * (
        np.exp(1j * sigma * u) - kappa)


@pytest.mark.parametrize("kind", [0, 1])
def test_linear_mode_equals_direct_linear_convolution(orc, kind):
    """With L >= n + support, the cyclic definition equals the linear
    convolution of the zero-extended signal with the textbook wavelet: no
    wrap-around at the edges (the cyclic result at L = n differs there)."""
    rng = np.random.default_rng(11)
    N, sfreq = 300, 1000.0
    freqs = np.array([4.0, 20.0, 60.0])
    cyc = np.array([3.0, 6.0, 10.0])
    x = rng.normal(size=N)
    S = orc.linear_support(sfreq, freqs, cyc)
    L = orc.pad_length(N, "linear", support=S)
    assert L >= N + S
    W = orc.cwt(x[None, :], sfreq, freqs, cyc, kind=kind, pad="linear")[0]
    Wc = orc.cwt(x[None, :], sfreq, freqs, cyc, kind=kind, pad="none")[0]
    t = np.arange(N)
    for fi, (f, sg) in enumerate(zip(freqs, cyc)):
        ref = np.array([np.sum(x * _time_morlet(tt - t, sfreq, f, sg, kind)) for tt in t])
        assert np.max(np.abs(W[fi] - ref)) <= 1e-11 * np.max(np.abs(ref))
    # the 4 Hz wavelet is longer than the signal: the cyclic result wraps
    assert np.max(np.abs(Wc[0] - W[0])) > 0.1 * np.max(np.abs(W[0]))


# ----------------------------------------------- sampled (user) wavelets --

def test_user_wavelet_brute_force_two_ffts(orc):
    """The two-FFT form IFFT(FFT(x_pad) FFT(psi_pad)), by numpy's FFT, for
    random complex wavelets of odd and even length and every pad mode."""
    rng = np.random.default_rng(5)
    for N, w, pad in ((37, 9, "smooth7"), (50, 12, "none"), (40, 7, "linear"), (33, 33, "pow2")):
        x = rng.normal(size=(2, N))
        wv = rng.normal(size=(3, w)) + 1j * rng.normal(size=(3, w))
        W = orc.cwt_user(x, wv, pad=pad)
        L = orc.pad_length(N, pad, support=max(w // 2, w - 1 - w // 2) + 1 if pad == "linear" else None)
        psi = np.zeros((3, L), complex)
        for j in range(w):
            psi[:, (j - w // 2) % L] = wv[:, j]
        xp = np.zeros((2, L))
        xp[:, :N] = x
        ref = np.fft.ifft(np.fft.fft(xp)[:, None, :] * np.fft.fft(psi)[None, :, :])[:, :, :N]
        assert np.max(np.abs(W - ref)) <= 1e-12 * np.max(np.abs(ref)), (N, w, pad)


def test_user_wavelet_sampled_morlet_matches_closed_form(orc):
    """Sampling the textbook time-domain Morlet over +-8 scales and passing it
    as a user wavelet gives the closed-form path's result (the two routes of
    "Fourier transformed formula"), up to the truncated tails (< 1e-12)."""
    N, sfreq = 1000, 1000.0
    freqs = np.array([10.0, 40.0])
    sig = 7.0
    x = synth.tones(N, sfreq, [(10.0, 1.0), (40.0, 0.5)], noise_sd=0.5, seed=3)
    W = orc.cwt(x[None, :], sfreq, freqs, sig)[0]
    for fi, f in enumerate(freqs):
        s = sig / (2 * math.pi * f)
        half = int(math.ceil(8 * s * sfreq))
        m = np.arange(-half, half + 1)
        # the closed form's inverse DFT is the wavelet periodised onto the
        # circle of L = N samples: fold the sampled wavelet the same way and
        # pass it as an L-sample user wavelet centred at L // 2
        circ = np.zeros(N, complex)
        np.add.at(circ, m % N, _time_morlet(m, sfreq, f, sig))
        wv = circ[(np.arange(N) - N // 2) % N]
        Wu = orc.cwt_user(x[None, :], wv[None, :], L=N)[0, 0]
        assert np.max(np.abs(Wu - W[fi])) <= 1e-12 * np.max(np.abs(W[fi])), f
