"""Seeded synthetic EEG inputs for tests and benchmarks.

This module holds only input generation: signals, analysis-frequency grids,
recording batches and session schedules.  It contains none of the CWT's
arithmetic, and both the oracle-side tests and the GPU path take their inputs
from here.  The paper measures on generated "random" and "EEG" data rather than
a public dataset, so synthetic inputs with EEG-like structure stand in for it:

* pink (1/f power) background noise at 20 uV rms,
* 10 Hz alpha bursts with Gaussian envelopes at Poisson onsets,
* pure tones for closed-form checks.
"""
import numpy as np

EEG_RMS_UV = 20.0


def tones(n, sfreq, comps, noise_sd=0.0, seed=None):
    """sum_k A_k sin(2 pi f_k t) + N(0, noise_sd^2); comps = [(f_k, A_k), ...]."""
    t = np.arange(n) / float(sfreq)
    x = np.zeros(n)
    for f, a in comps:
        x += a * np.sin(2.0 * np.pi * f * t)
    if noise_sd > 0:
        rng = np.random.default_rng(seed)
        x += rng.normal(0.0, noise_sd, size=n)
    return x


def two_tone_signal(seed=1):
    """1 channel, 1000 samples at 1000 Hz: sin 10 Hz + 0.5 sin 40 Hz + N(0, 0.5^2)."""
    return tones(1000, 1000.0, [(10.0, 1.0), (40.0, 0.5)], noise_sd=0.5, seed=seed)[None, :]


def pink_noise(rng, C, N, rms=EEG_RMS_UV):
    """Per channel: |G(f)| ~ f^-1/2 with uniform random phase, G[0] = 0, scaled to rms."""
    nb = N // 2 + 1
    k = np.arange(nb, dtype=np.float64)
    mag = np.zeros(nb)
    mag[1:] = k[1:] ** -0.5
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(C, nb))
    G = mag[None, :] * np.exp(1j * ph)
    x = np.fft.irfft(G, n=N, axis=1)
    sd = np.sqrt(np.mean(x * x, axis=1, keepdims=True))
    sd[sd == 0] = 1.0
    return x / sd * rms


def alpha_bursts(rng, C, N, sfreq, rate_hz=1.0, env_sd_s=0.15, peak=EEG_RMS_UV, f=10.0):
    """10 Hz bursts: Poisson onsets at rate_hz, Gaussian envelope, random phase.
    Each burst is evaluated within 8 envelope widths of its centre (beyond,
    its envelope is below exp(-32) of the peak)."""
    t = np.arange(N) / float(sfreq)
    dur = N / float(sfreq)
    half = int(np.ceil(8.0 * env_sd_s * sfreq))
    out = np.zeros((C, N))
    for c in range(C):
        n_b = rng.poisson(rate_hz * dur)
        for _ in range(n_b):
            t0 = rng.uniform(0.0, dur)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            i = int(t0 * sfreq)
            a, b = max(0, i - half), min(N, i + half + 1)
            tt = t[a:b] - t0
            out[c, a:b] += peak * np.exp(-0.5 * (tt / env_sd_s) ** 2) * np.cos(
                2.0 * np.pi * f * tt + ph)
    return out


def eeg(C, N, sfreq, seed):
    """[C, N] float32 synthetic EEG in microvolts (pink noise + alpha bursts)."""
    rng = np.random.default_rng(seed)
    x = pink_noise(rng, C, N) + alpha_bursts(rng, C, N, sfreq)
    return x.astype(np.float32)


def log_freqs(lo, hi, n):
    return np.logspace(np.log10(lo), np.log10(hi), n)


def eeg_cycles(freqs):
    """n_cycles = clip(f / 2, 3, 10) per analysis frequency."""
    return np.clip(np.asarray(freqs, dtype=np.float64) / 2.0, 3.0, 10.0)


def eeg_64ch(seed=2, C=64, N=4096, F=100):
    """64 ch x 4096 samples at 1000 Hz; 100 log-spaced freqs 1-100 Hz (seed 2)."""
    sfreq = 1000.0
    freqs = log_freqs(1.0, 100.0, F)
    return dict(x=eeg(C, N, sfreq, seed), sfreq=sfreq, freqs=freqs, n_cycles=eeg_cycles(freqs))


def batch_recordings(n=256, seed=4, n_lo=500, n_hi=20000, c_hi=128):
    """Heterogeneous recordings: uniform length, channel count, grid size and rate.

    Returns a list of dicts with N, C, sfreq, freqs, n_cycles and a per-recording
    signal seed.  Grids are log-spaced from 0.5 Hz to min(200, 0.45 sfreq).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.integers(n_lo, n_hi + 1))
        C = int(rng.integers(1, c_hi + 1))
        F = int(rng.integers(20, 151))
        sfreq = float(rng.choice([250.0, 500.0, 1000.0, 2048.0]))
        freqs = log_freqs(0.5, min(200.0, 0.45 * sfreq), F)
        out.append(dict(N=N, C=C, F=F, sfreq=sfreq, freqs=freqs, n_cycles=eeg_cycles(freqs),
                        seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


def session_schedule(n_mean, duration_s, mean_life_s=20.0, hop_s=0.05, seed=5):
    """Poisson session arrivals keeping about n_mean sessions alive.

    Arrival rate n_mean / mean_life_s; lifetimes exponential with mean
    mean_life_s; n_mean sessions are already open at t = 0.  Each session gets a
    random hop phase in [0, hop_s).  Returns a list of (t_open, t_close, phase).
    """
    rng = np.random.default_rng(seed)
    sess = []
    for _ in range(n_mean):
        sess.append((0.0, float(rng.exponential(mean_life_s)), float(rng.uniform(0, hop_s))))
    t = 0.0
    lam = n_mean / mean_life_s
    while True:
        t += float(rng.exponential(1.0 / lam))
        if t >= duration_s:
            break
        sess.append((t, t + float(rng.exponential(mean_life_s)), float(rng.uniform(0, hop_s))))
    return sess
