"""FP64 CPU oracle of the FFT-based Morlet CWT (Nakanishi, arXiv 2506.07793).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the GPU library and never imports it.

The heavy loops live in ``cwt_oracle.c`` (direct IDFT and direct cyclic
convolution, no FFT anywhere); this module marshals numpy arrays and adds the
plain reductions (power, band mean, trailing-hop mean).

Paper sections followed:
  * "Fourier transformed formula": W = IDFT(DFT(x_pad) * Psi_hat(omega)), which
    by the cyclic convolution theorem is the cyclic convolution of the padded
    signal with the inverse DFT of the sampled wavelet spectrum.  Computed here
    directly as that convolution.
  * Morlet / Gabor Fourier-domain equations (same section) for Psi_hat; the
    constants c and kappa, which the paper leaves implicit, are the unit-energy
    and zero-mean closed forms (see ``cwt_oracle.c``).
  * The generalized Morse wavelet equation (same section), read with the unit
    step for sign(omega) and alpha = 2 (e gamma / beta)^(beta / gamma).
  * "Fast Fourier transform": pad to the smallest 2*3*5*7-smooth length >= N.
  * "Precision": power |W|^2 and the real/imag/phase comparison metric.
  * Introduction: the EEG bands delta/theta/alpha/beta/gamma (edges are a
    stated reading, see ``DEFAULT_BANDS``).

Parity pins: every function here is checked in ``tests/test_oracle_pins.py``
against closed forms, quadrature, brute force and invariants.  The band
membership, band mean and streaming trailing-hop mean are pinned against the
closed form of exact-bin tones (whose beats make the power change within a
hop) with a hand-written band membership that puts a grid frequency on every
band edge; ``tests/test_oracle_mutants.py`` plants mistakes in them too.

``parity_errors`` compares in absolute terms when the reference is all zero
(for instance a Morlet transform of a one-sample signal: the wavelet spectrum
vanishes at zero frequency, so the whole transform is zero).
"""
import ctypes
import os

import numpy as np

from . import build as _build

MORLET = 0
GABOR = 1
GMW = 2

#: Generalized Morse wavelet parameters the paper uses (section "Precision").
GMW_BETA = 17.5
GMW_GAMMA = 3.0

#: EEG bands named in the paper's introduction; the edges (Hz) are a reading:
#: lo <= f < hi, except that the last band also includes f == hi.
DEFAULT_BANDS = ((1.0, 4.0), (4.0, 8.0), (8.0, 13.0), (13.0, 30.0), (30.0, 100.0))

_lib = None


def _configure(lib):
    """Declare the C signatures on a loaded copy of the oracle library."""
    i64, dbl, p_d, p_i64 = ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_double), \
        ctypes.POINTER(ctypes.c_int64)
    lib.orc_pad_smooth7.restype = i64
    lib.orc_pad_smooth7.argtypes = [i64]
    lib.orc_pad_pow2.restype = i64
    lib.orc_pad_pow2.argtypes = [i64]
    lib.orc_wavelet_constants.restype = None
    lib.orc_wavelet_constants.argtypes = [ctypes.c_int, dbl, p_d, p_d]
    lib.orc_mother_spectrum.restype = dbl
    lib.orc_mother_spectrum.argtypes = [ctypes.c_int, dbl, dbl]
    lib.orc_wavelet_spectrum.restype = None
    lib.orc_wavelet_spectrum.argtypes = [i64, dbl, dbl, dbl, ctypes.c_int, p_d]
    lib.orc_gmw_peak.restype = dbl
    lib.orc_gmw_peak.argtypes = [dbl, dbl]
    lib.orc_gmw_spectrum.restype = dbl
    lib.orc_gmw_spectrum.argtypes = [dbl, dbl, dbl]
    lib.orc_gmw_wavelet_spectrum.restype = None
    lib.orc_gmw_wavelet_spectrum.argtypes = [i64, dbl, dbl, dbl, dbl, p_d]
    lib.orc_idft_real_spectrum.restype = None
    lib.orc_idft_real_spectrum.argtypes = [i64, p_d, p_d, p_d]
    lib.orc_cwt_rows.restype = None
    lib.orc_cwt_rows.argtypes = [p_d, i64, i64, i64, p_d, p_d, i64, p_i64, p_i64, i64, i64,
                                 i64, p_d, p_d]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    _lib = _configure(ctypes.CDLL(_build.LIB))
    return _lib


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _kind(kind):
    if kind in (MORLET, "morlet"):
        return MORLET
    if kind in (GABOR, "gabor"):
        return GABOR
    if kind in (GMW, "gmw"):
        return GMW
    raise ValueError("unknown wavelet kind %r" % (kind,))


def num_threads():
    """Threads the oracle's OpenMP loops use."""
    return int(_load().orc_num_threads())


def linear_support(sfreq, freqs, n_cycles):
    """One-sided time support, in samples, of the widest Morlet / Gabor
    wavelet of a grid: its Gaussian envelope exp(-u^2/2), u = t / s, is below
    1e-12 of the peak for u > sqrt(2 ln 1e12); s = sigma / (2 pi f)."""
    freqs = np.asarray(freqs, dtype=np.float64)
    s = sigmas_for(freqs, n_cycles) / (2 * np.pi * freqs)
    return int(np.ceil(np.sqrt(2 * np.log(1e12)) * s.max() * sfreq)) + 1


def pad_length(n, mode="smooth7", explicit=None, support=None):
    """Padded FFT length for a signal of n samples ("Fast Fourier transform");
    "linear": the smooth length >= n + support (no cyclic wrap reaches the
    output; ``support`` from linear_support)."""
    lib = _load()
    if mode == "linear":
        if support is None:
            raise ValueError("linear padding needs the wavelet support")
        return int(lib.orc_pad_smooth7(int(n) + int(support)))
    if mode == "smooth7":
        return int(lib.orc_pad_smooth7(int(n)))
    if mode == "pow2":
        return int(lib.orc_pad_pow2(int(n)))
    if mode == "none":
        return int(n)
    if mode == "explicit":
        if explicit is None or explicit < n:
            raise ValueError("explicit length must be >= n")
        return int(explicit)
    raise ValueError("unknown pad mode %r" % (mode,))


def wavelet_constants(sigma, kind=MORLET):
    """(c_sigma, kappa_sigma) of the Morlet (or Gabor) Fourier-domain formula."""
    c = ctypes.c_double()
    k = ctypes.c_double()
    _load().orc_wavelet_constants(_kind(kind), float(sigma), ctypes.byref(c), ctypes.byref(k))
    return c.value, k.value


def mother_spectrum(sigma, u, kind=MORLET):
    """Psi_hat_sigma(u) of the mother wavelet (Morlet / Gabor equations)."""
    lib = _load()
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    return np.array([lib.orc_mother_spectrum(_kind(kind), float(sigma), float(v)) for v in u])


def gmw_peak(beta=GMW_BETA, gamma=GMW_GAMMA):
    """u_p = (beta / gamma)^(1 / gamma), where the GMW spectrum peaks."""
    return float(_load().orc_gmw_peak(float(beta), float(gamma)))


def gmw_spectrum(u, beta=GMW_BETA, gamma=GMW_GAMMA):
    """Generalized Morse wavelet in the Fourier domain (GMW equation of
    "Fourier transformed formula", read with the unit step and the peak-2
    normalisation alpha = 2 (e gamma / beta)^(beta / gamma))."""
    lib = _load()
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    return np.array([lib.orc_gmw_spectrum(float(beta), float(gamma), float(v)) for v in u])


def sigmas_for(freqs, n_cycles):
    """n_cycles is one number (the paper's sigma) or one value per frequency."""
    freqs = np.asarray(freqs, dtype=np.float64)
    s = np.asarray(n_cycles, dtype=np.float64)
    if s.ndim == 0:
        s = np.full(freqs.shape, float(s))
    if s.shape != freqs.shape:
        raise ValueError("n_cycles must be a scalar or one value per frequency")
    return s


def wavelet_spectrum(L, sfreq, f, sigma, kind=MORLET, beta=GMW_BETA, gamma=GMW_GAMMA):
    """H_f[b], b in [0, L): the scaled Fourier-domain wavelet on the DFT bins
    (sigma for Morlet / Gabor; beta and gamma for the GMW)."""
    H = np.empty(int(L), dtype=np.float64)
    if _kind(kind) == GMW:
        _load().orc_gmw_wavelet_spectrum(int(L), float(sfreq), float(f), float(beta),
                                         float(gamma), _ptr(H))
    else:
        _load().orc_wavelet_spectrum(int(L), float(sfreq), float(f), float(sigma), _kind(kind),
                                     _ptr(H))
    return H


def wavelet_bank(L, sfreq, freqs, n_cycles, kind=MORLET, beta=GMW_BETA, gamma=GMW_GAMMA):
    """[F, L] spectra for every analysis frequency."""
    freqs = np.asarray(freqs, dtype=np.float64)
    sig = sigmas_for(freqs, n_cycles if _kind(kind) != GMW else 0.0)
    return np.stack([wavelet_spectrum(L, sfreq, f, s, kind, beta, gamma)
                     for f, s in zip(freqs, sig)])


def wavelet_time(H):
    """h = IDFT(H) by the direct O(L^2) sum (complex128)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    L = H.shape[0]
    re = np.empty(L)
    im = np.empty(L)
    _load().orc_idft_real_spectrum(L, _ptr(H), _ptr(re), _ptr(im))
    return re + 1j * im


def cwt(x, sfreq, freqs, n_cycles, kind=MORLET, pad="smooth7", L=None, rows=None, t0=0,
        nt=None, beta=GMW_BETA, gamma=GMW_GAMMA):
    """Direct cyclic-convolution CWT in FP64.

    x: [C, N] (or [N]) real signal.  Returns complex128 [C, F, nt] with
    nt = N - t0 by default, or [len(rows), nt] when ``rows`` lists (c, f)
    index pairs.  ``L`` overrides the padded length (explicit padding).
    For the GMW (kind "gmw") n_cycles is not used; beta and gamma are.
    """
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[None, :]
    x = np.ascontiguousarray(x)
    C, N = x.shape
    freqs = np.asarray(freqs, dtype=np.float64)
    F = freqs.shape[0]
    if L is None:
        sup = linear_support(sfreq, freqs, n_cycles) if pad == "linear" else None
        L = pad_length(N, pad, support=sup)
    if L < N:
        raise ValueError("padded length shorter than the signal")
    if nt is None:
        nt = N - t0
    if not (0 <= t0 and t0 + nt <= N):
        raise ValueError("output window outside [0, N)")
    sig = sigmas_for(freqs, n_cycles if _kind(kind) != GMW else 0.0)
    if rows is None:
        rc, rf = np.meshgrid(np.arange(C), np.arange(F), indexing="ij")
        rc, rf = rc.ravel(), rf.ravel()
    else:
        rows = np.asarray(rows, dtype=np.int64).reshape(-1, 2)
        rc, rf = rows[:, 0], rows[:, 1]
    used = np.unique(rf)
    h_re = np.zeros((F, L))
    h_im = np.zeros((F, L))
    for f in used:
        h = wavelet_time(wavelet_spectrum(L, sfreq, freqs[f], sig[f], kind, beta, gamma))
        h_re[f], h_im[f] = h.real, h.imag
    rc = np.ascontiguousarray(rc, dtype=np.int64)
    rf = np.ascontiguousarray(rf, dtype=np.int64)
    n_rows = rc.shape[0]
    w_re = np.empty((n_rows, nt))
    w_im = np.empty((n_rows, nt))
    _load().orc_cwt_rows(_ptr(x), C, N, L, _ptr(h_re), _ptr(h_im), F,
                         _ptr(rc, ctypes.c_int64), _ptr(rf, ctypes.c_int64), n_rows, t0, nt,
                         _ptr(w_re), _ptr(w_im))
    W = w_re + 1j * w_im
    if rows is None:
        return W.reshape(C, F, nt)
    return W


def user_wavelet_time(wavelets, L):
    """Place sampled time-domain wavelets on a length-L circle: sample j of a
    wavelet of w samples sits at time (j - w // 2) / sfreq, i.e. at index
    (j - w // 2) mod L.  [F, w] complex -> [F, L] complex128."""
    wv = np.atleast_2d(np.asarray(wavelets, dtype=np.complex128))
    F, w = wv.shape
    if w > L:
        raise ValueError("wavelet longer than the padded length")
    h = np.zeros((F, L), dtype=np.complex128)
    idx = (np.arange(w) - w // 2) % L
    h[:, idx] = wv
    return h


def cwt_user(x, wavelets, pad="smooth7", L=None, rows=None, t0=0, nt=None):
    """CWT with sampled time-domain wavelets (the two-FFT form of "Fourier
    transformed formula": IFFT(FFT(x_pad) FFT(psi_pad)), i.e. the cyclic
    convolution of the padded signal with each placed wavelet), computed
    directly as that cyclic convolution.  "linear" padding uses the longest
    one-sided extent of the wavelets as the support."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[None, :]
    x = np.ascontiguousarray(x)
    C, N = x.shape
    wv = np.atleast_2d(np.asarray(wavelets, dtype=np.complex128))
    F, w = wv.shape
    if L is None:
        sup = max(w // 2, w - 1 - w // 2) + 1 if pad == "linear" else None
        L = pad_length(N, pad, support=sup)
    if nt is None:
        nt = N - t0
    h = user_wavelet_time(wv, L)
    h_re = np.ascontiguousarray(h.real)
    h_im = np.ascontiguousarray(h.imag)
    if rows is None:
        rc, rf = np.meshgrid(np.arange(C), np.arange(F), indexing="ij")
        rc, rf = rc.ravel(), rf.ravel()
    else:
        rows = np.asarray(rows, dtype=np.int64).reshape(-1, 2)
        rc, rf = rows[:, 0], rows[:, 1]
    rc = np.ascontiguousarray(rc, dtype=np.int64)
    rf = np.ascontiguousarray(rf, dtype=np.int64)
    n_rows = rc.shape[0]
    w_re = np.empty((n_rows, nt))
    w_im = np.empty((n_rows, nt))
    _load().orc_cwt_rows(_ptr(x), C, N, L, _ptr(h_re), _ptr(h_im), F,
                         _ptr(rc, ctypes.c_int64), _ptr(rf, ctypes.c_int64), n_rows, t0, nt,
                         _ptr(w_re), _ptr(w_im))
    W = w_re + 1j * w_im
    if rows is None:
        return W.reshape(C, F, nt)
    return W


def power(W):
    """|W|^2 (section "Precision" compares power values)."""
    return W.real ** 2 + W.imag ** 2


def band_groups(freqs, bands=DEFAULT_BANDS):
    """Frequency indices of each band: lo <= f < hi, the last band closed at hi."""
    freqs = np.asarray(freqs, dtype=np.float64)
    out = []
    for i, (lo, hi) in enumerate(bands):
        if i == len(bands) - 1:
            m = (freqs >= lo) & (freqs <= hi)
        else:
            m = (freqs >= lo) & (freqs < hi)
        out.append(np.nonzero(m)[0])
    return out


def band_power(P, groups):
    """Arithmetic mean of power over each band's frequencies: [C, F, T] -> [C, B, T]."""
    return np.stack([P[:, g, :].mean(axis=1) for g in groups], axis=1)


def stream_band_power(window, sfreq, freqs, n_cycles, hop, bands=DEFAULT_BANDS, kind=MORLET,
                      pad="smooth7"):
    """Band power of one sliding window, averaged over its last ``hop`` samples.

    window: [C, W] samples in time order (oldest first).  Returns [C, B].
    """
    window = np.asarray(window, dtype=np.float64)
    C, Wn = window.shape
    W = cwt(window, sfreq, freqs, n_cycles, kind=kind, pad=pad, t0=Wn - hop, nt=hop)
    bp = band_power(power(W), band_groups(freqs, bands))
    return bp.mean(axis=2)


def parity_errors(W_test, W_ref):
    """e_P = max|P_t - P_r| / max P_r and e_W = max|W_t - W_r| / max|W_r| (FP64)."""
    W_test = np.asarray(W_test).astype(np.complex128)
    P_t, P_r = power(W_test), power(W_ref)
    # An all-zero reference (e.g. a Morlet transform of a constant) is
    # compared in absolute terms.
    dP = float(np.max(np.abs(P_t - P_r)))
    dW = float(np.max(np.abs(W_test - W_ref)))
    e_P = dP / float(np.max(P_r)) if np.max(P_r) > 0 else dP
    e_W = dW / float(np.max(np.abs(W_ref))) if np.max(np.abs(W_ref)) > 0 else dW
    return e_P, e_W
