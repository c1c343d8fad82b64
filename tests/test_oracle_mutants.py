"""Planted mistakes in the oracle (on the CPU) must each fail at least one pin.

Each mutant is the oracle's C source with one plausible mistake substituted
in (a wrong sign, a dropped factor, a transposed index, a wrong constant).  It
is compiled into a temporary library, swapped in for the real one, and the
pins of ``test_oracle_pins.py`` are run against it.  The real oracle is
restored afterwards.  This shows that the pins are sensitive to the kinds of
error they are meant to catch.
"""
import ctypes
import importlib.util
import os
import subprocess

import pytest

import oracle
from oracle import build as obuild

HERE = os.path.dirname(os.path.abspath(__file__))

_spec = importlib.util.spec_from_file_location("_pins", os.path.join(HERE, "test_oracle_pins.py"))
pins = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(pins)

PIN_CALLS = [
    (pins.test_morlet_constants_unit_energy_and_admissible, dict(sigma=3.0)),
    (pins.test_morlet_constants_unit_energy_and_admissible, dict(sigma=7.0)),
    (pins.test_gabor_constants, {}),
    (pins.test_mother_spectrum_matches_closed_form, {}),
    (pins.test_pad_smooth7_against_sieve, {}),
    (pins.test_pad_pow2_and_explicit, {}),
    (pins.test_idft_of_spectrum_is_periodised_time_wavelet,
     dict(L=1000, sfreq=1000.0, f=10.0, sigma=7.0, kind=0)),
    (pins.test_idft_of_spectrum_is_periodised_time_wavelet,
     dict(L=4096, sfreq=1000.0, f=1.0, sigma=3.0, kind=0)),
    (pins.test_unit_energy_within_riemann_bound, dict(L=4096, sfreq=1000.0, f=50.0, sigma=10.0)),
    (pins.test_nyquist_bin_is_negative_frequency, {}),
    (pins.test_direct_matches_fft_cyclic_brute_force, dict(n=37, pad="smooth7", explicit=None,
                                                           kind=0)),
    (pins.test_direct_matches_fft_cyclic_brute_force, dict(n=50, pad="explicit", explicit=63,
                                                           kind=0)),
    (pins.test_two_tone_closed_form, {}),
    (pins.test_sinusoid_peak_amplitude_and_argmax, {}),
    (pins.test_cyclic_shift_equivariance, {}),
    (pins.test_dc_null_and_gabor_dc, {}),
    (pins.test_parseval, {}),
    (pins.test_gmw_peak_is_two_at_closed_form_location, dict(beta=17.5, gamma=3.0)),
    (pins.test_gmw_moments_match_gamma_functions, dict(beta=8.0, gamma=2.0)),
    (pins.test_gmw_vanishes_at_nonpositive_frequencies, {}),
    (pins.test_gmw_tone_closed_form, dict(beta=17.5, gamma=3.0)),
    (pins.test_band_groups_on_the_edges, {}),
    (pins.test_band_power_tone_closed_form, {}),
    (pins.test_stream_band_power_tone_closed_form, {}),
]

MUTANTS = {
    "kappa_sign": ("- kappa * exp(-0.5 * u * u)", "+ kappa * exp(-0.5 * u * u)"),
    "c_constant": ("2.0 * exp(-0.75 * sigma * sigma)", "2.0 * exp(-0.5 * sigma * sigma)"),
    "nyquist_sign": ("(2 * b < L) ? b : b - L;\n        double omega = 2.0 * M_PI * sfreq * (double)bt / (double)L;\n        H[b] = pref * orc_mother_spectrum",
                     "(2 * b <= L) ? b : b - L;\n        double omega = 2.0 * M_PI * sfreq * (double)bt / (double)L;\n        H[b] = pref * orc_mother_spectrum"),
    "gmw_nyquist_sign": ("(2 * b < L) ? b : b - L;\n        double omega = 2.0 * M_PI * sfreq * (double)bt / (double)L;\n        H[b] = pref * orc_gmw_spectrum",
                         "(2 * b <= L) ? b : b - L;\n        double omega = 2.0 * M_PI * sfreq * (double)bt / (double)L;\n        H[b] = pref * orc_gmw_spectrum"),
    "dropped_2pi_prefactor": ("sigma / (2.0 * M_PI * f);\n    double pref = sqrt(2.0 * M_PI * s * sfreq);",
                              "sigma / (2.0 * M_PI * f);\n    double pref = sqrt(s * sfreq);"),
    "gmw_dropped_2pi_prefactor": (
        "orc_gmw_peak(beta, gamma) / (2.0 * M_PI * f);\n    double pref = sqrt(2.0 * M_PI * s * sfreq);",
        "orc_gmw_peak(beta, gamma) / (2.0 * M_PI * f);\n    double pref = sqrt(s * sfreq);"),
    "scale_map": ("sigma / (2.0 * M_PI * f)", "sigma / (M_PI * f)"),
    "idft_direction": ("im += H[b] * sn[m];", "im -= H[b] * sn[m];"),
    "missing_1_over_L": ("h_re[j] = re / (double)L;", "h_re[j] = re;"),
    "transposed_conv_index": ("int64_t j = t - k;", "int64_t j = k - t;"),
    "conv_drops_last_sample": ("for (int64_t k = 0; k < N; ++k) {",
                               "for (int64_t k = 0; k + 1 < N; ++k) {"),
    "smooth_primes": ("{2, 3, 5, 7}", "{2, 3, 5, 11}"),
    "gabor_kappa": ("*kappa = 0.0;\n        *c = 1.0;", "*kappa = 0.0;\n        *c = 0.5;"),
    "exponent_half": ("exp(-0.5 * a * a)", "exp(-a * a)"),
    "gmw_alpha_exponent": ("pow(M_E * gamma / beta, beta / gamma)",
                           "pow(M_E * gamma / beta, gamma / beta)"),
    "gmw_no_step": ("if (u <= 0.0) return 0.0;", "if (u < -1e300) return 0.0;"),
    "gmw_peak_location": ("pow(beta / gamma, 1.0 / gamma)", "pow(beta / gamma, gamma)"),
    "gmw_exponent_param": ("exp(-pow(u, gamma))", "exp(-pow(u, beta))"),
}


def _build_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / ("mut_%s.c" % name)
    path.write_text(src.replace(old, new))
    lib = tmp_path / ("libmut_%s.so" % name)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(lib), str(path), "-lm"], check=True)
    return str(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    lib_path = _build_mutant(name, tmp_path)
    real = oracle._load()
    oracle._lib = oracle._configure(ctypes.CDLL(lib_path))
    failed = []
    try:
        for fn, kw in PIN_CALLS:
            try:
                fn(oracle, **kw)
            except AssertionError:
                failed.append(fn.__name__)
    finally:
        oracle._lib = real
    assert failed, "mutant %s passed every pin" % name


def test_real_oracle_passes_the_same_pins():
    for fn, kw in PIN_CALLS:
        fn(oracle, **kw)


# Planted mistakes in the oracle's Python reductions (band membership, band
# mean, power, the streaming trailing-hop window and its mean).  The mutated
# module source is loaded as a sibling module sharing the real C library.
PY_MUTANTS = {
    "band_sum_not_mean": ("P[:, g, :].mean(axis=1)", "P[:, g, :].sum(axis=1)"),
    "last_band_open_at_hi": ("(freqs >= lo) & (freqs <= hi)", "(freqs >= lo) & (freqs < hi)"),
    "band_lo_exclusive": ("m = (freqs >= lo) & (freqs < hi)", "m = (freqs > lo) & (freqs < hi)"),
    "band_hi_inclusive": ("m = (freqs >= lo) & (freqs < hi)", "m = (freqs >= lo) & (freqs <= hi)"),
    "power_drops_imag": ("W.real ** 2 + W.imag ** 2", "W.real ** 2"),
    "stream_window_one_early": ("t0=Wn - hop, nt=hop", "t0=Wn - hop - 1, nt=hop"),
    "stream_window_one_late": ("t0=Wn - hop, nt=hop", "t0=Wn - hop + 1, nt=hop - 1"),
    "stream_leading_hop": ("t0=Wn - hop, nt=hop", "t0=0, nt=hop"),
    "stream_hop_sum": ("return bp.mean(axis=2)", "return bp.sum(axis=2)"),
}


def _load_py_mutant(name):
    import importlib.util as iu
    import types
    old, new = PY_MUTANTS[name]
    src = open(oracle.__file__).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle._mutant_" + name)
    mod.__package__ = "oracle"
    mod.__file__ = oracle.__file__
    exec(compile(src.replace(old, new), oracle.__file__, "exec"), mod.__dict__)
    mod._lib = oracle._load()
    return mod


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_planted_reduction_mistake_fails_a_pin(name):
    mut = _load_py_mutant(name)
    failed = []
    for fn, kw in PIN_CALLS:
        try:
            fn(mut, **kw)
        except AssertionError:
            failed.append(fn.__name__)
    assert failed, "mutant %s passed every pin" % name
