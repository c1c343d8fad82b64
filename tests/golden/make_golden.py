"""Write ``two_tone_oracle_samples.txt`` from the FP64 oracle alone.

One channel, 1000 samples at 1000 Hz,
sin 10 Hz + 0.5 sin 40 Hz + N(0, 0.5^2) (seed 1), Morlet sigma = 7, 50 linear
frequencies 1-50 Hz, 2,3,5,7-smooth padding (L = 1000).  The file stores W at
a fixed set of (f, t) samples with 17 significant digits; the test-suite checks
the oracle still reproduces them (a regression guard on the oracle itself).
Run:  python tests/golden/make_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

SAMPLES_F = [0, 4, 9, 19, 29, 39, 49]
SAMPLES_T = [0, 1, 137, 499, 500, 862, 998, 999]


def main():
    x = synth.two_tone_signal()
    freqs = np.arange(1.0, 51.0)
    W = oracle.cwt(x, 1000.0, freqs, 7.0)[0]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "two_tone_oracle_samples.txt")
    with open(path, "w") as fh:
        fh.write("# Oracle W[f_index, t] for the two-tone signal (written by make_golden.py; FP64)\n")
        fh.write("# f_index t re im\n")
        for fi in SAMPLES_F:
            for t in SAMPLES_T:
                fh.write("%d %d %.17e %.17e\n" % (fi, t, W[fi, t].real, W[fi, t].imag))
    print(path)


if __name__ == "__main__":
    main()
