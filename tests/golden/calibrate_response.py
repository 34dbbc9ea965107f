"""Normalisation of the response stand-in (calls only the oracle and the input recipe).

The paper quotes SNR = 262 for its cosmic-string background (Eq. (cs) with
G mu = 1e-13, flat spectrum) over one year at the fiducial noise levels
(A_OMS = 7.9e-12 m/sqrt(Hz), A_TM = 2.4e-15 m s^-2/sqrt(Hz)), with the SNR of
Eq. (snr).  The response stand-in is linear in its normalisation zeta, so
zeta = 262 / SNR(zeta = 1).  Run:  python tests/golden/calibrate_response.py
"""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lps_oracle as O  # noqa: E402
from synth import workloads as W  # noqa: E402


def main():
    ds = W.make_dataset("year_912085bins_4096states")
    ds.R = W.response_standin(ds.f, zeta=1.0)
    params = np.array([7.9e-12, 2.4e-15, math.log10(0.55e-11), 0.0])
    snr1 = O.snr(ds, params)
    print(f"SNR(zeta=1) = {snr1:.6f}  ->  zeta = {262.0 / snr1:.5f}")


if __name__ == "__main__":
    main()
