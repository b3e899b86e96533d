"""Separation quality in dB.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Thesis Chapter 4, equations ch4_Qpd and ch4_Qr:
Q = 10 log10(||d_original||^2 / ||d_original - d_estimate||^2); the improvement
due to the Radon inversion is Q_R - Q_PD.
"""
import numpy as np


def q_db(d_original, d_estimate):
    d_original = np.asarray(d_original, dtype=np.float64)
    d_estimate = np.asarray(d_estimate, dtype=np.float64)
    num = float(np.sum(d_original * d_original))
    den = float(np.sum((d_original - d_estimate) ** 2))
    if den == 0.0:
        return float("inf")
    return 10.0 * np.log10(num / den)
