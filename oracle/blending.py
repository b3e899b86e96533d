"""FP64 oracle of numerical blending and pseudo-deblending (thesis Chapter
2, equations ch2_blending and pseudodeblending_equ; Chapter 4's synthetic
acquisition: one source vessel, dithered firing times, continuous records).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The unblended cube D[s][r][t] (source, receiver, time; nt samples per shot)
is recorded continuously: each receiver's record is
    b[r][tau] = sum_s D[s][r][tau - T_s]    (0 <= tau - T_s < nt)
with firing times T_s in samples (Gamma).  Pseudo-deblending is the adjoint:
    D~[s][r][t] = b[r][T_s + t]              (Gamma')
which leaves the other sources' energy in every shot window; sorted to
common receiver gathers it appears at random times (the dithering), which is
what the robust Radon inversion separates.
"""
import numpy as np


def record_length(fire, nt):
    return int(np.max(fire)) + nt


def blend(D, fire, nrec=None):
    D = np.asarray(D, np.float64)
    ns, nr, nt = D.shape
    nrec = nrec or record_length(fire, nt)
    b = np.zeros((nr, nrec))
    for s in range(ns):
        T = int(fire[s])
        n = max(0, min(nt, nrec - T))
        b[:, T:T + n] += D[s, :, :n]
    return b


def deblend(b, fire, nt):
    """[s][r][t] pseudo-deblended cube."""
    b = np.asarray(b, np.float64)
    nr, nrec = b.shape
    out = np.zeros((len(fire), nr, nt))
    for s, T in enumerate(fire):
        T = int(T)
        n = max(0, min(nt, nrec - T))
        out[s, :, :n] = b[:, T:T + n]
    return out
