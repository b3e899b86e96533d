"""Pins of the blending oracle (oracle/blending.py): the pseudo-deblending
is the adjoint of blending (dot-product test), a hand-worked two-shot
example, and deblending recovers a shot exactly where it does not overlap
its neighbours."""
import numpy as np

from oracle import blending as B
from synth import make_survey


def test_hand_example():
    D = np.zeros((2, 1, 4))
    D[0, 0] = [1, 2, 3, 4]
    D[1, 0] = [10, 20, 30, 40]
    b = B.blend(D, np.array([0, 2]))
    assert b.tolist() == [[1, 2, 13, 24, 30, 40]]
    Dt = B.deblend(b, np.array([0, 2]), 4)
    assert Dt[0, 0].tolist() == [1, 2, 13, 24] and Dt[1, 0].tolist() == [13, 24, 30, 40]


def test_deblend_is_adjoint_of_blend():
    rng = np.random.default_rng(1)
    D = rng.standard_normal((7, 3, 50))
    fire = np.sort(rng.integers(0, 120, 7))
    b = rng.standard_normal((3, B.record_length(fire, 50)))
    lhs = np.sum(B.blend(D, fire) * b)
    rhs = np.sum(D * B.deblend(b, fire, 50))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_isolated_shot_is_recovered():
    sv = make_survey(ns=6, nt=64, compression=0.0, dither_s=0.0)   # no overlap: shots back to back
    b = B.blend(sv.D, sv.fire)
    assert np.allclose(B.deblend(b, sv.fire, 64), sv.D, atol=0, rtol=0)
