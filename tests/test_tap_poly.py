"""The Stolt map's interpolation weights on the GPU (half-width R = 4) are
polynomials in delta = u - floor(u) (paper_1711_10214_amd/csrc/tap_poly.h,
written by gen_tap_poly.py).  Checked here against the Hann-windowed sinc
h(x) = sinc(x) (1/2 + 1/2 cos(pi x / R)) of the map's reading of the
interpolation kernel, evaluated in FP32 in the kernels' order (even and odd
parts in z^2, taps t and 1 - t from E +- z O)."""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1711_10214_amd", "csrc",
                   "tap_poly.h")
R = 4


def _read():
    txt = open(HDR).read()
    scale = float(re.search(r"kTapZScale = ([-0-9.e]+)f", txt).group(1))

    def table(name):
        body = re.search(name + r"\[4\]\[5\] = \{(.*?)\};", txt, re.S).group(1)
        rows = re.findall(r"\{([^}]*)\}", body)
        return np.array([[float(v.strip().rstrip("f")) for v in r.split(",")] for r in rows], np.float32)

    return np.float32(scale), table("kTapEven"), table("kTapOdd")


def _weights(delta):
    scale, E, O = _read()
    f = np.float32
    d = np.asarray(delta, f)
    z = (f(2) * scale) * d - scale
    w = z * z
    out = {}
    for q in range(4):
        e = E[q, 4] * w + E[q, 3]
        for k in (2, 1, 0):
            e = e * w + E[q, k]
        o = O[q, 4] * w + O[q, 3]
        for k in (2, 1, 0):
            o = o * w + O[q, k]
        out[q + 1] = z * o + e
        out[-q] = -z * o + e
    return np.array([out[t] for t in range(-R + 1, R + 1)], np.float64)


def _hann_sinc(x):
    return np.where(np.abs(x) < R, np.sinc(x) * (0.5 + 0.5 * np.cos(np.pi * x / R)), 0.0)


def test_polynomial_weights_match_the_windowed_sinc():
    d = np.linspace(-2e-3, 1 + 2e-3, 100001)
    got = _weights(d)
    want = np.array([_hann_sinc(d - t) for t in range(-R + 1, R + 1)])
    assert np.max(np.abs(got - want)) < 2e-7


def test_weights_at_integer_coordinates_and_partition():
    # u on a model bin: the tap at that bin has weight 1, the others ~0
    w0 = _weights([0.0])[:, 0]
    np.testing.assert_allclose(w0, [0, 0, 0, 1, 0, 0, 0, 0], atol=2e-7)
    # the windowed sinc's weights sum to ~1 at half-integer positions too
    wh = _weights([0.5])[:, 0]
    assert abs(wh.sum() - _hann_sinc(0.5 - np.arange(-R + 1, R + 1)).sum()) < 1e-6
