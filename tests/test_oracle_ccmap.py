"""Pins of the oracle's correlation map, eq. (15) at every shift (Sec. 5).

The map is a plain definition (a sum over the overlap of the two
mean-subtracted images), so each pin ties it to something other than the
oracle's own loop: a hand-worked 2 x 2 example, scipy's 2-D correlation of
the mean-subtracted images, and the properties Sec. 5 states (a shifted copy
peaks at its shift, C(f, a f) = a, the complement gives -1).  No GPU.
"""
import json
import os

import numpy as np
import pytest
import scipy.signal as ss

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _smooth_image(rng, H, W, C=3):
    """A non-periodic image with structure on several scales (a smoothed
    random field), float32 in [0, 1]."""
    a = rng.random((H + 8, W + 8, C))
    k = np.ones(5) / 5.0
    for ax in (0, 1):
        a = np.apply_along_axis(lambda v: np.convolve(v, k, mode="same"), ax, a)
    a = a[4:4 + H, 4:4 + W]
    a = (a - a.min()) / (a.max() - a.min())
    return a.astype(np.float32)


def test_hand_worked_2x2():
    with open(os.path.join(GOLDEN, "cc_map_2x2.json")) as fh:
        gold = json.load(fh)
    f = np.array(gold["f"], dtype=np.float32)
    g = np.array(gold["g"], dtype=np.float32)
    m, pk, dx, dy = O.cross_correlate_map(f, g, 1, 1)
    assert np.max(np.abs(m - np.array(gold["map"]))) <= 1e-15
    assert abs(pk - gold["peak"]) <= 1e-15
    assert (dx, dy) == (gold["peak_dx"], gold["peak_dy"])


@pytest.mark.parametrize("H,W,C,rx,ry", [(23, 31, 3, 5, 7), (16, 9, 1, 8, 0), (12, 12, 3, 11, 11)])
def test_map_matches_scipy_correlate2d(H, W, C, rx, ry):
    # the numerator of eq. (15) at shift (dx, dy) is scipy's full 2-D
    # correlation of g' with f' at index (H - 1 + dy, W - 1 + dx), summed
    # over channels; the denominator is sum f'^2
    rng = np.random.default_rng(H * 100 + W)
    f = rng.random((H, W, C)).astype(np.float32)
    g = rng.random((H, W, C)).astype(np.float32)
    fd, gd = f.astype(np.float64), g.astype(np.float64)
    fp = fd - fd.reshape(-1, C).mean(axis=0)
    gp = gd - gd.reshape(-1, C).mean(axis=0)
    num = sum(ss.correlate2d(gp[:, :, c], fp[:, :, c], mode="full") for c in range(C))
    want = num[H - 1 - ry:H + ry, W - 1 - rx:W + rx] / (fp * fp).sum()
    m, pk, dx, dy = O.cross_correlate_map(f, g, rx, ry)
    assert m.shape == (2 * ry + 1, 2 * rx + 1)
    assert np.max(np.abs(m - want)) <= 1e-13
    iy, ix = np.unravel_index(np.argmax(want), want.shape)
    assert (dx, dy) == (ix - rx, iy - ry)
    assert pk == m.max()


def test_column_window_matches_cropped_copy():
    # a window passed with the full row pitch equals the cropped image
    rng = np.random.default_rng(3)
    f = rng.random((20, 30, 3)).astype(np.float32)
    g = rng.random((20, 30, 3)).astype(np.float32)
    a = O.cross_correlate_map(f, g, 3, 2, cols=(7, 19))
    b = O.cross_correlate_map(np.ascontiguousarray(f[:, 7:19]), np.ascontiguousarray(g[:, 7:19]), 3, 2)
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]


@pytest.mark.parametrize("sx,sy", [(3, 0), (-2, 4), (5, -3)])
def test_shifted_copy_peaks_at_its_shift(sx, sy):
    # Sec. 5: an image identical to f but shifted within the frame gives the
    # maximum at that shift, below 100% for a finite photograph
    rng = np.random.default_rng(11)
    big = _smooth_image(rng, 80, 90)
    f = big[10:70, 10:80]
    g = big[10 - sy:70 - sy, 10 - sx:80 - sx]      # g(x + sx, y + sy) = f(x, y)
    m, pk, dx, dy = O.cross_correlate_map(f, g, 6, 6)
    assert (dx, dy) == (sx, sy)
    assert m[6, 6] < pk < 1.0
    assert pk > 0.8


def test_autocorrelation_scaling_and_complement():
    # C(f, f) peaks at (0, 0) with 100%; C(f, a f) = a C(f, f) at every shift;
    # the complement M - f gives -C(f, f) (Sec. 5)
    rng = np.random.default_rng(5)
    f = _smooth_image(rng, 40, 50)
    m1, pk, dx, dy = O.cross_correlate_map(f, f, 4, 4)
    assert (dx, dy) == (0, 0) and abs(pk - 1.0) <= 1e-15
    a = np.float32(0.25)            # a power of two: a f is exact in float32
    ma, _, _, _ = O.cross_correlate_map(f, a * f, 4, 4)
    assert np.max(np.abs(ma - 0.25 * m1)) <= 1e-15
    mc, _, _, _ = O.cross_correlate_map(f, np.float32(1.0) - f, 4, 4)
    assert np.max(np.abs(mc + m1)) <= 1e-7      # 1 - f rounds in float32


def test_zero_shift_equals_zero_shift_coefficient():
    rng = np.random.default_rng(9)
    f = rng.random((17, 21, 3)).astype(np.float32)
    g = rng.random((17, 21, 3)).astype(np.float32)
    m, _, _, _ = O.cross_correlate_map(f, g, 0, 0)
    c0, _ = O.cross_correlate(f, g)
    assert abs(m[0, 0] - c0) <= 1e-15
