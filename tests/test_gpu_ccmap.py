"""GPU parity of the correlation map (eq. (15) at every shift, Sec. 5)
against the oracle: every map entry within 1e-10, the peak value within
1e-10, and the peak's location holding the oracle's maximum to 1e-10 (where
two shifts tie to rounding either is correct).  Inputs are seeded synthetic
images.  Run on an MI355X (gfx950) only."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1012_5107_amd import binding
    return binding


def _smooth(rng, H, W, C=3):
    a = rng.random((H + 8, W + 8, C))
    k = np.ones(5) / 5.0
    for ax in (0, 1):
        a = np.apply_along_axis(lambda v: np.convolve(v, k, mode="same"), ax, a)
    a = a[4:4 + H, 4:4 + W]
    return ((a - a.min()) / (a.max() - a.min())).astype(np.float32)


def _compare(B, f, g, rx, ry, cols=None, name=""):
    print(f"[ccmap {name}] shape={f.shape} rx={rx} ry={ry} cols={cols}", flush=True)
    m_o, pk_o, dx_o, dy_o = O.cross_correlate_map(f, g, rx, ry, cols=cols)
    dev = torch.device("cuda", 0)
    m_g, pk_g, dx_g, dy_g = B.cross_correlate_map(torch.from_numpy(g).to(dev), torch.from_numpy(f).to(dev), rx, ry,
                                                  cols=cols)
    m_g = m_g.cpu().numpy()
    err = np.max(np.abs(m_g - m_o))
    print(f"[ccmap {name}] max|map err|={err:.2e} peak gpu={pk_g:.12f} ({dx_g},{dy_g}) "
          f"oracle={pk_o:.12f} ({dx_o},{dy_o})", flush=True)
    assert m_g.shape == m_o.shape
    assert err <= TOL
    assert abs(pk_g - pk_o) <= TOL
    assert m_o[dy_g + ry, dx_g + rx] >= pk_o - TOL
    return m_g, (pk_g, dx_g, dy_g)


@pytest.mark.parametrize("H,W,C,rx,ry", [(48, 64, 3, 8, 6), (37, 53, 1, 5, 9), (96, 80, 3, 40, 3)])
def test_map_matches_oracle_random(B, H, W, C, rx, ry):
    rng = np.random.default_rng(H * 1000 + W)
    f = rng.random((H, W, C)).astype(np.float32)
    g = (0.5 * f + 0.5 * rng.random((H, W, C))).astype(np.float32)
    _compare(B, f, g, rx, ry, name="random")


@pytest.mark.parametrize("sx,sy", [(4, 0), (-3, 5)])
def test_shifted_image_peaks_at_its_shift(B, sx, sy):
    rng = np.random.default_rng(21)
    big = _smooth(rng, 140, 150)
    f = np.ascontiguousarray(big[10:130, 10:140])
    g = np.ascontiguousarray(big[10 - sy:130 - sy, 10 - sx:140 - sx])
    _, (pk, dx, dy) = _compare(B, f, g, 8, 8, name="shifted")
    assert (dx, dy) == (sx, sy) and pk < 1.0


def test_column_window(B):
    # a column window passed with the row pitch (the field-of-view strips)
    rng = np.random.default_rng(4)
    f = _smooth(rng, 60, 90)
    g = _smooth(rng, 60, 90)
    _compare(B, f, g, 3, 4, cols=(31, 59), name="window")
    _compare(B, f, g, 0, 0, cols=(45, 46), name="one column")


def test_zero_shift_equals_cross_correlate(B):
    rng = np.random.default_rng(8)
    f = rng.random((33, 47, 3)).astype(np.float32)
    g = rng.random((33, 47, 3)).astype(np.float32)
    m, _ = _compare(B, f, g, 0, 0, name="zero shift")
    dev = torch.device("cuda", 0)
    c0, _ = B.cross_correlate(torch.from_numpy(g).to(dev), torch.from_numpy(f).to(dev))
    assert abs(m[0, 0] - c0) <= 1e-12


def test_largest_shifts(B):
    # every shift the window allows, and more than 256 shifts along a row
    # (several shifts per thread)
    rng = np.random.default_rng(13)
    f = rng.random((15, 20, 3)).astype(np.float32)
    g = rng.random((15, 20, 3)).astype(np.float32)
    _compare(B, f, g, 19, 14, name="all shifts")
    f = rng.random((6, 400, 1)).astype(np.float32)
    g = rng.random((6, 400, 1)).astype(np.float32)
    _compare(B, f, g, 300, 2, name="601 shifts")


def test_full_size_render_shape(B):
    # 512 x 512 x 3 with |dx|, |dy| <= 16, every entry against the oracle
    rng = np.random.default_rng(99)
    f = _smooth(rng, 512, 512)
    g = np.ascontiguousarray(np.roll(f, (2, -3), axis=(0, 1)) * np.float32(0.75))
    _, (pk, dx, dy) = _compare(B, f, g, 16, 16, name="512x512")
    assert (dx, dy) == (-3, 2)


def test_errors(B):
    dev = torch.device("cuda", 0)
    f = torch.ones((8, 8, 3), dtype=torch.float32, device=dev)
    g = torch.rand((8, 8, 3), dtype=torch.float32, device=dev)
    with pytest.raises(B.GcError) as e:
        B.cross_correlate_map(g, f, 2, 2)          # constant reference
    assert e.value.status == B.GC_EINVAL
    with pytest.raises(B.GcError) as e:
        B.cross_correlate_map(g, g, 8, 0)          # rx >= width
    assert e.value.status == B.GC_EINVAL
    wide = torch.rand((2, 4000, 3), dtype=torch.float32, device=dev)
    with pytest.raises(B.GcError) as e:
        B.cross_correlate_map(wide, wide, 1, 0)    # two rows exceed the LDS budget
    assert e.value.status == B.GC_EUNSUPPORTED
