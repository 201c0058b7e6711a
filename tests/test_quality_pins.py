"""CPU pins of the quality-metric oracle (oracle/quality.py): closed forms of
Eq. 3 and Eq. 4, the window geometry against scipy's box filter, and
invariances that follow from the definitions."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import quality as Q


def _rng_field(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_identical_fields_give_one_and_infinite_psnr():
    a = _rng_field((10, 12, 9), 1)
    assert Q.ssim(a, a) == pytest.approx(1.0, abs=1e-15)
    assert Q.psnr(a, a) == float("inf")


def test_psnr_of_a_constant_offset():
    a = _rng_field((9, 9, 9), 2)
    d = 0.01
    want = 20 * np.log10((a.max() - a.min()) / d)
    assert Q.psnr(a, a + d) == pytest.approx(want, rel=1e-12)
    assert Q.mse(a, a + d) == pytest.approx(d * d, rel=1e-12)


def test_single_window_closed_forms():
    """One 7^3 window: an offset changes only the luminance term,
    (2 mu1 mu2 + c1) / (mu1^2 + mu2^2 + c1); a field against its negation
    inside the same range gives the covariance term -s^2 ... closed forms."""
    a = _rng_field((7, 7, 7), 3)
    lo, rng = a.min(), a.max() - a.min()
    u = (a - lo) / rng
    c = 0.05 * rng
    mu1 = u.mean()
    mu2 = mu1 + c / rng
    want = (2 * mu1 * mu2 + Q.C1) / (mu1 ** 2 + mu2 ** 2 + Q.C1)
    assert Q.ssim(a, a + c) == pytest.approx(want, rel=1e-13)
    # mirrored field b = lo + hi - a: normalised v = 1 - u, equal variance, covariance -s^2
    b = lo + (a.max()) - a
    s2 = ((u - mu1) ** 2).sum() / (u.size - 1)
    muv = 1 - mu1
    want = (2 * mu1 * muv + Q.C1) * (-2 * s2 + Q.C2) / ((mu1 ** 2 + muv ** 2 + Q.C1) * (2 * s2 + Q.C2))
    assert Q.ssim(a, b) == pytest.approx(want, rel=1e-12)


def test_window_geometry_matches_a_box_filter():
    """Window means equal scipy's uniform filter (size 7) at the window
    centres 3, 5, 7, ... on every axis; the number of windows per axis is
    (n - 7) // 2 + 1, and a short axis is one whole-extent window."""
    shape = (12, 15, 20)
    a = _rng_field(shape, 4)
    lo, rng = a.min(), a.max() - a.min()
    st = Q.window_stats(a, a)
    assert st.shape[1:] == tuple((n - 7) // 2 + 1 for n in shape)
    box = ndimage.uniform_filter((a - lo) / rng, size=7, mode="constant")
    centres = np.ix_(*[np.arange(3, n - 3, 2) for n in shape])
    np.testing.assert_allclose(st[0], box[centres], rtol=0, atol=1e-13)
    flat = Q.window_stats(a[:1], a[:1])           # a 2-D field: windows of 1 x 7 x 7
    assert flat.shape[1:] == (1, (15 - 7) // 2 + 1, (20 - 7) // 2 + 1)
    short = Q.window_stats(a[:5, :6], a[:5, :6])  # axes of 5 and 6 voxels: one whole-extent window each
    assert short.shape[1:] == (1, 1, (20 - 7) // 2 + 1)
    sub = a[:5, :6]
    want = ((sub[:, :, :7] - sub.min()) / (sub.max() - sub.min())).mean()  # normalised by its own range
    np.testing.assert_allclose(short[0, 0, 0, 0], want, rtol=1e-14)


def test_sample_variance_divides_by_m_minus_one():
    a = _rng_field((7, 7, 7), 5)
    lo, rng = a.min(), a.max() - a.min()
    u = ((a - lo) / rng).ravel()
    st = Q.window_stats(a, a)
    assert st[2, 0, 0, 0] == pytest.approx(np.var(u, ddof=1), rel=1e-13)
    assert st[4, 0, 0, 0] == pytest.approx(np.var(u, ddof=1), rel=1e-13)


def test_invariant_to_a_common_affine_map():
    a = _rng_field((9, 11, 13), 6)
    b = a + 0.1 * _rng_field((9, 11, 13), 7)
    s = Q.ssim(a, b)
    assert Q.ssim(3.0 * a - 7.0, 3.0 * b - 7.0) == pytest.approx(s, rel=1e-12)
    assert Q.psnr(3.0 * a - 7.0, 3.0 * b - 7.0) == pytest.approx(Q.psnr(a, b), rel=1e-12)
    assert -1.0 <= Q.ssim(a, -b) <= s <= 1.0
