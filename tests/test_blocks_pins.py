"""CPU pins of the block-decomposed variants (oracle/blocks.py): on one block
all three strategies are the whole-field algorithm; the approximate variant's
step A sees its neighbours, so its boundary marks equal the whole field's;
embarrassingly parallel blocks equal the oracle on the cut-out blocks; the
block grid covers the field."""
import numpy as np
import pytest

import oracle
from oracle import blocks as B
from paper_2602_20097_amd import synth


def _field(shape, rel=1e-2, seed=61):
    x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, seed), rel)
    return xq, eb


@pytest.mark.parametrize("shape", [(12, 14, 16), (1, 30, 40)])
def test_one_block_is_the_whole_field(shape):
    xq, eb = _field(shape)
    r = oracle.qai(xq, eb)
    np.testing.assert_array_equal(B.ep(xq, eb, (1, 1, 1)), r["out"])
    out, tp = B.approximate(xq, eb, (1, 1, 1), taps=True)
    np.testing.assert_allclose(out, r["out"], rtol=0, atol=1e-12)   # step E in numpy vs the C oracle
    for k in ("b1", "sb", "s", "b2", "d1sq", "d2sq"):
        np.testing.assert_array_equal(tp[k], r[k].astype(np.int64), err_msg=k)


def test_block_bounds_cover_the_axis():
    for n, k in ((512, 2), (13, 3), (7, 7), (100, 6)):
        b = B.block_bounds(n, k)
        assert sum(e for _, e in b) == n and b[0][0] == 0
        assert all(b[i][0] + b[i][1] == b[i + 1][0] for i in range(k - 1))
        assert max(e for _, e in b) - min(e for _, e in b) <= 1


def test_approximate_step_a_equals_the_whole_field():
    xq, eb = _field((14, 18, 22), seed=62)
    r = oracle.qai(xq, eb)
    _, tp = B.approximate(xq, eb, (2, 2, 2), taps=True)
    np.testing.assert_array_equal(tp["b1"], r["b1"].astype(np.int64))
    np.testing.assert_array_equal(tp["sb"], r["sb"].astype(np.int64))


def test_ep_blocks_and_the_relaxed_bound():
    xq, eb = _field((14, 18, 22), seed=63)
    ep = B.ep(xq, eb, (2, 2, 2))
    r = oracle.qai(xq[:7, :9, :11].copy(), eb)
    np.testing.assert_array_equal(ep[:7, :9, :11], r["out"])
    ap = B.approximate(xq, eb, (2, 2, 2))
    ex = oracle.qai(xq, eb)["out"]
    x = xq.astype(np.float64)
    for o in (ep, ap, ex):
        assert np.abs(o - x).max() <= 0.9 * eb * (1 + 1e-6)
    assert not np.array_equal(ep, ex)


def test_exchange_of_signs_on_the_band_example():
    """Bands of 8 voxels (x_k = (k - 3.5)/8, eb = 0.5, so q = floor(k/8)) over
    28 voxels in two blocks [0, 14) and [14, 28).  Whole field: B1 = {7, 8, 15,
    16, 23, 24}, B2 = {11, 12, 19, 20}.  Block 0 does not see voxel 15, so its
    local first EDT gives S = - on 8..13; block 1 gives S(14) = + (from 15).
    The exchanged signs disagree across the face: B2 = {13, 14, 19, 20}, and
    on 9..12 (S = -, d1 = k - 8, d2 = 13 - k) the weight is (13 - k) / 5."""
    k = np.arange(28)
    xq = np.floor((k - 3.5) / 8.0 + 0.5).astype(np.float32)[None, None, :]   # x' = 2 eb q = q
    eb = 0.5
    c = float(np.float32(0.9)) * eb
    ex = oracle.qai(xq, eb)
    assert sorted(np.nonzero(ex["b1"][0, 0])[0].tolist()) == [7, 8, 15, 16, 23, 24]
    assert sorted(np.nonzero(ex["b2"][0, 0])[0].tolist()) == [11, 12, 19, 20]
    out, tp = B.approximate(xq, eb, (1, 1, 2), taps=True)
    assert sorted(np.nonzero(tp["b2"][0, 0])[0].tolist()) == [13, 14, 19, 20]
    assert tp["s"][0, 0, 8:14].tolist() == [-1] * 6 and tp["s"][0, 0, 14] == 1
    for kk in range(9, 13):
        assert out[0, 0, kk] == pytest.approx(float(xq[0, 0, kk]) - c * (13 - kk) / 5.0, abs=1e-12)
    assert out[0, 0, 13] == xq[0, 0, 13] and out[0, 0, 14] == xq[0, 0, 14]
