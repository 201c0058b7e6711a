"""CPU pins of the index code: the oracle's decoders invert the encoder on
smooth, rough, constant and extreme index fields, and a hand-made segment
decodes to its written values."""
import numpy as np
import pytest

from oracle import codec
from paper_2602_20097_amd import synth


@pytest.mark.parametrize("shape,kind", [((3, 4, 70), "smooth"), ((2, 5, 64), "rough"), ((1, 3, 31), "const"),
                                        ((2, 2, 33), "extreme"), ((1, 1, 1), "smooth")])
def test_decoders_invert_the_encoder(shape, kind):
    rng = np.random.default_rng(9)
    if kind == "smooth":
        q = np.rint(synth.grf(shape, 3.0, 5) * 40).astype(np.int32)
    elif kind == "rough":
        q = rng.integers(-300, 300, size=shape).astype(np.int32)
    elif kind == "const":
        q = np.full(shape, -17, np.int32)
    else:
        q = rng.choice(np.array([-(2 ** 21), 2 ** 21, 0, 1, -1], np.int32), size=shape)
    code = synth.encode_indices(q)
    np.testing.assert_array_equal(codec.decode_indices(code, shape), q)
    np.testing.assert_array_equal(codec.decode_indices_fast(code, shape), q)
    if kind == "const":
        assert (code["meta"] & 0xFF == 0).all() and code["payload"].size == 1
    if kind == "extreme":
        assert (code["meta"] & 0xFF).max() == 24   # a difference of +2^22 zigzags to 2^23: 24 bits


def test_hand_segment():
    """One row of 4 values 5, 6, 4, 4: differences +1, -2, 0 -> zigzag 2, 3, 0
    (then 28 zeros of padding), width 2 bits: payload word 0b00_11_10 = 14."""
    q = np.array([[[5, 6, 4, 4]]], np.int32)
    code = synth.encode_indices(q)
    assert code["base"].tolist() == [5]
    assert int(code["meta"][0]) == (0 << 8) | 2
    assert code["payload"][0] == 0b001110
    assert codec.decode_indices(code, q.shape).tolist() == q.tolist()


def test_smooth_fields_code_small():
    x32, xq, q, eb = synth.quantize(synth.grf((16, 32, 64), 11.0 / 3.0, 3), 1e-3)
    code = synth.encode_indices(q)
    assert code["nbytes"] < 0.4 * q.nbytes
