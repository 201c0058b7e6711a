"""The post-pass straight from coded indices (qai_mitigate_coded): the GPU
decoder reproduces the decompressed field bit for bit, the fused pass (the
first seed pass decodes the lines it reads and writes x' into out) gives
qai_mitigate_ex's result on that field bit for bit, for every supported line
geometry (ceil(nx/64) in {1, 2, 4, 8}; lines of 513..2048 voxels over two or
four waves), ragged last segments, and the shapes that decode first; the
indices are checked against the oracle's decoder and the output against the
oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2602_20097_amd as qai
from oracle import codec
from paper_2602_20097_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(24, 40, 64), (20, 30, 128), (16, 24, 256), (12, 20, 512), (8, 9, 70), (5, 7, 100), (10, 20, 384),
          (1, 100, 300), (1, 1, 90), (3, 40, 600), (4, 9, 1024), (3, 5, 1500), (2, 3, 2100)]


@pytest.mark.parametrize("shape", SHAPES)
def test_coded_pass_equals_the_plain_pass(shape):
    print(f"coded case {shape}", flush=True)
    x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, 81), 2e-3)
    code = synth.encode_indices(q)
    np.testing.assert_array_equal(codec.decode_indices_fast(code, q.shape), q)
    dc = qai.upload_code(code)
    t = torch.from_numpy(xq).cuda()
    dec = qai.decode(dc, eb)
    ref = qai.mitigate(t, eb)
    out = qai.mitigate_coded(dc, eb)
    torch.cuda.synchronize()
    assert torch.equal(dec.view(torch.int32), t.view(torch.int32))
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))


def test_coded_pass_against_the_oracle():
    x32, xq, q, eb = synth.quantize(synth.grf((16, 24, 256), 11.0 / 3.0, 82), 1e-3)
    code = synth.encode_indices(q)
    qd = codec.decode_indices(code, q.shape)
    xq_o = (2.0 * eb * qd).astype(np.float32)
    np.testing.assert_array_equal(xq_o, xq)
    r = oracle.qai(xq_o, eb)
    out = qai.mitigate_coded(qai.upload_code(code), eb).cpu().numpy().astype(np.float64)
    assert (np.abs(out - r["out"]) <= 1e-6 * np.maximum(np.abs(r["out"]), eb)).all()


def test_out_of_range_indices_raise_the_status_flag():
    q = np.zeros((6, 8, 64), np.int32)
    q[3, 4, 10] = (1 << 21) + 5
    code = synth.encode_indices(q)
    ws = qai.new_workspace(q.shape)
    qai.mitigate_coded(qai.upload_code(code), 0.5, workspace=ws)
    assert qai.device_status(ws) & qai.QAI_STATUS_QRANGE
    q[3, 4, 10] = 7
    ws2 = qai.new_workspace(q.shape)
    qai.mitigate_coded(qai.upload_code(synth.encode_indices(q)), 0.5, workspace=ws2)
    assert qai.device_status(ws2) == 0


@pytest.mark.parametrize("shape", [(4, 6, 512), (4, 6, 256), (3, 5, 128), (3, 5, 64), (2, 3, 600), (1, 2, 700)])
def test_wide_and_mixed_segment_widths(shape):
    """Rough rows (differences up to 2^21: widths past 12 bits, where a lane of
    eight voxels reads two words per difference) beside smooth ones, so that the
    lanes of one wave take both decode paths."""
    print(f"coded wide case {shape}", flush=True)
    rng = np.random.default_rng(83)
    x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, 84), 1e-3)
    q = q.copy()
    rough = rng.random(shape[:2]) < 0.5
    rough.flat[0], rough.flat[-1] = True, False
    noise = rng.integers(-(1 << 20), (1 << 20) + 1, size=shape, dtype=np.int64)
    q[rough] = np.clip(q[rough] + noise[rough], -(1 << 21), 1 << 21).astype(np.int32)
    xq = (2.0 * eb * q.astype(np.float64)).astype(np.float32)
    code = synth.encode_indices(q)
    meta = code["meta"].astype(np.int64)
    assert (meta & 0xFF).max() > 12 and (meta & 0xFF).min() <= 12
    dc = qai.upload_code(code)
    t = torch.from_numpy(xq).cuda()
    dec = qai.decode(dc, eb)
    ref = qai.mitigate(t, eb)
    out = qai.mitigate_coded(dc, eb)
    torch.cuda.synchronize()
    assert torch.equal(dec.view(torch.int32), t.view(torch.int32))
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
