"""GPU quality metrics (SSIM, Eq. 3; PSNR, Eq. 4) against the float64
oracle (oracle/quality.py) on QAI outputs and decompressed fields: several
tiles and z-chunks, ragged tiles, 2-D fields, axes shorter than the window,
equal fields and a constant original."""
import math

import numpy as np
import pytest
import torch

import paper_2602_20097_amd as qai
from oracle import quality as Q
from paper_2602_20097_amd import synth

pytestmark = pytest.mark.gpu


def _check(orig, dec):
    print(f"quality case {orig.shape}", flush=True)
    r = qai.quality(torch.from_numpy(orig).cuda(), torch.from_numpy(dec).cuda())
    want_s = Q.ssim(orig, dec)
    want_p = Q.psnr(orig, dec)
    assert abs(r["ssim"] - want_s) <= 1e-9, (r["ssim"], want_s)
    if math.isinf(want_p):
        assert math.isinf(r["psnr"]) and r["psnr"] > 0
    else:
        assert r["psnr"] == pytest.approx(want_p, rel=1e-9)
    assert r["mse"] == pytest.approx(Q.mse(orig, dec), rel=1e-9, abs=0.0)
    assert r["range"] == float(orig.max()) - float(orig.min())
    return r


@pytest.mark.parametrize("shape", [(24, 40, 56), (80, 40, 50), (9, 17, 33), (1, 300, 700), (5, 6, 30), (1, 1, 90)])
def test_quality_matches_the_oracle_on_qai_outputs(shape):
    x = synth.grf(shape, 3.0, 51)
    x32, xq, q, eb = synth.quantize(x, 1e-2)
    out = qai.mitigate(torch.from_numpy(xq).cuda(), eb).cpu().numpy()
    before = _check(x32, xq)
    after = _check(x32, out)
    print(f"{shape}: SSIM {before['ssim']:.4f} -> {after['ssim']:.4f}, "
          f"PSNR {before['psnr']:.2f} -> {after['psnr']:.2f}", flush=True)


def test_equal_and_constant_fields():
    x32 = synth.grf((16, 20, 24), 3.0, 52).astype(np.float32)
    r = _check(x32, x32)
    assert r["ssim"] == pytest.approx(1.0, abs=1e-12)
    c = np.full((8, 9, 10), 3.0, np.float32)
    r = qai.quality(torch.from_numpy(c).cuda(), torch.from_numpy(c + 1).cuda())
    assert math.isnan(r["ssim"]) and r["range"] == 0.0


def test_unaligned_inputs_take_the_scalar_path():
    x32 = synth.grf((10, 21, 31), 3.0, 53).astype(np.float32)
    y32 = (x32 + 0.01 * np.random.default_rng(3).standard_normal(x32.shape)).astype(np.float32)
    buf_a = torch.zeros(x32.size + 1, device="cuda")
    buf_b = torch.zeros(x32.size + 1, device="cuda")
    a = buf_a[1:].view(x32.shape)
    b = buf_b[1:].view(x32.shape)
    a.copy_(torch.from_numpy(x32))
    b.copy_(torch.from_numpy(y32))
    r = qai.quality(a, b)
    assert abs(r["ssim"] - Q.ssim(x32, y32)) <= 1e-9
    assert r["psnr"] == pytest.approx(Q.psnr(x32, y32), rel=1e-9)


def test_windows_need_two_voxels():
    t = torch.zeros((1, 1, 1), device="cuda")
    with pytest.raises(qai.QAIError):
        qai.quality(t, t)
