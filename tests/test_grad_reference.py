"""CPU pins of the FP64 reference the adjoint is checked against
(tests/_gradref.py): its forward is the oracle's step E, and its autograd
derivatives agree with central finite differences of the same float64
function -- exactly (up to rounding) in eta, where the output is affine, and to
O(h^2) in the IDW power p."""
import numpy as np
import torch

import oracle
from _gradref import reference_out
from paper_2602_20097_amd import synth


def _loss(xq, eb, r, g, eta, power):
    e = torch.tensor(eta, dtype=torch.float64, requires_grad=True)
    p = torch.tensor(power, dtype=torch.float64, requires_grad=True)
    out = reference_out(xq, eb, r, e, p)
    loss = (g * out).sum()
    loss.backward()
    return float(loss.detach()), float(e.grad), float(p.grad)


def test_reference_gradients_match_central_differences():
    x32, xq, q, eb = synth.quantize(synth.grf((20, 28, 36), 3.0, 21), 2e-2)
    g = torch.from_numpy(np.random.default_rng(5).standard_normal(xq.shape))
    for eta, power in ((0.9, 1.0), (0.6, 2.0), (1.1, 0.5)):
        r = oracle.qai(xq, eb, eta, power)
        # the reference's forward is the oracle's output
        out = reference_out(xq, eb, r, torch.tensor(float(np.float32(eta)), dtype=torch.float64),
                            torch.tensor(float(np.float32(power)), dtype=torch.float64))
        np.testing.assert_allclose(out.numpy(), r["out"], rtol=0, atol=1e-12)
        _, ge, gp = _loss(xq, eb, r, g, eta, power)
        assert ge != 0.0 and gp != 0.0
        h = 1e-3
        fe = (_loss(xq, eb, r, g, eta + h, power)[0] - _loss(xq, eb, r, g, eta - h, power)[0]) / (2 * h)
        fp = (_loss(xq, eb, r, g, eta, power + h)[0] - _loss(xq, eb, r, g, eta, power - h)[0]) / (2 * h)
        assert abs(fe - ge) <= 1e-6 * abs(ge), (eta, power, fe, ge)
        assert abs(fp - gp) <= 1e-6 * abs(gp), (eta, power, fp, gp)


def test_reference_eta_derivative_is_the_closed_form():
    """d out / d eta = w S eb, so dL/deta = sum g w S eb with the oracle's w."""
    x32, xq, q, eb = synth.quantize(synth.grf((16, 24, 32), 3.0, 22), 2e-2)
    r = oracle.qai(xq, eb, 0.9, 1.5)
    g = np.random.default_rng(6).standard_normal(xq.shape)
    _, ge, _ = _loss(xq, eb, r, torch.from_numpy(g), 0.9, 1.5)
    want = float((g * r["w"] * r["s"] * eb).sum())
    assert abs(ge - want) <= 1e-12 * max(1.0, abs(want))
