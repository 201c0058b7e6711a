"""FP64 reference of step E for the gradient tests: the exact distance
transforms and signs come from the CPU oracle, and the weight (Section V,
generalised to the IDW power p) is written out in float64 torch, so autograd
differentiates w = k1^-p / (k1^-p + k2^-p) with the pinned cases (on B1, on
B2, no B2, no B1) held constant."""
import numpy as np
import torch


def reference_out(xq, eb, r, eta, power):
    """Step E in float64 torch from the oracle's transforms; eta and power are
    0-dim float64 tensors (possibly requiring grad)."""
    d1 = torch.from_numpy(r["d1sq"].astype(np.float64))
    d2 = torch.from_numpy(r["d2sq"].astype(np.float64))
    s = torch.from_numpy(r["s"].astype(np.float64))
    x = torch.from_numpy(xq.astype(np.float64))
    on_b1 = d1 == 0
    on_b2 = d2 == 0
    no_b2 = d2 < 0
    no_b1 = d1 < 0
    general = ~(on_b1 | on_b2 | no_b2 | no_b1)
    k1 = torch.sqrt(torch.where(general, d1, torch.ones_like(d1)))
    k2 = torch.sqrt(torch.where(general, d2, torch.ones_like(d2)))
    wg = 1.0 / (1.0 + (k1 / k2) ** power)
    w = torch.where(on_b1 | (no_b2 & ~on_b2), torch.ones_like(d1), torch.zeros_like(d1))
    w = torch.where(general, wg, w)
    return x + w * s * eta * float(eb)
