"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compare it with the CPU oracle.

Bit-exact for the indices, masks, signs and squared distances; the
compensated output within 1e-6 * max(|out_oracle|, eb), the FP32-vs-FP64
tolerance derived in the design notes (FP32 relative error of C is a few
ulp of |C| <= 0.9 eb, plus half an ulp of |out| from the final add)."""
import numpy as np
import torch

import oracle

REL_TOL = 1e-6
KEYS = ("q", "b1", "sb", "s", "d1sq", "b2", "d2sq")


def gpu_run(xq, eb, eta=0.9, power=1.0):
    """Both forms of the call: with every tap (all passes written out) and
    without (the last EDT pass fused with step E); the outputs must agree
    bit for bit."""
    import paper_2602_20097_amd as qai
    t = torch.from_numpy(np.ascontiguousarray(xq, np.float32)).cuda()
    out, taps = qai.mitigate(t, eb, eta, power, taps=True)
    plain = qai.mitigate(t, eb, eta, power)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in taps.items()}
    res["out"] = out.cpu().numpy()
    res["out_plain"] = plain.cpu().numpy()
    return res


def assert_out_close(out, r, eb, label=""):
    """A GPU output (float32 array) against the oracle's within the tolerance."""
    err = np.abs(np.asarray(out, np.float64) - r["out"])
    lim = REL_TOL * np.maximum(np.abs(r["out"]), eb)
    assert (err <= lim).all(), f"{label}: out off by {err.max():.3g} (limit {lim[np.argmax(err - lim)]:.3g})"


def assert_parity(xq, eb, eta=0.9, power=1.0, label="", r=None):
    print(f"parity case {label} shape={xq.shape} eb={eb:.6g}", flush=True)
    g = gpu_run(xq, eb, eta, power)
    if r is None:
        r = oracle.qai(xq, eb, eta, power)
    for k in KEYS:
        a, b = g[k], r[k]
        if not np.array_equal(a.astype(np.int64), b.astype(np.int64)):
            bad = np.argwhere(a.astype(np.int64) != b.astype(np.int64))
            raise AssertionError(f"{label}: tap {k} differs at {len(bad)} voxels, first {bad[:5].tolist()}: "
                                 f"gpu {a[tuple(bad[0])]} oracle {b[tuple(bad[0])]}")
    assert np.array_equal(g["out_plain"].view(np.uint32), g["out"].view(np.uint32)), f"{label}: fused path differs"
    assert_out_close(g["out"], r, eb, label)
    np.testing.assert_allclose(g["w"], r["w"], rtol=0, atol=1e-6)
    return g, r
