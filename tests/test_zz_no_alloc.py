"""The allocation-free entry point qai_mitigate_noalloc, called through the C
ABI: its output must equal that of qai_mitigate_ex (the same kernels on a
caller-owned workspace) on two calls in a row, the second on a smaller field,
so that stale contents of the fixed scratch from the first call cannot leak
into the second; the smaller field is also checked against the CPU oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2602_20097_amd as qai
from paper_2602_20097_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _noalloc(field, eb, out, eta=None):
    L = qai.lib()
    prm = _lib.Params(float(eta), 1.0, 0) if eta is not None else None
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.qai_mitigate_noalloc(ctypes.c_void_p(field.data_ptr()), _lib.dims3(field.shape), ctypes.c_float(eb),
                                  ctypes.byref(prm) if prm is not None else None, ctypes.c_void_p(out.data_ptr()),
                                  stream)


def test_noalloc_matches_the_workspace_entry_point_on_two_calls():
    cases = [((40, 72, 100), 3.0, 1e-3, 0.9), ((24, 40, 56), 3.0, 1e-2, 0.7)]
    for k, (shape, beta, rel, eta) in enumerate(cases):
        print(f"noalloc call {k}: shape {shape} rel eb {rel} eta {eta}", flush=True)
        x = synth.grf(shape, beta, 777 + k)
        _, xq, _, eb = synth.quantize(x, rel)
        t = torch.from_numpy(xq).to("cuda:0")
        ref = qai.mitigate(t, eb, eta=eta)           # qai_mitigate_ex, torch workspace
        out = torch.full_like(t, float("nan"))
        _lib.check(_noalloc(t, eb, out, eta))
        torch.cuda.synchronize()
        # the same kernels: equal bit for bit, hence within the parity tolerance too
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), f"call {k} differs"
        if k == 1:
            r = oracle.qai(xq, eb, eta=eta)
            o = out.cpu().numpy().astype(np.float64)
            assert (np.abs(o - r["out"]) <= 1e-6 * np.maximum(np.abs(r["out"]), eb)).all()


def test_noalloc_in_place_and_2d():
    x = synth.grf((1, 300, 700), 11.0 / 3.0, 4321)
    _, xq, _, eb = synth.quantize(x, 1e-3)
    t = torch.from_numpy(xq).to("cuda:0")
    ref = qai.mitigate(t, eb)
    _lib.check(_noalloc(t, eb, t))                    # out == field
    torch.cuda.synchronize()
    assert torch.equal(t.view(torch.int32), ref.view(torch.int32))


def test_noalloc_rejects_fields_beyond_the_scratch():
    t = torch.empty(4, device="cuda:0")
    L = qai.lib()
    dims = _lib.Dims(512, 512, 512)
    assert L.qai_workspace_bytes(dims) > _lib.NOALLOC_SCRATCH_BYTES
    rc = L.qai_mitigate_noalloc(ctypes.c_void_p(t.data_ptr()), dims, ctypes.c_float(0.1), None,
                                ctypes.c_void_p(t.data_ptr()), None)
    assert rc == -3 and "scratch" in L.qai_last_error().decode()
