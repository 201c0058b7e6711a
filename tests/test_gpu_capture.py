"""A call captured into a graph (torch.cuda.graph on the caller's stream)
replays to the eager call's output bit for bit.  While its stream is being
captured the library keeps every launch on that stream (no side stream), and
the pass clears its status words with a kernel, so the graph holds kernel
nodes only.  Each replay is checked, with eager calls and synchronisations in
between, on a 3-D field (needed-voxel search) and a 2-D field (fused y pass)."""
import numpy as np
import pytest
import torch

from paper_2602_20097_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,rel", [((24, 40, 56), 1e-3), ((1, 90, 200), 1e-3)])
def test_captured_call_replays_like_the_eager_call(shape, rel):
    import paper_2602_20097_amd as qai
    x32, xq, q, eb = synth.quantize(synth.grf(shape, 3.0, 60 + shape[1]), rel)
    print(f"capture case shape={shape} rel={rel}", flush=True)
    f = torch.from_numpy(xq).cuda()
    ws = qai.new_workspace(f.shape)
    ref = qai.mitigate(f, eb, workspace=ws).clone()
    out = torch.empty_like(f)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        qai.mitigate(f, eb, out=out, workspace=ws)  # warm-up off the default stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        qai.mitigate(f, eb, out=out, workspace=ws)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), f"replay {rep}"
        # eager work on the same workspace between replays
        again = qai.mitigate(f, eb, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(again.view(torch.int32), ref.view(torch.int32))
    del g
    assert np.isfinite(ref.cpu().numpy()).all()
