"""Batched form (project addition): one graph launch over fields of uneven
shapes gives, for every field, exactly what the plain entry point gives, and
every field agrees with the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_20097_amd import synth

from _parity import assert_out_close, assert_parity

pytestmark = pytest.mark.gpu

SHAPES = [(7, 33, 65), (20, 50, 70), (1, 100, 300), (5, 16, 600), (9, 9, 9), (7, 33, 65), (3, 1, 200)]


def make_fields(host=False):
    out = []
    for i, s in enumerate(SHAPES):
        x32, xq, q, eb = synth.quantize(synth.grf(s, 2.0 + 0.3 * i, 900 + i), 10.0 ** (-2 - 0.25 * i))
        out.append((xq, eb) if host else (torch.from_numpy(xq).cuda(), eb))
    return out


def test_every_batched_field_matches_the_oracle():
    """Each output of one graph launch against the oracle on its own field
    (the tolerance of the plain path), besides being the plain path's bits."""
    import paper_2602_20097_amd as qai
    host = make_fields(host=True)
    fields = [(torch.from_numpy(xq).cuda(), eb) for xq, eb in host]
    plan = qai.BatchPlan([f for f, _ in fields], [eb for _, eb in fields], autotune=True)
    try:
        plan.launch()
        torch.cuda.synchronize()
        for i, ((xq, eb), o) in enumerate(zip(host, plan.outs)):
            print(f"batched field {i} shape {SHAPES[i]} eb {eb:.4g}", flush=True)
            r = oracle.qai(xq, eb)
            assert_out_close(o.cpu().numpy(), r, eb, f"batched field {i} {SHAPES[i]}")
            assert torch.equal(o, qai.mitigate(fields[i][0], eb))
    finally:
        plan.close()


# one field per shape class of the 48-field batch (16 each of 100x500x500,
# 256x384x384 and 128x128x1024; spectral exponents in [2, 4]) at the two ends
# of the batch's relative bounds, [1e-4, 1e-2]
W4_CLASSES = [((100, 500, 500), 2.0), ((256, 384, 384), 3.0), ((128, 128, 1024), 4.0)]


@pytest.mark.parametrize("rel", [1e-4, 1e-2])
def test_batch_shape_classes_full_parity(rel):
    """Full oracle parity (every intermediate bit-exact, out within tolerance)
    of one field per shape class of the 48-field batch, through the plain
    entry point; then the three fields as one autotuned batch plan, each
    output checked against the oracle and against the plain path bit for bit.
    The 128x128x1024 class takes the long-line seed kernels (x-lines longer
    than 512 voxels)."""
    import paper_2602_20097_amd as qai
    host, refs = [], []
    for i, (shape, beta) in enumerate(W4_CLASSES):
        x32, xq, q, eb = synth.quantize(synth.grf(shape, beta, 7700 + i), rel)
        r = oracle.qai(xq, eb)
        g, _ = assert_parity(xq, eb, label=f"class {shape} rel {rel}", r=r)
        assert np.array_equal(g["q"], q)
        host.append((xq, eb))
        refs.append((r["out"], g["out"]))
        del g, r
    fields = [torch.from_numpy(xq).cuda() for xq, _ in host]
    plan = qai.BatchPlan(fields, [eb for _, eb in host], autotune=True)
    try:
        for rep in range(2):
            print(f"class batch replay {rep} rel {rel}", flush=True)
            for o in plan.outs:
                o.fill_(float("nan"))
            plan.launch()
            torch.cuda.synchronize()
            for i, ((xq, eb), (ro, plain), o) in enumerate(zip(host, refs, plan.outs)):
                got = o.cpu().numpy()
                assert np.array_equal(got.view(np.uint32), plain.view(np.uint32)), (rep, i)
                assert_out_close(got, {"out": ro}, eb, f"batched class {W4_CLASSES[i][0]}")
    finally:
        plan.close()


@pytest.mark.parametrize("autotune", [False, True])
def test_graph_replays_match_the_plain_path(autotune):
    import paper_2602_20097_amd as qai
    fields = make_fields()
    ref = [qai.mitigate(f, eb) for f, eb in fields]
    plan = qai.BatchPlan([f for f, _ in fields], [eb for _, eb in fields], autotune=autotune)
    try:
        for rep in range(3):
            print(f"batch replay {rep} autotune={autotune}", flush=True)
            for o in plan.outs:
                o.fill_(float("nan"))
            plan.launch()
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(plan.outs, ref)):
                assert torch.equal(o, r), (rep, i, SHAPES[i])
            # the program's own eager work between replays
            extra = qai.mitigate(fields[1][0], fields[1][1])
            torch.cuda.synchronize()
            assert torch.equal(extra, ref[1])
        for o in plan.outs:
            o.zero_()
        plan.launch_per_field()
        torch.cuda.synchronize()
        for o, r in zip(plan.outs, ref):
            assert torch.equal(o, r)
        # fields of one shape share the tuning the autotuner picked
        assert plan.tuning(0) == plan.tuning(5)
    finally:
        plan.close()


def test_mitigate_batched_and_inputs_untouched():
    import paper_2602_20097_amd as qai
    fields = make_fields()
    before = [f.clone() for f, _ in fields]
    outs = qai.mitigate_batched([f for f, _ in fields], [eb for _, eb in fields])
    for (f, eb), o, b in zip(fields, outs, before):
        assert torch.equal(f, b)
        assert torch.equal(o, qai.mitigate(f, eb))


def test_batch_argument_errors():
    import paper_2602_20097_amd as qai
    f = torch.zeros((4, 5, 6), device="cuda")
    with pytest.raises(qai.QAIError):
        qai.BatchPlan([f], [0.0])
    with pytest.raises(qai.QAIError):
        qai.BatchPlan([f], [0.5], outs=[f])  # output overlapping its input
