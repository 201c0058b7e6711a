"""Batched form (project addition): one graph launch over fields of uneven
shapes gives, for every field, exactly what the plain entry point gives."""
import numpy as np
import pytest
import torch

from paper_2602_20097_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(7, 33, 65), (20, 50, 70), (1, 100, 300), (5, 16, 600), (9, 9, 9), (7, 33, 65), (3, 1, 200)]


def make_fields():
    out = []
    for i, s in enumerate(SHAPES):
        x32, xq, q, eb = synth.quantize(synth.grf(s, 2.0 + 0.3 * i, 900 + i), 10.0 ** (-2 - 0.25 * i))
        out.append((torch.from_numpy(xq).cuda(), eb))
    return out


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
