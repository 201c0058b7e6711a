"""Autotuner and per-shape tuning cache on the GPU: the tuned setting changes
nothing in the result (every candidate computes the same exact transforms),
the plain path uses the cached setting, and a saved and reloaded cache gives
the same setting and output."""
import numpy as np
import pytest
import torch

import oracle
import paper_2602_20097_amd as qai
from paper_2602_20097_amd import synth

pytestmark = pytest.mark.gpu


def _field(shape, rel, seed):
    _, xq, _, eb = synth.quantize(synth.grf(shape, 3.0, seed), rel)
    return torch.from_numpy(xq).to("cuda:0"), xq, eb


@pytest.mark.parametrize("shape", [(1, 200, 700), (20, 36, 600), (24, 40, 56)])
def test_autotuned_setting_is_used_and_changes_nothing(shape, tmp_path):
    qai.set_tuning(None)
    qai.tuning_cache_clear()
    t, xq, eb = _field(shape, 1e-2, 31)
    ref = qai.mitigate(t, eb)
    best = qai.autotune(t, eb)
    print(f"{shape}: tuned {best}", flush=True)
    assert qai.tuning_cache_size() == 1
    out = qai.mitigate(t, eb)
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
    r = oracle.qai(xq, eb)
    o = out.cpu().numpy().astype(np.float64)
    assert (np.abs(o - r["out"]) <= 1e-6 * np.maximum(np.abs(r["out"]), eb)).all()
    path = tmp_path / "cache.txt"
    qai.tuning_cache_save(path)
    qai.tuning_cache_clear()
    assert qai.tuning_cache_size() == 0
    qai.tuning_cache_load(path)
    assert qai.tuning_cache_size() == 1
    again = qai.mitigate(t, eb)
    torch.cuda.synchronize()
    assert torch.equal(again.view(torch.int32), ref.view(torch.int32))
    qai.tuning_cache_clear()


def test_batch_plan_takes_cached_settings():
    qai.set_tuning(None)
    qai.tuning_cache_clear()
    a, _, eb_a = _field((1, 200, 700), 1e-2, 41)
    b, _, eb_b = _field((16, 24, 40), 1e-3, 42)
    tuned = qai.autotune(a, eb_a)
    plan = qai.BatchPlan([a, b, a.clone()], [eb_a, eb_b, eb_a], autotune=True)
    outs = [o.clone() for o in plan.launch()]
    torch.cuda.synchronize()
    assert plan.tuning(0) == tuned and plan.tuning(2) == tuned
    assert qai.tuning_cache_size() == 2     # the second shape was tuned and cached by the plan
    for f, eb, o in ((a, eb_a, outs[0]), (b, eb_b, outs[1]), (a, eb_a, outs[2])):
        assert torch.equal(o.view(torch.int32), qai.mitigate(f, eb).view(torch.int32))
    plan.close()
    qai.tuning_cache_clear()
