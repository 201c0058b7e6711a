"""Benchmark of the QAI post-pass on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--no-regime] [--no-extra]
                    [--extra quality,blocks,coded,workloads,differentiable,batched]

A step is one full post-pass (Algorithm 4: boundary/sign stencil, two exact
EDTs, interpolation and compensation) over one synthetic field already
resident in HBM.  The workload defaults to the 512^3 Gaussian random field
(amplitude spectrum |k|^-11/3) pre-quantized at eb = 1e-3 x range -- the shape
of the paper's per-rank JHTDB blocks (Section VII-E2).

Prints ONE JSON line on stdout (everything else goes to stderr):
* value = field GB/s = 4 bytes x voxels x steps / elapsed (host clock around
  exactly K steps, bracketed by device synchronisation; no stage timing on);
* roofline = the dominant kernel's algorithmic bytes per launch / its mean
  duration (HIP events on the launch stream, from a separate staged run)
  against 8 TB/s;
* pipeline = the whole pass against the roofline: algorithmic (the 56 B/voxel
  budget of two separable 3-pass EDTs in 3-D, 40 B in 2-D, and the bytes this
  design must move), measured (rocprofv3 FETCH/WRITE bytes of every stage,
  while the kernels are the ones measured) and against a copy kernel;
* workloads = the other configurations of the metric (the 256x384x384 field at
  three bounds, the 2-D 1800x3600 field, the 256^3 field of the
  differentiable form with its adjoint, the 64^3 field), each with its regime,
  timed with the autotuner's setting for its shape (and with the default);
* quality = SSIM and PSNR on the GPU before and after the pass (also per
  workload: the eb-distortion sweep of the 256x384x384 field), and the metric
  kernels' rate;
* blocks = the paper's block strategies (embarrassingly parallel, approximate)
  on 2 x 2 x 2 blocks beside the exact pass: time and quality;
* coded = the pass from coded indices (decoded inside the first seed pass)
  against decoding first, with the code's bytes per voxel;
* batched = the 48-field uneven batch, one graph launch vs per-field launches;
* cpu_baseline = the CPU oracle on the host's cores and on one core.
"""
import argparse
import ctypes
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QAI post-pass GB/s of FP32 field and % HBM roofline, plain vs batched, 1 GPU"
HBM_PEAK_GBPS = 8000.0
# Byte budget of the separable pass: read x', write out, and the word round
# trips of two EDTs of three passes each (two in 2-D).
BUDGET_3D, BUDGET_2D = 56, 40
# The paper's CPU throughput (Section VII-E2, weak scaling, 64 ranks on two
# nodes of 2x AMD EPYC 7702, 512^3 FP32 blocks): 695.93 MB/s with the
# embarrassingly parallel decomposition, i.e. about 10.9 MB/s per core.
PAPER_CPU = {"mb_per_s": 695.93, "ranks": 64, "mb_per_s_per_core": round(695.93 / 64, 2),
             "hardware": "2 nodes x 2x AMD EPYC 7702 (64 cores each), one core per rank",
             "workload": "512^3 FP32 blocks of a turbulence field, embarrassingly parallel variant"}

# Algorithmic HBM bytes per voxel of each stage (reads + writes of the
# arrays the stage must touch once): the post-pass moves 44 B/voxel in 3-D.
STAGE_BYTES = {
    "seed1_xscan": 8,     # read x', write first-EDT words
    "edt1_y": 8,          # read + write words
    "edt1_z": 8,
    "edt1_yz": 8,         # 3-D: both passes as one search (read x-pass words, write final words)
    "edt1_fallback": 0,   # separable passes behind it, run only when a distance exceeds its disc
    "seed2_xscan": 8,     # read first-EDT words, write second-EDT words
    "edt2_y": 8,
    "edt2_z": 8,
    "interp": 16,         # read second-EDT words, first-EDT words, x'; write out
    "edt2_z_interp": 12,  # fused last pass: read first-EDT words, x'; write out (the z search reads the
                          # y-pass words only at the voxels whose weight needs d2, ~3% at 512^3)
    "edt2_z_stream": 12,  # its streaming phase alone, on a side stream beside the y pass
    "edt2_z_search": 0,   # its search phase: reads only at the voxels whose weight needs d2
    "edt2_z_sparse": 0,   # whole z pass + step E on the side stream, run instead of the search only
                          # where B1 covers under 60% (launches that return at once elsewhere)
    "edt2_y_interp": 12,  # 2-D: step E fused with the y pass done where the weight needs d2 (read
                          # first-EDT words, x'; write out; x-pass words read by the searches)
    "clear": 0,
}

EXTRAS = ("quality", "blocks", "coded", "workloads", "differentiable", "batched")
EXTRA_WORKLOADS = ["modes256x384x384_eb1e-4", "modes256x384x384_eb1e-3", "modes256x384x384_eb1e-2",
                   "grf2d_1800x3600_k11/3_eb1e-3", "grf256_k3_eb5e-3", "grf64_k3_eb1e-2"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def budget(shape):
    return BUDGET_3D if shape[0] > 1 else BUDGET_2D


def timed_steps(fn, steps, warmup, stream):
    """Warm up, then time exactly `steps` calls: host clock between two device
    synchronisations, plus one HIP event pair per step on the launch stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record(stream)
    for k in range(steps):
        fn()
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))
    trimmed = step_ms[1:-1] if len(step_ms) > 2 else step_ms
    return elapsed, {"median": float(np.median(step_ms)), "trimmed_mean": float(np.mean(trimmed)),
                     "min": step_ms[0], "max": step_ms[-1]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grf512_k11/3_eb1e-3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-regime", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the other workloads, the batch and the adjoint")
    ap.add_argument("--extra", default=",".join(EXTRAS),
                    help="comma-separated subset of the parts after the headline: " + ",".join(EXTRAS))
    args = ap.parse_args()
    extra = set() if args.no_extra else {e for e in args.extra.split(",") if e}
    unknown = extra - set(EXTRAS)
    if unknown:
        ap.error(f"unknown --extra parts {sorted(unknown)}")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(fields would shard by slabs, see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2602_20097_amd as qai
    from paper_2602_20097_amd import synth

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    qai.lib()  # fail loudly if the HIP library is not built

    t0 = time.time()
    x32, xq, q, eb = synth.make_workload(args.workload)
    shape = xq.shape
    nvox = int(np.prod(shape))
    log(f"workload {args.workload} shape {shape} eb {eb:.6g} generated in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    field = torch.from_numpy(xq).to(dev)
    out = torch.empty_like(field)
    ws = qai.new_workspace(shape, dev)
    stream = torch.cuda.current_stream()

    # copy-kernel bandwidth (the achievable HBM rate) on buffers of the field's size
    src = torch.empty(nvox, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    qai.copy_probe(src, dst)
    copy_s, _ = timed_steps(lambda: qai.copy_probe(src, dst), 10, 1, stream)
    copy_gbps = 10 * 8.0 * nvox / copy_s / 1e9
    del src, dst

    # timed region: exactly K full post-passes, no stage timing
    run = lambda: qai.mitigate(field, eb, out=out, workspace=ws)  # noqa: E731
    elapsed, step = timed_steps(run, args.steps, args.warmup, stream)
    ms_step = elapsed * 1e3 / args.steps
    value = 4.0 * nvox * args.steps / elapsed / 1e9
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, field {value:.1f} GB/s "
        f"(device median {step['median']:.3f} ms)")

    # a separate run with per-stage HIP events (for the kernel roofline)
    qai.profile(True)
    qai.stage_times(reset=True)
    for _ in range(args.steps):
        run()
    stages = qai.stage_times(reset=True)
    qai.profile(False)
    per_launch = {k: v / args.steps for k, v in stages.items()}
    dom = max((k for k in per_launch if STAGE_BYTES.get(k, 0) > 0), key=lambda k: per_launch[k])
    dom_ms = per_launch[dom]
    dom_bytes = STAGE_BYTES[dom] * nvox
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    own_alg = sum(STAGE_BYTES.get(k, 0) for k in per_launch) * nvox
    for k, v in per_launch.items():
        bw = STAGE_BYTES.get(k, 0) * nvox / (v * 1e-3) / 1e9 if v > 0 else 0.0
        log(f"  stage {k:16s} {v * 1e3:9.1f} us  {bw:8.1f} GB/s alg")

    traffic, measured = read_traffic(args.workload, list(per_launch))
    dom_traffic = traffic.get(dom) if traffic else None
    bud = budget(shape) * nvox
    t_s = ms_step * 1e-3
    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "shape": list(shape), "voxels": nvox, "eb": eb,
                   "eb_rel": synth.WORKLOADS[args.workload]["rel"], "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": dom_traffic, "kernel": dom,
                     "kernel_ms": round(dom_ms, 4), "alg_bytes_per_launch": dom_bytes},
        "pipeline": {
            "budget_bytes_per_voxel": budget(shape),
            "frac_of_peak_budget": round(bud / t_s / 1e9 / HBM_PEAK_GBPS, 4),
            "alg_bytes_per_voxel": own_alg // nvox,
            "frac_of_peak_alg": round(own_alg / t_s / 1e9 / HBM_PEAK_GBPS, 4),
            "measured_bytes_per_voxel": round(measured / nvox, 2) if measured else None,
            "frac_of_peak_measured": round(measured / t_s / 1e9 / HBM_PEAK_GBPS, 4) if measured else None,
            "measured_within_guard": (measured <= 1.25 * bud) if measured else None,
            "frac_of_copy_budget": round(bud / t_s / 1e9 / copy_gbps, 4),
            "copy_GBps": round(copy_gbps, 1),
            "stages_us": {k: round(v * 1e3, 1) for k, v in per_launch.items()},
            "stage_sum_ms": round(sum(per_launch.values()), 4),
            "side_stream_stages": [k for k in per_launch if k == "edt2_z_stream"],
            "step_ms_median": round(step["median"], 4),
            "step_ms_trimmed_mean": round(step["trimmed_mean"], 4)},
    }
    if not args.no_regime:
        res["regime"] = regime_stats(qai, field, x32, eb, dev)
    if "quality" in extra:
        res["quality"] = bench_quality(qai, field, out, x32, dev, max(5, args.steps // 2))
    if "blocks" in extra and shape[0] > 1:
        del ws
        torch.cuda.empty_cache()
        res["blocks"] = bench_blocks(qai, field, x32, eb, dev, ms_step, max(3, args.steps // 4))
    if "coded" in extra:
        res["coded"] = bench_coded(qai, synth, q, eb, field, dev, ms_step, max(5, args.steps // 2))
    del field, out
    torch.cuda.empty_cache()

    if "workloads" in extra:
        res["workloads"] = {}
        for name in EXTRA_WORKLOADS:
            res["workloads"][name] = bench_workload(qai, synth, dev, name, max(5, args.steps // 2), args.no_regime)
            torch.cuda.empty_cache()
    if "differentiable" in extra:
        res["differentiable"] = bench_grad(qai, synth, dev, max(5, args.steps // 2))
        torch.cuda.empty_cache()
    if "batched" in extra:
        res["batched"] = bench_batched(qai, synth, dev, max(3, args.steps // 4))
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(xq, eb)

    print(json.dumps(res), flush=True)


def read_traffic(workload, stages):
    """Stage bytes from profiles/traffic.json (rocprofv3 FETCH_SIZE/WRITE_SIZE,
    scaled by the copy probe), used only while the kernel sources hash to the
    revision they were measured on.  Returns ({stage: bytes}, pass total or None)."""
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tfile):
        return {}, None
    try:
        with open(tfile) as fh:
            tr = json.load(fh)
    except Exception:
        return {}, None
    rev = kernel_rev()
    out = {}
    for st in stages:
        e = tr.get(f"{workload}:{st}")
        if e and e.get("kernel_rev") == rev:
            out[st] = e["bytes_per_launch"]
    total = sum(out.values()) if all(st in out for st in stages) else None
    return out, total


def bench_quality(qai, field, out, x32, dev, reps):
    """SSIM (Eq. 3) and PSNR (Eq. 4) on the GPU of the decompressed and the
    compensated field against the original, and the metric kernels' rate
    (two passes over two fields: 16 B/voxel)."""
    import torch
    x = torch.from_numpy(x32).to(dev)
    before = qai.quality(x, field)
    after = qai.quality(x, out)
    s = torch.cuda.current_stream()
    el, step = timed_steps(lambda: qai.quality(x, out, sync=False), reps, 1, s)
    ms = el * 1e3 / reps
    n = x.numel()
    log(f"quality: SSIM {before['ssim']:.4f} -> {after['ssim']:.4f}, PSNR {before['psnr']:.2f} -> "
        f"{after['psnr']:.2f} dB; metric pass {ms:.3f} ms")
    return {"ssim_before": round(before["ssim"], 6), "ssim_after": round(after["ssim"], 6),
            "psnr_before": round(before["psnr"], 4), "psnr_after": round(after["psnr"], 4),
            "metric_ms": round(ms, 4), "metric_GBps_alg": round(16.0 * n / (ms * 1e-3) / 1e9, 1),
            "metric_frac_of_peak": round(16.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}


def bench_blocks(qai, field, x32, eb, dev, exact_ms, reps, blocks=(2, 2, 2)):
    """The paper's block strategies (Section VI-B) with the field cut into
    2 x 2 x 2 blocks: time and quality of embarrassingly parallel and
    approximate beside the exact (whole-field) pass."""
    import torch
    x = torch.from_numpy(x32).to(dev)
    s = torch.cuda.current_stream()
    res = {"blocks": list(blocks), "exact_ms": round(exact_ms, 4)}
    exact = qai.mitigate(field, eb)
    q = qai.quality(x, exact)
    res["exact_ssim"], res["exact_psnr"] = round(q["ssim"], 6), round(q["psnr"], 4)
    for mode in ("ep", "approximate"):
        o = torch.empty_like(field)
        el, _ = timed_steps(lambda: qai.mitigate_blocks(field, eb, blocks, mode=mode, out=o), reps, 1, s)
        q = qai.quality(x, o)
        differ = float((o != exact).float().mean())
        res[mode] = {"ms": round(el * 1e3 / reps, 4), "ssim": round(q["ssim"], 6), "psnr": round(q["psnr"], 4),
                     "frac_voxels_differing_from_exact": round(differ, 6)}
        log(f"blocks {mode}: {el * 1e3 / reps:.3f} ms, SSIM {q['ssim']:.5f}, PSNR {q['psnr']:.3f}, "
            f"{differ:.4%} of voxels differ from the exact pass")
    return res


def bench_coded(qai, synth, q, eb, field, dev, plain_ms, reps):
    """The post-pass from coded indices (segment code, decoded inside the first
    seed pass) against decoding to x' first and running the plain pass; the
    bytes of the code per voxel beside the 4 of x'."""
    import torch
    t0 = time.time()
    code = synth.encode_indices(q)
    dc = qai.upload_code(code, dev)
    n = int(q.size)
    log(f"coded: {code['nbytes'] / n:.3f} B/voxel of code, encoded in {time.time() - t0:.1f}s")
    out = torch.empty_like(field)
    xd = torch.empty_like(field)
    ws = qai.new_workspace(field.shape, dev)
    s = torch.cuda.current_stream()
    f_el, _ = timed_steps(lambda: qai.mitigate_coded(dc, eb, out=out, workspace=ws), reps, 2, s)
    ok = bool(torch.equal(out.view(torch.int32), qai.mitigate(field, eb).view(torch.int32)))

    def unfused():
        qai.decode(dc, eb, out=xd)
        qai.mitigate(xd, eb, out=out, workspace=ws)
    u_el, _ = timed_steps(unfused, reps, 2, s)
    d_el, _ = timed_steps(lambda: qai.decode(dc, eb, out=xd), reps, 2, s)
    fused_ms, unf_ms, dec_ms = f_el * 1e3 / reps, u_el * 1e3 / reps, d_el * 1e3 / reps
    log(f"coded: fused {fused_ms:.3f} ms, decode + plain {unf_ms:.3f} ms (decode {dec_ms:.3f} ms); "
        f"plain on x' {plain_ms:.3f} ms; equal to the plain pass: {ok}")
    return {"code_bytes_per_voxel": round(code["nbytes"] / n, 4), "fused_ms": round(fused_ms, 4),
            "decode_then_plain_ms": round(unf_ms, 4), "decode_ms": round(dec_ms, 4),
            "plain_ms": round(plain_ms, 4), "fused_GBps": round(4.0 * n / (fused_ms * 1e-3) / 1e9, 2),
            "equal_to_plain": ok}


def bench_workload(qai, synth, dev, name, steps, no_regime):
    """One of the metric's other configurations: the default setting, then the
    autotuner's setting for the shape (cached, used by the same call)."""
    import torch
    x32, xq, q, eb = synth.make_workload(name)
    n = int(np.prod(xq.shape))
    t = torch.from_numpy(xq).to(dev)
    out = torch.empty_like(t)
    ws = qai.new_workspace(t.shape, dev)
    s = torch.cuda.current_stream()
    run = lambda: qai.mitigate(t, eb, out=out, workspace=ws)  # noqa: E731
    el_def, _ = timed_steps(run, steps, 3, s)
    tuned = qai.autotune(t, eb)
    elapsed, step = timed_steps(run, steps, 3, s)
    qai.tuning_cache_clear()
    ms = elapsed * 1e3 / steps
    bud = budget(xq.shape) * n
    entry = {"shape": list(xq.shape), "voxels": n, "eb": eb, "ms": round(ms, 4),
             "device_ms_median": round(step["median"], 4),
             "GBps": round(4.0 * n / (ms * 1e-3) / 1e9, 2),
             "budget_bytes_per_voxel": budget(xq.shape),
             "frac_of_peak_budget": round(bud / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
             "default_setting_ms": round(el_def * 1e3 / steps, 4), "tuned": tuned}
    if not no_regime:
        entry["regime"] = regime_stats(qai, t, x32, eb, dev)
    if min(xq.shape[1:]) >= 2:
        x = torch.from_numpy(x32).to(dev)
        qb, qa = qai.quality(x, t), qai.quality(x, out)
        entry["quality"] = {"ssim_before": round(qb["ssim"], 6), "ssim_after": round(qa["ssim"], 6),
                            "psnr_before": round(qb["psnr"], 4), "psnr_after": round(qa["psnr"], 4)}
    log(f"workload {name}: {ms:.3f} ms, {entry['GBps']} GB/s, {entry['frac_of_peak_budget']:.3f} of peak")
    return entry


def bench_grad(qai, synth, dev, steps):
    """Forward (workspace kept) + adjoint on the 256^3 differentiable-form field."""
    import torch
    name = "grf256_k3_eb5e-3"
    x32, xq, q, eb = synth.make_workload(name)
    n = int(np.prod(xq.shape))
    t = torch.from_numpy(xq).to(dev)
    out = torch.empty_like(t)
    ws = qai.new_workspace(t.shape, dev)
    g = torch.randn_like(t)
    s = torch.cuda.current_stream()
    qai.mitigate(t, eb, out=out, workspace=ws)
    f_el, _ = timed_steps(lambda: qai.mitigate(t, eb, out=out, workspace=ws), steps, 2, s)
    b_el, bstep = timed_steps(lambda: qai.backward(g, ws, t.shape, eb), steps, 2, s)
    fwd, bwd = f_el * 1e3 / steps, b_el * 1e3 / steps
    log(f"differentiable {name}: forward {fwd:.3f} ms, adjoint {bwd:.3f} ms")
    return {"workload": name, "voxels": n, "forward_ms": round(fwd, 4), "adjoint_ms": round(bwd, 4),
            "adjoint_device_ms_median": round(bstep["median"], 4),
            "adjoint_GBps_alg": round(12.0 * n / (bwd * 1e-3) / 1e9, 1),
            "adjoint_frac_of_peak": round(12.0 * n / (bwd * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}


def bench_batched(qai, synth, dev, reps):
    """The 48-field uneven batch: one graph launch vs the same kernels launched
    field by field (autotuned per shape)."""
    import torch
    t0 = time.time()
    fields, ebs = [], []
    for spec in synth.batch_specs():
        x32, xq, q, eb = synth.make_batch_field(spec)
        fields.append(torch.from_numpy(xq).to(dev))
        ebs.append(eb)
    nvox = sum(int(f.numel()) for f in fields)
    log(f"batch of {len(fields)} fields, {nvox} voxels, generated in {time.time() - t0:.1f}s")
    t1 = time.time()
    plan = qai.BatchPlan(fields, ebs, autotune=True, tune_each=True)
    log(f"batch plan (autotuned per shape, pass choice per field) in {time.time() - t1:.1f}s")
    s = torch.cuda.current_stream()
    g_el, gstep = timed_steps(plan.launch, reps, 1, s)
    p_el, _ = timed_steps(plan.launch_per_field, reps, 1, s)
    graph_ms, per_ms = g_el * 1e3 / reps, p_el * 1e3 / reps
    tunes = {}
    for i, f in enumerate(fields):
        tunes.setdefault("x".join(map(str, f.shape)), plan.tuning(i))
    plan.close()
    bud = BUDGET_3D * nvox
    log(f"batched: graph {graph_ms:.2f} ms, per-field launches {per_ms:.2f} ms")
    return {"fields": len(fields), "voxels": nvox, "graph_ms": round(graph_ms, 3),
            "graph_device_ms_median": round(gstep["median"], 3), "per_field_ms": round(per_ms, 3),
            "value": round(4.0 * nvox / (graph_ms * 1e-3) / 1e9, 2), "unit": "GB/s",
            "per_field_GBps": round(4.0 * nvox / (per_ms * 1e-3) / 1e9, 2),
            "frac_of_peak_budget": round(bud / (graph_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "per_field_frac_of_peak_budget": round(bud / (per_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "tuning": tunes}


def kernel_rev():
    """Hash of the plain pass's kernel sources: traffic counters are only
    reused while it holds."""
    from paper_2602_20097_amd.profsum import kernel_rev as rev
    return rev()


def regime_stats(qai, field, x32, eb, dev):
    import torch
    out, t = qai.mitigate(field, eb, taps=True)
    torch.cuda.synchronize()
    x = torch.from_numpy(x32).to(dev)
    f = lambda m: float(m.float().mean())  # noqa: E731
    b1 = t["b1"] == 1
    sb = t["sb"]
    d1 = t["d1sq"][t["d1sq"] >= 0].double().sqrt()
    d2 = t["d2sq"][t["d2sq"] >= 0].double().sqrt()
    err0 = x.double() - field.double()
    err1 = x.double() - out.double()
    rng = float(x.max() - x.min())
    sel = b1 & (sb != 0)
    agree = f(torch.sign(err0[sel]) == sb[sel].double()) if bool(sel.any()) else None
    mse0, mse1 = float((err0 ** 2).mean()), float((err1 ** 2).mean())
    return {"b1": round(f(b1), 4), "sb_nonzero": round(f(sb != 0), 4), "b2": round(f(t["b2"] == 1), 4),
            "s_nonzero": round(f(t["s"] != 0), 4), "c_nonzero": round(f(out != field), 4),
            "d1_mean": round(float(d1.mean()), 3) if d1.numel() else None,
            "d1_max": round(float(d1.max()), 2) if d1.numel() else None,
            "d2_mean": round(float(d2.mean()), 3) if d2.numel() else None,
            "d2_max": round(float(d2.max()), 2) if d2.numel() else None,
            "sign_agreement": round(agree, 4) if agree is not None else None,
            "psnr_before": round(20 * np.log10(rng / np.sqrt(mse0)), 3),
            "psnr_after": round(20 * np.log10(rng / np.sqrt(mse1)), 3),
            "max_err_over_eb": round(float(err1.abs().max()) / eb, 5)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of the calling thread's later parallel
    regions (the oracle's runtime is libgomp)."""
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def _oracle_rate(oracle, xq, eb, target_s):
    """The oracle on a bounded z-slab of the field sized from a 4-plane probe to
    take about target_s (the whole field, repeated, when it takes less)."""
    nz = xq.shape[0]
    probe = xq[: min(nz, 4)]
    t = time.perf_counter()
    oracle.qai(probe, eb)
    per_plane = (time.perf_counter() - t) / probe.shape[0]
    planes = int(min(nz, max(4, target_s / max(per_plane, 1e-9))))
    slab = xq[:planes]
    reps, dt = 0, 0.0
    while reps == 0 or (planes == nz and dt < target_s and reps < 64):
        t = time.perf_counter()
        oracle.qai(slab, eb)
        dt += time.perf_counter() - t
        reps += 1
    what = "the whole field" if planes == nz else f"z-slab {list(slab.shape)} ({planes}/{nz} planes)"
    return 4.0 * slab.size * reps / dt / 1e9, dt, f"{what}, {reps} run(s)"


def cpu_baseline(xq, eb):
    """The CPU oracle, as it stands, on bounded samples of the same field: all
    host threads (about 15 s) and one thread (about 8 s)."""
    import oracle
    oracle.qai(xq[: min(xq.shape[0], 2)], eb)  # load / build outside the timing
    threads = oracle.max_threads()
    gbps, dt, what = _oracle_rate(oracle, xq, eb, 15.0)
    one = None
    if _omp_threads(1):
        g1, dt1, what1 = _oracle_rate(oracle, xq, eb, 8.0)
        _omp_threads(threads)
        one = {"value": round(g1, 6), "unit": "GB/s", "mb_per_s": round(g1 * 1e3, 3), "seconds": round(dt1, 3),
               "sample": what1}
    return {"value": round(gbps, 5), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}, full Algorithm 4 in FP64 C/OpenMP with every intermediate kept, {dt:.2f} s",
            "seconds": round(dt, 3), "mb_per_s": round(gbps * 1e3, 2), "cpu_model": cpu_model(),
            "one_thread": one, "paper_cpu": PAPER_CPU}


if __name__ == "__main__":
    main()
