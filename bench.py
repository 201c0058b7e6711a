"""Benchmark of the QAI post-pass on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--no-regime]

A step is one full post-pass (Algorithm 4: boundary/sign stencil, two exact
EDTs, interpolation and compensation) over one synthetic field already
resident in HBM.  The workload defaults to the 512^3 Gaussian random field
(amplitude spectrum |k|^-11/3) pre-quantized at eb = 1e-3 x range -- the shape
of the paper's per-rank JHTDB blocks (Section VII-E2).

Prints ONE JSON line on stdout (everything else goes to stderr):
value = field GB/s = 4 bytes x voxels x steps / elapsed; roofline = the
dominant kernel's algorithmic bytes per launch / its mean duration (HIP
events on the launch stream over the timed region) against 8 TB/s;
cpu_baseline = the CPU oracle timed on a bounded slab of the same field.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QAI post-pass GB/s of FP32 field and % HBM roofline, plain vs batched, 1 GPU"
HBM_PEAK_GBPS = 8000.0

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
    "clear": 0,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grf512_k11/3_eb1e-3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-regime", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="also time the 48-field uneven batch (graph launch vs per-field launches)")
    ap.add_argument("--grad", action="store_true",
                    help="also time forward + adjoint on the 256^3 field of the differentiable form")
    args = ap.parse_args()
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

    for _ in range(args.warmup):
        qai.mitigate(field, eb, out=out, workspace=ws)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")

    # copy-kernel bandwidth (the achievable HBM rate) on buffers of the field's size
    src = torch.empty(nvox, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    qai.copy_probe(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        qai.copy_probe(src, dst)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 10 * 8.0 * nvox / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    # timed region: K full post-passes, stage and step events on the launch stream
    qai.profile(True)
    qai.stage_times(reset=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    marks[0].record(stream)
    for k in range(args.steps):
        qai.mitigate(field, eb, out=out, workspace=ws)
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    step_ms = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps))
    trimmed = step_ms[1:-1] if len(step_ms) > 2 else step_ms
    stages = qai.stage_times(reset=True)
    qai.profile(False)
    ms_step = elapsed * 1e3 / args.steps
    value = 4.0 * nvox * args.steps / elapsed / 1e9
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, field {value:.1f} GB/s")

    per_launch = {k: v / args.steps for k, v in stages.items()}
    dom = max((k for k in per_launch if STAGE_BYTES.get(k, 0) > 0), key=lambda k: per_launch[k])
    dom_ms = per_launch[dom]
    dom_bytes = STAGE_BYTES[dom] * nvox
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    total_alg = sum(STAGE_BYTES.get(k, 0) for k in per_launch) * nvox
    stage_sum_ms = sum(per_launch.values())
    for k, v in per_launch.items():
        bw = STAGE_BYTES.get(k, 0) * nvox / (v * 1e-3) / 1e9 if v > 0 else 0.0
        log(f"  stage {k:16s} {v * 1e3:9.1f} us  {bw:8.1f} GB/s alg")

    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            with open(tfile) as fh:
                tr = json.load(fh)
            key = f"{args.workload}:{dom}"
            if key in tr and tr[key].get("kernel_rev") == kernel_rev():
                traffic = tr[key]["bytes_per_launch"]
        except Exception:
            traffic = None

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
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic, "kernel": dom,
                     "kernel_ms": round(dom_ms, 4), "alg_bytes_per_launch": dom_bytes},
        "pipeline": {"alg_bytes_per_voxel": total_alg // nvox,
                     "alg_GBps": round(total_alg / (ms_step * 1e-3) / 1e9, 1),
                     "frac_of_peak": round(total_alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                     "frac_of_copy": round(total_alg / (ms_step * 1e-3) / 1e9 / copy_gbps, 4),
                     "copy_GBps": round(copy_gbps, 1), "stage_sum_ms": round(stage_sum_ms, 4),
                     "stages_us": {k: round(v * 1e3, 1) for k, v in per_launch.items()},
                     "step_ms_median": round(float(np.median(step_ms)), 4),
                     "step_ms_trimmed_mean": round(float(np.mean(trimmed)), 4)},
    }

    if not args.no_regime:
        res["regime"] = regime_stats(qai, field, x32, eb, dev)

    if args.grad:
        res["differentiable"] = bench_grad(qai, synth, dev, args.steps, args.warmup)
    if args.batched:
        del field, out, ws
        torch.cuda.empty_cache()
        res["batched"] = bench_batched(qai, synth, dev, max(3, args.steps // 4))

    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(xq, eb)

    print(json.dumps(res), flush=True)


def _time(fn, reps, stream):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def bench_grad(qai, synth, dev, steps, warmup):
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
    for _ in range(warmup):
        qai.mitigate(t, eb, out=out, workspace=ws)
        qai.backward(g, ws, t.shape, eb)
    fwd = _time(lambda: qai.mitigate(t, eb, out=out, workspace=ws), steps, s)
    bwd = _time(lambda: qai.backward(g, ws, t.shape, eb), steps, s)
    log(f"differentiable {name}: forward {fwd:.3f} ms, adjoint {bwd:.3f} ms")
    return {"workload": name, "voxels": n, "forward_ms": round(fwd, 4), "adjoint_ms": round(bwd, 4),
            "adjoint_GBps_alg": round(12.0 * n / (bwd * 1e-3) / 1e9, 1)}


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
    plan = qai.BatchPlan(fields, ebs, autotune=True)
    s = torch.cuda.current_stream()
    plan.launch()
    plan.launch_per_field()
    graph_ms = _time(plan.launch, reps, s)
    per_ms = _time(plan.launch_per_field, reps, s)
    tunes = {}
    for i, f in enumerate(fields):
        tunes.setdefault("x".join(map(str, f.shape)), plan.tuning(i))
    plan.close()
    log(f"batched: graph {graph_ms:.2f} ms, per-field launches {per_ms:.2f} ms")
    return {"fields": len(fields), "voxels": nvox, "graph_ms": round(graph_ms, 3), "per_field_ms": round(per_ms, 3),
            "value": round(4.0 * nvox / (graph_ms * 1e-3) / 1e9, 2), "unit": "GB/s",
            "per_field_GBps": round(4.0 * nvox / (per_ms * 1e-3) / 1e9, 2), "tuning": tunes}


def kernel_rev():
    """Hash of the kernel sources: traffic counters are only reused while it holds."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2602_20097_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


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


def cpu_baseline(xq, eb, target_s=15.0):
    """The CPU oracle, as it stands, on a bounded sample of the same field: a
    16-plane probe sets a z-slab that takes about target_s; when the whole
    field takes less, the whole field is run repeatedly for about target_s."""
    import oracle
    nz = xq.shape[0]
    oracle.qai(xq[: min(nz, 2)], eb)  # load / build outside the timing
    probe = xq[: min(nz, 16)]
    t = time.perf_counter()
    oracle.qai(probe, eb)
    per_plane = (time.perf_counter() - t) / probe.shape[0]
    planes = int(min(nz, max(16, target_s / max(per_plane, 1e-9))))
    slab = xq[:planes]
    reps, dt = 0, 0.0
    while reps == 0 or (planes == nz and dt < target_s and reps < 64):
        t = time.perf_counter()
        oracle.qai(slab, eb)
        dt += time.perf_counter() - t
        reps += 1
    gbps = 4.0 * slab.size * reps / dt / 1e9
    what = "the whole field" if planes == nz else f"z-slab {list(slab.shape)} ({planes}/{nz} planes)"
    return {"value": round(gbps, 5), "unit": "GB/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{what}, {reps} run(s), {slab.size * reps} voxels in total; full Algorithm 4 in FP64 "
                      f"C/OpenMP with every intermediate kept, {dt:.2f} s",
            "seconds": round(dt, 3), "mb_per_s": round(gbps * 1e3, 2)}


if __name__ == "__main__":
    main()
