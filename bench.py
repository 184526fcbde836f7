"""Throughput of one forward+backward rendering step on one MI355X.

A step is the whole rendering path for one camera: collection pass
(preprocess, depth sort, tile binning and sort, raster), texturing pass
(hash grid + MLP + composite), the L2 image-loss gradient, and the backward
of both passes (hash-grid, MLP and surfel gradients). Inputs are resident in
HBM before the timed region.

Workload: 400k surfels (ground plane + 50 boxes, depths 0.5-50 m, scales
spanning three decades), 1920x1080, K=4, hash grid 16 x 2^19 x 2,
MLP 32-64-64-3. The headline form stores the grid in FP16 and runs the MLP
on BF16 matrix cores; the FP32 form (FP32 grid, FP32 matrix cores) is timed
beside it.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpix/s fwd+bwd at 400k surfels 1080p K=4 (BF16 vs FP32); % HBM roofline"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3}  # dense matrix peaks of the MI355X per operand type
# VALU peak: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz = 39.3e12 lane-instructions/s (packed FP32 is off)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane-instructions per (pixel, surfel) pair the collection pass tests, from SQ_INSTS_VALU x 64 over the
# tested pairs of the 1080p frame: the forward evaluates the pair (27 on the gamma = 1 path up to the alpha
# threshold) and updates the K-buffer and colour of composited pairs; the backward re-evaluates the pair, forms
# its 16 record gradients and sums them across the wave once per surfel.
RASTER_OPS_PER_PAIR = {"raster_forward": 38, "raster_backward": 76}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def method_work(phase, st):
    """(bound, HBM bytes, matrix flops, VALU lane-ops) the launches of `phase` in one step must move / compute.

    Bytes count what the method reads and writes: each input once and each output once at its storage width,
    the hash table once per camera (its re-reads are cache traffic), atomically updated buffers as a read and a
    write, and the binning and sort arrays the tile rasteriser needs. They do not count this design's own
    intermediates (the per-level feature gradients and the hash-scatter records); those appear only in the
    measured traffic. Per-surfel kernels run once per camera (C cameras)."""
    N, C, P, K, I, T = st["N"], st["C"], st["P"], st["K"], st["I"], st["n_tiles"]
    S = P * K
    L = st["L"]
    table = L * st["T"] * st["F"] * st["tb"]
    gtable = L * st["T"] * st["F"] * 4
    mlp_flops = 2.0 * S * (st["in"] * st["H"] + st["H"] * st["H"] + 3 * st["H"])
    rec = 80
    pairs = st["pairs"]
    hbm = {
        "preprocess": C * N * (60 + 4 + 4 + 16 + rec),
        "depth_sort": C * N * (8 + 4 * 16),
        "instance_scan": C * N * 12,
        "duplicate": C * N * 24 + I * 8,
        "tile_sort": I * 16 * st["tile_passes"],
        "tile_ranges": I * 4 + T * 8,
        "raster_forward": I * (4 + rec) + T * 8 + P * (12 + 12 * K + 8),
        "texture_forward": S * 12 + P * 24 + C * table,
        "zero_record_grads": C * N * 64,
        "texture_backward": S * 16 + P * 12 + C * table,
        # the table gradient: each level's slice read and written once
        "hash_backward": 2 * gtable,
        "raster_backward": I * (4 + rec) + T * 8 + P * (28 + 24 * K) + C * N * 120,
        "preprocess_backward": C * N * (36 + 4 + 64 + 2 * 60),
    }
    flops = {"texture_forward": mlp_flops, "texture_backward": 3.0 * mlp_flops}
    valu = {k: pairs * v for k, v in RASTER_OPS_PER_PAIR.items()}
    bound = "mfma" if phase in flops else ("alu" if phase in valu else "hbm")
    return bound, float(hbm.get(phase, 0)), float(flops.get(phase, 0.0)), float(valu.get(phase, 0.0))


# Kernel phases that together form one method step of the table: the hash-grid gradient is one pass of the
# method (its bytes are the table slice) that this design splits over several launches.
PHASE_GROUPS = {"hash_backward": ("scatter_bin", "scatter_reduce")}


def rooflines(phases, steps, st, form):
    """Per method phase: bound, achieved vs peak, from the HIP-event time per step of its launches."""
    per_step = {k: v[0] / steps for k, v in phases.items()}
    launches = {k: v[1] // steps for k, v in phases.items()}
    for grp, members in PHASE_GROUPS.items():
        if any(m in per_step for m in members):
            per_step[grp] = sum(per_step.pop(m, 0.0) for m in members)
            launches[grp] = sum(launches.pop(m, 0) for m in members)
    out = {}
    for ph, ms in per_step.items():
        if ms <= 0:
            continue
        bound, nbytes, nflops, nvalu = method_work(ph, st)
        t = ms / 1000.0
        r = {"ms_per_step": round(ms, 4), "launches_per_step": int(launches[ph]),
             "hbm_gbs": round(nbytes / t / 1e9, 1), "hbm_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4),
             "bytes_per_step": nbytes}
        if nflops:
            peak = MFMA_PEAK_TFLOPS[form]
            r.update(mfma_tflops=round(nflops / t / 1e12, 2), mfma_peak=peak,
                     mfma_frac=round(nflops / t / 1e12 / peak, 4))
        if nvalu:
            r.update(valu_tops=round(nvalu / t / 1e12, 2), valu_frac=round(nvalu / t / 1e12 / VALU_PEAK_TOPS, 4))
        r["bound"] = bound
        out[ph] = r
    return out


def kernel_source_digest():
    """SHA-256 of the HIP sources with comments and blank lines removed (a comment edit does not change the
    kernels); hardware byte counts are only quoted for the code they were taken on."""
    import hashlib
    import re
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2512_13796_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".h")):
            t = open(os.path.join(src, name), encoding="utf-8").read()
            t = re.sub(r"/\*.*?\*/", "", t, flags=re.S)
            t = re.sub(r"//[^\n]*", "", t)
            h.update("\n".join(ln.rstrip() for ln in t.splitlines() if ln.strip()).encode())
    return h.hexdigest()


def measured_traffic(phase):
    """HBM bytes per launch of `phase` from the committed FETCH_SIZE / WRITE_SIZE profile (each scaled by the
    same counter's reading for a plain copy of known size), or None if there is none for the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    k = rec.get("phases", {}).get(phase)
    return None if k is None else k.get("bytes_per_launch")


WORKLOADS = {
    # name: (config, description)
    "outdoor": (3, "outdoor 400k surfels 1920x1080 K=4, grid 16x2^19x2 fp16, MLP 32-64-64-3 bf16"),
    "multiview": (4, "planes 300k surfels, 16 orbit cameras 640x480..1920x1080 in one call, K=4, grid 16x2^19x2 fp32, "
                     "MLP 32-64-64-3 fp32"),
    "large": (5, "outdoor 1M surfels 2560x1440 K=8, grid 16x2^21x2 bf16, MLP 32-128-128-3 bf16"),
}


def setup(form, workload="outdoor"):
    import torch

    import paper_2512_13796_amd as nx
    import scenes

    config = WORKLOADS[workload][0]
    if form == "fp32":
        wl = scenes.make_workload(config, feat_dtype=torch.float32, mlp_dtype=torch.float32)
    else:
        wl = scenes.make_workload(config)  # the workload's own storage dtypes
    dev = torch.device("cuda:0")
    surf = tuple(t.to(dev).contiguous() for t in wl.scene.tensors())
    table = wl.grid.table.to(dev).contiguous()
    weights = [w.to(dev).contiguous() for w in wl.mlp.weights]
    target = torch.cat([t.reshape(-1, 3) for t in wl.target]).to(dev).contiguous()
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype)
    z = lambda t: torch.zeros(t.shape, device=dev, dtype=torch.float32)
    grads = {"means": z(surf[0]), "quats": z(surf[1]), "scales": z(surf[2]), "opacities": z(surf[3]),
             "gammas": z(surf[4]), "colors": z(surf[5]), "table": z(table), "mlp": [z(w) for w in weights]}
    return nx, wl, ctx, surf, table, weights, target, grads


def make_step(nx, wl, ctx, surf, table, weights, target, grads):
    cams = wl.cameras if len(wl.cameras) > 1 else wl.cameras[0]
    P = sum(c.width * c.height for c in wl.cameras)
    scale = 2.0 / (3.0 * P)
    state = {}

    def step():
        res = nx.render_forward(ctx, surf, cams, table, wl.grid.level_scales, weights)
        g = (res.image - target).mul_(scale)
        for k, t in grads.items():
            if k == "mlp":
                for w in t:
                    w.zero_()
            else:
                t.zero_()
        nx.render_backward(ctx, surf, res, table, wl.grid.level_scales, weights, g, None, None, grads)
        state["res"] = res
        return res

    return step, state


def _median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def time_form(form, steps, warmup, workload="outdoor"):
    import torch

    nx, wl, ctx, surf, table, weights, target, grads = setup(form, workload)
    step, state = make_step(nx, wl, ctx, surf, table, weights, target, grads)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the collection pass's LDS batch, tuned for these cameras (untimed)
    batch = nx.autotune_raster(ctx, surf, state["res"], reps=3) if warmup > 0 else None
    ctx.timing(True)
    ctx.timing_reset()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        step()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev[0].elapsed_time(ev[-1]) / steps
    median = _median([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    phases = ctx.timings()
    ctx.timing(False)
    res = state["res"]
    cams = wl.cameras
    st = {"N": wl.scene.n, "C": len(cams), "P": sum(c.width * c.height for c in cams), "K": wl.K,
          "I": res.n_instances, "n_tiles": sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams),
          "L": wl.grid.levels, "T": 1 << wl.grid.log2_size, "F": wl.grid.feat, "tb": table.element_size(),
          "in": weights[0].shape[1], "H": weights[0].shape[0], "tile_passes": 2,
          "width": cams[0].width, "height": cams[0].height, "pairs": int(res.n_iter.to(torch.int64).sum()),
          "raster_batch": batch}
    st["workload_stats"] = workload_stats(res, wl, K=wl.K)
    return {"ms": ms, "ms_median": median, "wall_ms": 1000.0 * wall / steps, "phases": phases, "stats": st,
            "workload": wl}


def time_graph(form, steps, warmup, workload="outdoor"):
    """The same step captured once in a HIP graph (through torch.cuda.CUDAGraph) and replayed: the forward runs
    the sync-free entry point with this frame's per-camera instance count as its bound, so the whole step
    (forward, loss gradient, zeroing, backward) is one graph launch. The replays' outputs are checked against
    an eager step first."""
    import torch

    nx, wl, ctx, surf, table, weights, target, grads = setup(form, workload)
    cams = wl.cameras if len(wl.cameras) > 1 else wl.cameras[0]
    ls = wl.grid.level_scales
    P = sum(c.width * c.height for c in wl.cameras)
    scale = 2.0 / (3.0 * P)
    counts = nx.workspace_size_exact(ctx, surf, cams)[1]
    cap = max(counts)
    ws = torch.empty(nx.workspace_size(ctx, wl.scene.n, cams, cap), device="cuda", dtype=torch.uint8)
    state = {}

    def step():
        res = nx.render_forward(ctx, surf, cams, table, ls, weights, workspace=ws, max_instances=cap)
        g = (res.image - target).mul_(scale)
        for k, t in grads.items():
            for x in (t if k == "mlp" else [t]):
                x.zero_()
        nx.render_backward(ctx, surf, res, table, ls, weights, g, None, None, grads)
        state["res"] = res

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # eager warm-up off the default stream (creates the backward's streams)
        for _ in range(max(warmup, 1)):
            step()
        nx.autotune_raster(ctx, surf, state["res"], reps=3)
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = state["res"].image.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    res = state["res"]
    for _ in range(max(warmup, 1)):
        graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(res.image, eager), "graph replay differs from the eager step"
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        graph.replay()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1]) / steps
    median = _median([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    return {"ms_per_step": round(ms, 4), "ms_median": round(median, 4),
            "value": round(P / (ms / 1000.0) / 1e6, 2), "instances_bound_per_camera": cap}


def workload_stats(res, wl, K):
    """Per-frame statistics of the rendered workload (outside the timed region)."""
    import torch

    P = res.image.shape[0]
    n_iter = res.n_iter.to(torch.int64)
    out = {"instances": int(res.n_instances),
           "tiles_per_surfel": round(float(res.n_instances) / max(wl.scene.n * len(wl.cameras), 1), 3),
           "tested_pairs_per_pixel": round(float(n_iter.sum()) / P, 2)}
    if K > 0:
        filled = (res.ids[:, :K] >= 0).sum(dim=1)
        out["mean_selected_per_pixel"] = round(float(filled.double().mean()), 3)
        out["frac_pixels_under_K"] = round(float((filled < K).double().mean()), 4)
        out["mean_selected_weight"] = round(float(res.weights[:, :K].sum(dim=1).double().mean()), 4)
    out["mean_T_final"] = round(float(res.t_final.double().mean()), 4)
    return out


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sample_pixels=4096, seed=0):
    """The FP64 oracle, as it stands, on a bounded pixel sample of the same workload: one forward + backward
    call (every surfel tested per pixel) with a fixed upstream image gradient of the L2 loss's size."""
    import numpy as np
    import torch

    import oracle
    import scenes

    wl = scenes.make_workload(3)
    cam = wl.cameras[0]
    P = cam.width * cam.height
    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(P, sample_pixels, replace=False))
    g = rng.uniform(-1.0, 1.0, (sample_pixels, 3)) * (2.0 / (3.0 * P))
    t0 = time.perf_counter()
    oracle.render_and_grad(wl.scene, cam, wl.grid, wl.mlp, wl.K, pixels=pix, grad_image=g)
    dt = time.perf_counter() - t0
    return {"value": sample_pixels / dt / 1e6, "unit": "Mpix/s", "cores": torch.get_num_threads(),
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{sample_pixels} random pixels of the 1920x1080 400k-surfel frame, one forward+backward call "
                      f"of the FP64 oracle on {torch.get_num_threads()} threads: {dt:.1f} s",
            "full_frame_s_extrapolated": round(dt * P / sample_pixels, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip timing the step as a replayed HIP graph")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="outdoor",
                    help="outdoor (the headline: 400k surfels, 1080p), multiview (16 cameras in one call) or large "
                         "(1M surfels, 1440p, K=8, hidden 128); the last two print their own line without the FP32 "
                         "form and the CPU baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain elementwise copy of MIB MiB (read MIB, write MIB) three times, as the "
                         "reference for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the rendering path has no multi-GPU code); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    log(f"{args.workload} ...")
    bf = time_form("native", args.steps, args.warmup, args.workload)
    st = bf["stats"]
    P = st["P"]
    value = P / (bf["ms"] / 1000.0) / 1e6
    per_step = {k: v[0] / args.steps for k, v in bf["phases"].items()}
    form = {"outdoor": "bf16", "multiview": "f32", "large": "bf16"}[args.workload]
    roofs = rooflines(bf["phases"], args.steps, st, form)
    dom = max(roofs, key=lambda k: roofs[k]["ms_per_step"])
    rd = roofs[dom]
    launches = max(rd["launches_per_step"], 1)
    avg_s = rd["ms_per_step"] / 1000.0 / launches
    if rd["bound"] == "mfma":
        achieved, peak, unit = rd["mfma_tflops"], rd["mfma_peak"], "TFLOP/s"
    elif rd["bound"] == "alu":
        achieved, peak, unit = rd["valu_tops"], round(VALU_PEAK_TOPS, 2), "T VALU lane-ops/s"
    else:
        achieved, peak, unit = rd["hbm_gbs"], HBM_PEAK_GBS, "GB/s"
    roof = {"kernel": dom, "bound": rd["bound"], "achieved": achieved, "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 5),
            "traffic": measured_traffic(dom) if args.workload == "outdoor" else None,
            "avg_ms": round(avg_s * 1000.0, 4), "launches_per_step": launches,
            "algorithmic_bytes_per_launch": rd["bytes_per_step"] / launches}
    if rd["bound"] != "hbm":
        roof["hbm_frac"] = rd["hbm_frac"]
    cfg = {"workload": WORKLOADS[args.workload][1], "surfels": st["N"], "cameras": st["C"], "pixels": P,
           "K": st["K"], "instances": st["I"], "raster_lds_batch": st["raster_batch"], "stats": st["workload_stats"]}
    if st["C"] == 1:
        cfg.update(width=st["width"], height=st["height"])
    dtype = form
    line = {
        "metric": METRIC if args.workload == "outdoor" else "Mpix/s fwd+bwd",
        "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(bf["ms"], 4), "ms_median": round(bf["ms_median"], 4),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": cfg,
        "roofline": roof,
        "raster": {k: {f: roofs[k].get(f) for f in ("ms_per_step", "hbm_frac", "valu_frac")}
                   for k in ("raster_forward", "raster_backward") if k in roofs},
        "rooflines": roofs,
        "phases_ms_per_step": {k: round(v, 4) for k, v in sorted(per_step.items(), key=lambda kv: -kv[1])},
    }
    if not args.no_graph:
        log("graph replay ...")
        line["graph_replay"] = time_graph("native", args.steps, args.warmup, args.workload)
        if args.workload == "multiview":
            # the batched uneven views are measured as one replayed graph per step; the eager figure stays beside it
            line["eager"] = {"value": line["value"], "ms_per_step": line["ms_per_step"],
                             "ms_median": line["ms_median"]}
            for f in ("value", "ms_per_step", "ms_median"):
                line[f] = line["graph_replay"][f]
    if args.workload != "outdoor":
        args.no_fp32 = True
        args.no_cpu_baseline = True
    if not args.no_fp32:
        log("fp32 form ...")
        f32 = time_form("fp32", max(3, args.steps // 2), max(1, args.warmup // 2), args.workload)
        n32 = max(3, args.steps // 2)
        ph32 = {k: v[0] / n32 for k, v in f32["phases"].items()}
        r32 = rooflines(f32["phases"], n32, f32["stats"], "f32")
        line["fp32_form"] = {"value": round(P / (f32["ms"] / 1000.0) / 1e6, 2), "ms_per_step": round(f32["ms"], 4),
                             "phases_ms_per_step": {k: round(v, 4)
                                                    for k, v in sorted(ph32.items(), key=lambda kv: -kv[1])},
                             "mfma": {k: {f: r32[k].get(f) for f in ("mfma_tflops", "mfma_peak", "mfma_frac")}
                                      for k in ("texture_forward", "texture_backward") if k in r32}}
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        line["copy_calibration_mib"] = args.copy_calibration
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
