"""Benchmark of the dynamic EM ray tracer on the 2x2 km city workload.

A step is one discovery frame of the whole hot path: per-frame geometry
(moving vehicles, dynamic LBVH rebuild, receiver and edge LBVHs), 16 Tx x 1M
rays traced through K = 5 bounces with receiver and edge capture, the
discovered keys merged with the path cache, exact validation of every
candidate plus line of sight for all 160,000 links, field evaluation at two
carriers and the per-link reduction.  value = primary rays per step / step
time (Mrays/s).  Inputs are synthetic (seeded generator) and resident on the
GPU before the timed region starts.

Prints one JSON line.  Extra keys: cached-frame and 10-frame-schedule
ms/frame (the paper's Table II analogue), the roofline of the dominant kernel
(the bounce kernel; its HBM traffic comes from the committed counter summary
profiles/k_bounce_city_traffic.txt while the kernel sources are unchanged),
the oracle timed on the host cores, the adjoint against the plain forward
step (8-material district) and 64 uneven cities stepped as one batch against
the same cities stepped one after the other.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32, published (packed)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # without packed FP32 instructions, which this library does not use
# Counted work of the closest-hit traversal, FP32 operations as the code performs them (fma = 2):
FLOP_PER_NODE = 34  # binary node (dynamic tree): two boxes x (6 fma + 4 min/max + 1 scale)
FLOP_PER_WIDE_BOX = 29  # child box of a 4-wide node (static tree): 6 fma decode + 6 fma + 4 min/max + 1 scale
FLOP_PER_TRI = 35  # watertight triangle test (shear, edge functions, determinant, distance)


def committed_traffic():
    """HBM bytes per bounce launch from the committed counter summary, or
    None when the bounce kernel's sources (or the builder of the trees it
    reads) changed since it was measured."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_bounce_city_traffic.txt")
    try:
        kv = dict(ln.split(": ", 1) for ln in open(path).read().splitlines() if ": " in ln and ln[0].isalpha())
        m = hashlib.sha256()
        for f in ("trace.hip", "emrt_dev.h", "bvh.hip"):
            m.update(open(os.path.join(ROOT, "paper_2303_10521_amd", "csrc", f), "rb").read())
        if m.hexdigest() != kv.get("kernel_source_sha256", "").strip():
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _ev_ms(torch, fn, reps, stream=None):
    """Mean device time of fn() over reps calls (events on the stream)."""
    stream = stream or torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_adjoint(torch, np, reps: int = 3) -> dict:
    """Adjoint vs plain forward on the 8-material district: one discovery
    step forward, then emrt_backward of a loss of every link's H and P_coh."""
    from paper_2303_10521_amd import Tracer
    from synth import workload

    w = workload("adjoint")
    sc = w.scene
    fr = sc.frame(0.0)
    kw = dict(freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections, rays_per_tx=w.rays_per_tx,
              diffraction=int(w.diffraction), diff_max_leg_m=w.diff_max_leg, path_capacity=1 << 22)
    plain = Tracer(sc, sc.n_tx, sc.n_rx, **kw)
    plain_bytes = plain.workspace.numel()
    plain.close()
    tr = Tracer(sc, sc.n_tx, sc.n_rx, adjoint_materials=len(sc.materials), **kw)
    tr.set_frame(fr)
    nf, nl = len(w.freqs_hz), sc.n_tx * sc.n_rx
    rng = np.random.default_rng(0)
    GH = torch.as_tensor(rng.normal(size=(nf, nl)) + 1j * rng.normal(size=(nf, nl))).cuda()
    GP = torch.as_tensor(rng.normal(size=(nf, nl))).cuda()
    tr.step(True)
    tr.backward(GH, GP)
    fwd = _ev_ms(torch, lambda: tr.step(True), reps)
    bwd = _ev_ms(torch, lambda: tr.backward(GH, GP), reps)
    st = tr.stats()
    out = {
        "workload": f"district with 8 materials: {len(sc.tris)} triangles, {sc.n_tx} Tx x {w.rays_per_tx} rays, "
                    f"{sc.n_rx} Rx, K={w.max_reflections}, diffraction",
        "forward_ms": round(fwd, 3),
        "backward_ms": round(bwd, 3),
        "backward_over_forward": round(bwd / fwd, 4),
        "valid_paths": int(st["n_valid"]),
        "workspace_bytes": int(tr.workspace.numel()),
        "plain_workspace_bytes": int(plain_bytes),
    }
    tr.close()
    return out


def bench_batched(torch, reps: int = 3) -> dict:
    """64 uneven cities: one batched discovery step (multi-scene bounce
    launches, graph replay, autotuned launch shape) vs the 64 cities stepped
    one after the other."""
    from paper_2303_10521_amd import Batch, Tracer
    from synth.city import batch_city

    ws = [batch_city(i) for i in range(64)]
    trs = []
    for w in ws:
        sc = w.scene
        trs.append(Tracer(sc, sc.n_tx, sc.n_rx, freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections,
                          rays_per_tx=w.rays_per_tx, diffraction=int(w.diffraction), path_capacity=1 << 20))
        trs[-1].set_frame(sc.frame(0.0))
    rays = sum(w.rays_per_tx * w.scene.n_tx for w in ws)

    def plain_step():
        for t in trs:
            t.step(True)

    plain_step()
    plain_ms = _ev_ms(torch, plain_step, reps)
    b = Batch(trs)
    tune = b.autotune(repeats=3, cache=os.environ.get("EMRT_TUNE_CACHE"))
    b.step(True)
    batched_ms = _ev_ms(torch, lambda: b.step(True), reps, b.stream)
    rc = b.sync()
    b.close()
    for t in trs:
        t.close()
    return {
        "cities": len(ws),
        "rays_per_step": int(rays),
        "plain_ms_per_step": round(plain_ms, 3),
        "batched_ms_per_step": round(batched_ms, 3),
        "plain_mrays_s": round(rays / (plain_ms * 1e-3) / 1e6, 3),
        "batched_mrays_s": round(rays / (batched_ms * 1e-3) / 1e6, 3),
        "speedup": round(plain_ms / batched_ms, 3),
        "grid": tune["grid"],
        "streams": tune["streams"],
        "chunk": tune["chunk"],
        "tuned": "cache" if tune["from_cache"] else f"timed ({tune['repeats']} repeats per combination, median)",
        "status": rc,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="city")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=200, help="oracle traces every n-th launch direction")
    ap.add_argument("--timed-only", action="store_true", help="skip extra measurements (for profiler runs)")
    ap.add_argument("--no-extras", action="store_true", help="skip the adjoint and batched measurements")
    ap.add_argument("--cached-only", action="store_true",
                    help="time cached (revalidation) frames only, after one discovery frame (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 1 GiB device-to-device before the warm-up (reference dispatch for HBM counters)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint measurement (8-material district; for profiler runs)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched measurement (64 cities; for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (the path is not sharded "
                                   "across GPUs)"}))
        return 2

    import numpy as np
    import torch

    from paper_2303_10521_amd import Tracer
    from synth import workload

    if args.adjoint_only:
        if args.calibrate_copy:
            src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
        print(json.dumps({"mode": "adjoint only", "adjoint": bench_adjoint(torch, np, reps=1)}))
        return 0
    if args.batched_only:
        print(json.dumps({"mode": "batched only", "batched": bench_batched(torch)}))
        return 0

    w = workload(args.workload)
    sc = w.scene
    n_frames = max(args.steps + args.warmup, 12)
    frames = [sc.frame(i * w.frame_dt) for i in range(n_frames)]
    tr = Tracer(sc, sc.n_tx, sc.n_rx, freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections,
                rays_per_tx=w.rays_per_tx, diffraction=int(w.diffraction), diff_max_leg_m=w.diff_max_leg,
                path_capacity=1 << 23)
    stream = torch.cuda.current_stream()
    rays = sc.n_tx * w.rays_per_tx

    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.cached_only:
        tr.set_frame(frames[0], 0)
        tr.step(True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(args.steps):
            f = 1 + k % (n_frames - 1)
            tr.set_frame(frames[f], f)
            tr.step(False)
        e1.record(stream)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "cached frames", "steps": args.steps,
                          "ms_per_frame_cached": round(e0.elapsed_time(e1) / args.steps, 3),
                          "cache_keys": int(tr.stats()["n_cache"])}))
        return 0

    # warmup
    for i in range(args.warmup):
        tr.set_frame(frames[i], i)
        tr.step(True)
    torch.cuda.synchronize()

    # timed discovery steps, kernel events on the library stream
    tr.set_instrumentation(stats=False, timing=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        f = args.warmup + k
        tr.set_frame(frames[f], f)
        tr.step(True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    st = tr.stats()  # kernel events recorded on the library stream during the timed steps
    bounce_ms, bounce_launches, validate_ms = st["bounce_ms"], st["bounce_launches"], st["validate_ms"]
    tr.set_instrumentation(stats=False, timing=False)
    value = rays / (ms_per_step * 1e-3) / 1e6

    out = {
        "metric": "Mrays/s and ms/frame (2x2 km, 10k Rx); batched & adjoint vs plain",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 geometry / f64 fields",
        "data": "synthetic (seeded Manhattan-grid generator)",
        "config": {
            "workload": f"{args.workload}: {2 * sc.extent / 1000:.0f}x{2 * sc.extent / 1000:.0f} km grid, "
                        f"{len(sc.tris)} triangles, {sc.n_dynamic} moving vehicles, {sc.n_tx} Tx x "
                        f"{w.rays_per_tx} rays, {sc.n_rx} Rx, K={w.max_reflections}, "
                        f"diffraction={int(w.diffraction)}, {len(w.freqs_hz)} carriers",
            "rays_per_step": rays,
            "step": "discovery frame",
            "wall_s": round(wall, 3),
        },
    }

    if not args.timed_only:
        # counted traversal work of the same steps (instrumented, untimed)
        tr.set_instrumentation(stats=True, timing=False)
        nodes = boxes = tris = segs = 0
        for k in range(args.steps):
            f = args.warmup + k
            tr.set_frame(frames[f], f)
            tr.step(True)
            st = tr.stats()
            nodes += st["node_visits"]
            boxes += st["wide_box_tests"]
            tris += st["tri_tests"]
            segs += st["segments"]
        tr.set_instrumentation(stats=False, timing=False)
        flops = FLOP_PER_NODE * nodes + FLOP_PER_WIDE_BOX * boxes + FLOP_PER_TRI * tris
        achieved = flops / (bounce_ms * 1e-3) / 1e12 if bounce_ms > 0 else 0.0
        out["roofline"] = {
            "kernel": "k_bounce (closest hit + receiver/edge capture + reflect + compaction)",
            "bound": "alu",
            "limiter": "latency of divergent traversal (dependent node loads; VALU issue about 80% of slots, 61% of lanes active)",
            "achieved": round(achieved, 4),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 5),
            "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 5),
            "traffic": committed_traffic(),
            "avg_launch_ms": round(bounce_ms / max(bounce_launches, 1), 4),
            "flops_per_launch": int(flops / max(bounce_launches, 1)),
            "segments_per_step": int(segs / args.steps),
            "wide_box_tests_per_segment": round(boxes / max(segs, 1), 2),
            "node_visits_per_segment": round(nodes / max(segs, 1), 2),
            "tri_tests_per_segment": round(tris / max(segs, 1), 2),
            "static_tree_area": round(float(st["static_tree_area"]), 2),
        }
        out["validate_ms_per_step"] = round(validate_ms / args.steps, 3)
        out["bounce_ms_per_step"] = round(bounce_ms / args.steps, 3)

        # cached frames and the 10-frame schedule (1 discovery + 9 cached)
        tr.set_frame(frames[0], 0)
        tr.step(True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for f in range(1, 10):
            tr.set_frame(frames[f], f)
            tr.step(False)
        e1.record(stream)
        torch.cuda.synchronize()
        cached_ms = e0.elapsed_time(e1) / 9
        out["ms_per_frame_cached"] = round(cached_ms, 3)
        out["ms_per_frame_schedule10"] = round((ms_per_step + 9 * cached_ms) / 10, 3)
        out["discovery_over_cached"] = round(ms_per_step / cached_ms, 2)

    if not args.no_cpu_baseline and not args.timed_only:
        from oracle import oracle as orc

        os_ = orc.OracleScene(sc)
        fr = frames[0]
        g = os_.geometry(fr.obj_xform)
        ids = np.arange(0, w.rays_per_tx, args.cpu_stride, dtype=np.int32)
        t = time.perf_counter()
        n = 0
        for tx in range(sc.n_tx):
            orc.trace(os_, g, fr.tx_pos[tx], w.rays_per_tx, ids, w.max_reflections, fr.rx_pos, 1.0,
                      bool(w.diffraction), want_robust=False)
            n += len(ids)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": round(n / dt / 1e6, 6),
            "unit": "Mrays/s",
            "cores": orc.num_threads(),
            "kind": "oracle",
            "sample": f"every {args.cpu_stride}th launch direction of each of the {sc.n_tx} transmitters "
                      f"({n} rays, K={w.max_reflections}, brute-force closest hit, receiver and edge capture; "
                      f"{dt:.1f} s)",
        }
    tr.close()
    if not args.timed_only and not args.no_extras:
        out["adjoint"] = bench_adjoint(torch, np)
        out["batched"] = bench_batched(torch)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
