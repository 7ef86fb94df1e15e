"""Benchmark of one REFINE prune step on one MI355X.

A step is the whole path on one batch: refine_stats -> refine_score ->
refine_select -> refine_compact, enqueued on one stream, on the medium
synthetic workload (3M Gaussians x 200 cameras, prune ratio 0.5), inputs
resident in HBM before timing starts.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload medium]
                  [--no-cpu-baseline]

value = Gaussian-view evaluations per second of the whole step
(N * |V| / step time); ms_per_step is the time of one 3M-Gaussian prune.
The roofline object describes refine_score (the dominant launch), timed
with HIP events on its own stream over the timed region.  cpu_baseline
times the FP64 CPU oracle on the host's cores on the same workload.
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

# Algorithmic work of the scoring, per (primitive, view) pair and per
# primitive (FLOP; FMA = 2, mul/add/rcp/sqrt = 1, compares/min/max = 0), and
# bytes per primitive (14 fp32 attribute planes read, one fp32 score written).
FLOP_PER_PAIR = {0: 103, 1: 25, 2: 22}
# a pair screened out after its first step: camera-space centre 18, d z 4, bound 1
FLOP_PER_SCREENED_PAIR = 23
BYTES_PER_PRIM = 14 * 4 + 4
PEAK_FP32_TFLOPS = 157.3      # MI355X dense FP32 vector, vendor figure
# VALU issue: 256 CU x 4 SIMD x 2.4 GHz / 2 cycles per wave64 FP32 instruction
# (the same hardware rate that gives 157.3 TFLOP/s with FMAs)
PEAK_VALU_GINSTS = 1228.8
PEAK_HBM_GBS = 8000.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


# Sources of the view-loop kernels: HBM traffic measured with rocprofv3
# counters is reported only while these are unchanged.
KERNEL_SOURCES = ("paper_2606_09074_amd/csrc/score.hip", "paper_2606_09074_amd/csrc/refine_internal.hpp")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_counters(kernel: str, workload: str) -> dict:
    """Per-launch counter figures of `kernel` on `workload` from the committed
    summary profiles/<kernel>_<workload>_traffic.md: HBM bytes (FETCH_SIZE x
    2.0 + WRITE_SIZE x 1.0, see profiles/copy-1GiB_traffic-calibration.md)
    and VALU instructions (SQ_INSTS_VALU).  Empty when there is no summary or
    the kernel sources changed after it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return {}
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                if k.strip() in ("sources_sha256", "hbm_bytes_per_launch", "valu_insts_per_launch"):
                    fields[k.strip()] = v.strip().strip("`")
    if fields.pop("sources_sha256", None) != kernel_sources_sha256():
        return {}
    out = {}
    for k, v in fields.items():
        try:
            out[k] = int(v)
        except ValueError:
            pass
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="medium", choices=["small", "medium", "large"])
    ap.add_argument("--ratio", type=float, default=None)
    ap.add_argument("--score-path", default="auto", choices=["auto", "direct", "binned"],
                    help="refine_score scheduling (results are bit-identical across paths)")
    ap.add_argument("--records-per-lane", type=int, default=0, choices=[0, 1, 2],
                    help="binned records each lane of the view loop holds (0: the library's default)")
    ap.add_argument("--views-per-iteration", type=int, default=0, choices=[0, 1, 2],
                    help="views the binned view loop evaluates per iteration (0: the library's default)")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16-f16"],
                    help="scene storage: FP32 planes, or BF16 geometry/opacity + FP16 SH (arithmetic is FP32 either way)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=240,
                    help="prune jobs per storage format in the served-latency run (0: skip it)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate of the served jobs (1/s)")
    ap.add_argument("--serve-slots", type=int, default=4, help="jobs in flight at once (one HIP stream each)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 times) and exit: the reference "
                         "kernel for scaling HBM traffic counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: this build runs the path on a single MI355X "
              f"(--gpus {args.gpus} requested); the multi-GPU sharding is described in DESIGN.md",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2606_09074_amd import _lib, api, synth

    _lib.load()
    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        return 2
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)
        return 0
    spec = synth.SPECS[args.workload]
    ratio = args.ratio if args.ratio is not None else spec.ratios[0]
    log(f"bench: generating {spec.name} (n={spec.n}, V={spec.n_views}), ratio {ratio}")
    planes_np = synth.make_planes(spec)
    cams_np = synth.make_cameras(spec)
    if args.storage == "bf16-f16":
        stored_np = synth.quantize_bf16_f16(planes_np)
        planes_np = synth.dequantize_bf16_f16(stored_np)   # the values the 2-byte scene holds
    else:
        stored_np = planes_np
    n, V = spec.n, cams_np.shape[0]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    planes = torch.from_numpy(stored_np).to(dev)
    cams = torch.from_numpy(cams_np).to(dev)
    params = _lib.default_params()
    params.score_path = {"auto": _lib.PATH_AUTO, "direct": _lib.PATH_DIRECT, "binned": _lib.PATH_BINNED}[args.score_path]
    params.records_per_lane = args.records_per_lane
    params.views_per_iteration = args.views_per_iteration
    ws = api.workspace(n, V, dev)
    st = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
    scores = torch.empty(n, dtype=torch.float32, device=dev)
    keep = torch.empty(n, dtype=torch.uint8, device=dev)
    n_keep = torch.empty(1, dtype=torch.int64, device=dev)
    cap = n - api.prune_count(n, ratio)
    out = torch.empty((59, max(cap, 1)), dtype=planes.dtype, device=dev)
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    phases = ("stats", "prepare", "views", "select", "compact")
    n_ev = max(args.steps, 1)
    ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_ev)]
          for k in phases}

    def step(j: int | None, marked=("views",)):
        def mark(k, e):
            if j is not None and k in marked:
                ev[k][j][e].record(stream)
        mark("stats", 0)
        api.refine_stats(planes, st, ws, params, stream=stream)
        mark("stats", 1)
        mark("prepare", 0)
        api.refine_score_prepare(planes, cams, st, ws, params, stream=stream)
        mark("prepare", 1)
        mark("views", 0)
        api.refine_score_views(planes, V, st, scores, ws, params, stream=stream)
        mark("views", 1)
        mark("select", 0)
        api.refine_select(scores, keep, ws, ratio=ratio, n_keep_out=n_keep, stream=stream)
        mark("select", 1)
        mark("compact", 0)
        api.refine_compact(planes, keep, out, ws, index_map_out=idx, capacity=cap, stream=stream)
        mark("compact", 1)

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    log(f"bench: warmup done ({args.warmup} steps); timing {args.steps} steps")

    # timed region: wall clock around K steps; HIP events on the launch stream
    # bracket the view loop (the dominant kernel) in every step
    t0 = time.perf_counter()
    for j in range(args.steps):
        step(j)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    views_ms = [a.elapsed_time(b) for a, b in ev["views"][:args.steps]]
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n * V / (ms_per_step / 1e3)

    # per-phase breakdown from a separate, untimed pass with events around every call
    for j in range(args.steps):
        step(j, marked=phases)
    torch.cuda.synchronize()
    avg = {k: float(np.mean([a.elapsed_time(b) for a, b in ev[k][:args.steps]])) for k in phases}
    avg["views"] = float(np.mean(views_ms))
    log(f"bench: {ms_per_step:.3f} ms/step, phases {avg}")

    # pairs the view loop evaluated in full, and pairs it screened out after
    # their first step (culled pairs are in neither), read once after the timed region
    evaluated = torch.zeros(2, dtype=torch.int64, device=dev)
    api.refine_score_views(planes, V, st, scores, ws, params, evaluated_out=evaluated, stream=stream)
    torch.cuda.synchronize()
    n_eval, n_screened = (int(x) for x in evaluated.cpu().tolist())

    # roofline of the view loop (the dominant kernel): ALU-bound FP32 work it
    # actually performed, over its event-timed duration
    t_views = avg["views"] / 1e3
    flops = FLOP_PER_PAIR[params.proj_mode] * n_eval + FLOP_PER_SCREENED_PAIR * n_screened
    achieved_tflops = flops / t_views / 1e12
    kname = "score_binned" if n_eval < n * V else "score_direct"
    counters = profiled_counters(kname, spec.name) if params.proj_mode == 0 else {}
    traffic = counters.get("hbm_bytes_per_launch")
    valu = counters.get("valu_insts_per_launch")
    valu_issue = None
    if valu:
        rate = valu / t_views / 1e9
        valu_issue = {"insts_per_launch": valu, "achieved": round(rate, 1), "peak": PEAK_VALU_GINSTS,
                      "unit": "G wave-instructions/s", "frac": round(rate / PEAK_VALU_GINSTS, 4)}
    roofline = {"bound": "alu", "kernel": kname,
                "achieved": round(achieved_tflops, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4), "traffic": traffic, "valu_issue": valu_issue,
                "flop_per_pair": FLOP_PER_PAIR[params.proj_mode], "pairs_evaluated": n_eval,
                "flop_per_screened_pair": FLOP_PER_SCREENED_PAIR, "pairs_screened": n_screened,
                "pairs_total": n * V, "views_ms": round(avg["views"], 4), "prepare_ms": round(avg["prepare"], 4)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("bench: timing the FP64 CPU oracle on the same workload")
        oracle.build(force=False)
        prm = oracle.Params()
        tc0 = time.perf_counter()
        F = oracle.stats(planes_np, eta=prm.eta)
        lam = oracle.lam(F, prm)
        D, _, _, _ = oracle.score(planes_np, cams_np, lam, prm)
        keep_o, _ = oracle.select(D, oracle.n_prune(n, ratio))
        oracle.compact(planes_np, keep_o)
        tc = time.perf_counter() - tc0
        cpu = {"value": round(n * V / tc, 1), "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"full {spec.name} prune (stats+score+select+compact), {tc:.2f} s",
               "ms_per_prune": round(tc * 1e3, 1)}

    serving = serve_bench(args) if args.serve_jobs > 0 else None

    line = {"metric": "Gaussian-view evals/s", "value": round(value, 1), "unit": "evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": spec.name, "n": n, "views": V, "ratio": ratio, "storage": args.storage,
                       "step": "stats+score+select+compact", "score_path": args.score_path, "records_per_lane": args.records_per_lane,
                       "views_per_iteration": args.views_per_iteration,
                       "ms_per_prune": round(ms_per_step, 4)},
            "phases_ms": {k: round(v, 4) for k, v in avg.items()},
            "roofline": roofline, "cpu_baseline": cpu, "serving": serving}
    print(json.dumps(line), flush=True)
    return 0


def serve_bench(args) -> dict:
    """Served latency: Poisson arrivals of prune jobs on resident, prepared
    scenes (paper_2606_09074_amd.serve), once with FP32 scenes and once with
    the same scenes in 2-byte storage, once more with FP32 scenes where every
    job runs the whole path, then a burst of the same jobs with and without
    overlap.  Latency = completion seen by the host - arrival time."""
    import numpy as np
    import torch

    from paper_2606_09074_amd import serve, synth
    dev = torch.device("cuda:0")
    specs = synth.serve_scene_specs(8)
    log(f"serve: generating {len(specs)} resident scenes, n = {[sp.n for sp in specs]}")
    f32, b16 = [], []
    for sp in specs:
        pl = synth.make_planes(sp)
        f32.append(torch.from_numpy(pl).to(dev))
        b16.append(torch.from_numpy(synth.quantize_bf16_f16(pl)).to(dev))
    arrivals, reqs = synth.serve_requests(args.serve_jobs, len(specs), rate=args.serve_rate)
    cams = {}
    for _, V, _ in reqs:
        if V not in cams:
            cams[V] = torch.from_numpy(synth.ring_cameras(V)).to(dev)
    torch.cuda.synchronize()

    tuner = serve.Tuner()
    buckets = sorted({(serve.bucket_of(sp.n, V)) for sp in specs for V in (64, 128, 256)})
    tuner.tune(f32[-1], lambda V: torch.from_numpy(synth.ring_cameras(V)).to(dev), buckets, reps=3)
    log(f"serve: tuned {len(buckets)} buckets: {sorted(tuner.table.items())}")

    def run(scenes, arr, slots, prepare=True, pack=True):
        srv = serve.Server(dev, slots=slots, tuner=tuner, prepare_scenes=prepare,
                           pack_max_n=(1 << 20) if pack else 0)
        for t in scenes:
            srv.add_scene(t)
        # warm the allocator and the kernels on every scene
        for j in range(len(scenes)):
            srv.submit(j, cams[reqs[0][1]], 0.5)
        srv.drain()
        keeps = {}

        def done(job):
            keeps[job.id] = job.keep[:job.n]
            job.out = job.index_map = job.scores = None
        jobs = [(sc, cams[V], r) for sc, V, r in reqs]
        t0 = time.perf_counter()
        fin = serve.run_open_loop(srv, jobs, arr, on_done=done)
        span = time.perf_counter() - t0
        torch.cuda.synchronize()
        lat = [j.latency * 1e3 for j in fin]
        dev_ms = [j.device_ms for j in fin]
        first = min(j.id for j in fin)
        order = [keeps[first + i] for i in range(len(fin))]
        evals = sum(scenes[sc].shape[1] * V for sc, V, _ in reqs)
        return {"p50_ms": round(serve.percentile(lat, 0.5), 3), "p99_ms": round(serve.percentile(lat, 0.99), 3),
                "mean_ms": round(float(np.mean(lat)), 3), "max_ms": round(float(np.max(lat)), 3),
                "device_p50_ms": round(serve.percentile(dev_ms, 0.5), 3),
                "device_p99_ms": round(serve.percentile(dev_ms, 0.99), 3),
                "jobs_per_s": round(len(fin) / span, 2), "evals_per_s": round(evals / span, 1)}, order

    log(f"serve: {len(reqs)} jobs at {args.serve_rate}/s, FP32 scenes")
    r32, k32 = run(f32, arrivals, args.serve_slots)
    log(f"serve: same jobs, BF16/FP16 scenes")
    r16, k16 = run(b16, arrivals, args.serve_slots)
    log(f"serve: same jobs, FP32 scenes, every job on the whole path (no prepared scenes)")
    r32u, _ = run(f32, arrivals, args.serve_slots, prepare=False)
    jac = []
    for a, b in zip(k32, k16):
        a, b = a.bool(), b.bool()
        jac.append(float((a & b).sum().item()) / max(float((a | b).sum().item()), 1.0))
    burst = np.zeros(len(reqs))
    log("serve: burst (all jobs at once), with and without overlap")
    b4, _ = run(f32, burst, args.serve_slots)
    b4n, _ = run(f32, burst, args.serve_slots, pack=False)
    b1, _ = run(f32, burst, 1, pack=False)
    # the same jobs on small resident scenes (20k..200k Gaussians), where
    # launches rather than arithmetic set the pace: packed vs one launch
    # sequence per job
    small_specs = synth.serve_scene_specs(8, n_range=(20_000, 200_000))
    small = [torch.from_numpy(synth.make_planes(sp)).to(dev) for sp in small_specs]
    log("serve: burst on small scenes, packed and unpacked")
    s4, _ = run(small, burst, args.serve_slots)
    s4n, _ = run(small, burst, args.serve_slots, pack=False)
    return {"workload": "resident scenes n=0.25M..4.9M (log-uniform strata), 50..300 ring views, ratio 0.3..0.9",
            "jobs": len(reqs), "rate_per_s": args.serve_rate, "slots": args.serve_slots,
            "latency_clock": "host: arrival to observed completion",
            "f32": r32, "bf16_f16": r16, "f32_whole_path": r32u,
            "kept_jaccard_bf16_vs_f32": {"min": round(min(jac), 5), "mean": round(float(np.mean(jac)), 5)},
            "burst": {"slots": args.serve_slots, "jobs_per_s": b4["jobs_per_s"], "evals_per_s": b4["evals_per_s"],
                      "unpacked_jobs_per_s": b4n["jobs_per_s"], "one_slot_unpacked_jobs_per_s": b1["jobs_per_s"]},
            "burst_small_scenes": {"n": "20k..200k", "packed_jobs_per_s": s4["jobs_per_s"],
                                   "unpacked_jobs_per_s": s4n["jobs_per_s"]}}


if __name__ == "__main__":
    sys.exit(main())
