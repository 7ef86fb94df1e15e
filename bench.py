"""Benchmark of one REFINE prune step on one MI355X.

A step is the whole path on one batch: refine_stats -> refine_score ->
refine_select -> refine_compact, enqueued on one stream, on the medium
synthetic workload (3M Gaussians x 200 cameras, prune ratio 0.5), inputs
resident in HBM before timing starts.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload medium]
                  [--no-cpu-baseline]

value = Gaussian-view evaluations per second of the whole step
(N * |V| / step time); ms_per_step is the time of one 3M-Gaussian prune.
The roofline object describes the view loop (the dominant kernel, the one
launch of refine_score_views), timed with HIP events on its launch stream in
every timed step.  cpu_baseline times the FP64 CPU oracle on the host's
cores on the same workload (all threads, and one thread on a sample);
precision reports each 2-byte storage's prune time and its error against
that oracle; other_workloads the small (50k x 16) and large (6M x 300)
prunes; serving the served latencies (paper_2606_09074_amd.serve).
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

# Algorithmic work of the scoring per (primitive, view) pair (FLOP; FMA = 2,
# mul/add/rcp/sqrt = 1, compares/min/max = 0), from the per-pair ledger of
# the projected-covariance evaluation: transform 18, reciprocal 1, x/z and
# y/z 2, u and v 4, Jacobian 4, J R_v 18, (J R_v) L 30, a b c 15, largest
# eigenvalue and radius 11, footprint box 4, projection term 6, accumulate 1
# = 114 (the kernel's square-root-free gate executes a few less).  DEPTH
# and NONE modes change only the projection term (1/(z^2 + eta): 1 FLOP
# from the shared reciprocal; or 1): the gate still needs the projected
# covariance for the footprint radius.
FLOP_PER_PAIR = {0: 114, 1: 109, 2: 108}
# a pair screened out after its first step: camera-space centre 18, d z 4, bound 1
FLOP_PER_SCREENED_PAIR = 23
BYTES_PER_PRIM = 14 * 4 + 4
PEAK_FP32_TFLOPS = 157.3      # MI355X dense FP32 vector, vendor figure
# VALU issue: 256 CU x 4 SIMD x 2.4 GHz / 2 cycles per wave64 FP32 instruction
# (the same hardware rate that gives 157.3 TFLOP/s with FMAs)
PEAK_VALU_GINSTS = 1228.8
PEAK_HBM_GBS = 8000.0
# The paper's own figures (Sec. 4.2, Table 2, Table B.1), context only: they
# compare pruning methods on another GPU and include reading and saving the
# scene, so no ratio to them is reported.
PAPER_CONTEXT = {
    "hardware": "RTX 3090 (named by the paper)",
    "prune_s_mipnerf360_ratio_0.5": 3.85, "primitives_mipnerf360_derived": 3.36e6, "views_subsampled": 64,
    "evals_per_s_derived": 5.6e7, "includes_io": True,
    "claims": "about 3,000x fewer FLOPs than the Hessian-based PUP method; up to about 20x lower latency "
              "than the rendering-based methods compared",
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


# Sources of the view-loop kernels and the build that compiles them: HBM
# traffic measured with rocprofv3 counters is reported only while these are
# unchanged.
KERNEL_SOURCES = ("paper_2606_09074_amd/csrc/score.hip", "paper_2606_09074_amd/csrc/refine_internal.hpp",
                  "paper_2606_09074_amd/build.py")


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
    ap.add_argument("--waves-per-block", type=int, default=0, choices=[0, 1, 2, 4, 8],
                    help="waves per block of the binned view loop (0: the library's default)")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16-f16", "f16"],
                    help="scene storage: FP32 planes, BF16 geometry/opacity + FP16 SH, or FP16 throughout "
                         "(arithmetic is FP32 either way)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the prune times of the small and large workloads")
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
        print(f"bench.py measures one GPU: the path runs on a single MI355X (--gpus {args.gpus} requested); "
              f"sharding over several GPUs is a design that is not built", file=sys.stderr)
        return 2

    import torch

    from paper_2606_09074_amd import _lib, synth

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
    stored_np = STORAGES[args.storage][0](planes_np)
    planes_np = STORAGES[args.storage][1](stored_np)   # the values the scene holds
    n, V = spec.n, cams_np.shape[0]
    dev = torch.device("cuda:0")
    params = _lib.default_params()
    params.score_path = {"auto": _lib.PATH_AUTO, "direct": _lib.PATH_DIRECT, "binned": _lib.PATH_BINNED}[args.score_path]
    params.records_per_lane = args.records_per_lane
    params.views_per_iteration = args.views_per_iteration
    params.waves_per_block = args.waves_per_block
    run = Pruner(torch.from_numpy(stored_np).to(dev), torch.from_numpy(cams_np).to(dev), ratio, params)
    res = run.time(args.steps, args.warmup)
    ms_per_step = res["ms_per_step"]
    value = n * V / (ms_per_step / 1e3)
    avg = res["phases_ms"]
    log(f"bench: {ms_per_step:.3f} ms/step, phases {avg}")
    cold_ms = run.cold(args.steps)
    log(f"bench: {cold_ms:.3f} ms per prune after a 1 GiB cache flush")
    n_eval, n_screened = run.pair_counts()

    # roofline of the view loop (the dominant kernel, the only launch of
    # refine_score_views): FP32 work it performed, over its event-timed
    # duration on the launch stream
    t_views = avg["views"] / 1e3
    flops = FLOP_PER_PAIR[params.proj_mode] * n_eval + FLOP_PER_SCREENED_PAIR * n_screened
    achieved_tflops = flops / t_views / 1e12
    kname = "score_binned" if n_eval < n * V else "score_direct"
    counters = profiled_counters(kname, spec.name) if (params.proj_mode == 0 and args.storage == "f32") else {}
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

    # the other workloads: the small one (50k x 16, launch-bound) and the
    # large one (6M x 300), same path and parameters
    others = {}
    if not args.no_other_workloads:
        for name in ("small", "large"):
            if name == args.workload:
                continue
            sp = synth.SPECS[name]
            log(f"bench: {sp.name}")
            pr = Pruner(torch.from_numpy(STORAGES[args.storage][0](synth.make_planes(sp))).to(dev),
                        torch.from_numpy(synth.make_cameras(sp)).to(dev), sp.ratios[0], params)
            r = pr.time(args.steps, args.warmup)
            others[sp.name] = {"ms_per_prune": r["ms_per_step"], "ratio": sp.ratios[0],
                               "evals_per_s": round(sp.n * sp.n_views / (r["ms_per_step"] / 1e3), 1),
                               "phases_ms": r["phases_ms"]}
            del pr
            torch.cuda.empty_cache()
        # the paper's own cost setting (Table B.1) on this workload: the
        # depth-only projection term (Eq. 17) over 64 subsampled views
        if args.workload == "medium" and args.storage == "f32":
            pp = _lib.default_params()
            pp.proj_mode, pp.n_sub_views = _lib.PROJ_DEPTH, 64
            log("bench: paper configuration (depth-only term, 64 views)")
            pr = Pruner(run.planes, run.cams, ratio, pp)
            r = pr.time(args.steps, args.warmup)
            others[f"{spec.name}-depth-64-views"] = {
                "ms_per_prune": r["ms_per_step"], "ratio": ratio, "views_evaluated": 64,
                "evals_per_s": round(n * 64 / (r["ms_per_step"] / 1e3), 1), "phases_ms": r["phases_ms"]}
            del pr
            torch.cuda.empty_cache()

    cpu = None
    precision = None
    if not args.no_cpu_baseline:
        cpu, D_oracle = cpu_baseline(spec, planes_np, cams_np, ratio)
        # each 2-byte storage of this workload: its prune time, and its
        # scores and kept sets against the FP64 oracle on the FP32 scene
        if args.storage == "f32" and args.workload == "medium":
            precision = {}
            for st_name in ("bf16-f16", "f16"):
                q = STORAGES[st_name][0](planes_np)
                pr = Pruner(torch.from_numpy(q).to(dev), run.cams, ratio, params)
                r = pr.time(args.steps, args.warmup)
                precision[st_name] = {"ms_per_prune": r["ms_per_step"], "phases_ms": r["phases_ms"],
                                      **storage_error(pr.score_only(), D_oracle, spec.n)}
                del pr
                torch.cuda.empty_cache()
            precision["f32"] = storage_error(run.score_only(), D_oracle, spec.n)

    serving = serve_bench(args) if args.serve_jobs > 0 else None

    line = {"metric": "Gaussian-view evals/s", "value": round(value, 1), "unit": "evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": spec.name, "n": n, "views": V, "ratio": ratio, "storage": args.storage,
                       "step": "stats+score+select+compact", "score_path": args.score_path,
                       "records_per_lane": args.records_per_lane, "views_per_iteration": args.views_per_iteration,
                       "waves_per_block": args.waves_per_block, "ms_per_prune": round(ms_per_step, 4)},
            "phases_ms": {k: round(v, 4) for k, v in avg.items()},
            "cold_cache": {"ms_per_prune": round(cold_ms, 4), "flush": "1 GiB read before each prune",
                           "clock": "HIP events around the prune on its stream"},
            "paper_context": PAPER_CONTEXT,
            "roofline": roofline, "cpu_baseline": cpu, "precision": precision, "other_workloads": others,
            "serving": serving}
    print(json.dumps(line), flush=True)
    return 0


def _identity(x):
    return x


def _storages():
    from paper_2606_09074_amd import synth
    return {"f32": (_identity, _identity),
            "bf16-f16": (synth.quantize_bf16_f16, synth.dequantize_bf16_f16),
            "f16": (synth.quantize_f16, synth.dequantize_f16)}


class _LazyStorages(dict):
    def __missing__(self, key):
        self.update(_storages())
        return dict.__getitem__(self, key)


STORAGES = _LazyStorages()


class Pruner:
    """One resident scene and its buffers: times whole prune steps (stats ->
    prepare -> views -> select -> compact on one stream, inputs in HBM)."""

    PHASES = ("stats", "prepare", "views", "select", "compact")

    def __init__(self, planes, cams, ratio, params):
        import torch

        from paper_2606_09074_amd import _lib, api
        self.torch, self.api = torch, api
        self.planes, self.cams, self.ratio, self.params = planes, cams, ratio, params
        dev = planes.device
        self.n, self.V = planes.shape[1], cams.shape[0]
        self.stream = torch.cuda.current_stream(dev)
        self.ws = api.workspace(self.n, self.V, dev)
        self.st = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
        self.scores = torch.empty(self.n, dtype=torch.float32, device=dev)
        self.keep = torch.empty(self.n, dtype=torch.uint8, device=dev)
        self.n_keep = torch.empty(1, dtype=torch.int64, device=dev)
        self.cap = self.n - api.prune_count(self.n, ratio)
        self.out = torch.empty((59, max(self.cap, 1)), dtype=planes.dtype, device=dev)
        self.idx = torch.empty(max(self.cap, 1), dtype=torch.int32, device=dev)
        torch.cuda.synchronize()

    def step(self, ev=None, j=0, marked=("views",)):
        api, s, prm = self.api, self.stream, self.params

        def mark(k, e):
            if ev is not None and k in marked:
                ev[k][j][e].record(s)
        mark("stats", 0)
        api.refine_stats(self.planes, self.st, self.ws, prm, stream=s)
        mark("stats", 1)
        mark("prepare", 0)
        api.refine_score_prepare(self.planes, self.cams, self.st, self.ws, prm, stream=s)
        mark("prepare", 1)
        mark("views", 0)
        api.refine_score_views(self.planes, self.V, self.st, self.scores, self.ws, prm, stream=s)
        mark("views", 1)
        mark("select", 0)
        api.refine_select(self.scores, self.keep, self.ws, ratio=self.ratio, n_keep_out=self.n_keep, stream=s)
        mark("select", 1)
        mark("compact", 0)
        api.refine_compact(self.planes, self.keep, self.out, self.ws, index_map_out=self.idx, capacity=self.cap,
                           stream=s)
        mark("compact", 1)

    def time(self, steps, warmup) -> dict:
        """K timed steps bracketed by synchronisations (wall clock), with HIP
        events on the launch stream around every view loop; then the same
        number of untimed steps with events around every phase."""
        import numpy as np
        torch = self.torch
        n_ev = max(steps, 1)
        ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_ev)]
              for k in self.PHASES}
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(steps):
            self.step(ev, j)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        views_ms = [a.elapsed_time(b) for a, b in ev["views"][:steps]]
        for j in range(steps):
            self.step(ev, j, marked=self.PHASES)
        torch.cuda.synchronize()
        avg = {k: float(np.mean([a.elapsed_time(b) for a, b in ev[k][:steps]])) for k in self.PHASES}
        avg["views"] = float(np.mean(views_ms))
        return {"ms_per_step": round((t1 - t0) * 1e3 / max(steps, 1), 4), "phases_ms": {k: round(v, 4) for k, v in avg.items()}}

    def cold(self, steps) -> float:
        """Mean time of a prune that starts with a cold last-level cache: a
        1 GiB read (which evicts the 256 MB cache) precedes each prune, and
        HIP events on the launch stream bracket the prune alone."""
        import numpy as np
        torch = self.torch
        flush = torch.ones(1 << 28, dtype=torch.float32, device=self.planes.device)
        ms = []
        for _ in range(max(steps, 1)):
            flush.sum()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(self.stream)
            self.step()
            b.record(self.stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        del flush
        return float(np.mean(ms))

    def pair_counts(self):
        """Pairs the view loop evaluated in full and pairs it screened out
        after their first step (culled pairs are in neither)."""
        torch = self.torch
        evaluated = torch.zeros(2, dtype=torch.int64, device=self.planes.device)
        self.api.refine_score_views(self.planes, self.V, self.st, self.scores, self.ws, self.params,
                                    evaluated_out=evaluated, stream=self.stream)
        torch.cuda.synchronize()
        return tuple(int(x) for x in evaluated.cpu().tolist())

    def score_only(self):
        """Scores of one step, on the host."""
        self.step()
        self.torch.cuda.synchronize()
        return self.scores.cpu().numpy().copy()


def storage_error(scores, D, n) -> dict:
    """Score relative error and kept-set Jaccard at beta 0.5 and 0.9 of GPU
    scores against the FP64 oracle's scores of the FP32 scene (ranking by
    (score, index), as the library's selection does)."""
    import numpy as np
    s = scores.astype(np.float64)
    nz = D > 0
    rel = np.abs(s[nz] - D[nz]) / D[nz]
    out = {"score_rel_err_median": float(np.median(rel)), "score_rel_err_p99": float(np.quantile(rel, 0.99))}
    idx = np.arange(n)
    for beta in (0.5, 0.9):
        k = int(np.floor(beta * n + 0.5))
        ka = np.ones(n, bool)
        ka[np.lexsort((idx, scores.astype(np.float32)))[:k]] = False
        kb = np.ones(n, bool)
        kb[np.lexsort((idx, D))[:k]] = False
        out[f"jaccard_vs_oracle_{beta}"] = round(float((ka & kb).sum()) / float((ka | kb).sum()), 6)
    return {k: (round(v, 8) if isinstance(v, float) else v) for k, v in out.items()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_mhz() -> float | None:
    """The first logical CPU's current clock from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("cpu MHz"):
                    return round(float(line.split(":", 1)[1]), 1)
    except (OSError, ValueError):
        pass
    return None


def cpu_baseline(spec, planes_np, cams_np, ratio):
    """The FP64 oracle as it stands, timed on the host: the whole prune of
    the workload on all its OpenMP threads, and one thread on a bounded
    sample (every 8th primitive; the per-primitive work is independent, so
    its rate is that of the whole).  Returns the baseline and the oracle's
    scores (kept for the precision report)."""
    import subprocess

    import oracle
    log("bench: timing the FP64 CPU oracle on the same workload")
    oracle.build(force=False)
    prm = oracle.Params()
    n, V = planes_np.shape[1], cams_np.shape[0]
    tc0 = time.perf_counter()
    F = oracle.stats(planes_np, eta=prm.eta)
    lam = oracle.lam(F, prm)
    D, _, _, _ = oracle.score(planes_np, cams_np, lam, prm)
    keep_o, _ = oracle.select(D, oracle.n_prune(n, ratio))
    oracle.compact(planes_np, keep_o)
    tc = time.perf_counter() - tc0
    # one thread, in a child process (OMP_NUM_THREADS=1) that draws the same
    # scene and times the oracle's scoring of every 8th primitive
    code = ("import sys, time, numpy as np; sys.path.insert(0, %r); import oracle; "
            "from paper_2606_09074_amd import synth; sp = synth.SPECS[%r]; pl = synth.make_planes(sp); "
            "cm = synth.make_cameras(sp); prm = oracle.Params(); idx = np.arange(0, sp.n, 8); "
            "t0 = time.perf_counter(); F = oracle.stats(pl, eta=prm.eta); lam = oracle.lam(F, prm); "
            "oracle.score(pl, cm, lam, prm, idx=idx); print(time.perf_counter() - t0, idx.size, oracle.num_threads())"
            ) % (ROOT, {"medium-3M-x200": "medium", "small-50k-x16": "small", "large-6M-x300": "large"}[spec.name])
    env = dict(os.environ, OMP_NUM_THREADS="1")
    single = None
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300,
                             check=True).stdout.split()
        t1, m, thr = float(out[0]), int(out[1]), int(out[2])
        single = {"value": round(m * V / t1, 1), "unit": "evals/s", "cores": thr,
                  "sample": f"statistics of all {n} + scores of every 8th primitive ({m}) x {V} views, {t1:.2f} s"}
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        log(f"bench: single-thread oracle leg failed: {e}")
    cpu = {"value": round(n * V / tc, 1), "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"full {spec.name} prune (stats+score+select+compact), {tc:.2f} s",
           "ms_per_prune": round(tc * 1e3, 1), "cpu_model": cpu_model(), "cpu_mhz": cpu_mhz(),
           "logical_cpus_visible": os.cpu_count(), "single_thread": single}
    return cpu, D


def serve_bench(args) -> dict:
    """Served latency: Poisson arrivals of prune jobs on resident, prepared
    scenes (paper_2606_09074_amd.serve) with the scenes in FP32, BF16/FP16
    and FP16 storage, once more with FP32 scenes where every job runs the
    whole path; then the same jobs as a burst (capacity, with and without
    overlap and packing) and, with FP32 and FP16 scenes, Poisson arrivals at
    70% of the burst capacity, where jobs overlap on the device.  Latency =
    completion seen by the host - arrival time."""
    import numpy as np
    import torch

    from paper_2606_09074_amd import serve, synth
    dev = torch.device("cuda:0")
    specs = synth.serve_scene_specs(8)
    log(f"serve: generating {len(specs)} resident scenes, n = {[sp.n for sp in specs]}")
    stores = {"f32": [], "bf16_f16": [], "f16": []}
    for sp in specs:
        pl = synth.make_planes(sp)
        stores["f32"].append(torch.from_numpy(pl).to(dev))
        stores["bf16_f16"].append(torch.from_numpy(synth.quantize_bf16_f16(pl)).to(dev))
        stores["f16"].append(torch.from_numpy(synth.quantize_f16(pl)).to(dev))
    arrivals, reqs = synth.serve_requests(args.serve_jobs, len(specs), rate=args.serve_rate)
    cams = {}
    for _, V, _ in reqs:
        if V not in cams:
            cams[V] = torch.from_numpy(synth.ring_cameras(V)).to(dev)
    torch.cuda.synchronize()

    tuner = serve.Tuner()
    buckets = sorted({(serve.bucket_of(sp.n, V)) for sp in specs for V in (64, 128, 256)})
    tuner.tune(stores["f32"][-1], lambda V: torch.from_numpy(synth.ring_cameras(V)).to(dev), buckets, reps=3,
               prepared=True)
    log(f"serve: tuned {len(buckets)} buckets on prepared scenes: {sorted(tuner.table.items())}")

    def run(scenes, arr, slots, prepare=True, pack=True):
        srv = serve.Server(dev, slots=slots, tuner=tuner, prepare_scenes=prepare,
                           pack_max_n=(1 << 20) if pack else 0)
        for t in scenes:
            srv.add_scene(t)
        # steady state: the kernels, and the caching allocator of every slot
        # stream, warmed by one untimed burst of the same jobs (a server that
        # has run for a while no longer grows its pools per job)
        for sc, V, r in reqs:
            srv.submit(sc, cams[V], r)
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

    def jaccard(ka, kb):
        out = []
        for a, b in zip(ka, kb):
            a, b = a.bool(), b.bool()
            out.append(float((a & b).sum().item()) / max(float((a | b).sum().item()), 1.0))
        return {"min": round(min(out), 5), "mean": round(float(np.mean(out)), 5)}

    res, keeps = {}, {}
    for name in ("f32", "bf16_f16", "f16"):
        log(f"serve: {len(reqs)} jobs at {args.serve_rate}/s, {name} scenes")
        res[name], keeps[name] = run(stores[name], arrivals, args.serve_slots)
    log("serve: same jobs, FP32 scenes, every job on the whole path (no prepared scenes)")
    res["f32_whole_path"], _ = run(stores["f32"], arrivals, args.serve_slots, prepare=False)
    burst = np.zeros(len(reqs))
    log("serve: burst (all jobs at once), with and without overlap")
    b4, _ = run(stores["f32"], burst, args.serve_slots)
    b4n, _ = run(stores["f32"], burst, args.serve_slots, pack=False)
    b1, _ = run(stores["f32"], burst, 1, pack=False)
    # Poisson arrivals at 70% of the burst capacity: jobs arrive while others
    # are on the device and overlap there
    busy_rate = round(0.7 * b4["jobs_per_s"], 1)
    busy_arr, _ = synth.serve_requests(args.serve_jobs, len(specs), rate=busy_rate)
    log(f"serve: same jobs at {busy_rate}/s (70% of the burst capacity), FP32 and FP16 scenes")
    busy32, _ = run(stores["f32"], busy_arr, args.serve_slots)
    busy16, _ = run(stores["f16"], busy_arr, args.serve_slots)
    # the same jobs on small resident scenes (20k..200k Gaussians), where
    # launches rather than arithmetic set the pace: packed vs one launch
    # sequence per job
    small_specs = synth.serve_scene_specs(8, n_range=(20_000, 200_000))
    small = [torch.from_numpy(synth.make_planes(sp)).to(dev) for sp in small_specs]
    log("serve: burst on small scenes, packed and unpacked")
    s4, _ = run(small, burst, args.serve_slots)
    s4n, _ = run(small, burst, args.serve_slots, pack=False)
    return {"workload": f"8 resident scenes n=0.2M..6M (log-spaced, ends included), 50..300 ring views, "
                        f"ratio 0.3..0.9, Poisson arrivals",
            "jobs": len(reqs), "rate_per_s": args.serve_rate, "slots": args.serve_slots,
            "latency_clock": "host: arrival to observed completion",
            **res,
            "kept_jaccard_vs_f32": {"bf16_f16": jaccard(keeps["bf16_f16"], keeps["f32"]),
                                    "f16": jaccard(keeps["f16"], keeps["f32"])},
            "overlapping_load": {"rate_per_s": busy_rate, "f32": busy32, "f16": busy16},
            "burst": {"slots": args.serve_slots, "jobs_per_s": b4["jobs_per_s"], "evals_per_s": b4["evals_per_s"],
                      "unpacked_jobs_per_s": b4n["jobs_per_s"], "one_slot_unpacked_jobs_per_s": b1["jobs_per_s"]},
            "burst_small_scenes": {"n": "20k..200k", "packed_jobs_per_s": s4["jobs_per_s"],
                                   "unpacked_jobs_per_s": s4n["jobs_per_s"]}}


if __name__ == "__main__":
    sys.exit(main())
