"""Serving prune jobs on one GPU: resident scenes, continuous batching.

A job is one prune (paper Sec. 3.3: score every primitive, remove the
bottom beta * N) of a scene that stays resident in device memory, seen
from the job's own camera set.  The server

* keeps scenes resident (``add_scene``), each plane padded to a multiple of
  8 elements so the library's 16-byte-load kernels apply, together with what
  scoring needs of the scene alone: its statistics and its spatially binned,
  activated copy (``refine_score_prepare``), which do not depend on the
  cameras -- a job then only rebuilds the camera tables
  (``refine_score_cameras``) before the view loop;
* takes jobs as they arrive (``submit``), in arrival order;
* admits the head of the queue as soon as an in-flight slot and enough
  device memory are free: a job reserves its workspace, scores, mask,
  survivor planes and index map (``job_bytes``) against a budget, which by
  default is the device's memory less the resident scenes and a reserve;
* runs an admitted job's camera tables and view loop on its scene's stream
  (they write the scene's prepared workspace, so jobs on one scene take
  their turns there) and its selection and compaction on the slot's own HIP
  stream, with its own small workspace; jobs that arrive while others run
  overlap on the device -- a small scene does not fill the 256 compute
  units, and its launches interleave with the others'.  Jobs with their own
  parameters, or more views than a scene was prepared for, run the whole
  path (stats, prepare, views, select, compact) on the slot's stream;
* packs small scenes: when two or more small jobs (default parameters, at
  most ``pack_max_n`` primitives) wait at the head of the queue, up to
  ``max_pack`` of them go to one slot as one ``refine_prune_batch`` -- one
  grouped launch per kernel (9 in all) for all of them, its job table
  copied from the slot's pinned staging buffer without blocking the host;
* notices completions by polling an event recorded after each launch unit's
  last call, then frees the slot and the reservation and admits the next
  jobs.

Each job's results do not depend on what runs beside it: the library's
reductions have fixed orders (FP64 statistics summed per tile in a fixed
order, per-primitive view sums in view order within 64-view blocks,
integer selection), so a job
gives bit-identical scores, mask and survivors alone and in the mix.

``Tuner`` picks, per (primitive count, view count) bucket, the execution
choice of the view loop -- direct, or binned with one or two primitives per
lane, one or two views per iteration and 2, 4 or 8 waves (128 to 1024
primitives) per block -- by timing, on a scene of the bucket's size, the
calls the server makes for such a job: the camera tables and the view loop
on a prepared scene, or statistics and the whole scoring otherwise.
Choices never change results, only speed; the table can be saved and
reloaded.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import math
import time
from typing import Optional

import numpy as np

N_PLANES = 59
STRIDE_ALIGN = 8      # elements: 16-byte aligned planes for 2- and 4-byte storage


# ------------------------------------------------------------------ policy

def job_bytes(n: int, n_views: int, n_keep: int, elem_bytes: int, workspace_bytes: int) -> int:
    """Device bytes a job holds while in flight: workspace, FP32 scores, the
    keep mask, the survivors' planes, the index map and the small outputs."""
    return int(workspace_bytes + 4 * n + n + N_PLANES * elem_bytes * n_keep + 4 * n_keep + 18 * 4 * n_views
               + 256 + 96 + 64)


class Admission:
    """First-come first-served admission against in-flight slots and a byte
    budget.  The head of the queue blocks the ones behind it, so a large job
    is never starved by a stream of small ones.  No device calls: the
    policy is plain bookkeeping."""

    def __init__(self, budget_bytes: int, slots: int):
        if slots < 1 or budget_bytes <= 0:
            raise ValueError("need at least one slot and a positive budget")
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.in_use = 0
        self.inflight = 0

    def fits_ever(self, nbytes: int) -> bool:
        return nbytes <= self.budget

    def can_admit(self, nbytes: int) -> bool:
        return self.inflight < self.slots and self.in_use + nbytes <= self.budget

    def admit(self, nbytes: int) -> None:
        if not self.can_admit(nbytes):
            raise RuntimeError("admission without room")
        self.in_use += nbytes
        self.inflight += 1

    def release(self, nbytes: int) -> None:
        if self.inflight < 1 or nbytes > self.in_use:
            raise RuntimeError("release without a matching admission")
        self.in_use -= nbytes
        self.inflight -= 1


def poisson_arrivals(rate_per_s: float, count: int, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process."""
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def percentile(values, q: float) -> float:
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.quantile(v, q))


# ------------------------------------------------------------------- tuner

def bucket_of(n: int, n_views: int) -> tuple[int, int]:
    """(round(log2 n), round(log2 V)) of a job."""
    return (int(round(math.log2(max(n, 1)))), int(round(math.log2(max(n_views, 1)))))


# execution choices of the view loop: (score_path, records_per_lane,
# views_per_iteration, waves_per_block) -- primitives per lane, views per
# iteration and waves per block of the binned loop, or the direct loop
CANDIDATES = ((1, 0, 0, 0),) + tuple((2, ppl, vpi, w) for ppl in (1, 2) for vpi in (1, 2) for w in (2, 4, 8))


def apply_choice(prm, cand) -> None:
    """Set a tuner choice (path, records per lane[, views per iteration[,
    waves per block]]) on a params struct (tables saved before the later
    entries were tuned have fewer)."""
    prm.score_path, prm.records_per_lane = cand[0], cand[1]
    prm.views_per_iteration = cand[2] if len(cand) > 2 else 0
    prm.waves_per_block = cand[3] if len(cand) > 3 else 0


class Tuner:
    """Per-bucket choice of the view loop's execution (never its results)."""

    def __init__(self, table: Optional[dict] = None):
        self.table: dict[tuple[int, int], tuple[int, ...]] = dict(table or {})

    def choice(self, n: int, n_views: int) -> Optional[tuple[int, ...]]:
        return self.table.get(bucket_of(n, n_views))

    def save(self, path: str) -> None:
        with open(path, "w") as f:
            json.dump({f"{a},{b}": list(v) for (a, b), v in sorted(self.table.items())}, f, indent=1)

    @classmethod
    def load(cls, path: str) -> "Tuner":
        with open(path) as f:
            raw = json.load(f)
        return cls({tuple(int(x) for x in k.split(",")): tuple(v) for k, v in raw.items()})

    def tune(self, planes, cams_for_views, buckets, reps: int = 3, stream=None, log=None,
             prepared: bool = True) -> None:
        """Time every candidate on prefixes of `planes` (a resident scene
        tensor at least as large as the biggest bucket) with camera sets from
        `cams_for_views(V)`, keep the fastest per bucket.  With `prepared`
        (a server that prepares its scenes) a candidate is timed on what a
        job on a prepared scene runs, the camera tables (with the culling and
        group order) and the view loop; otherwise on the statistics and the
        whole scoring a job runs from scratch."""
        import torch

        from . import _lib, api
        dev = planes.device
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        for (lb_n, lb_v) in buckets:
            n = min(1 << lb_n, planes.shape[1])
            V = 1 << lb_v
            cams = cams_for_views(V)
            ws = api.workspace(n, V, dev)
            st = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
            scores = torch.empty(n, dtype=torch.float32, device=dev)
            if prepared:   # the scene as Server._prepare leaves it
                prm0 = _lib.default_params()
                prm0.score_path = _lib.PATH_BINNED
                api.refine_stats(planes, st, ws, prm0, n=n, stream=s)
                api.refine_score_prepare(planes, cams, st, ws, prm0, n=n, stream=s)
            best = None
            for cand in CANDIDATES:
                prm = _lib.default_params()
                apply_choice(prm, cand)
                times = []
                for r in range(reps + 1):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(s)
                    if prepared:
                        api.refine_score_cameras(planes, cams, ws, prm, n=n, stream=s)
                        api.refine_score_views(planes, V, st, scores, ws, prm, n=n, stream=s)
                    else:
                        api.refine_stats(planes, st, ws, prm, n=n, stream=s)
                        api.refine_score(planes, cams, st, scores, ws, prm, n=n, stream=s)
                    e1.record(s)
                    e1.synchronize()
                    if r:
                        times.append(e0.elapsed_time(e1))
                t = float(np.median(times))
                if best is None or t < best[0]:
                    best = (t, cand)
            self.table[(lb_n, lb_v)] = best[1]
            if log:
                log(f"tuner: bucket n=2^{lb_n} V=2^{lb_v} -> path {best[1][0]} ppl {best[1][1]} vpi {best[1][2]} "
                    f"waves {best[1][3]} ({best[0]:.3f} ms)")


# ------------------------------------------------------------------ server

@dataclasses.dataclass
class Job:
    id: int
    scene: int
    cams: object                  # device tensor [V, 18]
    ratio: float
    params: object                # _lib.Params
    t_arrival: float
    n: int = 0
    n_keep: int = 0
    nbytes: int = 0
    on_prepared: bool = False     # scored on its scene's prepared workspace
    packable: bool = False        # may share a grouped launch with other small jobs
    t_admit: float = 0.0
    t_done: float = 0.0
    slot: int = -1
    start_event: object = None
    done_event: object = None
    stats: object = None
    scores: object = None
    keep: object = None
    out: object = None
    index_map: object = None
    n_out: object = None
    workspace: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def device_ms(self) -> float:
        """Stream time from the job's first call to its last (finished jobs)."""
        return self.start_event.elapsed_time(self.done_event)


class Server:
    """Continuous-batching prune server on one device (see module doc)."""

    def __init__(self, device="cuda:0", slots: int = 4, budget_bytes: Optional[int] = None,
                 reserve_bytes: int = 8 << 30, tuner: Optional[Tuner] = None, prepare_scenes: bool = True,
                 max_views: int = 512, pack_max_n: int = 1 << 20, max_pack: int = 32):
        import torch

        from . import _lib
        _lib.load()
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]   # default priority
        self.free_slots = collections.deque(range(slots))
        self.scenes: dict[int, object] = {}      # id -> padded [59, stride] tensor
        self.scene_n: dict[int, int] = {}
        self.prepared: dict[int, tuple] = {}      # id -> (stats, workspace, stream)
        self.max_views = int(max_views)
        self.prepare_scenes = bool(prepare_scenes)
        self.scene_bytes = 0
        self.reserve = int(reserve_bytes)
        self.explicit_budget = budget_bytes
        self.admission = Admission(self._budget(), slots)
        self.queue: collections.deque[Job] = collections.deque()
        self.running: list[tuple] = []           # launch units: (jobs, nbytes, slot, done event)
        self.pack_max_n = int(pack_max_n)
        self.max_pack = int(max_pack)
        self.tuner = tuner
        self._next_id = 0
        # per slot: the pinned host buffer a packed launch's job table is
        # copied from (a slot's next launch waits for its previous one to end)
        from . import api
        self.staging = [api.batch_staging(self.max_pack) for _ in range(slots)]

    def _budget(self) -> int:
        if self.explicit_budget is not None:
            return int(self.explicit_budget)
        total = self.torch.cuda.get_device_properties(self.device).total_memory
        return max(int(total - self.scene_bytes - self.reserve), 1)

    # scenes ---------------------------------------------------------------
    def add_scene(self, planes, n: Optional[int] = None) -> int:
        """Keep the first n primitives of a [59, stride] scene tensor (float32,
        or int16 2-byte storage) resident; returns its id.  A stride that is
        not a multiple of STRIDE_ALIGN is padded (one device copy)."""
        from . import api
        api.storage_dtypes(planes)
        if planes.device != self.device:
            raise ValueError("scenes must live on the server's device")
        n = planes.shape[1] if n is None else int(n)
        if planes.stride(1) != 1 or planes.stride(0) % STRIDE_ALIGN or planes.data_ptr() % 16:
            stride = -(-max(n, 1) // STRIDE_ALIGN) * STRIDE_ALIGN
            padded = self.torch.zeros((N_PLANES, stride), dtype=planes.dtype, device=self.device)
            padded[:, :n] = planes[:, :n]
            planes = padded
        sid = len(self.scenes)
        self.scenes[sid] = planes
        self.scene_n[sid] = n
        self.scene_bytes += planes.numel() * planes.element_size()
        if self.prepare_scenes and n > 0:
            self._prepare(sid)
        if self.explicit_budget is None:
            self.admission.budget = self._budget()
        return sid

    def _prepare(self, sid: int) -> None:
        """Statistics and the binned copy of scene `sid` with the default
        parameters, in a workspace sized for max_views cameras."""
        from . import _lib, api
        torch = self.torch
        planes, n = self.scenes[sid], self.scene_n[sid]
        prm = _lib.default_params()
        prm.score_path = _lib.PATH_BINNED
        s = torch.cuda.Stream(self.device)
        ws = api.workspace(n, self.max_views, self.device)
        st = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=self.device)
        one_cam = torch.zeros((1, 18), dtype=torch.float32, device=self.device)
        one_cam[0, 0] = one_cam[0, 4] = one_cam[0, 8] = 1.0
        one_cam[0, 11] = 1.0
        one_cam[0, 12:18] = torch.tensor([1.0, 1.0, 0.5, 0.5, 1.0, 1.0])
        s.wait_stream(torch.cuda.current_stream(self.device))
        api.refine_stats(planes, st, ws, prm, n=n, stream=s)
        api.refine_score_prepare(planes, one_cam, st, ws, prm, n=n, stream=s)
        s.synchronize()
        self.prepared[sid] = (st, ws, s)
        self.scene_bytes += ws.numel()
        if self.explicit_budget is None:
            self.admission.budget = self._budget()

    # jobs -----------------------------------------------------------------
    def submit(self, scene: int, cams, ratio: float, params=None, t_arrival: Optional[float] = None) -> Job:
        from . import _lib, api
        if scene not in self.scenes:
            raise KeyError(f"no resident scene {scene}")
        planes = self.scenes[scene]
        n = self.scene_n[scene]
        V = cams.shape[0]
        prm = params if params is not None else _lib.default_params()
        if self.tuner is not None and params is None:
            c = self.tuner.choice(n, V)
            if c is not None:
                apply_choice(prm, c)
        n_keep = n - api.prune_count(n, ratio)
        job = Job(self._next_id, scene, cams, float(ratio), prm,
                  time.perf_counter() if t_arrival is None else t_arrival, n=n, n_keep=n_keep)
        job.on_prepared = params is None and scene in self.prepared and V <= self.max_views
        job.packable = params is None and n <= self.pack_max_n
        job.nbytes = job_bytes(n, V, n_keep, planes.element_size(),
                               api.workspace_size(n, 0 if job.on_prepared else V))
        if not self.admission.fits_ever(job.nbytes):
            raise ValueError(f"job needs {job.nbytes} bytes, more than the budget {self.admission.budget}")
        self._next_id += 1
        self.queue.append(job)
        return job

    def _launch(self, job: Job) -> None:
        from . import _lib, api
        torch = self.torch
        slot = self.free_slots.popleft()
        s = self.streams[slot]
        planes = self.scenes[job.scene]
        n, V = job.n, job.cams.shape[0]
        dev = self.device
        with torch.cuda.stream(s):
            job.workspace = api.workspace(n, 0 if job.on_prepared else V, dev)
            job.stats = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
            job.scores = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
            job.keep = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
            out_stride = -(-max(job.n_keep, 1) // STRIDE_ALIGN) * STRIDE_ALIGN
            job.out = torch.empty((N_PLANES, out_stride), dtype=planes.dtype, device=dev)
            job.index_map = torch.empty(max(job.n_keep, 1), dtype=torch.int32, device=dev)
            job.n_out = torch.empty(1, dtype=torch.int64, device=dev)
        job.start_event = torch.cuda.Event(enable_timing=True)
        if job.on_prepared:
            st, pws, ss = self.prepared[job.scene]
            # the camera table may have been written on another stream; the
            # slot's own stream is idle (a slot is freed only once its last
            # job's done event has completed), so nothing else is waited for
            ss.wait_stream(torch.cuda.current_stream(dev))
            job.start_event.record(ss)
            job.stats = st
            api.refine_score_cameras(planes, job.cams, pws, job.params, n=n, stream=ss)
            api.refine_score_views(planes, V, st, job.scores, pws, job.params, n=n, stream=ss)
            scored = torch.cuda.Event()
            scored.record(ss)
            s.wait_event(scored)
        else:
            s.wait_stream(torch.cuda.current_stream(dev))
            job.start_event.record(s)
            api.refine_stats(planes, job.stats, job.workspace, job.params, n=n, stream=s)
            api.refine_score(planes, job.cams, job.stats, job.scores, job.workspace, job.params, n=n, stream=s)
        api.refine_select(job.scores, job.keep, job.workspace, ratio=job.ratio, n=n, stream=s)
        api.refine_compact(planes, job.keep, job.out, job.workspace, index_map_out=job.index_map,
                           n_out=job.n_out, n=n, capacity=job.n_keep, stream=s)
        job.done_event = torch.cuda.Event(enable_timing=True)
        job.done_event.record(s)
        job.slot = slot
        job.t_admit = time.perf_counter()
        self.running.append(([job], job.nbytes, slot, job.done_event))

    def _launch_pack(self, jobs: list) -> None:
        """Prune `jobs` (small, default parameters) with one grouped launch per
        kernel on one slot."""
        from . import _lib, api
        torch = self.torch
        slot = self.free_slots.popleft()
        s = self.streams[slot]
        dev = self.device
        descs = []
        with torch.cuda.stream(s):
            for job in jobs:
                planes = self.scenes[job.scene]
                n = job.n
                job.stats = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
                job.scores = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
                job.keep = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
                out_stride = -(-max(job.n_keep, 1) // STRIDE_ALIGN) * STRIDE_ALIGN
                job.out = torch.empty((N_PLANES, out_stride), dtype=planes.dtype, device=dev)
                job.index_map = torch.empty(max(job.n_keep, 1), dtype=torch.int32, device=dev)
                job.n_out = torch.empty(1, dtype=torch.int64, device=dev)
                descs.append({"planes": planes, "n": n, "cams": job.cams, "ratio": job.ratio, "stats": job.stats,
                              "scores": job.scores, "keep": job.keep, "out": job.out, "capacity": job.n_keep,
                              "index_map": job.index_map, "n_out": job.n_out})
            prm = _lib.default_params()
            ws = torch.empty(max(api.batch_workspace_size(descs, prm), 1), dtype=torch.uint8, device=dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        start = torch.cuda.Event(enable_timing=True)
        start.record(s)
        api.refine_prune_batch(descs, ws, prm, stream=s, staging=self.staging[slot])
        done = torch.cuda.Event(enable_timing=True)
        done.record(s)
        now = time.perf_counter()
        nbytes = sum(j.nbytes for j in jobs)
        for job in jobs:
            job.start_event, job.done_event, job.slot, job.t_admit = start, done, slot, now
            job.workspace = ws
        self.running.append((list(jobs), nbytes, slot, done))

    def step(self) -> list[Job]:
        """Retire finished jobs, then admit queued ones while they fit.
        Returns the jobs that finished in this step."""
        done = []
        still = []
        for unit in self.running:
            jobs, nbytes, slot, event = unit
            if event.query():
                t = time.perf_counter()
                self.admission.release(nbytes)
                self.free_slots.append(slot)
                for job in jobs:
                    job.t_done = t
                    # the workspace goes back to the allocator, on the job's stream
                    job.workspace = None
                    done.append(job)
            else:
                still.append(unit)
        self.running = still
        while self.queue:
            pack = self._pack_at_head()
            if len(pack) >= 2:
                nbytes = sum(j.nbytes for j in pack)
                if not self.admission.can_admit(nbytes):
                    break
                for _ in pack:
                    self.queue.popleft()
                self.admission.admit(nbytes)
                self._launch_pack(pack)
                continue
            if not self.admission.can_admit(self.queue[0].nbytes):
                break
            job = self.queue.popleft()
            self.admission.admit(job.nbytes)
            self._launch(job)
        return done

    def _pack_at_head(self) -> list:
        """The packable jobs at the head of the queue, in order, up to
        max_pack and within the memory left."""
        pack, nbytes = [], 0
        room = self.admission.budget - self.admission.in_use
        for job in self.queue:
            if not job.packable or len(pack) >= self.max_pack or nbytes + job.nbytes > room:
                break
            pack.append(job)
            nbytes += job.nbytes
        return pack

    def idle(self) -> bool:
        return not self.queue and not self.running

    def drain(self) -> list[Job]:
        out = []
        while not self.idle():
            out.extend(self.step())
        return out


def run_open_loop(server: Server, requests, arrivals, on_done=None) -> list[Job]:
    """Submit `requests` [(scene, cams, ratio)] at host times `arrivals`
    (seconds from the start), stepping the server in between; returns the
    finished jobs in completion order."""
    t0 = time.perf_counter()
    finished = []
    i = 0
    total = len(requests)
    while len(finished) < total:
        now = time.perf_counter() - t0
        while i < total and arrivals[i] <= now:
            scene, cams, ratio = requests[i]
            server.submit(scene, cams, ratio, t_arrival=t0 + arrivals[i])
            i += 1
        for job in server.step():
            finished.append(job)
            if on_done:
                on_done(job)
    return finished
