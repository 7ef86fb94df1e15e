"""Python front end of the REFINE library, one function per C entry point.

PyTorch provides device memory and the current HIP stream; every step of
the computation runs in the library's HIP kernels.  The functions only
check tensor shapes/dtypes/devices and pass pointers.

A scene is a [59, stride] tensor: float32 for FP32 storage; int16 holding
the raw bits of BF16 planes 0..10 and FP16 planes 11..58 (the mixed 2-byte
storage; see synth.quantize_bf16_f16); or float16 for FP16 planes
throughout (the half 2-byte storage; see synth.quantize_f16).
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import Params, Scene, Stats, check, default_params

__all__ = ["Params", "default_params", "workspace", "workspace_size", "prune_count", "refine_stats",
           "refine_stats_noalloc",
           "refine_score", "refine_score_prepare", "refine_score_cameras", "refine_score_views", "refine_select",
           "refine_compact",
           "refine_prune_batch", "batch_staging", "stats_from_tensor", "prune", "prune_batch", "version"]


def version() -> str:
    return _lib.load().refine_version().decode()


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def storage_dtypes(planes: torch.Tensor) -> tuple[int, int]:
    """(dtype, sh_dtype) of a scene tensor."""
    if planes.dtype == torch.float32:
        return _lib.REFINE_F32, _lib.REFINE_F32
    if planes.dtype == torch.int16:
        return _lib.REFINE_BF16, _lib.REFINE_F16
    if planes.dtype == torch.float16:
        return _lib.REFINE_F16, _lib.REFINE_F16
    raise ValueError("scene planes must be float32, float16, or int16 bit patterns of BF16 (planes 0..10) and "
                     "FP16 (11..58)")


def _scene(planes: torch.Tensor, n: Optional[int] = None) -> Scene:
    if planes.dim() != 2 or planes.shape[0] != 59:
        raise ValueError("scene planes must be a [59, stride] tensor")
    dt, sh = storage_dtypes(planes)
    if not planes.is_cuda:
        raise ValueError("scene planes must live on the GPU")
    if planes.stride(1) != 1 or planes.stride(0) < planes.shape[1]:
        raise ValueError("scene planes must be row-contiguous")
    stride = planes.stride(0)
    n = planes.shape[1] if n is None else int(n)
    return Scene(n, stride, dt, sh, ctypes.c_void_p(planes.data_ptr()))


def workspace_size(n: int, n_views: int) -> int:
    out = ctypes.c_size_t(0)
    check(_lib.load().refine_workspace_size(int(n), int(n_views), ctypes.byref(out)), "refine_workspace_size")
    return int(out.value)


def workspace(n: int, n_views: int, device="cuda") -> torch.Tensor:
    """A workspace tensor for scenes of up to n primitives and n_views cameras."""
    return torch.empty(max(workspace_size(n, n_views), 1), dtype=torch.uint8, device=device)


def prune_count(n: int, ratio: float) -> int:
    k = _lib.load().refine_prune_count(int(n), float(ratio))
    if k < 0:
        raise ValueError("prune ratio must lie in (0, 1)")
    return int(k)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def refine_stats(planes: torch.Tensor, stats_out: torch.Tensor, ws: torch.Tensor,
                 params: Optional[Params] = None, n: Optional[int] = None, stream=None) -> None:
    """Enqueue the scene statistics; ``stats_out`` is a uint8 tensor of
    ``_lib.STATS_BYTES`` bytes on the GPU."""
    params = params or default_params()
    sc = _scene(planes, n)
    if stats_out.numel() * stats_out.element_size() < _lib.STATS_BYTES or not stats_out.is_cuda:
        raise ValueError("stats_out too small or not on the GPU")
    check(_lib.load().refine_stats(ctypes.byref(sc), ctypes.byref(params), _ptr(stats_out), _ptr(ws),
                                   ws.numel(), _stream_ptr(stream)), "refine_stats")


def refine_stats_noalloc(planes: torch.Tensor, stats_out: torch.Tensor, params: Optional[Params] = None,
                         n: Optional[int] = None, stream=None) -> None:
    """refine_stats on the library's fixed device array instead of a
    workspace (n <= _lib.STATS_NOALLOC_MAX_N; calls on one GPU must not
    overlap)."""
    params = params or default_params()
    sc = _scene(planes, n)
    if stats_out.numel() * stats_out.element_size() < _lib.STATS_BYTES or not stats_out.is_cuda:
        raise ValueError("stats_out too small or not on the GPU")
    check(_lib.load().refine_stats_noalloc(ctypes.byref(sc), ctypes.byref(params), _ptr(stats_out),
                                           _stream_ptr(stream)), "refine_stats_noalloc")


def refine_score(planes: torch.Tensor, cams: torch.Tensor, stats: torch.Tensor, scores_out: torch.Tensor,
                 ws: torch.Tensor, params: Optional[Params] = None, n: Optional[int] = None, stream=None) -> None:
    params = params or default_params()
    sc = _scene(planes, n)
    if cams.dim() != 2 or cams.shape[1] != 18 or cams.dtype != torch.float32 or not cams.is_cuda \
            or not cams.is_contiguous():
        raise ValueError("cams must be a contiguous float32 [V, 18] GPU tensor")
    if scores_out.dtype != torch.float32 or scores_out.numel() < sc.n or not scores_out.is_cuda:
        raise ValueError("scores_out must be a float32 GPU tensor of at least n elements")
    check(_lib.load().refine_score(ctypes.byref(sc), _ptr(cams), cams.shape[0], ctypes.byref(params),
                                   _ptr(stats), _ptr(scores_out), _ptr(ws), ws.numel(), _stream_ptr(stream)),
          "refine_score")


def _check_cams(cams: torch.Tensor) -> None:
    if cams.dim() != 2 or cams.shape[1] != 18 or cams.dtype != torch.float32 or not cams.is_cuda \
            or not cams.is_contiguous():
        raise ValueError("cams must be a contiguous float32 [V, 18] GPU tensor")


def refine_score_prepare(planes: torch.Tensor, cams: torch.Tensor, stats: torch.Tensor, ws: torch.Tensor,
                         params: Optional[Params] = None, n: Optional[int] = None, stream=None) -> None:
    """First phase of refine_score: view tables and (binned path) the binned scene copy in ``ws``."""
    params = params or default_params()
    sc = _scene(planes, n)
    _check_cams(cams)
    check(_lib.load().refine_score_prepare(ctypes.byref(sc), _ptr(cams), cams.shape[0], ctypes.byref(params),
                                           _ptr(stats), _ptr(ws), ws.numel(), _stream_ptr(stream)),
          "refine_score_prepare")


def refine_score_cameras(planes: torch.Tensor, cams: torch.Tensor, ws: torch.Tensor,
                         params: Optional[Params] = None, n: Optional[int] = None, stream=None) -> None:
    """Rebuild only the per-view tables in ``ws`` for a new camera set; the
    binned scene copy from an earlier refine_score_prepare is kept."""
    params = params or default_params()
    sc = _scene(planes, n)
    _check_cams(cams)
    check(_lib.load().refine_score_cameras(ctypes.byref(sc), _ptr(cams), cams.shape[0], ctypes.byref(params),
                                           _ptr(ws), ws.numel(), _stream_ptr(stream)), "refine_score_cameras")


def refine_score_views(planes: torch.Tensor, n_views: int, stats: torch.Tensor, scores_out: torch.Tensor,
                       ws: torch.Tensor, params: Optional[Params] = None, evaluated_out: Optional[torch.Tensor] = None,
                       n: Optional[int] = None, stream=None) -> None:
    """Second phase of refine_score: the view loop over the prepared workspace."""
    params = params or default_params()
    sc = _scene(planes, n)
    if scores_out.dtype != torch.float32 or scores_out.numel() < sc.n or not scores_out.is_cuda:
        raise ValueError("scores_out must be a float32 GPU tensor of at least n elements")
    if evaluated_out is not None and (evaluated_out.dtype != torch.int64 or not evaluated_out.is_cuda
                                      or evaluated_out.numel() < 2):
        raise ValueError("evaluated_out must be an int64 GPU tensor of 2 elements (evaluated, screened)")
    check(_lib.load().refine_score_views(ctypes.byref(sc), int(n_views), ctypes.byref(params), _ptr(stats),
                                         _ptr(scores_out), _ptr(evaluated_out), _ptr(ws), ws.numel(),
                                         _stream_ptr(stream)), "refine_score_views")


def refine_select(scores: torch.Tensor, keep_out: torch.Tensor, ws: torch.Tensor, ratio: float = 0.5,
                  n_prune: int = -1, n_keep_out: Optional[torch.Tensor] = None,
                  threshold_out: Optional[torch.Tensor] = None, n: Optional[int] = None, stream=None) -> None:
    n = scores.numel() if n is None else int(n)
    if scores.dtype != torch.float32 or not scores.is_cuda or keep_out.dtype not in (torch.uint8, torch.bool) \
            or keep_out.numel() < n or not keep_out.is_cuda:
        raise ValueError("scores must be float32 and keep_out uint8/bool [n], both on the GPU")
    check(_lib.load().refine_select(_ptr(scores), n, float(ratio), int(n_prune), _ptr(keep_out),
                                    _ptr(n_keep_out), _ptr(threshold_out), _ptr(ws), ws.numel(),
                                    _stream_ptr(stream)), "refine_select")


def refine_compact(planes: torch.Tensor, keep: torch.Tensor, out_planes: torch.Tensor, ws: torch.Tensor,
                   index_map_out: Optional[torch.Tensor] = None, n_out: Optional[torch.Tensor] = None,
                   n: Optional[int] = None, capacity: Optional[int] = None, stream=None) -> None:
    src = _scene(planes, n)
    dst = _scene(out_planes, capacity)
    if index_map_out is not None and (index_map_out.dtype != torch.int32 or index_map_out.numel() < dst.n):
        raise ValueError("index_map_out must be int32 with at least capacity elements")
    check(_lib.load().refine_compact(ctypes.byref(src), _ptr(keep), ctypes.byref(dst), _ptr(index_map_out),
                                     _ptr(n_out), _ptr(ws), ws.numel(), _stream_ptr(stream)), "refine_compact")


def stats_from_tensor(stats: torch.Tensor) -> dict:
    """Read a refine_stats_t back to the host (synchronises)."""
    raw = bytes(stats[:_lib.STATS_BYTES].cpu().numpy().tobytes())
    s = Stats.from_buffer_copy(raw)
    return {"ybar": s.ybar, "f_col": s.f_col, "f_opa": s.f_opa, "f_gem": s.f_gem, "lambda": list(s.lam),
            "n": s.n, "n_nonfinite": s.n_nonfinite, "bbox_min": list(s.bbox_min), "bbox_max": list(s.bbox_max)}


def prune(planes: torch.Tensor, cams: torch.Tensor, ratio: float, params: Optional[Params] = None,
          ws: Optional[torch.Tensor] = None, stream=None) -> dict:
    """Stats -> score -> select -> compact on one stream; returns the device
    tensors (scores, keep mask, survivors, index map, n_keep)."""
    n = planes.shape[1]
    V = cams.shape[0]
    dev = planes.device
    ws = ws if ws is not None else workspace(n, V, dev)
    st = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
    scores = torch.empty(n, dtype=torch.float32, device=dev)
    keep = torch.empty(n, dtype=torch.uint8, device=dev)
    n_keep = torch.empty(1, dtype=torch.int64, device=dev)
    cap = n - prune_count(n, ratio)
    out = torch.empty((59, max(cap, 1)), dtype=planes.dtype, device=dev)
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    refine_stats(planes, st, ws, params, stream=stream)
    refine_score(planes, cams, st, scores, ws, params, stream=stream)
    refine_select(scores, keep, ws, ratio=ratio, n_keep_out=n_keep, stream=stream)
    refine_compact(planes, keep, out, ws, index_map_out=idx, capacity=cap, stream=stream)
    return {"stats": st, "scores": scores, "keep": keep, "out": out[:, :cap], "index_map": idx[:cap],
            "n_keep": n_keep}


def _batch_jobs(jobs) -> "ctypes.Array":
    arr = (_lib.PruneJob * len(jobs))()
    for k, j in enumerate(jobs):
        _check_cams(j["cams"])
        n = j.get("n")
        arr[k].scene = _scene(j["planes"], n)
        arr[k].cams = j["cams"].data_ptr()
        arr[k].n_views = j["cams"].shape[0]
        arr[k].reserved = 0
        arr[k].ratio = float(j["ratio"])
        arr[k].stats = j["stats"].data_ptr()
        arr[k].scores = j["scores"].data_ptr()
        arr[k].keep = j["keep"].data_ptr()
        arr[k].n_keep = j["n_keep"].data_ptr() if j.get("n_keep") is not None else None
        arr[k].out = _scene(j["out"], j.get("capacity"))
        arr[k].index_map = j["index_map"].data_ptr() if j.get("index_map") is not None else None
        arr[k].n_out = j["n_out"].data_ptr() if j.get("n_out") is not None else None
    return arr


def batch_workspace_size(jobs, params: Optional[Params] = None) -> int:
    arr = _batch_jobs(jobs)
    out = ctypes.c_size_t(0)
    check(_lib.load().refine_prune_batch_workspace_size(arr, len(jobs), ctypes.byref(params or default_params()),
                                                        ctypes.byref(out)), "refine_prune_batch_workspace_size")
    return int(out.value)


def batch_staging(n_jobs: int) -> torch.Tensor:
    """A pinned host buffer for refine_prune_batch's job table (n_jobs jobs)."""
    return torch.empty(max(n_jobs, 1) * _lib.BATCH_STAGING_BYTES_PER_JOB, dtype=torch.uint8, pin_memory=True)


def refine_prune_batch(jobs, ws: torch.Tensor, params: Optional[Params] = None, stream=None,
                       staging: Optional[torch.Tensor] = None) -> None:
    """Enqueue the batched prune of ``jobs`` (dicts of tensors: planes, cams,
    ratio, stats, scores, keep, out, optional n, n_keep, capacity, index_map,
    n_out) in one grouped launch per kernel.  ``staging`` (from
    batch_staging) makes the job-table copy asynchronous; it must stay
    untouched until the stream has passed this call."""
    arr = _batch_jobs(jobs)
    if staging is not None and (staging.is_cuda or not staging.is_pinned()):
        raise ValueError("staging must be a pinned host tensor (batch_staging)")
    check(_lib.load().refine_prune_batch(arr, len(jobs), ctypes.byref(params or default_params()), _ptr(ws),
                                         ws.numel(), _ptr(staging),
                                         staging.numel() if staging is not None else 0, _stream_ptr(stream)),
          "refine_prune_batch")


def prune_batch(scenes, cams, ratios, params: Optional[Params] = None, stream=None) -> list:
    """Allocate the outputs and prune several resident scenes in one batch;
    returns one dict of device tensors per scene (as ``prune``)."""
    jobs = []
    for planes, c, r in zip(scenes, cams, ratios):
        n = planes.shape[1]
        dev = planes.device
        cap = n - prune_count(n, r)
        jobs.append({"planes": planes, "cams": c, "ratio": r,
                     "stats": torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev),
                     "scores": torch.empty(n, dtype=torch.float32, device=dev),
                     "keep": torch.empty(n, dtype=torch.uint8, device=dev),
                     "n_keep": torch.empty(1, dtype=torch.int64, device=dev),
                     "out": torch.empty((59, max(cap, 1)), dtype=planes.dtype, device=dev), "capacity": cap,
                     "index_map": torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                     "n_out": torch.empty(1, dtype=torch.int64, device=dev)})
    ws = torch.empty(max(batch_workspace_size(jobs, params), 1), dtype=torch.uint8, device=scenes[0].device)
    staging = batch_staging(len(jobs))
    refine_prune_batch(jobs, ws, params, stream, staging=staging)
    for j in jobs:
        j["workspace"] = ws
        j["staging"] = staging      # in use until the stream has passed the call
    return jobs
