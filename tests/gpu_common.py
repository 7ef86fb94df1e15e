"""Helpers of the GPU parity tests: run the library through its C ABI on
seeded inputs, run the oracle on the same inputs, compare."""
from __future__ import annotations

import functools
import sys

import numpy as np

from tests.helpers import (ABS_TOL, CLAMP_K, E_COL, E_LNGEM, E_OPA, ETA, REL_TOL, Z_NEAR, within_interval)


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_params(**kw):
    from paper_2606_09074_amd import _lib
    p = _lib.Params(ETA, Z_NEAR, CLAMP_K, E_COL, E_OPA, E_LNGEM, 0, 0, 0, 0, 0, 0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def oracle_params(**kw):
    import oracle
    return oracle.Params(eta=ETA, z_near=Z_NEAR, clamp_k=CLAMP_K, e_col=E_COL, e_opa=E_OPA, e_lngem=E_LNGEM,
                         **kw)


def run_gpu(planes: np.ndarray, cams: np.ndarray, n: int | None = None, ratio: float | None = None,
            n_prune: int = -1, params=None, repeat: int = 1) -> dict:
    """Stats, score and (optionally) select + compact on cuda:0."""
    import torch

    from paper_2606_09074_amd import _lib, api
    n = planes.shape[1] if n is None else n
    dev = torch.device("cuda:0")
    pl = torch.from_numpy(np.ascontiguousarray(planes)).to(dev)
    cm = torch.from_numpy(np.ascontiguousarray(cams)).to(dev)
    ws = api.workspace(n, cams.shape[0], dev)
    st = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
    scores = torch.full((max(n, 1),), float("nan"), dtype=torch.float32, device=dev)
    params = params or gpu_params()
    res = {}
    outs = []
    for _ in range(repeat):
        api.refine_stats(pl, st, ws, params, n=n)
        api.refine_score(pl, cm, st, scores, ws, params, n=n)
        outs.append(scores[:n].cpu().numpy().copy())
    torch.cuda.synchronize()
    res["stats"] = api.stats_from_tensor(st)
    res["scores"] = outs[0]
    res["runs"] = outs
    if ratio is not None or n_prune >= 0:
        keep = torch.full((max(n, 1),), 7, dtype=torch.uint8, device=dev)
        nk = torch.full((1,), -1, dtype=torch.int64, device=dev)
        thr = torch.zeros(1, dtype=torch.int32, device=dev)
        api.refine_select(scores, keep, ws, ratio=ratio if ratio is not None else 0.5, n_prune=n_prune,
                          n_keep_out=nk, threshold_out=thr, n=n)
        k = int(nk.item())
        cap = max(k, 0)
        if pl.dtype == torch.float32:
            out = torch.full((59, max(cap, 1) + 3), float("nan"), dtype=pl.dtype, device=dev)
        else:   # 2-byte storage: a fill bit pattern
            out = torch.full((59, max(cap, 1) + 3), INT16_FILL, dtype=torch.int16, device=dev).view(pl.dtype)
        idx = torch.full((max(cap, 1) + 3,), -7, dtype=torch.int32, device=dev)
        nout = torch.full((1,), -1, dtype=torch.int64, device=dev)
        api.refine_compact(pl, keep, out, ws, index_map_out=idx, n_out=nout, n=n, capacity=cap)
        torch.cuda.synchronize()
        res["keep"] = keep[:n].cpu().numpy()
        res["n_keep"] = k
        res["threshold"] = int(thr.item()) & 0xFFFFFFFF
        res["out"] = out.cpu().numpy()
        res["index_map"] = idx.cpu().numpy()
        res["n_out"] = int(nout.item())
        res["capacity"] = cap
    return res


# the bit pattern run_gpu pre-fills a 2-byte compaction output with (float32: NaN)
INT16_FILL = -12345


def oracle_all(planes, cams, n=None, **kw):
    """Stats, lambda and scores (with ambiguity intervals) from the oracle."""
    import oracle
    prm = oracle_params(**kw)
    F = oracle.stats(planes, n=n, eta=prm.eta)
    lam = oracle.lam(F, prm)
    D, lo, hi, na = oracle.score(planes, cams, lam, prm, n=n)
    return F, lam, D, lo, hi


STATS_RTOL = 1e-6


def check_stats(gs, F, lam, what, **kw):
    """Features (FP32 per-primitive terms, FP64 sums) within STATS_RTOL of the
    oracle's; lambda equal, to FP64 rounding, to Eq. 18-19 applied to the
    GPU's own features (the derivation is FP64 on both sides, while its
    logarithm amplifies the features' FP32 error by 1/|ln(F_gem + eta)|,
    about 9 where F_gem + eta is near 0.9), and within a loose bound of the
    oracle's lambda."""
    import oracle
    for k in ("ybar", "f_col", "f_opa", "f_gem"):
        assert abs(gs[k] - F[k]) <= STATS_RTOL * abs(F[k]) + 1e-15, (what, k, gs[k], F[k])
    if gs["n"] > 0:
        lam_gpu_features = oracle.lam({k: gs[k] for k in ("ybar", "f_col", "f_opa", "f_gem")}, oracle_params(**kw))
        np.testing.assert_allclose(gs["lambda"], lam_gpu_features, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gs["lambda"], lam, rtol=50 * STATS_RTOL, atol=1e-12)


def check_compact(planes, n, r):
    """Survivors bit-exact in the storage type, index map exact, nothing
    written beyond n_keep."""
    keep = r["keep"].astype(bool)
    k = int(keep.sum())
    assert r["n_keep"] == k and r["n_out"] == k
    bits = np.uint32 if planes.dtype.itemsize == 4 else np.uint16
    ref = planes[:, :n][:, keep]
    np.testing.assert_array_equal(r["out"][:, :k].view(bits), ref.view(bits))
    np.testing.assert_array_equal(r["index_map"][:k], np.nonzero(keep)[0].astype(np.int32))
    tail = r["out"][:, k:]
    assert (np.all(np.isnan(tail)) if planes.dtype == np.float32 else np.all(tail.view(np.int16) == INT16_FILL))
    assert np.all(r["index_map"][k:] == -7)


def float_keys(x: np.ndarray) -> np.ndarray:
    """Order-preserving uint32 keys of float32 values (numpy, for checks)."""
    x = np.asarray(x, dtype=np.float32).copy()
    x[x == 0] = 0.0                      # -0 -> +0
    u = x.view(np.uint32).astype(np.uint64)
    key = np.where(u & 0x80000000, (~u) & 0xFFFFFFFF, u | 0x80000000)
    key[np.isnan(x)] = 0xFFFFFFFF
    return key.astype(np.uint64)


def expected_keep_from_scores(scores: np.ndarray, n_prune: int) -> np.ndarray:
    n = scores.size
    order = np.lexsort((np.arange(n), float_keys(scores)))
    keep = np.ones(n, dtype=np.uint8)
    keep[order[:n_prune]] = 0
    return keep


def check_scores(gpu: np.ndarray, D: np.ndarray, lo: np.ndarray, hi: np.ndarray, what: str) -> dict:
    ok = within_interval(gpu, lo, hi)
    bad = np.nonzero(~ok)[0]
    rel = np.abs(gpu.astype(np.float64) - D) / np.maximum(np.abs(D), ABS_TOL / REL_TOL)
    amb = lo != hi
    summary = {"n": gpu.size, "max_rel_unambiguous": float(rel[~amb].max()) if (~amb).any() else 0.0,
               "n_interval": int(amb.sum()), "n_fail": int(bad.size)}
    log(f"[{what}] {summary}")
    if bad.size:
        j = bad[:10]
        raise AssertionError(f"{what}: {bad.size} scores outside tolerance; idx {j}, gpu {gpu[j]}, "
                             f"oracle {D[j]}, lo {lo[j]}, hi {hi[j]}")
    return summary


def check_mask_vs_oracle(keep_gpu, D, lo, hi, n_prune: int, what: str) -> int:
    import oracle
    n = D.size
    keep_o, order = oracle.select(D, n_prune)
    assert int(keep_gpu.sum()) == int(keep_o.sum()) == n - n_prune
    if n_prune == 0 or n_prune == n:
        np.testing.assert_array_equal(keep_gpu, keep_o)
        return 0
    tau_lo = D[order[n_prune - 1]]
    tau_hi = D[order[n_prune]]
    tol = lambda x: np.maximum(REL_TOL * np.abs(x), ABS_TOL)
    border = (lo - tol(lo) <= tau_hi + tol(tau_hi)) & (hi + tol(hi) >= tau_lo - tol(tau_lo))
    diff = keep_gpu.astype(bool) != keep_o.astype(bool)
    bad = diff & ~border
    log(f"[{what}] mask differs on {int(diff.sum())} primitives, {int(border.sum())} borderline")
    assert not bad.any(), f"{what}: {int(bad.sum())} non-borderline mask differences, e.g. {np.nonzero(bad)[0][:10]}"
    return int(diff.sum())


@functools.lru_cache(maxsize=4)
def workload(name: str, n: int | None = None):
    from paper_2606_09074_amd import synth
    spec = synth.SPECS[name]
    if n is not None:
        spec = spec.with_n(n)
    return synth.make_planes(spec), synth.make_cameras(spec), spec


@functools.lru_cache(maxsize=2)
def oracle_workload(name: str):
    """Oracle statistics, weights and scores (with intervals) of a whole
    named workload in FP32 storage, computed once per test session."""
    planes, cams, _ = workload(name)
    return oracle_all(planes, cams)
