"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Scores: |D_gpu - D_ref| <= max(1e-4 |D_ref|, 1e-7), widened to the oracle's
[D_lo, D_hi] where a gate decision lies within FP32 reach.  Masks: equal to a
stable sort of the GPU's own scores (bit-exact) and to the oracle's mask
except for primitives within tolerance of the threshold.  Compaction:
bit-exact given the mask.  Scene statistics: relative 1e-6 (per-primitive
FP32 terms, FP64 sums).
"""
import numpy as np
import pytest

from tests.gpu_common import (check_compact, check_mask_vs_oracle, check_scores, check_stats,
                              expected_keep_from_scores, gpu_params, log, oracle_all, oracle_params, run_gpu,
                              workload)
from tests.helpers import camera, planes_from_prims, raw_prim, within_interval

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_09074_amd import _lib
    _lib.load()


def test_small_workload_full_pipeline():
    planes, cams, spec = workload("small")
    log(f"small: n={spec.n} V={cams.shape[0]}")
    F, lam, D, lo, hi = oracle_all(planes, cams)
    import oracle
    n_prune = oracle.n_prune(spec.n, 0.5)
    r = run_gpu(planes, cams, ratio=0.5)
    check_stats(r["stats"], F, lam, "small")
    assert r["stats"]["n"] == spec.n and r["stats"]["n_nonfinite"] == 0
    check_scores(r["scores"], D, lo, hi, "small scores")
    np.testing.assert_array_equal(r["keep"], expected_keep_from_scores(r["scores"], n_prune))
    check_mask_vs_oracle(r["keep"], D, lo, hi, n_prune, "small mask")
    check_compact(planes, spec.n, r)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 256, 257, 4095, 4096, 4097, 9000])
def test_ragged_sizes(n):
    planes, cams, _ = workload("small")
    sub = np.ascontiguousarray(planes[:, :n])
    F, lam, D, lo, hi = oracle_all(sub, cams)
    r = run_gpu(sub, cams, ratio=0.5)
    check_stats(r["stats"], F, lam, f"n={n}")
    check_scores(r["scores"], D, lo, hi, f"n={n}")
    import oracle
    n_prune = oracle.n_prune(n, 0.5)
    np.testing.assert_array_equal(r["keep"], expected_keep_from_scores(r["scores"], n_prune))
    check_compact(sub, n, r)


def test_padded_stride():
    from paper_2606_09074_amd import synth
    spec = synth.SMALL.with_n(5000)
    planes = synth.make_planes(spec, stride=5000 + 37)
    planes[:, 5000:] = np.nan                       # padding must never be read
    cams = synth.make_cameras(spec)
    F, lam, D, lo, hi = oracle_all(planes, cams, n=5000)
    r = run_gpu(planes, cams, n=5000, ratio=0.3)
    check_stats(r["stats"], F, lam, "padded")
    assert r["stats"]["n_nonfinite"] == 0
    check_scores(r["scores"], D, lo, hi, "padded")
    check_compact(planes, 5000, r)


def test_empty_scene():
    planes = np.zeros((59, 4), dtype=np.float32)
    cams = workload("small")[1]
    r = run_gpu(planes, cams, n=0, ratio=0.5)
    assert r["stats"]["n"] == 0 and r["stats"]["lambda"] == [1 / 3] * 3
    assert r["n_keep"] == 0 and r["n_out"] == 0


@pytest.mark.parametrize("mode", [dict(proj_mode=1), dict(proj_mode=2), dict(vis_mode=1), dict(equal_lambda=1),
                                  dict(n_sub_views=5), dict(proj_mode=1, vis_mode=1, n_sub_views=7)])
def test_method_switches(mode):
    planes, cams, _ = workload("small")
    sub = np.ascontiguousarray(planes[:, :20000])
    F, lam, D, lo, hi = oracle_all(sub, cams, **mode)
    r = run_gpu(sub, cams, params=gpu_params(**mode))
    check_stats(r["stats"], F, lam, str(mode), **mode)
    check_scores(r["scores"], D, lo, hi, str(mode))


def test_opacity_only_ranking():
    """score_kind = OPACITY: D = alpha against the oracle, the mask against
    the oracle's and against a stable sort of the GPU's own scores, compaction
    exact; the prepare/views split and the binned path request change
    nothing."""
    import oracle
    planes, cams, spec = workload("small")
    F, lam, D, lo, hi = oracle_all(planes, cams, score_kind=1)
    n_prune = oracle.n_prune(spec.n, 0.7)
    r = run_gpu(planes, cams, ratio=0.7, params=gpu_params(score_kind=1))
    check_scores(r["scores"], D, lo, hi, "opacity-only scores")
    np.testing.assert_array_equal(r["keep"], expected_keep_from_scores(r["scores"], n_prune))
    check_mask_vs_oracle(r["keep"], D, lo, hi, n_prune, "opacity-only mask")
    check_compact(planes, spec.n, r)
    b = run_gpu(planes, cams[:1], params=gpu_params(score_kind=1, score_path=2))
    np.testing.assert_array_equal(b["scores"].view(np.uint32), r["scores"].view(np.uint32))


def test_single_and_many_views():
    planes, cams, spec = workload("small")
    sub = np.ascontiguousarray(planes[:, :8000])
    for rig in (cams[:1], np.concatenate([cams] * 40)):   # 1 and 640 views
        F, lam, D, lo, hi = oracle_all(sub, rig)
        r = run_gpu(sub, rig)
        check_scores(r["scores"], D, lo, hi, f"V={rig.shape[0]}")


def test_hand_built_degenerate_primitives():
    """Identity-less quaternion, isotropic and needle-like scales, primitives
    on the optical axis, at the near plane, behind and far outside."""
    prims = [raw_prim(mu=(0, 0, 3.0), quat=(0, 0, 0, 0)),
             raw_prim(mu=(0, 0, 3.0), log_scale=(-1.0, -9.0, -9.0), quat=(0.3, 0.5, -0.2, 0.7)),
             raw_prim(mu=(0.01, -0.02, 0.2), log_scale=(-3, -3, -3)),
             raw_prim(mu=(0, 0, -5.0)),
             raw_prim(mu=(500.0, 0, 3.0)),
             raw_prim(mu=(0.2, 0.1, 1.5), log_scale=(-8, -2, -8), logit=8.0, dc=(3, -3, 1)),
             raw_prim(mu=(0, 0, 40.0), logit=-9.0)]
    planes = planes_from_prims(prims)
    cams = np.stack([camera(), camera(t=(0.1, 0.0, 0.5), fx=500.0, fy=450.0)])
    F, lam, D, lo, hi = oracle_all(planes, cams)
    r = run_gpu(planes, cams, n_prune=3)
    check_stats(r["stats"], F, lam, "hand-built")
    check_scores(r["scores"], D, lo, hi, "hand-built")
    assert r["scores"][3] == 0.0 and r["scores"][4] == 0.0
    np.testing.assert_array_equal(r["keep"], expected_keep_from_scores(r["scores"], 3))


def test_nonfinite_inputs_are_counted():
    planes, cams, _ = workload("small")
    sub = np.ascontiguousarray(planes[:, :3000])
    sub[0, 5] = np.nan
    sub[4, 17] = np.inf
    sub[9, 17] = -np.inf
    sub[13, 2999] = np.nan
    sub[30, 100] = np.nan                 # higher SH: not read by the scoring
    r = run_gpu(sub, cams)
    import oracle
    assert r["stats"]["n_nonfinite"] == oracle.nonfinite(sub) == 3


def test_deterministic_and_permutation_consistent():
    planes, cams, _ = workload("small")
    r = run_gpu(planes, cams, repeat=3)
    for other in r["runs"][1:]:
        np.testing.assert_array_equal(other.view(np.uint32), r["runs"][0].view(np.uint32))
    perm = np.random.default_rng(9).permutation(planes.shape[1])
    rp = run_gpu(np.ascontiguousarray(planes[:, perm]), cams)
    np.testing.assert_array_equal(rp["scores"].view(np.uint32), r["scores"][perm].view(np.uint32))


@pytest.mark.slow
@pytest.mark.parametrize("n", [16_777_216 + 4096 * 3 + 17])
def test_select_many_tiles(n):
    """More than 4096 tiles: the per-tile counts of threshold keys go through
    the separate scan; ties spread over many tiles; the threshold key and the
    kept count are exact."""
    import torch

    from paper_2606_09074_amd import api
    rng = np.random.default_rng(5)
    vals = (rng.integers(0, 3000, size=n) * np.float32(0.25)).astype(np.float32)   # heavy ties
    n_prune = int(n * 0.37)
    dev = torch.device("cuda:0")
    s = torch.from_numpy(vals).to(dev)
    keep = torch.empty(n, dtype=torch.uint8, device=dev)
    nk = torch.empty(1, dtype=torch.int64, device=dev)
    thr = torch.empty(1, dtype=torch.int32, device=dev)
    ws = api.workspace(n, 1, dev)
    log(f"select n={n} tiles={(n + 4095) // 4096}")
    api.refine_select(s, keep, ws, n_prune=n_prune, n_keep_out=nk, threshold_out=thr)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(keep.cpu().numpy(), expected_keep_from_scores(vals, n_prune))
    assert int(nk.item()) == n - n_prune


@pytest.mark.parametrize("n_prune", [0, 1, 2, 4999, 5000])
def test_select_edges_and_ties(n_prune):
    import torch

    from paper_2606_09074_amd import api
    n = 5000
    rng = np.random.default_rng(n_prune)
    vals = rng.integers(0, 5, size=n).astype(np.float32) * np.float32(0.5)
    vals[::7] = -0.0
    vals[::11] = 0.0
    vals[3] = np.nan
    vals[9] = -np.float32(2.5)
    vals[10] = np.inf
    dev = torch.device("cuda:0")
    s = torch.from_numpy(vals).to(dev)
    keep = torch.empty(n, dtype=torch.uint8, device=dev)
    nk = torch.empty(1, dtype=torch.int64, device=dev)
    ws = api.workspace(n, 1, dev)
    api.refine_select(s, keep, ws, n_prune=n_prune, n_keep_out=nk)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(keep.cpu().numpy(), expected_keep_from_scores(vals, n_prune))
    assert int(nk.item()) == n - n_prune


def test_select_ties_across_tiles_reused_workspace():
    """Ties at the threshold spread over ~250 tiles (the equal keys before
    each tile come from the last histogram pass's per-tile rows), on one
    workspace reused by calls that prune many, none, then a few."""
    import torch

    from paper_2606_09074_amd import api
    n = 1_000_003
    rng = np.random.default_rng(77)
    vals = (rng.integers(0, 40, size=n) * np.float32(0.25)).astype(np.float32)
    vals[rng.integers(0, n, size=50)] = -0.0
    dev = torch.device("cuda:0")
    s = torch.from_numpy(vals).to(dev)
    ws = api.workspace(n, 1, dev)
    for n_prune in (int(n * 0.61) + 5, 0, 123_457, 1):
        log(f"select ties n={n} n_prune={n_prune}")
        keep = torch.empty(n, dtype=torch.uint8, device=dev)
        nk = torch.empty(1, dtype=torch.int64, device=dev)
        api.refine_select(s, keep, ws, n_prune=n_prune, n_keep_out=nk)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(keep.cpu().numpy(), expected_keep_from_scores(vals, n_prune))
        assert int(nk.item()) == n - n_prune


def test_select_all_equal_scores():
    import torch

    from paper_2606_09074_amd import api
    n = 10007
    dev = torch.device("cuda:0")
    s = torch.full((n,), 0.125, dtype=torch.float32, device=dev)
    keep = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = api.workspace(n, 1, dev)
    api.refine_select(s, keep, ws, ratio=0.37)
    k = api.prune_count(n, 0.37)
    got = keep.cpu().numpy()
    assert got[:k].sum() == 0 and got[k:].all()


def test_compact_capacity_smaller_than_survivors():
    import torch

    from paper_2606_09074_amd import api
    planes, _, _ = workload("small")
    n = 9000
    dev = torch.device("cuda:0")
    pl = torch.from_numpy(np.ascontiguousarray(planes[:, :n])).to(dev)
    keep_np = (np.random.default_rng(2).random(n) < 0.5).astype(np.uint8)
    keep = torch.from_numpy(keep_np).to(dev)
    cap = 1000
    out = torch.full((59, cap + 5), float("nan"), dtype=torch.float32, device=dev)
    idx = torch.full((cap + 5,), -7, dtype=torch.int32, device=dev)
    nout = torch.empty(1, dtype=torch.int64, device=dev)
    ws = api.workspace(n, 1, dev)
    api.refine_compact(pl, keep, out, ws, index_map_out=idx, n_out=nout, capacity=cap)
    torch.cuda.synchronize()
    sel = np.nonzero(keep_np)[0]
    assert int(nout.item()) == sel.size
    np.testing.assert_array_equal(out.cpu().numpy()[:, :cap], planes[:, sel[:cap]])
    np.testing.assert_array_equal(idx.cpu().numpy()[:cap], sel[:cap])
    assert np.all(np.isnan(out.cpu().numpy()[:, cap:])) and np.all(idx.cpu().numpy()[cap:] == -7)


@pytest.mark.slow
@pytest.mark.parametrize("ratio", [0.5, 0.9])
def test_medium_workload_full_parity(ratio):
    """3M primitives x 200 views: every score against the oracle."""
    planes, cams, spec = workload("medium")
    log(f"medium: n={spec.n} V={cams.shape[0]} ratio={ratio}")
    key = ("medium",)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle_all(planes, cams)
    F, lam, D, lo, hi = _ORACLE_CACHE[key]
    import oracle
    n_prune = oracle.n_prune(spec.n, ratio)
    r = run_gpu(planes, cams, ratio=ratio)
    if ratio == 0.5:
        d = run_gpu(planes, cams, params=gpu_params(score_path=1))
        np.testing.assert_array_equal(r["scores"].view(np.uint32), d["scores"].view(np.uint32))
    check_stats(r["stats"], F, lam, "medium")
    summary = check_scores(r["scores"], D, lo, hi, "medium scores")
    assert summary["n_interval"] <= 1e-3 * spec.n
    np.testing.assert_array_equal(r["keep"], expected_keep_from_scores(r["scores"], n_prune))
    check_mask_vs_oracle(r["keep"], D, lo, hi, n_prune, f"medium mask beta={ratio}")
    check_compact(planes, spec.n, r)


_ORACLE_CACHE = {}


@pytest.mark.slow
def test_paper_configuration_at_full_size():
    """The paper's own cost setting (Table B.1): the depth-only projection
    term of Eq. 17 over 64 subsampled views, on the 3M-primitive, 200-view
    workload: every score against the oracle in the same mode, the mask at
    beta 0.5 against the oracle's, and the binned path equal to the direct
    one."""
    import oracle
    planes, cams, spec = workload("medium")
    mode = dict(proj_mode=1, n_sub_views=64)
    F, lam, D, lo, hi = oracle_all(planes, cams, **mode)
    n_prune = oracle.n_prune(spec.n, 0.5)
    r = run_gpu(planes, cams, ratio=0.5, params=gpu_params(**mode))
    d = run_gpu(planes, cams, params=gpu_params(score_path=1, **mode))
    np.testing.assert_array_equal(r["scores"].view(np.uint32), d["scores"].view(np.uint32))
    check_stats(r["stats"], F, lam, "paper configuration", **mode)
    summary = check_scores(r["scores"], D, lo, hi, "paper configuration scores")
    assert summary["n_interval"] <= 1e-3 * spec.n
    np.testing.assert_array_equal(r["keep"], expected_keep_from_scores(r["scores"], n_prune))
    check_mask_vs_oracle(r["keep"], D, lo, hi, n_prune, "paper configuration mask")
    check_compact(planes, spec.n, r)


@pytest.mark.slow
def test_large_workload_full_parity():
    """6M primitives x 300 views at beta 0.66: every score against the
    oracle, the mask against the oracle's (identical except borderline) and
    against a stable sort of the GPU's own scores, compaction exact."""
    import oracle
    planes, cams, spec = workload("large")
    log(f"large: n={spec.n} V={cams.shape[0]}")
    F, lam, D, lo, hi = oracle_all(planes, cams)
    n_prune = oracle.n_prune(spec.n, 0.66)
    r = run_gpu(planes, cams, ratio=0.66)
    check_stats(r["stats"], F, lam, "large")
    summary = check_scores(r["scores"], D, lo, hi, "large scores")
    # 300 views give each primitive 1.5 times the chances of a flagged view
    # of the 200-view workload, whose bound is 0.1%
    assert summary["n_interval"] <= 1.5e-3 * spec.n
    np.testing.assert_array_equal(r["keep"], expected_keep_from_scores(r["scores"], n_prune))
    check_mask_vs_oracle(r["keep"], D, lo, hi, n_prune, "large mask beta=0.66")
    check_compact(planes, spec.n, r)


def _paths(planes, cams, n=None, **kw):
    direct = run_gpu(planes, cams, n=n, params=gpu_params(score_path=1, **kw))
    binned = run_gpu(planes, cams, n=n, params=gpu_params(score_path=2, **kw))
    return direct, binned


@pytest.mark.parametrize("name,n,mode", [("small", None, {}), ("small", 9000, {}), ("small", 777, {}),
                                         ("small", None, dict(proj_mode=1)), ("small", None, dict(proj_mode=2)),
                                         ("small", None, dict(vis_mode=1, n_sub_views=6)),
                                         ("medium", 400_000, {}), ("small", 9000, dict(records_per_lane=2)),
                                         ("medium", 400_000, dict(records_per_lane=2)),
                                         ("small", 9000, dict(records_per_lane=1, views_per_iteration=2)),
                                         ("medium", 400_000, dict(records_per_lane=2, views_per_iteration=2)),
                                         ("small", 9000, dict(waves_per_block=1)),
                                         ("small", None, dict(records_per_lane=1, waves_per_block=2)),
                                         ("medium", 400_000, dict(records_per_lane=2, waves_per_block=8)),
                                         ("medium", 400_000, dict(records_per_lane=1, views_per_iteration=2,
                                                                  waves_per_block=8))])
def test_binned_and_direct_paths_bit_identical(name, n, mode):
    """Culling skips only (group, view) pairs whose every primitive is gated
    out, so the binned path must reproduce the direct path bit for bit."""
    planes, cams, spec = workload(name)
    sub = np.ascontiguousarray(planes[:, :n]) if n else planes
    d, b = _paths(sub, cams, **mode)
    np.testing.assert_array_equal(b["scores"].view(np.uint32), d["scores"].view(np.uint32))
    log(f"[paths {name} n={sub.shape[1]} {mode}] identical; nonzero {int((d['scores'] > 0).sum())}")


def _edge_scene(n, seed):
    """Primitives just outside the image of camera() (320 x 240, f = 300),
    each with 3 s f / z between 0.5 and 1.0 times its distance to the image
    edge (off-axis Jacobians make the actual radius larger), some
    needle-like and rotated, plus some at the near plane: about half of
    them score, so the culling bound and the loop's screen are exercised at
    the gate's boundary."""
    from tests.helpers import planes_from_prims, raw_prim
    rng = np.random.default_rng(seed)
    prims = []
    for i in range(n):
        z = rng.uniform(1.0, 8.0)
        d = rng.uniform(0.5, 40.0)
        side = rng.integers(4)
        u = -d if side == 0 else (320.0 + d if side == 1 else rng.uniform(0.0, 320.0))
        v = -d if side == 2 else (240.0 + d if side == 3 else rng.uniform(0.0, 240.0))
        if i % 10 == 0:   # at the near plane
            z = rng.uniform(0.15, 0.25)
        x, y = (u - 160.0) * z / 300.0, (v - 120.0) * z / 300.0
        s = rng.uniform(0.5, 1.0) * d * z / (3.0 * 300.0)
        ls = np.log(np.full(3, s))
        q = (1.0, 0.0, 0.0, 0.0)
        if i % 3 == 0:    # needle-like, rotated
            ls = ls + np.log(np.array([2.0, 0.3, 0.3]))
            q = tuple(rng.normal(size=4))
        prims.append(raw_prim(mu=(x, y, z), log_scale=tuple(ls), quat=q, logit=rng.normal(),
                              dc=tuple(rng.normal(scale=0.5, size=3))))
    return planes_from_prims(prims)


@pytest.mark.parametrize("mode", [{}, dict(records_per_lane=1), dict(views_per_iteration=2)])
def test_binned_matches_direct_at_the_gate_boundary(mode):
    """Binned and direct paths stay bit-identical when many pairs sit at the
    footprint gate's boundary, where the culling bound and the view loop's
    screen are tightest."""
    planes = _edge_scene(12_000, 31)
    # the reference camera and small shifts of it, so each primitive meets
    # the boundary at several distances
    cams = np.stack([camera(t=(dx, dy, 0.0)) for dx, dy in
                     [(0, 0), (0.01, 0), (-0.01, 0), (0, 0.01), (0, -0.01), (0.02, 0.02)]])
    d, b = _paths(planes, cams, **mode)
    np.testing.assert_array_equal(b["scores"].view(np.uint32), d["scores"].view(np.uint32))
    frac = float((d["scores"] > 0).mean())
    log(f"[gate boundary {mode}] identical; scored > 0: {frac:.3f}")
    assert 0.2 < frac < 0.95   # the scene straddles the boundary


@pytest.mark.parametrize("rec,vpi", [(1, 1), (2, 1), (2, 2)])
@pytest.mark.parametrize("n,v", [(5, 3), (777, 1), (9000, 65), (9000, 640)])
def test_binned_view_masks_and_chunks(n, v, rec, vpi):
    """The binned view phase at its edges: fewer primitives than one group,
    a single view, a second mask word holding one view, and more views than
    one LDS camera chunk (several mask words and chunks per group)."""
    planes, cams, _ = workload("small")
    sub = np.ascontiguousarray(planes[:, :n])
    rig = np.ascontiguousarray(np.concatenate([cams] * (v // cams.shape[0] + 1))[:v])
    d, b = _paths(sub, rig, records_per_lane=rec, views_per_iteration=vpi)
    np.testing.assert_array_equal(b["scores"].view(np.uint32), d["scores"].view(np.uint32))
    if n >= 777 and vpi == 1:
        F, lam, D, lo, hi = oracle_all(sub, rig)
        check_scores(b["scores"], D, lo, hi, f"binned n={n} V={v} rec={rec}")


def test_maximum_view_count():
    """The largest camera set a call takes, 2^20 views (16384 mask words and
    4096 LDS camera chunks per group), on 64 primitives: both paths
    bit-identical and within the rounding bound of their FP32 view sums of
    the oracle.  Each primitive's sum adds 64-view blocks in order, each block
    summed in order, so to first order its relative error stays below
    (64 + V/64 + 2) * 2^-24 (about 1e-3 here; a plain running sum would
    allow V * 2^-24 = 6%).  The rig repeats the 16 ring cameras, so the
    oracle's scores also equal its scores for the 16 cameras alone."""
    planes, cams, _ = workload("small")
    n, V = 64, 1 << 20
    sub = np.ascontiguousarray(planes[:, :n])
    rig = np.ascontiguousarray(np.tile(cams, (V // cams.shape[0], 1)))
    assert rig.shape == (V, 18)
    log(f"[max views] n={n} V={V}")
    d, b = _paths(sub, rig)
    np.testing.assert_array_equal(b["scores"].view(np.uint32), d["scores"].view(np.uint32))
    F, lam, D, lo, hi = oracle_all(sub, rig)
    D16 = oracle_all(sub, cams)[2]
    # the oracle's own FP64 running sum over V views: within V * 2^-53
    np.testing.assert_allclose(D, D16, rtol=V * 2.0 ** -53, atol=1e-300)
    bound = (64 + V // 64 + 2) * 2.0 ** -24
    ok = within_interval(d["scores"], lo, hi, rel=bound)
    amb = lo != hi
    live = (D > 0) & ~amb
    rel = np.abs(d["scores"].astype(np.float64) - D)[live] / D[live]
    log(f"[max views] {int(live.sum())} unambiguous nonzero scores, max rel error {rel.max():.2e} "
        f"(bound {bound:.2e}); {int(amb.sum())} with intervals")
    assert live.sum() >= 16
    assert ok.all(), np.nonzero(~ok)[0]


def test_binned_path_with_degenerate_and_nonfinite_inputs():
    planes, cams, _ = workload("small")
    sub = np.ascontiguousarray(planes[:, :20000])
    sub[:, 100:164] = sub[:, 100:101]          # 64 identical primitives
    sub[3:6, 200] = -30.0                      # vanishing scales
    sub[3, 201] = 4.0                          # a huge one
    sub[0, 300] = np.nan
    sub[1, 301] = np.inf
    sub[2, 302] = -np.inf
    sub[6:10, 400] = 0.0                       # zero quaternion
    d, b = _paths(sub, cams)
    fin = np.isfinite(d["scores"])
    np.testing.assert_array_equal(np.isfinite(b["scores"]), fin)
    np.testing.assert_array_equal(b["scores"][fin].view(np.uint32), d["scores"][fin].view(np.uint32))
    assert d["stats"]["n_nonfinite"] == 3


def test_stats_bounding_box():
    planes, cams, _ = workload("small")
    sub = np.ascontiguousarray(planes[:, :10000])
    sub[0, 7] = np.inf
    sub[1, 8] = np.nan
    r = run_gpu(sub, cams)
    mu = sub[0:3].astype(np.float64)
    for a in range(3):
        v = mu[a][np.isfinite(mu[a])]
        assert r["stats"]["bbox_min"][a] == np.float32(v.min())
        assert r["stats"]["bbox_max"][a] == np.float32(v.max())


@pytest.mark.parametrize("path", [1, 2])
def test_two_phase_scoring(path):
    """refine_score_prepare + refine_score_views (twice) equals refine_score;
    the counts: n |V| evaluated and none screened on the direct path; on the
    binned path some of each, together fewer than n |V| (culled pairs are
    in neither)."""
    import torch

    from paper_2606_09074_amd import _lib, api
    planes, cams, _ = workload("medium")
    n = 300_000
    sub = np.ascontiguousarray(planes[:, :n])
    ref = run_gpu(sub, cams, params=gpu_params(score_path=path))["scores"]
    dev = torch.device("cuda:0")
    pl = torch.from_numpy(sub).to(dev)
    cm = torch.from_numpy(cams).to(dev)
    ws = api.workspace(n, cams.shape[0], dev)
    st = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
    prm = gpu_params(score_path=path)
    api.refine_stats(pl, st, ws, prm)
    api.refine_score_prepare(pl, cm, st, ws, prm)
    ev = torch.full((2,), -1, dtype=torch.int64, device=dev)
    for _ in range(2):
        out = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
        api.refine_score_views(pl, cams.shape[0], st, out, ws, prm, evaluated_out=ev)
        np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    total = n * cams.shape[0]
    got, screened = (int(x) for x in ev.cpu().tolist())
    log(f"[two-phase path={path}] evaluated {got}, screened {screened} of {total} pairs ({got / total:.3f})")
    if path == 1:
        assert got == total and screened == 0
    else:
        assert 0 < got and 0 < screened and got + screened < total


@pytest.mark.parametrize("n,stride,mask_offset,cap_frac", [(9000, 9000, 0, 1.0), (8999, 9000, 0, 1.0),
                                                          (8999, 9000, 0, 0.3), (9000, 9001, 0, 1.0),
                                                          (9000, 9000, 1, 1.0), (4096 * 3, 4096 * 3, 0, 0.5)])
def test_compact_vector_and_scalar_kernels(n, stride, mask_offset, cap_frac):
    """The 16-byte path (aligned planes and mask) and the scalar fallback
    (odd stride, unaligned mask) give the same bit-exact survivors."""
    import torch

    from paper_2606_09074_amd import api
    from paper_2606_09074_amd import synth
    planes = synth.make_planes(synth.SMALL.with_n(n), stride=stride)
    dev = torch.device("cuda:0")
    pl = torch.from_numpy(planes).to(dev)
    keep_np = (np.random.default_rng(n + stride).random(n) < 0.45).astype(np.uint8)
    buf = torch.zeros(n + 8, dtype=torch.uint8, device=dev)
    keep = buf[mask_offset:mask_offset + n]
    keep.copy_(torch.from_numpy(keep_np).to(dev))
    sel = np.nonzero(keep_np)[0]
    cap = int(sel.size * cap_frac)
    out = torch.full((59, cap + 4), float("nan"), dtype=torch.float32, device=dev)
    idx = torch.full((cap + 4,), -7, dtype=torch.int32, device=dev)
    nout = torch.empty(1, dtype=torch.int64, device=dev)
    ws = api.workspace(n, 1, dev)
    api.refine_compact(pl, keep, out, ws, index_map_out=idx, n_out=nout, n=n, capacity=cap)
    torch.cuda.synchronize()
    assert int(nout.item()) == sel.size
    o = out.cpu().numpy()
    np.testing.assert_array_equal(o[:, :cap].view(np.uint32), planes[:, sel[:cap]].view(np.uint32))
    np.testing.assert_array_equal(idx.cpu().numpy()[:cap], sel[:cap])
    assert np.all(np.isnan(o[:, cap:])) and np.all(idx.cpu().numpy()[cap:] == -7)


@pytest.mark.parametrize("path,rec", [(1, 0), (2, 1), (2, 2)])
def test_rescoring_with_new_cameras(path, rec):
    """A scene prepared once and scored for further camera sets (camera tables
    rebuilt only) gives the same scores, bit for bit, as scoring each camera
    set from scratch; and those match the oracle."""
    import torch

    from paper_2606_09074_amd import _lib, api, synth
    planes, camsA, spec = workload("small")
    camsB = synth.ring_cameras(7)                       # fewer views, another rig
    camsC = np.ascontiguousarray(camsA[::-1][:13])
    dev = torch.device("cuda:0")
    pl = torch.from_numpy(planes).to(dev)
    prm = gpu_params(score_path=path, records_per_lane=rec)
    ws = api.workspace(spec.n, 16, dev)
    st = torch.empty(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
    api.refine_stats(pl, st, ws, prm)
    out = {}
    tA = torch.from_numpy(camsA).to(dev)
    api.refine_score_prepare(pl, tA, st, ws, prm)
    for name, c in (("A", camsA), ("B", camsB), ("C", camsC), ("A2", camsA)):
        tc = torch.from_numpy(c).to(dev)
        if name != "A":
            api.refine_score_cameras(pl, tc, ws, prm)
        sc = torch.empty(spec.n, dtype=torch.float32, device=dev)
        api.refine_score_views(pl, c.shape[0], st, sc, ws, prm)
        out[name] = sc.cpu().numpy()
    for name, c in (("A", camsA), ("B", camsB), ("C", camsC)):
        fresh = run_gpu(planes, c, params=gpu_params(score_path=path, records_per_lane=rec))["scores"]
        np.testing.assert_array_equal(out[name].view(np.uint32), fresh.view(np.uint32))
        F, lam, D, lo, hi = oracle_all(planes, c)
        check_scores(out[name], D, lo, hi, f"rescored {name} path={path} ppl={rec}")
    np.testing.assert_array_equal(out["A2"].view(np.uint32), out["A"].view(np.uint32))
