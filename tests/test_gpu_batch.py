"""Batched pruning (one grouped launch per kernel for many scenes) gives,
for every job, the same statistics, scores, mask and survivors, bit for
bit, as the single-scene calls with the direct scoring path; and the scores
match the oracle."""
import numpy as np
import pytest

from paper_2606_09074_amd import synth
from tests.gpu_common import check_scores, gpu_params, log, oracle_all, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_09074_amd import _lib
    _lib.load()


def _jobs():
    """Ragged sizes, both storages, several rigs and ratios, one padded stride
    (scalar compaction), one output below the survivor count."""
    base = synth.make_planes(synth.SMALL)
    spec = [  # (n, stride, storage, views, ratio, capacity fraction)
        (1, 1, "f32", 16, 0.5, 1.0), (777, 777, "f32", 7, 0.3, 1.0), (4096, 4096, "mixed", 16, 0.9, 1.0),
        (4097, 4103, "f32", 33, 0.5, 1.0), (20000, 20000, "mixed", 50, 0.66, 1.0),
        (50000, 50000, "f32", 16, 0.5, 0.8), (9001, 9003, "mixed", 5, 0.41, 1.0),
        (12345, 12352, "half", 24, 0.5, 1.0), (3001, 3003, "half", 9, 0.7, 0.9)]
    out = []
    for n, stride, store, V, ratio, capf in spec:
        pl = np.zeros((59, stride), np.float32)
        pl[:, :n] = base[:, :n]
        if store == "mixed":
            pl = synth.quantize_bf16_f16(pl)
        elif store == "half":
            pl = synth.quantize_f16(pl)
        out.append((pl, n, synth.ring_cameras(V), ratio, capf))
    return out


def test_batch_matches_single_scene_calls():
    import torch

    from paper_2606_09074_amd import _lib, api
    dev = torch.device("cuda:0")
    jobs, singles = [], []
    for pl_np, n, cams_np, ratio, capf in _jobs():
        pl = torch.from_numpy(pl_np).to(dev)
        cams = torch.from_numpy(cams_np).to(dev)
        cap = int((n - api.prune_count(n, ratio)) * capf)
        out = (torch.full((59, cap + 3), float("nan"), dtype=pl.dtype, device=dev) if pl.dtype == torch.float32
               else torch.full((59, cap + 3), -12345, dtype=torch.int16, device=dev).view(pl.dtype))
        jobs.append({"planes": pl, "n": n, "cams": cams, "ratio": ratio,
                     "stats": torch.zeros(_lib.STATS_BYTES, dtype=torch.uint8, device=dev),
                     "scores": torch.full((n,), float("nan"), dtype=torch.float32, device=dev),
                     "keep": torch.full((n,), 7, dtype=torch.uint8, device=dev),
                     "n_keep": torch.full((1,), -1, dtype=torch.int64, device=dev),
                     "out": out, "capacity": cap,
                     "index_map": torch.full((cap + 3,), -7, dtype=torch.int32, device=dev),
                     "n_out": torch.full((1,), -1, dtype=torch.int64, device=dev)})
        singles.append(run_gpu(pl_np, cams_np, n=n, ratio=ratio, params=gpu_params(score_path=1)))
    prm = gpu_params()
    ws = torch.empty(api.batch_workspace_size(jobs, prm), dtype=torch.uint8, device=dev)
    log(f"batch of {len(jobs)} jobs, n = {[j['n'] for j in jobs]}, workspace {ws.numel()} B")
    api.refine_prune_batch(jobs, ws, prm)
    torch.cuda.synchronize()
    for j, r, (pl_np, n, cams_np, ratio, capf) in zip(jobs, singles, _jobs()):
        what = f"job n={n} V={cams_np.shape[0]} ratio={ratio} {pl_np.dtype}"
        st = api.stats_from_tensor(j["stats"])
        for k in ("ybar", "f_col", "f_opa", "f_gem", "lambda", "n", "n_nonfinite", "bbox_min", "bbox_max"):
            assert st[k] == r["stats"][k], (what, k)
        np.testing.assert_array_equal(j["scores"].cpu().numpy().view(np.uint32), r["scores"].view(np.uint32))
        keep = j["keep"].cpu().numpy()
        np.testing.assert_array_equal(keep, r["keep"])
        k = int(keep.sum())
        assert int(j["n_keep"].item()) == k and int(j["n_out"].item()) == k
        cap = j["capacity"]
        sel = np.nonzero(keep)[0][:cap]
        out = j["out"].cpu().numpy()
        bits = np.uint32 if pl_np.dtype == np.float32 else np.uint16
        np.testing.assert_array_equal(out[:, :cap].view(bits), pl_np[:, sel].view(bits))
        np.testing.assert_array_equal(j["index_map"].cpu().numpy()[:cap], sel.astype(np.int32))
        tail = out[:, cap:]
        assert np.all(np.isnan(tail)) if pl_np.dtype == np.float32 else np.all(tail.view(np.int16) == -12345)
        deq = {np.dtype(np.float32): lambda x: x, np.dtype(np.int16): synth.dequantize_bf16_f16,
               np.dtype(np.float16): synth.dequantize_f16}[pl_np.dtype](pl_np)
        F, lam, D, lo, hi = oracle_all(deq, cams_np, n=n)
        check_scores(j["scores"].cpu().numpy(), D, lo, hi, what)


@pytest.mark.parametrize("mode", [dict(proj_mode=1), dict(proj_mode=2, vis_mode=1), dict(n_sub_views=5, equal_lambda=1),
                                  dict(score_kind=1)])
def test_batch_method_switches(mode):
    """The batch applies the shared parameters like the single calls do."""
    import torch

    from paper_2606_09074_amd import api
    dev = torch.device("cuda:0")
    base = synth.make_planes(synth.SMALL)
    scenes_np = [np.ascontiguousarray(base[:, a:a + n]) for a, n in ((0, 3000), (5000, 12345), (20000, 777))]
    cams_np = [synth.ring_cameras(V) for V in (16, 9, 31)]
    ratios = [0.5, 0.25, 0.75]
    prm = gpu_params(**mode)
    res = api.prune_batch([torch.from_numpy(p).to(dev) for p in scenes_np],
                          [torch.from_numpy(c).to(dev) for c in cams_np], ratios, params=prm)
    torch.cuda.synchronize()
    for r, p, c, ratio in zip(res, scenes_np, cams_np, ratios):
        single = run_gpu(p, c, ratio=ratio, params=gpu_params(score_path=1, **mode))
        np.testing.assert_array_equal(r["scores"].cpu().numpy().view(np.uint32), single["scores"].view(np.uint32))
        np.testing.assert_array_equal(r["keep"].cpu().numpy(), single["keep"])
        F, lam, D, lo, hi = oracle_all(p, c, **mode)
        check_scores(r["scores"].cpu().numpy(), D, lo, hi, f"batch {mode} n={p.shape[1]}")


def test_batch_nonfinite_inputs():
    """Non-finite inputs are counted per job and give the single-call results."""
    import torch

    from paper_2606_09074_amd import api
    dev = torch.device("cuda:0")
    base = synth.make_planes(synth.SMALL)
    a = np.ascontiguousarray(base[:, :3000]).copy()
    b = np.ascontiguousarray(base[:, 3000:9000]).copy()
    a[0, 7] = np.nan
    a[4, 100] = np.inf
    b[12, 5] = -np.inf
    cams = synth.ring_cameras(16)
    res = api.prune_batch([torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)],
                          [torch.from_numpy(cams).to(dev)] * 2, [0.5, 0.5])
    torch.cuda.synchronize()
    for r, p, bad in zip(res, (a, b), (2, 1)):
        st = api.stats_from_tensor(r["stats"])
        assert st["n_nonfinite"] == bad
        single = run_gpu(p, cams, ratio=0.5, params=gpu_params(score_path=1))
        np.testing.assert_array_equal(r["scores"].cpu().numpy().view(np.uint32), single["scores"].view(np.uint32))
        np.testing.assert_array_equal(r["keep"].cpu().numpy(), single["keep"])
