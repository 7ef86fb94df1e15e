"""refine_stats_noalloc (the statistics on the library's fixed device array,
for callers that cannot allocate) against refine_stats with a workspace:
the same bytes of refine_stats_t, on two calls in a row with the second
smaller, through the C ABI; and one call captured in a HIP graph, replayed
on new contents."""
import numpy as np
import pytest

from tests.gpu_common import gpu_params, log, workload

pytestmark = pytest.mark.gpu


def _stats_pair(planes_np, n, params):
    import torch

    from paper_2606_09074_amd import _lib, api
    dev = torch.device("cuda:0")
    pl = torch.from_numpy(np.ascontiguousarray(planes_np)).to(dev)
    ws = api.workspace(n, 0, dev)
    ref = torch.full((_lib.STATS_BYTES,), 0xA5, dtype=torch.uint8, device=dev)
    got = torch.full((_lib.STATS_BYTES,), 0x5A, dtype=torch.uint8, device=dev)
    api.refine_stats(pl, ref, ws, params, n=n)
    api.refine_stats_noalloc(pl, got, params, n=n)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_stats_match_workspace_stats_twice():
    import torch
    planes, _, spec = workload("medium")
    prm = gpu_params()
    # 3M primitives (733 tiles), then a smaller ragged scene on the same
    # array: the second call must not see the first call's partials
    for n in (spec.n, 123_457, 1):
        log(f"noalloc stats n={n}")
        ref, got = _stats_pair(planes[:, :n], n, prm)
        np.testing.assert_array_equal(got, ref)
    del torch


def test_noalloc_stats_other_storage_and_switches():
    from paper_2606_09074_amd import synth
    planes, _, _ = workload("small")
    q = synth.quantize_bf16_f16(planes[:, :20000])
    for pl, prm in ((q, gpu_params()), (planes[:, :9001], gpu_params(equal_lambda=1))):
        n = pl.shape[1]
        log(f"noalloc stats n={n} dtype={pl.dtype}")
        ref, got = _stats_pair(pl, n, prm)
        np.testing.assert_array_equal(got, ref)


def test_noalloc_stats_rejects_scenes_beyond_its_array():
    import torch

    from paper_2606_09074_amd import _lib, api
    dev = torch.device("cuda:0")
    pl = torch.zeros((59, 8), dtype=torch.float32, device=dev)
    st = torch.zeros(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
    with pytest.raises(_lib.RefineError) as e:
        # n is checked against the array before anything is enqueued: the
        # planes (too short for this n) are never read
        sc = api._scene(pl)
        sc.n = _lib.STATS_NOALLOC_MAX_N + 1
        sc.stride = sc.n
        _lib.check(_lib.load().refine_stats_noalloc(api.ctypes.byref(sc), api.ctypes.byref(gpu_params()),
                                                    api._ptr(st), api._stream_ptr(None)), "refine_stats_noalloc")
    assert e.value.status == _lib.REFINE_E_UNSUPPORTED


def test_noalloc_stats_replayed_from_a_graph():
    """The use the allocation-free entry point exists for: one call captured
    in a graph and replayed on new scene contents, written eagerly between
    the replays; every replay gives the bytes refine_stats with a workspace
    gives on the same contents."""
    import torch

    from paper_2606_09074_amd import _lib, api
    planes, _, _ = workload("small")
    n = 40_000
    dev = torch.device("cuda:0")
    prm = gpu_params()
    pl = torch.from_numpy(np.ascontiguousarray(planes[:, :n])).to(dev)
    got = torch.zeros(_lib.STATS_BYTES, dtype=torch.uint8, device=dev)
    # the first call on the device resolves the array's address (before capture)
    api.refine_stats_noalloc(pl, got, prm, n=n)
    torch.cuda.synchronize()
    side = torch.cuda.Stream(dev)   # default priority
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        api.refine_stats_noalloc(pl, got, prm, n=n)
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    log("noalloc stats: capturing one call")
    with torch.cuda.graph(graph):
        api.refine_stats_noalloc(pl, got, prm, n=n)
    torch.cuda.synchronize()
    ws = api.workspace(n, 0, dev)
    ref = torch.zeros_like(got)
    rng = np.random.default_rng(5)
    for r in range(4):
        # new contents each time: other primitives of the scene, scales shifted
        pick = rng.permutation(planes.shape[1])[:n]
        new = np.ascontiguousarray(planes[:, pick])
        new[3:6] += np.float32(0.25 * r)
        pl.copy_(torch.from_numpy(new))
        got.fill_(0x5A)
        torch.cuda.synchronize()
        graph.replay()
        api.refine_stats(pl, ref, ws, prm, n=n)
        torch.cuda.synchronize()
        log(f"noalloc stats: replay {r}")
        np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())
    del graph
