"""refine_stats_noalloc (the statistics on the library's fixed device array,
for callers that cannot allocate) against refine_stats with a workspace:
the same bytes of refine_stats_t, on two calls in a row with the second
smaller, through the C ABI."""
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
