"""GPU parity of the 2-byte scene storage (planes 0..10 BF16, planes 11..58
FP16, FP32 arithmetic) against the FP64 oracle on the dequantised inputs,
with the same tolerances as the FP32 storage; and the effect of the storage
itself (scores and kept sets against the FP32 scene).

The storage changes the inputs, not the arithmetic: the oracle runs on the
exact values the 2-byte planes hold, so the parity bar is unchanged.
"""
import numpy as np
import pytest

from paper_2606_09074_amd import synth
from tests.gpu_common import (check_compact, check_mask_vs_oracle, check_scores, check_stats,
                              expected_keep_from_scores, gpu_params, log, oracle_all, run_gpu, workload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_09074_amd import _lib
    _lib.load()


def _mixed(planes):
    q = synth.quantize_bf16_f16(planes)
    return q, synth.dequantize_bf16_f16(q)


def _pipeline(q, deq, cams, n, ratios, what):
    """Stats, scores, then for each ratio the mask and compaction, all
    against the oracle on the dequantised scene; returns the last run."""
    import oracle
    F, lam, D, lo, hi = oracle_all(deq, cams, n=n)
    r = None
    for ratio in np.atleast_1d(ratios):
        n_prune = oracle.n_prune(n, float(ratio))
        r = run_gpu(q, cams, n=n, ratio=float(ratio))
        check_stats(r["stats"], F, lam, what)
        assert r["stats"]["n"] == n and r["stats"]["n_nonfinite"] == 0
        check_scores(r["scores"], D, lo, hi, f"{what} scores")
        np.testing.assert_array_equal(r["keep"], expected_keep_from_scores(r["scores"], n_prune))
        check_mask_vs_oracle(r["keep"], D, lo, hi, n_prune, f"{what} mask beta={float(ratio)}")
        check_compact(q, n, r)
    return r


def test_small_mixed_full_pipeline():
    planes, cams, spec = workload("small")
    q, deq = _mixed(planes)
    log(f"small mixed: n={spec.n} V={cams.shape[0]}")
    _pipeline(q, deq, cams, spec.n, 0.5, "small mixed")


@pytest.mark.parametrize("n", [1, 65, 4095, 4097, 9000])
def test_mixed_ragged_sizes(n):
    planes, cams, _ = workload("small")
    q, deq = _mixed(np.ascontiguousarray(planes[:, :n]))
    log(f"mixed ragged n={n}")
    _pipeline(q, deq, cams, n, 0.5, f"mixed n={n}")


@pytest.mark.parametrize("stride_pad", [0, 3])
def test_mixed_padded_stride(stride_pad):
    """stride % 4 == 3 sends the compaction to its scalar kernel."""
    planes, cams, _ = workload("small")
    n = 5000
    q, deq = _mixed(np.ascontiguousarray(planes[:, :n]))
    qp = np.full((59, n + stride_pad), 0x7C01, dtype=np.int16)   # FP16 NaN / BF16 huge: must never be read
    qp[:, :n] = q
    log(f"mixed padded stride {n + stride_pad}")
    _pipeline(qp, deq, cams, n, 0.3, f"mixed stride={n + stride_pad}")


@pytest.mark.parametrize("name,n", [("small", None), ("medium", 400_000)])
def test_mixed_binned_and_direct_paths_bit_identical(name, n):
    planes, cams, _ = workload(name)
    q, _ = _mixed(np.ascontiguousarray(planes[:, :n]) if n else planes)
    d = run_gpu(q, cams, params=gpu_params(score_path=1))
    b = run_gpu(q, cams, params=gpu_params(score_path=2))
    np.testing.assert_array_equal(b["scores"].view(np.uint32), d["scores"].view(np.uint32))
    log(f"[mixed paths {name} n={q.shape[1]}] identical")


def test_mixed_nonfinite_inputs_are_counted():
    planes, cams, _ = workload("small")
    q, deq = _mixed(np.ascontiguousarray(planes[:, :2000]))
    q[0, 5] = np.int16(0x7FC0)                  # BF16 NaN centre
    q[12, 17] = np.int16(0x7C00)                 # FP16 +inf colour
    q[40, 23] = np.int16(0x7C00)                 # higher SH: not read by the scoring
    r = run_gpu(q, cams)
    assert r["stats"]["n_nonfinite"] == 2


def _jaccard(a, b):
    a, b = a.astype(bool), b.astype(bool)
    return float((a & b).sum()) / float((a | b).sum())


@pytest.mark.slow
def test_medium_mixed_parity_and_storage_effect():
    """3M x 200: every score of the 2-byte scene against the oracle on the
    dequantised scene; then the storage effect against the FP32 scene (kept-set
    Jaccard at beta 0.5 and 0.9, score relative error)."""
    planes, cams, spec = workload("medium")
    q, deq = _mixed(planes)
    log(f"medium mixed: n={spec.n} V={cams.shape[0]}")
    r16 = _pipeline(q, deq, cams, spec.n, (0.9, 0.5), "medium mixed")
    r32 = run_gpu(planes, cams)
    s16, s32 = r16["scores"].astype(np.float64), r32["scores"].astype(np.float64)
    nz = s32 > 0
    rel = np.abs(s16[nz] - s32[nz]) / s32[nz]
    out = {"rel_median": float(np.median(rel)), "rel_p99": float(np.quantile(rel, 0.99))}
    for beta in (0.5, 0.9):
        k = int(np.floor(beta * spec.n + 0.5))
        out[f"jaccard_kept_{beta}"] = _jaccard(expected_keep_from_scores(r16["scores"], k),
                                               expected_keep_from_scores(r32["scores"], k))
    log(f"[medium storage effect] {out}")
    # BF16 centres move by up to 2^-9 |x| (0.04 world units at |x| = 20): the
    # storage shifts scores by ~0.3% typically; the kept sets stay close
    assert out["jaccard_kept_0.5"] >= 0.99 and out["jaccard_kept_0.9"] >= 0.98, out


@pytest.mark.parametrize("n,stride,mask_offset,even_out,cap_frac",
                         [(9000, 9000, 0, True, 1.0),      # 16-byte loads, paired 2-byte stores
                          (9000, 9000, 0, False, 1.0),     # odd output stride: single 2-byte stores
                          (8999, 9008, 0, True, 0.6),      # ragged tail, capacity below the survivors
                          (9001, 9003, 1, True, 1.0),      # stride not a multiple of 8, unaligned mask: scalar
                          (20000, 20000, 0, True, 0.97)])
def test_mixed_compact_kernels(n, stride, mask_offset, even_out, cap_frac):
    """2-byte compaction: the 16-byte-load kernel with paired or single stores
    and the scalar fallback copy the survivors bit for bit, stably (tiles
    start at odd and even output offsets)."""
    import torch

    from paper_2606_09074_amd import api
    planes = synth.quantize_bf16_f16(synth.make_planes(synth.SMALL.with_n(n), stride=stride))
    dev = torch.device("cuda:0")
    pl = torch.from_numpy(planes).to(dev)
    keep_np = (np.random.default_rng(n + stride).random(n) < 0.45).astype(np.uint8)
    buf = torch.zeros(n + 8, dtype=torch.uint8, device=dev)
    keep = buf[mask_offset:mask_offset + n]
    keep.copy_(torch.from_numpy(keep_np).to(dev))
    sel = np.nonzero(keep_np)[0]
    cap = int(sel.size * cap_frac)
    out_stride = cap + 2 + ((cap + (0 if even_out else 1)) % 2)
    assert (out_stride % 2 == 0) == even_out
    out = torch.full((59, out_stride), -12345, dtype=torch.int16, device=dev)
    idx = torch.full((out_stride,), -7, dtype=torch.int32, device=dev)
    nout = torch.empty(1, dtype=torch.int64, device=dev)
    ws = api.workspace(n, 1, dev)
    log(f"mixed compact n={n} stride={stride} out_stride={out_stride} cap={cap}")
    api.refine_compact(pl, keep, out, ws, index_map_out=idx, n_out=nout, n=n, capacity=cap)
    torch.cuda.synchronize()
    assert int(nout.item()) == sel.size
    o = out.cpu().numpy()
    np.testing.assert_array_equal(o[:, :cap], planes[:, sel[:cap]])
    np.testing.assert_array_equal(idx.cpu().numpy()[:cap], sel[:cap])
    assert np.all(o[:, cap:] == -12345) and np.all(idx.cpu().numpy()[cap:] == -7)
