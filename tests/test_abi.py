"""C-ABI boundary checks that need no GPU: the library loads, exports every
function the header declares, and rejects invalid arguments on the host
before any HIP call (these calls never reach a kernel launch)."""
import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "refine.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2606_09074_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2606_09074_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(refine_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_function_is_exported(lib):
    from paper_2606_09074_amd import _lib
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(refine_\w+)$", out, flags=re.M))
    for name in names:
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_struct_sizes_match_header():
    from paper_2606_09074_amd import _lib
    assert ctypes.sizeof(_lib.Scene) == 32
    assert ctypes.sizeof(_lib.Params) == 88
    assert ctypes.sizeof(_lib.Stats) == 96


def test_version_status_defaults(lib):
    from paper_2606_09074_amd import _lib
    assert b"gfx950" in lib.refine_version()
    assert lib.refine_status_string(_lib.REFINE_E_WORKSPACE).startswith(b"REFINE_E_WORKSPACE")
    p = _lib.default_params()
    from tests.helpers import CLAMP_K, E_COL, E_LNGEM, E_OPA, ETA, Z_NEAR
    assert (p.eta, p.z_near, p.clamp_k, p.e_col, p.e_opa, p.e_lngem) == (ETA, Z_NEAR, CLAMP_K, E_COL, E_OPA,
                                                                          E_LNGEM)
    assert (p.proj_mode, p.vis_mode, p.equal_lambda, p.n_sub_views, p.score_path, p.records_per_lane,
            p.views_per_iteration) == (0,) * 7


def test_prune_count(lib):
    assert lib.refine_prune_count(5, 0.5) == 3
    assert lib.refine_prune_count(3_000_000, 0.9) == 2_700_000
    assert lib.refine_prune_count(6_000_000, 0.66) == 3_960_000
    for bad in (0.0, 1.0, -0.1, float("nan"), float("inf")):
        assert lib.refine_prune_count(10, bad) == -1
    assert lib.refine_prune_count(-1, 0.5) == -1


def test_workspace_size(lib):
    from paper_2606_09074_amd import _lib
    sz = ctypes.c_size_t()
    assert lib.refine_workspace_size(3_000_000, 200, ctypes.byref(sz)) == 0
    big = sz.value
    assert lib.refine_workspace_size(1000, 16, ctypes.byref(sz)) == 0
    assert 0 < sz.value < big
    assert lib.refine_workspace_size(-1, 16, ctypes.byref(sz)) == _lib.REFINE_E_INVALID
    assert lib.refine_workspace_size(10, -1, ctypes.byref(sz)) == _lib.REFINE_E_INVALID
    assert lib.refine_workspace_size(1 << 31, 16, ctypes.byref(sz)) == _lib.REFINE_E_UNSUPPORTED
    assert lib.refine_workspace_size(10, 16, None) == _lib.REFINE_E_INVALID
    # no cameras: only what stats, select and compact use (no binned scene copy)
    assert lib.refine_workspace_size(3_000_000, 0, ctypes.byref(sz)) == 0
    assert 0 < sz.value < big // 50


FAKE = 0x10000   # never dereferenced: every call below fails validation first


def _scene(n=100, stride=None, dtype=0, sh_dtype=0, planes=FAKE):
    from paper_2606_09074_amd import _lib
    return _lib.Scene(n, n if stride is None else stride, dtype, sh_dtype, ctypes.c_void_p(planes))


def test_stats_validation(lib):
    from paper_2606_09074_amd import _lib
    p = _lib.default_params()
    ws_ok = 1 << 30
    E = _lib.REFINE_E_INVALID
    call = lambda sc, prm=p, out=FAKE, ws=FAKE, wsb=ws_ok: lib.refine_stats(
        ctypes.byref(sc) if sc is not None else None, ctypes.byref(prm) if prm is not None else None,
        out, ws, wsb, None)
    assert call(None) == E
    assert call(_scene(n=-1)) == E
    assert call(_scene(n=10, stride=5)) == E
    assert call(_scene(planes=0)) == E
    # storage pairs: unknown dtypes are invalid, known but unsupported pairs unsupported
    assert call(_scene(dtype=7)) == E
    assert call(_scene(sh_dtype=-1)) == E
    U = _lib.REFINE_E_UNSUPPORTED
    F32, BF16, F16 = _lib.REFINE_F32, _lib.REFINE_BF16, _lib.REFINE_F16
    for dt, sh in ((F32, BF16), (F32, F16), (BF16, F32), (BF16, BF16), (F16, F32), (F16, BF16)):
        assert call(_scene(dtype=dt, sh_dtype=sh)) == U, (dt, sh)
    assert call(_scene(n=1 << 31)) == _lib.REFINE_E_UNSUPPORTED
    assert call(_scene(), prm=None) == E
    assert call(_scene(), out=None) == E
    assert call(_scene(), ws=None) == _lib.REFINE_E_WORKSPACE
    assert call(_scene(), wsb=16) == _lib.REFINE_E_WORKSPACE
    for field, bad in (("eta", 0.0), ("eta", float("nan")), ("z_near", -1.0), ("clamp_k", 0.0),
                       ("e_col", 0.0), ("e_lngem", float("inf")), ("proj_mode", 3), ("vis_mode", -1),
                       ("equal_lambda", 2), ("n_sub_views", -5), ("score_path", 3), ("records_per_lane", 3),
                       ("records_per_lane", -1), ("views_per_iteration", 3), ("views_per_iteration", -1),
                       ("waves_per_block", 3), ("waves_per_block", 16), ("waves_per_block", -1), ("score_kind", 2)):
        q = _lib.default_params()
        setattr(q, field, bad)
        assert call(_scene(), prm=q) == E, field


def test_score_validation(lib):
    from paper_2606_09074_amd import _lib
    p = _lib.default_params()
    E = _lib.REFINE_E_INVALID
    sc = _scene()

    def call(nv=16, cams=FAKE, stats=FAKE, scores=FAKE, ws=FAKE, wsb=1 << 30, scene=sc):
        return lib.refine_score(ctypes.byref(scene), cams, nv, ctypes.byref(p), stats, scores, ws, wsb, None)
    assert call(nv=0) == E
    assert call(nv=-3) == E
    assert call(cams=None) == E
    assert call(stats=None) == E
    assert call(scores=None) == E
    assert call(nv=(1 << 20) + 1) == _lib.REFINE_E_UNSUPPORTED
    assert call(wsb=100) == _lib.REFINE_E_WORKSPACE


def test_two_phase_validation(lib):
    from paper_2606_09074_amd import _lib
    p = _lib.default_params()
    E = _lib.REFINE_E_INVALID
    sc = _scene()
    assert lib.refine_score_prepare(ctypes.byref(sc), None, 16, ctypes.byref(p), FAKE, FAKE, 1 << 30, None) == E
    assert lib.refine_score_prepare(ctypes.byref(sc), FAKE, 0, ctypes.byref(p), FAKE, FAKE, 1 << 30, None) == E
    assert lib.refine_score_prepare(ctypes.byref(sc), FAKE, 16, ctypes.byref(p), None, FAKE, 1 << 30, None) == E
    assert lib.refine_score_prepare(ctypes.byref(sc), FAKE, 16, ctypes.byref(p), FAKE, FAKE, 64,
                                    None) == _lib.REFINE_E_WORKSPACE
    assert lib.refine_score_views(ctypes.byref(sc), 16, ctypes.byref(p), FAKE, None, None, FAKE, 1 << 30, None) == E
    assert lib.refine_score_views(ctypes.byref(sc), -1, ctypes.byref(p), FAKE, FAKE, None, FAKE, 1 << 30, None) == E
    assert lib.refine_score_views(ctypes.byref(sc), 16, None, FAKE, FAKE, None, FAKE, 1 << 30, None) == E
    cams = lib.refine_score_cameras
    assert cams(None, FAKE, 16, ctypes.byref(p), FAKE, 1 << 30, None) == E
    assert cams(ctypes.byref(sc), None, 16, ctypes.byref(p), FAKE, 1 << 30, None) == E
    assert cams(ctypes.byref(sc), FAKE, 0, ctypes.byref(p), FAKE, 1 << 30, None) == E
    assert cams(ctypes.byref(sc), FAKE, 16, None, FAKE, 1 << 30, None) == E
    assert cams(ctypes.byref(sc), FAKE, 16, ctypes.byref(p), FAKE, 64, None) == _lib.REFINE_E_WORKSPACE
    assert cams(ctypes.byref(sc), FAKE, 16, ctypes.byref(p), None, 1 << 30, None) == _lib.REFINE_E_WORKSPACE
    # a workspace sized for 16 views has no room for the tables of 17
    need = ctypes.c_size_t(0)
    assert lib.refine_workspace_size(100, 16, ctypes.byref(need)) == 0
    big = ctypes.c_size_t(0)
    assert lib.refine_workspace_size(100, 17, ctypes.byref(big)) == 0
    if big.value > need.value:
        assert cams(ctypes.byref(sc), FAKE, 17, ctypes.byref(p), FAKE, need.value, None) == _lib.REFINE_E_WORKSPACE


def test_select_validation(lib):
    from paper_2606_09074_amd import _lib
    E = _lib.REFINE_E_INVALID

    def call(n=100, ratio=0.5, ov=-1, scores=FAKE, keep=FAKE, wsb=1 << 30, ws=FAKE):
        return lib.refine_select(scores, n, ratio, ov, keep, None, None, ws, wsb, None)
    for r in (0.0, 1.0, 1.5, -0.2, float("nan")):
        assert call(ratio=r) == E
    assert call(ov=101) == E
    assert call(n=-1) == E
    assert call(scores=None) == E
    assert call(keep=None) == E
    assert call(wsb=10) == _lib.REFINE_E_WORKSPACE


def test_compact_validation(lib):
    from paper_2606_09074_amd import _lib
    E = _lib.REFINE_E_INVALID
    sin = _scene(n=100)

    def call(src=sin, dst=None, keep=FAKE, ws=FAKE, wsb=1 << 30):
        dst = dst if dst is not None else _scene(n=50, planes=0x4000000)
        return lib.refine_compact(ctypes.byref(src), keep, ctypes.byref(dst), None, None, ws, wsb, None)
    assert call(keep=None) == E
    assert call(dst=_scene(n=50, planes=FAKE + 64)) == E                 # overlapping buffers
    assert call(dst=_scene(n=50, dtype=7, planes=0x4000000)) == E
    # in and out must share the storage pair
    mixed = dict(dtype=_lib.REFINE_BF16, sh_dtype=_lib.REFINE_F16)
    assert call(dst=_scene(n=50, planes=0x4000000, **mixed)) == E
    assert call(src=_scene(n=100, **mixed)) == E
    # 2-byte scenes: 59 planes x 100 x 2 B = 11800 B, so an output 2 B before the end overlaps
    assert call(src=_scene(n=100, **mixed), dst=_scene(n=50, planes=FAKE + 11798, **mixed)) == E
    assert call(dst=_scene(n=50, stride=10, planes=0x4000000)) == E
    assert call(wsb=8) == _lib.REFINE_E_WORKSPACE


def test_batch_validation(lib):
    from paper_2606_09074_amd import _lib
    E, U, W = _lib.REFINE_E_INVALID, _lib.REFINE_E_UNSUPPORTED, _lib.REFINE_E_WORKSPACE
    p = _lib.default_params()

    def job(**kw):
        j = _lib.PruneJob()
        j.scene = _scene(n=kw.get("n", 100), dtype=kw.get("dtype", 0), sh_dtype=kw.get("sh_dtype", 0))
        j.cams = kw.get("cams", FAKE)
        j.n_views = kw.get("nv", 16)
        j.reserved = kw.get("reserved", 0)
        j.ratio = kw.get("ratio", 0.5)
        j.stats, j.scores, j.keep = kw.get("stats", FAKE), kw.get("scores", FAKE), kw.get("keep", FAKE)
        j.out = _scene(n=50, planes=0x4000000, dtype=kw.get("odtype", 0), sh_dtype=kw.get("osh", 0))
        return j

    def size(*jobs, prm=p):
        arr = (_lib.PruneJob * len(jobs))(*jobs)
        out = ctypes.c_size_t(0)
        return lib.refine_prune_batch_workspace_size(arr, len(jobs), ctypes.byref(prm), ctypes.byref(out)), out.value

    def run(*jobs, wsb=1 << 30, ws=FAKE, staging=None, stb=0):
        arr = (_lib.PruneJob * len(jobs))(*jobs)
        return lib.refine_prune_batch(arr, len(jobs), ctypes.byref(p), ws, wsb, staging, stb, None)
    rc, b1 = size(job())
    assert rc == 0 and b1 > 0
    rc, b2 = size(job(), job(n=5000))
    assert rc == 0 and b2 > b1
    assert lib.refine_prune_batch_workspace_size(None, 1, ctypes.byref(p), ctypes.byref(ctypes.c_size_t())) == E
    arr = (_lib.PruneJob * 1)(job())
    assert lib.refine_prune_batch_workspace_size(arr, 0, ctypes.byref(p), ctypes.byref(ctypes.c_size_t())) == E
    for bad in (dict(n=0), dict(ratio=1.0), dict(ratio=0.0), dict(cams=0), dict(nv=0), dict(stats=0),
                dict(scores=0), dict(keep=0), dict(reserved=1), dict(odtype=1, osh=2)):
        assert size(job(**bad))[0] == E, bad
        assert run(job(**bad)) == E, bad
    assert size(job(n=4096 * 4096 + 1))[0] == U
    assert run(job(), wsb=b1 - 1) == W
    assert run(job(), ws=0) == W
    # a staging buffer too small for the job table, or misaligned, is refused before any copy
    assert run(job(), job(), staging=FAKE, stb=_lib.BATCH_STAGING_BYTES_PER_JOB) == W
    assert run(job(), staging=FAKE + 4, stb=_lib.BATCH_STAGING_BYTES_PER_JOB) == E


def test_stats_noalloc_validation(lib):
    """The allocation-free statistics call validates like refine_stats and
    rejects scenes beyond its fixed array, all before touching HIP."""
    from paper_2606_09074_amd import _lib
    p = _lib.default_params()
    E, U = _lib.REFINE_E_INVALID, _lib.REFINE_E_UNSUPPORTED
    call = lambda sc, prm=p, out=FAKE: lib.refine_stats_noalloc(
        ctypes.byref(sc) if sc is not None else None, ctypes.byref(prm) if prm is not None else None, out, None)
    assert call(None) == E
    assert call(_scene(n=-1)) == E
    assert call(_scene(planes=0)) == E
    assert call(_scene(), prm=None) == E
    assert call(_scene(), out=None) == E
    bad = _lib.default_params()
    bad.eta = 0.0
    assert call(_scene(), prm=bad) == E
    assert _lib.STATS_NOALLOC_MAX_N == 1 << 26
    assert call(_scene(n=_lib.STATS_NOALLOC_MAX_N + 1)) == U
    assert call(_scene(n=1 << 31)) == U
