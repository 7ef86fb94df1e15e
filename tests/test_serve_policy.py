"""Host-side serving logic (no device): admission bookkeeping, the job
memory model, the serving workload draws and the tuner table."""
import numpy as np
import pytest

from paper_2606_09074_amd import serve, synth


def test_admission_slots_and_budget():
    a = serve.Admission(budget_bytes=1000, slots=2)
    assert a.can_admit(600)
    a.admit(600)
    assert not a.can_admit(500)          # bytes
    assert a.can_admit(400)
    a.admit(400)
    assert not a.can_admit(0)            # slots
    a.release(600)
    assert a.can_admit(600) and not a.can_admit(601)
    assert not a.fits_ever(1001) and a.fits_ever(1000)
    with pytest.raises(RuntimeError):
        a.admit(700)
    a.release(400)
    with pytest.raises(RuntimeError):
        a.release(1)


def test_fifo_head_blocks_until_it_fits():
    """Simulated queue: the large head job waits for memory instead of being
    passed by smaller ones, and every job is admitted exactly once."""
    a = serve.Admission(budget_bytes=100, slots=3)
    queue = [60, 50, 10, 10, 90, 5]
    running, order = [], []
    t = 0
    while queue or running:
        # the oldest running job finishes every tick
        if running:
            a.release(running.pop(0))
        while queue and a.can_admit(queue[0]):
            nb = queue.pop(0)
            a.admit(nb)
            running.append(nb)
            order.append(nb)
        assert a.in_use <= 100 and a.inflight <= 3
        t += 1
    assert order == [60, 50, 10, 10, 90, 5]


def test_job_bytes_counts_every_buffer():
    n, V, k = 1_000_000, 200, 400_000
    b4 = serve.job_bytes(n, V, k, 4, workspace_bytes=12345)
    b2 = serve.job_bytes(n, V, k, 2, workspace_bytes=12345)
    assert b4 - b2 == 59 * 2 * k                 # survivor planes scale with the element size
    assert b4 >= 12345 + 4 * n + n + 59 * 4 * k + 4 * k


def test_serving_workload_draws():
    specs = synth.serve_scene_specs(8)
    ns = np.array([s.n for s in specs], dtype=np.float64)
    # both ends of the law's range, equal log spacing between them
    assert ns[0] == 200_000 and ns[-1] == 6_000_000
    np.testing.assert_allclose(np.diff(np.log(ns)), np.log(30.0) / 7, rtol=1e-4)
    assert len({s.seed for s in specs}) == 8
    arr, jobs = synth.serve_requests(4000, n_scenes=5)
    assert np.all(np.diff(arr) > 0)
    assert abs(4000 / arr[-1] - 20.0) < 1.5       # Poisson rate
    v = np.array([j[1] for j in jobs]); r = np.array([j[2] for j in jobs])
    assert v.min() >= 50 and v.max() <= 300 and r.min() >= 0.3 and r.max() <= 0.9
    assert set(j[0] for j in jobs) == set(range(5))
    assert synth.ring_cameras(77).shape == (77, 18)


def test_tuner_table_round_trip(tmp_path):
    t = serve.Tuner({(18, 6): (1, 0), (22, 8): (2, 1)})
    p = tmp_path / "tune.json"
    t.save(str(p))
    u = serve.Tuner.load(str(p))
    assert u.table == t.table
    assert u.choice(300_000, 64) == (1, 0)        # round(log2) buckets
    assert u.choice(4_000_000, 250) == (2, 1)
    assert u.choice(10, 10) is None
    assert serve.percentile([1, 2, 3, 4], 0.5) == 2.5


def test_tuner_candidates_and_choices():
    """Every candidate is a valid parameter set for the library's view loop
    (path, records per lane, views per iteration, waves per block), the
    direct path is among them, and older tables with fewer entries apply
    with the library's defaults for the rest."""
    from paper_2606_09074_amd import _lib
    assert (1, 0, 0, 0) in serve.CANDIDATES
    assert len(set(serve.CANDIDATES)) == len(serve.CANDIDATES) == 13
    for c in serve.CANDIDATES:
        p = _lib.Params()
        serve.apply_choice(p, c)
        assert (p.score_path, p.records_per_lane, p.views_per_iteration, p.waves_per_block) == c
        assert p.waves_per_block in (0, 2, 4, 8) and p.records_per_lane in (0, 1, 2)
    p = _lib.Params()
    serve.apply_choice(p, (2, 2))
    assert (p.score_path, p.records_per_lane, p.views_per_iteration, p.waves_per_block) == (2, 2, 0, 0)
