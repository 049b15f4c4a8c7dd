"""Serving path (rpa_submit / rpa_poll): continuous batching with HBM admission.

A job's result must not depend on what runs beside it: every job runs the same kernels
on buffers it owns, so its energy and integrand are compared bit for bit with the
synchronous call on the same inputs, and each served energy is also checked against the
CPU oracle (FP64: 1e-10 relative; reduced precision: its stated bound per cell).
"""
import sys
import threading
import time

import numpy as np
import pytest

from oracle import rpa_oracle as orc
from paper_2505_06021_amd import inputs

pytestmark = pytest.mark.gpu
TOL_E_MIXED = {1: 1e-6, 2: 2e-5, 3: 1e-6}


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def small_jobs():
    specs = [((1, 1, 1), 4, 20, 96, 8), ((2, 2, 1), 3, 12, 130, 9), ((1, 1, 1), 6, 40, 200, 12),
             ((2, 2, 1), 5, 22, 64, 10), ((3, 3, 1), 2, 10, 77, 8), ((1, 1, 1), 8, 30, 256, 16)]
    return [inputs.make_system(f"j{i}", g, no, nv, na, nw, 500 + i, is_complex=True, sigma=0.1)
            for i, (g, no, nv, na, nw) in enumerate(specs)]


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_results_alone_equal_results_in_the_mix(prec):
    from paper_2505_06021_amd import rpa
    jobs = small_jobs()
    oracle = [orc.energy(s) for s in jobs]
    with rpa.Context(0) as ctx:
        say(f"alone prec={prec}")
        alone = [ctx.energy(s, prec=prec) for s in jobs]
        say("submit all")
        ids = [ctx.submit(s, prec=prec) for s in jobs]
        for s, jid, (E, eps), (E_ref, g_ref) in zip(jobs, ids, alone, oracle):
            r = None
            t0 = time.time()
            while r is None:
                r = ctx.poll(jid, timeout_ms=1000, nq=s.nq, nw=s.nw)
                assert time.time() - t0 < 60
            res, g = r
            assert res["status"] == 0
            assert res["E"] == E, (s.name, res["E"], E)
            assert np.array_equal(g, eps)
            if prec == 0:
                assert abs(res["E"] - E_ref) <= 1e-10 * abs(E_ref), s.name
                for q in range(s.nq):
                    assert np.max(np.abs(g[q] - g_ref[q])) <= 1e-10 * np.max(np.abs(g_ref[q]))
            else:
                assert abs(res["E"] - E_ref) <= TOL_E_MIXED[prec], s.name
            assert res["t_submit"] <= res["t_start"] <= res["t_done"]
            assert res["npoints"] == s.nq * s.nw
        st = ctx.stats()
        assert st["jobs_done"] == len(jobs) and st["jobs_queued"] == 0 and st["jobs_running"] == 0
        # the small jobs' split contractions went through the cross-job fuser (and the
        # results above are bit-identical to the unfused synchronous ones); FP64 and FP32
        # fuse only their paired configuration, which the tuner may or may not pick for
        # these shapes (test_fused_groups_of_several_jobs_equal_their_solo_results fixes it)
        say(f"fused launches {st['fused_launches']} carrying {st['fused_groups']} sub-batches, "
            f"{st['solo_groups']} alone")
        if prec in (2, 3):
            assert st["fused_launches"] >= 1 and st["fused_groups"] >= st["fused_launches"]


def test_admission_respects_the_hbm_limit():
    from paper_2505_06021_amd import rpa
    jobs = small_jobs()
    biggest = 0
    with rpa.Context(0) as probe:
        ids = [probe.submit(s) for s in jobs]
        for s, jid in zip(jobs, ids):
            res, _ = probe.poll(jid, timeout_ms=-1, nq=s.nq, nw=s.nw)
            biggest = max(biggest, res["hbm_bytes"])
    limit = int(biggest * 1.5)     # at most one of the larger jobs at a time
    say(f"limit {limit}")
    with rpa.Context(0, hbm_limit=limit) as ctx:
        ids = [ctx.submit(s) for s in jobs]
        for s, jid in zip(jobs, ids):
            res, _ = ctx.poll(jid, timeout_ms=-1, nq=s.nq, nw=s.nw)
            assert res["status"] == 0
        st = ctx.stats()
        assert st["hbm_high_water"] <= limit
        assert st["jobs_done"] == len(jobs)


def test_job_that_can_never_fit_is_refused_at_submit():
    from paper_2505_06021_amd import rpa
    with rpa.Context(0, hbm_limit=1 << 20) as ctx:
        with pytest.raises(rpa.RpaError) as e:
            ctx.submit(small_jobs()[2])
        assert e.value.code == rpa.RPA_E_NOMEM


def test_poll_unknown_and_consumed_jobs():
    from paper_2505_06021_amd import rpa
    with rpa.Context(0) as ctx:
        with pytest.raises(rpa.RpaError) as e:
            ctx.poll(12345, timeout_ms=0)
        assert e.value.code == rpa.RPA_E_UNKNOWN_JOB
        s = small_jobs()[0]
        jid = ctx.submit(s)
        assert ctx.poll(jid, timeout_ms=-1, nq=s.nq, nw=s.nw) is not None
        with pytest.raises(rpa.RpaError) as e:
            ctx.poll(jid, timeout_ms=0)
        assert e.value.code == rpa.RPA_E_UNKNOWN_JOB


def test_finalize_with_pending_jobs_returns():
    from paper_2505_06021_amd import rpa
    ctx = rpa.Context(0)
    for s in small_jobs() * 3:
        ctx.submit(s)
    t0 = time.time()
    ctx.close()          # cancels queued jobs, waits for the running ones
    assert time.time() - t0 < 120


@pytest.mark.parametrize("prec", [0, 2])
def test_workspace_of_synchronous_calls_does_not_block_admission(prec):
    # a synchronous call leaves its grow-only workspace allocated; a job that only fits
    # without it must still be admitted (the scheduler releases the idle workspace)
    from paper_2505_06021_amd import rpa
    s = small_jobs()[5]
    with rpa.Context(0) as probe:
        jid = probe.submit(s, prec=prec)
        res, _ = probe.poll(jid, timeout_ms=-1, nq=s.nq, nw=s.nw)
        need = res["hbm_bytes"]
    limit = int(need * 1.2)
    say(f"limit {limit} need {need}")
    with rpa.Context(0, hbm_limit=limit) as ctx:
        E, _ = ctx.energy(s, prec=prec)
        jid = ctx.submit(s, prec=prec)
        t0 = time.time()
        r = None
        while r is None:
            r = ctx.poll(jid, timeout_ms=1000, nq=s.nq, nw=s.nw)
            assert time.time() - t0 < 60, "job never admitted"
        res, _ = r
        assert res["status"] == 0 and res["E"] == E


def test_synchronous_calls_while_jobs_are_served():
    """rpa_energy calls from a second thread while jobs are submitted and polled: the
    synchronous workspace and the jobs' reservations share one HBM limit, and neither
    side's results change."""
    from paper_2505_06021_amd import rpa
    jobs = small_jobs()
    sync_sys = small_jobs()[1]
    with rpa.Context(0) as ctx:
        alone = [ctx.energy(s) for s in jobs]
        ref_sync = ctx.energy(sync_sys)
        got_sync, errors = [], []

        def sync_loop():
            try:
                for _ in range(6):
                    got_sync.append(ctx.energy(sync_sys))
            except Exception as e:          # reported below
                errors.append(e)

        say("synchronous calls beside served jobs")
        th = threading.Thread(target=sync_loop)
        th.start()
        ids = [ctx.submit(s) for s in jobs]
        for s, jid, (E, eps) in zip(jobs, ids, alone):
            res, g = ctx.poll(jid, timeout_ms=-1, nq=s.nq, nw=s.nw)
            assert res["status"] == 0 and res["E"] == E and np.array_equal(g, eps), s.name
        th.join(timeout=120)
        assert not th.is_alive() and not errors, errors
        assert len(got_sync) == 6
        for E, eps in got_sync:
            assert E == ref_sync[0] and np.array_equal(eps, ref_sync[1])


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_groups_of_several_jobs_equal_their_solo_results(monkeypatch, prec):
    # a long fusion window and eight small jobs submitted at once: the fuser puts several
    # jobs' paired contractions into one launch; each result stays bit for bit its own
    from paper_2505_06021_amd import rpa
    monkeypatch.setenv("RPA_FUSE_WINDOW_US", "20000")
    monkeypatch.setenv("RPA_SERVE_WORKERS", "8")
    monkeypatch.setenv("RPA_CHI0_CFG", "t64k16w2")     # the paired configurations are the
    monkeypatch.setenv("RPA_F32_TILE", "64w2")         # ones the fuser groups
    specs = [((1, 1, 1), 3, 12, 100 + 17 * i, 4 + (i % 3)) for i in range(8)]
    jobs = [inputs.make_system(f"f{i}", g, no, nv, na, nw, 700 + i, is_complex=True, sigma=0.1)
            for i, (g, no, nv, na, nw) in enumerate(specs)]
    with rpa.Context(0) as ctx:
        alone = [ctx.energy(s, prec=prec) for s in jobs]
        say(f"eight jobs at once prec={prec}")
        ids = [ctx.submit(s, prec=prec) for s in jobs]
        for s, jid, (E, eps) in zip(jobs, ids, alone):
            res, g = ctx.poll(jid, timeout_ms=-1, nq=s.nq, nw=s.nw)
            assert res["status"] == 0 and res["E"] == E and np.array_equal(g, eps), s.name
        st = ctx.stats()
    say(f"  fused launches {st['fused_launches']}, groups {st['fused_groups']}")
    assert st["fused_groups"] > st["fused_launches"] >= 1
