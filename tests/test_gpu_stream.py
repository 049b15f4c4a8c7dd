"""Streaming a q in k-chunks (the on-the-fly generation of the coefficients of the RPA
algorithm section): when one q's B slab, its copies and the point buffers do not fit the
context's HBM limit, the pipeline generates B for a chunk of k-points at a time,
contracts it for every point of the batch and adds the chunks' chi0 in chunk order.
Results equal the oracle to the FP64 bar (1e-10 relative) and the reduced precisions to
their bounds; the chunked sum differs from the whole-slab one by rounding only.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import rpa_oracle as orc
from paper_2505_06021_amd import inputs

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL_E = {1: 1e-6, 2: 2e-5, 3: 1e-6}


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def check_grid(got, ref, tol=1e-10):
    for q in range(ref.shape[0]):
        scale = np.max(np.abs(ref[q]))
        assert np.max(np.abs(got[q] - ref[q])) <= tol * scale, q


def test_streamed_q_matches_golden_fp64():
    # the 3x3x1 N_aux 384 slab's q slab is 99 MB: a 40 MB limit streams every q in
    # chunks of a few k-points
    from paper_2505_06021_amd import rpa
    g = json.load(open(os.path.join(GOLD, "slab3x3_naux384.json")))
    s = inputs.slab_3x3_384()
    say("streamed energy FP64, 40 MB limit")
    with rpa.Context(0, hbm_limit=40 * 2 ** 20) as c:
        E, eps = c.energy(s)
        st = c.stats()
    assert st["hbm_high_water"] <= 40 * 2 ** 20
    assert abs(E - g["E"]) <= 1e-10 * abs(g["E"])
    check_grid(eps, np.array(g["eps"]))


def test_streamed_points_explicit_host_B_and_ragged_chunks():
    # explicit host B copied chunk by chunk; 5 k-points of a 5x1x1 grid leave a ragged last
    # chunk; the oracle runs live
    from paper_2505_06021_amd import rpa
    # a q slab of 9.6 MB against a 6 MB limit: chunks of two k-points, the last one single
    s = inputs.make_system("stream5", (5, 1, 1), 8, 100, 150, 4, 61, is_complex=True, sigma=0.04).materialize_B()
    E_ref, g_ref = orc.energy(s)
    slab = s.M * s.naux * 16
    limit = 6 * 2 ** 20
    say(f"streamed energy FP64 explicit B, limit {limit} (slab {slab})")
    with rpa.Context(0, hbm_limit=limit) as c:
        E, eps = c.energy(s)
    assert abs(E - E_ref) <= 1e-10 * abs(E_ref)
    check_grid(eps, g_ref)


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_streamed_reduced_precision(prec):
    from paper_2505_06021_amd import rpa
    s = inputs.slab_3x3_384()
    with rpa.Context(0) as free:
        E64, _ = free.energy(s)
        E0, eps0 = free.energy(s, prec=prec)
    say(f"streamed energy prec={prec}, 60 MB limit")
    with rpa.Context(0, hbm_limit=60 * 2 ** 20) as c:
        E, eps = c.energy(s, prec=prec)
    say(f"  dE vs FP64 {abs(E - E64):.3e}, vs unstreamed {abs(E - E0):.3e}")
    assert abs(E - E64) <= TOL_E[prec]
    assert np.max(np.abs(eps - eps0)) <= 1e-6 * np.max(np.abs(eps0))


def test_streamed_device_B_mixed():
    # a caller's device B is read in place; the FP32 copy is made chunk by chunk
    from paper_2505_06021_amd import rpa
    # M = 3200 rows: the FP32 copy of a q is 5 MB, one k-point's 1.3 MB
    s = inputs.make_system("streamdev", (2, 2, 1), 8, 100, 200, 3, 62, is_complex=True, sigma=0.05).materialize_B()
    E_ref, _ = orc.energy(s)
    with rpa.Context(0, hbm_limit=4 * 2 ** 20) as c:
        say("streamed energy FP32 device B")
        E, _ = c.energy(s, prec=1, device=True)
        E64, g64 = c.energy(s, device=True)
    assert abs(E64 - E_ref) <= 1e-10 * abs(E_ref)
    assert abs(E - E_ref) <= 1e-6


def test_nothing_fits_is_an_error():
    from paper_2505_06021_amd import rpa
    s = inputs.slab_3x3_384()
    with rpa.Context(0, hbm_limit=4 * 2 ** 20) as c:     # less than one k-point's rows
        with pytest.raises(rpa.RpaError) as e:
            c.energy(s)
        assert e.value.code == rpa.RPA_E_NOMEM


def test_served_job_streams_when_a_q_does_not_fit():
    # a 100 MB limit cannot hold a whole q of the N_aux 384 slab with its twelve points
    # (about 160 MB): the job is admitted with its one-k-point footprint and streamed
    from paper_2505_06021_amd import rpa
    g = json.load(open(os.path.join(GOLD, "slab3x3_naux384.json")))
    s = inputs.slab_3x3_384()
    say("served streamed job, 100 MB limit")
    with rpa.Context(0, hbm_limit=100 * 2 ** 20) as c:
        jid = c.submit(s)
        res, eps = c.poll(jid, timeout_ms=-1, nq=s.nq, nw=s.nw)
        st = c.stats()
    assert res["status"] == 0
    assert res["hbm_bytes"] <= 100 * 2 ** 20 and st["hbm_high_water"] <= 100 * 2 ** 20
    assert abs(res["E"] - g["E"]) <= 1e-10 * abs(g["E"])
    check_grid(eps, np.array(g["eps"]))
