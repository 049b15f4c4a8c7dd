"""Full-size parity on sampled points: the 6x6x1 N_aux = 1200 and 3x3x1 N_aux = 2400 slabs,
with B streamed from the device Philox generator, and the 3x3x1 N_aux = 384 slab given in an
atomic-orbital basis (N_bas 144, B from the device MO transform), in the launch configuration of the
full energy (rpa_points groups the sampled points by q exactly like rpa_energy).

The oracle values are stored (tests/golden/*_sampled.json, written by make_golden.py from
the oracle alone).  The scale of a point is the largest |eps| among the sampled points of
its q (ln det(1 - Pi) and Tr Pi cancel at large omega, so a point's own |eps| is no scale
there; the full grids are checked the same way with every frequency of the q).
FP64: |d eps| <= 1e-10 scale.  Reduced precision: |d eps| <= 1e-8 scale (FP32 and
split-FP16) and 2e-7 scale (split-BF16); eps at these sizes is O(1e3 - 1e4) Ha at the
lowest frequency.

The largest auxiliary basis of the paper's basis-convergence study (Sec. 4, N_aux 4070: 64
tile rows of 64 with a 38-row tail, Pi and the Cholesky at that size) is checked against
the live oracle on a Gamma-only system with a short contraction (M = 128 rows), so that
the oracle finishes in seconds: E and the eps grid in FP64, chi0 element by element, and
the reduced precisions on the eps grid with the tolerances above.  The largest regular
k-grid of the paper's studies (17 x 17, Sec. 4: 289 k- and q-points, so 289 slabs, 289 weight
rows and k (+) q rows that wrap in both directions) is checked the same way with small
bands and N_aux.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2505_06021_amd import inputs

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {0: 1e-10, 1: 1e-8, 2: 2e-7, 3: 1e-8}


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_06021_amd import rpa
    c = rpa.Context(0)
    yield c
    c.close()


CASES = [("slab6x6_naux1200_sampled", inputs.slab_6x6_1200),
         ("slab3x3_naux2400_sampled", inputs.slab_3x3_2400),
         ("slab3x3_ao_naux384_sampled", inputs.slab_3x3_ao_384)]


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_sampled_points_full_size(ctx, name, make, prec):
    path = os.path.join(GOLD, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{name}.json not generated")
    g = json.load(open(path))
    s = make()
    iq = [p["iq"] for p in g["points"]]
    om = [p["omega"] for p in g["points"]]
    ref = np.array([p["eps"] for p in g["points"]])
    say(f"{name} prec={prec} points={list(zip(iq, om))}")
    got = ctx.points(s, iq, om, prec=prec)
    scale = np.array([max(abs(r) for q, r in zip(iq, ref) if q == qq) for qq in iq])
    rel = np.abs(got - ref) / scale
    say(f"  eps {got}  err / scale {rel}")
    assert np.all(rel <= TOL[prec])


def rel_rows(a, b):
    """Element by element: max_PQ |a_PQ - b_PQ| / max_Q' |b_PQ'| (each row's own scale)."""
    return float(np.max(np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)))


@pytest.fixture(scope="module")
def aux4070():
    from oracle import rpa_oracle as orc
    say("oracle at N_aux 4070")
    s = inputs.make_system("aux4070", (1, 1, 1), 4, 32, 4070, 2, 4070, is_complex=True)
    E_ref, g_ref = orc.energy(s)
    chi_ref = orc.chi0(s, 0, s.omega[1])
    return s, E_ref, g_ref, chi_ref


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_largest_paper_aux_basis(ctx, aux4070, prec):
    s, E_ref, g_ref, chi_ref = aux4070
    say(f"N_aux 4070 prec={prec}")
    E, eps = ctx.energy(s, prec=prec)
    scale = np.max(np.abs(g_ref))
    assert np.max(np.abs(eps - g_ref)) <= TOL[prec] * scale
    if prec == 0:
        assert abs(E - E_ref) <= 1e-10 * abs(E_ref)
        chi = ctx.chi0(s, 0, s.omega[1])
        assert rel_rows(chi, chi_ref) <= 1e-12


@pytest.fixture(scope="module")
def grid17():
    from oracle import rpa_oracle as orc
    say("oracle on the 17x17x1 grid")
    s = inputs.make_system("k17", (17, 17, 1), 2, 4, 40, 2, 1717, is_complex=True)
    E_ref, g_ref = orc.energy(s)
    return s, E_ref, g_ref


@pytest.mark.parametrize("prec", [0, 1])
def test_largest_paper_k_grid(ctx, grid17, prec):
    s, E_ref, g_ref = grid17
    say(f"17x17x1 grid prec={prec}")
    E, eps = ctx.energy(s, prec=prec)
    for q in range(s.nq):
        assert np.max(np.abs(eps[q] - g_ref[q])) <= TOL[prec] * np.max(np.abs(g_ref[q])), q
    if prec == 0:
        assert abs(E - E_ref) <= 1e-10 * abs(E_ref)
