"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Tolerances (FP64 path):
  chi0    ||chi0_gpu - chi0_oracle||_F <= 1e-12 ||chi0_oracle||_F
  eps     |eps_gpu(q,w) - eps_oracle(q,w)| <= 1e-10 max_w' |eps_oracle(q,w')|  (scale-aware:
          ln det(1 - Pi) and Tr Pi cancel at large w, so a point's own |eps| is no scale)
  E       |E_gpu - E_oracle| <= 1e-10 |E_oracle|
Philox words are compared bit for bit; B values to a few ulp (the device and host
transcendental functions may differ in the last bit).
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from oracle import rpa_oracle as orc
from paper_2505_06021_amd import inputs

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_06021_amd import rpa
    c = rpa.Context(0)
    yield c
    c.close()


def rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def rel_rows(a, b):
    """Element by element: max_PQ |a_PQ - b_PQ| / max_Q' |b_PQ'| (each row's own scale)."""
    return float(np.max(np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)))


def ragged_system(seed=31, nw=5):
    # N = 150 spans three 64-wide tiles with a ragged tail; M = 4*3*7 = 84 is not a
    # multiple of the 16-row K step
    return inputs.make_system("ragged", (2, 2, 1), 3, 7, 150, nw, seed, is_complex=True, sigma=0.15)


# ---------------------------------------------------------------- Philox (a1)

def test_philox_words_bitwise(ctx):
    say("philox words")
    for seed, nk, iq, ik, e0, n in [(7, 9, 0, 0, 0, 4096), (2 ** 40 + 5, 9, 8, 3, 12345, 1000),
                                    (123, 36, 35, 35, 2 ** 32 - 100, 300)]:
        dev = ctx.philox_words(seed, nk, iq, ik, e0, n)
        host = inputs.philox_words(seed, nk, iq, ik, e0, n)
        assert np.array_equal(dev, host), (seed, iq, ik, e0)


@pytest.mark.parametrize("cplx", [True, False])
def test_philox_B_matches_host(ctx, cplx):
    say(f"philox B complex={cplx}")
    dev = ctx.philox_B(99, 0.03, 9, 4, 7, 5, 112, 96, is_complex=cplx)
    host = inputs.philox_B_block(99, 0.03, 9, 4, 7, 5, 112, 96, cplx)
    assert np.max(np.abs(dev - host)) <= 1e-14 * 0.03 * 8


# ---------------------------------------------------------------- chi0 (a2, a3)

def test_chi0_gamma_real_explicit_B(ctx):
    say("chi0 Gamma real 128")
    s = inputs.gamma_real_128().materialize_B()
    for j in (0, 3, 7):
        ref = orc.chi0(s, 0, s.omega[j])
        got = ctx.chi0(s, 0, s.omega[j])
        assert got.dtype == np.float64
        assert rel_fro(got, ref) <= 1e-12
        assert rel_rows(got, ref) <= 1e-12


def test_chi0_ragged_tiles_philox(ctx):
    say("chi0 ragged N=150 M=84")
    s = ragged_system()
    for iq in (0, 3):
        for om in (0.0, 0.77, 40.0):
            ref = orc.chi0(s, iq, om)
            got = ctx.chi0(s, iq, om)
            assert rel_fro(got, ref) <= 1e-12, (iq, om)
            assert rel_rows(got, ref) <= 1e-12, (iq, om)
            assert np.abs(got - got.conj().T).max() == 0.0


def test_chi0_slab384_sampled(ctx):
    say("chi0 slab 3x3 naux 384")
    s = inputs.slab_3x3_384()
    for iq, j in [(0, 0), (4, 11)]:
        ref = orc.chi0(s, iq, s.omega[j])
        got = ctx.chi0(s, iq, s.omega[j])
        assert rel_fro(got, ref) <= 1e-12
        assert rel_rows(got, ref) <= 1e-12


def test_chi0_split_count_capped_by_hbm_limit(monkeypatch):
    """rpa_chi0 under an HBM limit that holds only a few of the row splits' partial
    planes: the capped split count still gives the oracle's chi0 (and the one-split
    result to rounding)."""
    from paper_2505_06021_amd import rpa
    say("chi0 split count under a tight HBM limit")
    s = inputs.slab_3x3_384()
    iq, om = 2, s.omega[3]
    ref = orc.chi0(s, iq, om)
    N, M = s.naux, s.M
    plane = N * N * 16
    # B slab, weight table, output and descriptors, plus three partial planes
    limit = M * N * 16 + M * 8 + 2 * plane + (1 << 20) + 3 * plane
    with rpa.Context(0, hbm_limit=limit) as c:
        got = c.chi0(s, iq, om, device=False)
    assert rel_fro(got, ref) <= 1e-12
    assert rel_rows(got, ref) <= 1e-12
    monkeypatch.setenv("RPA_CHI0_KSPLIT", "1")
    with rpa.Context(0) as c:
        one = c.chi0(s, iq, om, device=False)
    assert rel_rows(got, one) <= 1e-13


def test_chi0_device_memspace_equals_host(ctx):
    say("chi0 device memspace")
    s = ragged_system(nw=2)
    a = ctx.chi0(s, 1, 0.5, device=False)
    b = ctx.chi0(s, 1, 0.5, device=True)
    assert np.array_equal(a, b)


def test_chi0_single_aux_and_single_transition(ctx):
    say("chi0 degenerate sizes")
    s = inputs.make_system("deg", (1, 1, 1), 1, 1, 1, 3, 5, is_complex=True, sigma=0.4, periodic=False)
    ref = orc.chi0(s, 0, 0.3)
    got = ctx.chi0(s, 0, 0.3)
    assert rel_fro(got, ref) <= 1e-14


# ---------------------------------------------------------------- Pi (a4)

@pytest.mark.parametrize("n,cplx", [(1, True), (100, True), (200, True), (130, False)])
def test_pi_sandwich(ctx, n, cplx):
    say(f"pi n={n} complex={cplx}")
    rng = np.random.default_rng(n)
    if cplx:
        v = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        c = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    else:
        v = rng.standard_normal((n, n))
        c = rng.standard_normal((n, n))
    v = v + v.conj().T
    c = c + c.conj().T
    ref = orc.pi_matrix(v, c)
    got = ctx.pi(v, c)
    assert rel_fro(got, ref) <= 1e-13


# ---------------------------------------------------------------- Tr ln (a5)

def pis_of(s, pts):
    return [orc.pi_matrix(s.vhalf[iq], orc.chi0(s, iq, s.omega[j])) for iq, j in pts]


@pytest.mark.parametrize("n", [1, 16, 17, 64, 65, 129, 150, 384, 700])
def test_trln_matches_oracle(ctx, n):
    say(f"trln n={n}")
    s = inputs.make_system("t", (1, 1, 1), 4, 30, n, 6, 100 + n, is_complex=True, sigma=0.2,
                           periodic=False)
    pis = np.stack(pis_of(s, [(0, j) for j in range(s.nw)]))
    ref = np.array([orc.trace_log(p) for p in pis])
    got = ctx.trln(pis)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-10 * scale


@pytest.mark.parametrize("n", [1, 17, 150, 384])
def test_trln_single_workgroup_matches_oracle(ctx, monkeypatch, n):
    # RPA_TRLN_SINGLE=1: the one-workgroup-per-matrix factorisation instead of the blocked one
    say(f"trln single-workgroup n={n}")
    monkeypatch.setenv("RPA_TRLN_SINGLE", "1")
    s = inputs.make_system("t", (1, 1, 1), 4, 30, n, 6, 300 + n, is_complex=True, sigma=0.2,
                           periodic=False)
    pis = np.stack(pis_of(s, [(0, j) for j in range(s.nw)]))
    ref = np.array([orc.trace_log(p) for p in pis])
    got = ctx.trln(pis)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_energy_single_workgroup_trln_matches_oracle(ctx, monkeypatch):
    say("energy with the single-workgroup Cholesky")
    monkeypatch.setenv("RPA_TRLN_SINGLE", "1")
    s = ragged_system(nw=4)
    E_ref, g_ref = orc.energy(s)
    E, eps = ctx.energy(s)
    assert abs(E - E_ref) <= 1e-10 * abs(E_ref)
    check_grid(eps, g_ref)


def test_trln_real_input(ctx):
    say("trln real")
    s = inputs.gamma_real_128().materialize_B()
    pis = np.stack(pis_of(s, [(0, 0), (0, 5)]))
    ref = np.array([orc.trace_log(p) for p in pis])
    assert np.max(np.abs(ctx.trln(pis) - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,col", [(40, 17), (200, 130), (20, 0), (70, 63), (100, 79), (130, 64)])
def test_trln_not_positive_definite_is_an_error(ctx, n, col):
    from paper_2505_06021_amd import rpa
    say(f"trln not SPD n={n} col={col}")
    pi = np.zeros((3, n, n), dtype=np.complex128)
    pi[1, col, col] = 2.0     # 1 - Pi_1 has a negative pivot at column `col`
    with pytest.raises(rpa.RpaError) as e:
        ctx.trln(pi)
    assert e.value.code == rpa.RPA_E_NOTSPD
    assert f"matrix 1 (column {col})" in str(e.value)


def test_trln_batch_mixed_sizes_of_values(ctx):
    """Matrices of very different norms in one batch do not interact."""
    say("trln batch independence")
    s = inputs.make_system("t", (1, 1, 1), 4, 30, 200, 6, 77, is_complex=True, sigma=0.2, periodic=False)
    pis = np.stack(pis_of(s, [(0, j) for j in range(s.nw)]))
    one = np.array([ctx.trln(p)[0] for p in pis])
    allb = ctx.trln(pis)
    assert np.array_equal(one, allb)


# ---------------------------------------------------------------- energy (a1-a6)

def check_grid(got, ref):
    for q in range(ref.shape[0]):
        scale = np.max(np.abs(ref[q]))
        assert np.max(np.abs(got[q] - ref[q])) <= 1e-10 * scale, q


def test_energy_gamma_real_golden(ctx):
    say("energy Gamma real 128 (explicit B and Philox)")
    g = json.load(open(os.path.join(GOLD, "gamma_real_naux128.json")))
    s = inputs.gamma_real_128()
    E, eps = ctx.energy(s)                       # B from the device Philox stream
    assert abs(E - g["E"]) <= 1e-10 * abs(g["E"])
    check_grid(eps, np.array(g["eps"]))
    s.materialize_B()
    E2, _ = ctx.energy(s)                        # explicit B from host memory
    assert abs(E2 - g["E"]) <= 1e-10 * abs(g["E"])


def test_energy_slab384_golden(ctx):
    say("energy slab 3x3 naux 384")
    g = json.load(open(os.path.join(GOLD, "slab3x3_naux384.json")))
    s = inputs.slab_3x3_384()
    E, eps = ctx.energy(s)
    assert abs(E - g["E"]) <= 1e-10 * abs(g["E"])
    check_grid(eps, np.array(g["eps"]))


def test_energy_ragged_live_oracle(ctx):
    say("energy ragged live oracle")
    s = ragged_system(nw=6)
    E_ref, g_ref = orc.energy(s)
    E, eps = ctx.energy(s)
    assert abs(E - E_ref) <= 1e-10 * abs(E_ref)
    check_grid(eps, g_ref)


def test_energy_device_inputs_bitwise_equal(ctx):
    say("energy device inputs")
    s = ragged_system(nw=4)
    a = ctx.energy(s, device=False)
    b = ctx.energy(s, device=True)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_points_subset_equals_energy_grid(ctx):
    say("points subset")
    s = ragged_system(nw=4)
    E, eps = ctx.energy(s)
    iq = [3, 0, 2, 3]
    j = [1, 0, 3, 2]
    got = ctx.points(s, iq, s.omega[j])
    assert np.array_equal(got, eps[iq, j])


def test_energy_repeatable_bitwise(ctx):
    say("energy repeatable")
    s = ragged_system(nw=3)
    a = ctx.energy(s)
    b = ctx.energy(s)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------- errors

def test_argument_errors(ctx):
    from paper_2505_06021_amd import rpa
    say("argument errors")
    s = ragged_system(nw=2)
    s.kq = s.kq.copy()
    s.kq[1, 2] = 99                      # out-of-range k (+) q index is refused on the host
    with pytest.raises(rpa.RpaError) as e:
        ctx.energy(s)
    assert e.value.code == rpa.RPA_E_ARG
    s = ragged_system(nw=2)
    s.eps_occ = s.eps_occ + 5.0          # metallic: negative transition energies
    with pytest.raises(rpa.RpaError) as e:
        ctx.energy(s)
    assert e.value.code == rpa.RPA_E_ARG
    with pytest.raises(rpa.RpaError) as e:
        ctx.chi0(ragged_system(nw=2), 7, 0.1)
    assert e.value.code == rpa.RPA_E_ARG


def test_degenerate_and_out_of_range_inputs_are_errors(ctx):
    # empty frequency grid, a negative node, N_aux beyond the supported 16384, a negative
    # occupied-row count, a k (+) q row beyond a dual grid's occupied energies
    from paper_2505_06021_amd import rpa
    say("degenerate inputs")
    cases = []
    s = ragged_system(nw=2)
    s.omega, s.weight = s.omega[:0], s.weight[:0]
    cases.append(s)
    s = ragged_system(nw=2)
    s.omega = s.omega.copy()
    s.omega[0] = -1.0
    cases.append(s)
    s = ragged_system(nw=2)
    s.naux = 16385
    cases.append(s)
    s = inputs.make_dual_system("dual_err", (2, 2, 1), 2, 3, 8, 2, 5, frac=0.1)
    s.eps_occ = s.eps_occ[: s.nk]      # only the regular grid's rows: displaced k (+) q out of range
    cases.append(s)
    for s in cases:
        with pytest.raises(rpa.RpaError) as e:
            ctx.energy(s)
        assert e.value.code == rpa.RPA_E_ARG, s.name


def test_hbm_limit_is_enforced():
    from paper_2505_06021_amd import rpa
    say("hbm limit")
    with rpa.Context(0, hbm_limit=1 << 20) as c:
        s = ragged_system(nw=2)
        with pytest.raises(rpa.RpaError) as e:
            c.energy(s)
        assert e.value.code == rpa.RPA_E_NOMEM


@pytest.mark.parametrize("prec", [0, 2])
def test_energy_two_lanes(ctx, monkeypatch, prec):
    # RPA_LANES=2 runs alternate batches on a second stream with their own buffers
    say(f"energy on two lanes prec={prec}")
    s = inputs.slab_3x3_384()
    E1, eps1 = ctx.energy(s, prec=prec)
    monkeypatch.setenv("RPA_LANES", "2")
    E2, eps2 = ctx.energy(s, prec=prec)
    tol = 1e-10 if prec == 0 else 2e-5
    assert abs(E2 - E1) <= tol * (abs(E1) if prec == 0 else 1.0)
    assert np.max(np.abs(eps2 - eps1)) <= (1e-10 if prec == 0 else 1e-6) * np.max(np.abs(eps1))
    if prec == 0:
        g = json.load(open(os.path.join(GOLD, "slab3x3_naux384.json")))
        assert abs(E2 - g["E"]) <= 1e-10 * abs(g["E"])
