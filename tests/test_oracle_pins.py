"""Pins of the CPU oracle against closed forms, library routines and invariants.

Each pin is written as a function returning an error measure so that the planted-mistake
test at the bottom can check that a plausible slip in any oracle step breaks at least one.
"""
import math

import numpy as np
import pytest

from oracle import rpa_oracle as orc
from paper_2505_06021_amd import inputs
from tests import pins


def tiny_complex(seed=3, nw=8):
    return inputs.make_system("tiny_c", (2, 2, 1), 2, 3, 5, nw, seed, is_complex=True, sigma=0.2)


def small_complex(seed=5, nw=48):
    return inputs.make_system("small_c", (2, 2, 1), 3, 6, 14, nw, seed, is_complex=True, sigma=0.12)


def small_real(seed=6, nw=48):
    return inputs.make_system("small_r", (1, 1, 1), 4, 9, 16, nw, seed, is_complex=False,
                              sigma=0.08, periodic=False)


# ---------------------------------------------------------------- pin functions

def err_chi0_bruteforce(sysm):
    worst = 0.0
    for iq in range(sysm.nq):
        for om in (0.0, 0.37, 5.0):
            ref = pins.chi0_bruteforce(sysm, iq, om)
            got = orc.chi0(sysm, iq, om)
            worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
    return worst


def err_plasmon(sysm):
    e_or, _ = orc.energy(sysm)
    e_ex = pins.plasmon_energy(sysm)
    return abs(e_or - e_ex) / abs(e_ex)


def err_trace_log_eig(sysm):
    """Error relative to the largest |eps| of the q (eps cancels catastrophically at large omega)."""
    worst = 0.0
    for iq in range(sysm.nq):
        errs, scale = [], 0.0
        for j in (0, sysm.nw // 2, sysm.nw - 1):
            c = orc.chi0(sysm, iq, sysm.omega[j])
            p = orc.pi_matrix(sysm.vhalf[iq], c)
            ref = pins.trace_log_eig(p)
            errs.append(abs(orc.trace_log(p) - ref))
            scale = max(scale, abs(ref))
        worst = max(worst, max(errs) / scale)
    return worst


def err_logdet_algebra(sysm):
    """ln det(1 - Pi) = ln det(V^-1 - chi0) + ln det V and Tr Pi = sum_PQ chi0_PQ V_QP."""
    worst = 0.0
    for iq in range(sysm.nq):
        vh = sysm.vhalf[iq]
        V = vh @ vh
        for om in (0.1, 2.0):
            c = orc.chi0(sysm, iq, om)
            p = orc.pi_matrix(vh, c)
            e_or = orc.trace_log(p)
            s1, l1 = np.linalg.slogdet(np.linalg.inv(V) - c)
            s2, l2 = np.linalg.slogdet(V)
            tr = float(np.real(np.sum(c * V.T)))
            ref = float(l1 + l2) + tr
            worst = max(worst, abs(e_or - ref) / abs(ref))
    return worst


def err_ring_mp2(sysm):
    """E(lambda V)/lambda^2 -> E2 as lambda -> 0 (three-point Richardson in lambda).

    lambda = 1e-3 balances the O(lambda^3) remainder against the absolute rounding floor of
    ln det + Tr at tiny Pi, which the large tail weights of the omega map amplify.
    """
    lam = 1e-3
    vh0 = sysm.vhalf.copy()
    vals = []
    for s in (lam, 2 * lam, 4 * lam):
        sysm.vhalf = vh0 * math.sqrt(s)
        e, _ = orc.energy(sysm)
        vals.append(e / (s * s))
    sysm.vhalf = vh0
    e2_num = (8.0 * vals[0] - 6.0 * vals[1] + vals[2]) / 3.0
    e2_ex = pins.ring_mp2_energy(sysm)
    return abs(e2_num - e2_ex) / abs(e2_ex)


# ---------------------------------------------------------------- the pins

def test_chi0_matches_bruteforce_loops():
    assert err_chi0_bruteforce(tiny_complex()) < 1e-13


def test_chi0_real_system_bruteforce():
    s = inputs.make_system("tiny_r", (1, 1, 1), 2, 3, 4, 4, 9, is_complex=False, sigma=0.3,
                           periodic=False)
    assert err_chi0_bruteforce(s) < 1e-13


def test_chi0_hermitian_and_real_at_gamma():
    s = small_complex(nw=4)
    for iq in range(s.nq):
        c = orc.chi0(s, iq, 0.7)
        assert np.abs(c - c.conj().T).max() <= 1e-15 * np.abs(c).max()
    r = small_real(nw=4)
    c = orc.chi0(r, 0, 0.7)
    assert c.dtype == np.float64
    assert np.abs(c - c.T).max() <= 1e-15 * np.abs(c).max()


def test_trace_log_equals_eigenvalue_route():
    assert err_trace_log_eig(small_complex(nw=8)) < 1e-11
    assert err_trace_log_eig(small_real(nw=8)) < 1e-11


def test_trace_log_single_aux_function():
    for p in (-1e-6, -0.3, -5.0, -120.0):
        pi = np.array([[p]])
        ref = math.log1p(-p) + p
        # 2 ln L_11 with L_11 = sqrt(1 - p) carries the absolute rounding of ln near 1
        assert abs(orc.trace_log(pi) - ref) <= 1e-14 * abs(ref) + 4.5e-16


def test_logdet_algebra_without_sandwich():
    assert err_logdet_algebra(small_complex(nw=4)) < 1e-10
    assert err_logdet_algebra(small_real(nw=4)) < 1e-10


def test_pi_negative_semidefinite_and_point_bounds():
    s = small_complex(nw=16)
    for iq in range(s.nq):
        prev = -np.inf
        for j in range(s.nw):
            c = orc.chi0(s, iq, s.omega[j])
            p = orc.pi_matrix(s.vhalf[iq], c)
            lam = np.linalg.eigvalsh(p)
            assert lam.max() <= 1e-14 * abs(lam).max()
            L = np.linalg.cholesky(np.eye(s.naux) - p)
            assert np.real(np.diagonal(L)).min() >= 1.0 - 1e-14
            e = orc.trace_log(p)
            assert e <= 0.0
            tr2 = float(np.real(np.trace(p @ p)))
            assert e >= -0.5 * tr2 * (1 + 1e-12)
            assert e >= prev - 1e-14 * abs(e)   # omega nodes are increasing
            prev = e


def test_energy_matches_plasmon_closed_form_complex():
    assert err_plasmon(small_complex(nw=48)) < 1e-9


def test_energy_matches_plasmon_closed_form_real():
    assert err_plasmon(small_real(nw=48)) < 1e-9


def test_quadrature_converges_to_plasmon():
    base = small_complex(nw=8)
    ex = pins.plasmon_energy(base)
    errs = []
    for nw in (4, 8, 16, 32):
        base.omega, base.weight = inputs.frequency_grid(nw)
        e, _ = orc.energy(base)
        errs.append(abs(e - ex))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-8 * abs(ex)


def test_two_level_closed_form():
    s = inputs.make_system("two", (1, 1, 1), 1, 1, 7, 48, 11, is_complex=True, sigma=0.6,
                           periodic=False)
    d = s.eps_virt[0, 0] - s.eps_occ[0, 0]
    b = s.B_block(0, 0).reshape(-1)
    V = s.vhalf[0] @ s.vhalf[0]
    K = float(np.real(b @ V @ b.conj()))      # zeta_k = 1
    exact = 0.5 * (math.sqrt(d * d + 4 * d * K) - d - 2 * K)
    e, _ = orc.energy(s)
    assert abs(e - exact) <= 1e-9 * abs(exact)


def test_second_order_ring_limit():
    assert err_ring_mp2(small_complex(nw=64)) < 1e-5
    assert err_ring_mp2(small_real(nw=64)) < 1e-5


def test_gauss_legendre_map_integrates_known_functions():
    om, w = inputs.frequency_grid(32)
    assert abs(np.sum(w / (1.0 + om) ** 2) - 1.0) < 1e-13
    for d in (0.15, 1.0, 3.0):
        assert abs(np.sum(w * d / (d * d + om * om)) - math.pi / 2) < 1e-6
    om8, w8 = inputs.frequency_grid(8)
    assert np.all(np.diff(om8) > 0) and np.all(w8 > 0)


def test_energy_order_and_zeta_weights():
    s = small_complex(nw=8)
    e, g = orc.energy(s)
    manual = sum(s.zeta_q[q] * s.weight[j] * g[q, j] for q in range(s.nq) for j in range(s.nw))
    assert abs(e - manual / (2 * math.pi)) <= 1e-14 * abs(e)
    assert e < 0.0


# ---------------------------------------------------------------- planted mistakes

def _mut_weight_sign(delta, omega):
    return 4.0 * delta / (delta * delta + omega * omega)


def _mut_weight_factor(delta, omega):
    return -2.0 * delta / (delta * delta + omega * omega)


def _mut_weight_omega(delta, omega):
    return -4.0 * delta / (delta * delta + omega)


def _mut_transition_index(eps_occ, eps_virt, kq, iq):
    return eps_virt[:, None, :] - eps_occ[:, :, None]          # drops k (+) q


def _mut_pi_transpose(vhalf_q, chi0_q):
    return vhalf_q @ chi0_q.T @ vhalf_q


def _mut_pi_one_sided(vhalf_q, chi0_q):
    return vhalf_q @ vhalf_q @ chi0_q


def _mut_trace_sign(pi):
    n = pi.shape[0]
    L = np.linalg.cholesky(np.eye(n, dtype=pi.dtype) - pi)
    return 2.0 * float(np.sum(np.log(np.real(np.diagonal(L))))) - float(np.real(np.trace(pi)))


def _mut_trace_half(pi):
    n = pi.shape[0]
    L = np.linalg.cholesky(np.eye(n, dtype=pi.dtype) - pi)
    return float(np.sum(np.log(np.real(np.diagonal(L))))) + float(np.real(np.trace(pi)))


def _mut_quad_nopi(eps_qw, zeta_q, weight):
    return math.fsum(zeta_q[q] * weight[j] * eps_qw[q, j] for q in range(eps_qw.shape[0])
                     for j in range(eps_qw.shape[1]))


def _mut_quad_noq(eps_qw, zeta_q, weight):
    return math.fsum(weight[j] * eps_qw[q, j] / (2 * math.pi) for q in range(eps_qw.shape[0])
                     for j in range(eps_qw.shape[1]))


def _mut_chi0_conj(system, iq, omega, row_block=None):
    return np.conj(_orig_chi0(system, iq, omega, row_block))


def _mut_chi0_zeta(system, iq, omega, row_block=None):
    s = system.zeta_k.copy()
    system.zeta_k = np.ones_like(s)
    try:
        return _orig_chi0(system, iq, omega, row_block)
    finally:
        system.zeta_k = s


_orig_chi0 = orc.chi0

MUTATIONS = [
    ("frequency_weight", _mut_weight_sign),
    ("frequency_weight", _mut_weight_factor),
    ("frequency_weight", _mut_weight_omega),
    ("transition_energies", _mut_transition_index),
    ("pi_matrix", _mut_pi_transpose),
    ("pi_matrix", _mut_pi_one_sided),
    ("trace_log", _mut_trace_sign),
    ("trace_log", _mut_trace_half),
    ("quadrature", _mut_quad_nopi),
    ("quadrature", _mut_quad_noq),
    ("chi0", _mut_chi0_conj),
    ("chi0", _mut_chi0_zeta),
]


@pytest.mark.parametrize("name,fn", MUTATIONS, ids=[f"{n}:{f.__name__}" for n, f in MUTATIONS])
def test_pins_catch_planted_mistake(monkeypatch, name, fn):
    monkeypatch.setattr(orc, name, fn)
    s_c = tiny_complex(nw=24)
    s_r = small_real(nw=24)
    checks = [
        lambda: err_chi0_bruteforce(s_c) > 1e-8,
        lambda: err_plasmon(s_c) > 1e-5,
        lambda: err_plasmon(s_r) > 1e-5,
        lambda: err_logdet_algebra(s_c) > 1e-8,
        lambda: err_trace_log_eig(s_c) > 1e-8,
    ]
    caught = False
    for chk in checks:
        try:
            if chk():
                caught = True
                break
        except (np.linalg.LinAlgError, ValueError, FloatingPointError):
            caught = True
            break
    assert caught, f"planted mistake in {name} went unnoticed"
