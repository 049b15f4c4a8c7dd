"""Dual k/q grids (Sec. 3.2): the grid construction and the oracle on such grids.

Pins: the size relation the section states (|K_G| = (N_add + 1) |K_reg| for a regular
K_reg, e.g. (10 x 10) x 5 in 2D), the travel relation k_j + q = k_i for every pair,
Gamma absent from Q_G, weights summing to one; with zero displacement the dual grids
reproduce the regular-grid energy exactly (Gamma's weight shared by N_add copies of it);
the oracle on a dual system matches the plasmon closed form and brute-force chi0.
"""
import numpy as np
import pytest

from oracle import rpa_oracle as orc
from paper_2505_06021_amd import inputs
from tests import pins


@pytest.mark.parametrize("grid,nadd", [((3, 3, 1), 4), ((4, 4, 1), 4), ((10, 10, 1), 4), ((2, 2, 2), 8),
                                       ((5, 1, 1), 2)])
def test_dual_grid_sizes(grid, nadd):
    kr, kqq, kg, kq, z = inputs.dual_grids(grid)
    nk = int(np.prod(grid))
    assert len(kr) == nk
    assert len(kqq) == nk - 1 + nadd
    assert len(kg) == (nadd + 1) * nk
    assert kq.shape == (len(kqq), nk) and kq.min() >= 0 and kq.max() == len(kg) - 1


@pytest.mark.parametrize("grid", [(3, 3, 1), (2, 2, 2), (4, 1, 1)])
def test_travel_relation_and_displacements(grid):
    frac = 0.1
    kr, kqq, kg, kq, z = inputs.dual_grids(grid, frac)
    n = np.array(grid)
    for iq in range(len(kqq)):
        for ik in range(len(kr)):
            d = (kg[kq[iq, ik]] - kr[ik] - kqq[iq] + 0.5) % 1.0 - 0.5
            assert np.abs(d).max() < 1e-9
    # no q at Gamma; the displaced points are all sign choices of +-frac/N_i on the
    # directions with more than one point
    folded = (kqq + 0.5) % 1.0 - 0.5
    assert np.abs(folded).sum(axis=1).min() > 0.0
    nreg = int(np.prod(grid)) - 1
    disp = folded[nreg:]
    dirs = [d for d in range(3) if n[d] > 1]
    want = {tuple(np.round([s[d] if d in dirs else 0.0 for d in range(3)], 12))
            for s in [np.array([sx, sy, sz]) * frac / n for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]}
    assert {tuple(np.round(x, 12)) for x in disp} == want


def test_dual_weights():
    kr, kqq, kg, kq, z = inputs.dual_grids((3, 3, 1))
    assert abs(z.sum() - 1.0) < 1e-15
    assert np.allclose(z[:8], 1.0 / 9) and np.allclose(z[8:], 1.0 / 36)


def test_zero_displacement_reproduces_regular_energy():
    reg = inputs.make_system("reg", (2, 2, 1), 2, 3, 6, 6, 11, is_complex=True, sigma=0.2).materialize_B()
    dual = inputs.make_dual_system("dual0", (2, 2, 1), 2, 3, 6, 6, 11, frac=0.0, sigma=0.2)
    assert dual.nk_occ == reg.nk and dual.nq == 3 + 4
    # Gamma's B and V^(1/2) for the four displaced copies of Gamma, the regular q's otherwise
    src = [1, 2, 3, 0, 0, 0, 0]
    assert np.array_equal(dual.kq[3:], np.tile(np.arange(4, dtype=np.int32), (4, 1)))
    dual.B = reg.B[src]
    dual.vhalf = reg.vhalf[src]
    dual.eps_occ = reg.eps_occ.copy()
    dual.eps_virt = reg.eps_virt.copy()
    e_reg = orc.energy(reg)[0]
    e_dual = orc.energy(dual)[0]
    assert abs(e_dual - e_reg) <= 1e-13 * abs(e_reg)


def small_dual(nw=48):
    return inputs.make_dual_system("small_dual", (2, 2, 1), 2, 4, 10, nw, 5, frac=0.1, sigma=0.15)


def test_dual_oracle_matches_plasmon_closed_form():
    s = small_dual()
    e = orc.energy(s)[0]
    ex = pins.plasmon_energy(s)
    assert abs(e - ex) <= 1e-9 * abs(ex)


def test_dual_chi0_matches_bruteforce_at_displaced_q():
    s = small_dual(nw=4)
    iq = s.nq - 1          # a displaced q: every k + q lies outside K_reg
    assert s.kq[iq].min() >= s.nk
    ref = pins.chi0_bruteforce(s, iq, s.omega[2])
    got = orc.chi0(s, iq, s.omega[2])
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
