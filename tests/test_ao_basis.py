"""Systems given in an atomic-orbital basis: the periodic projector and the MO transform
of the pair-fit coefficients (Sec. 2.2, Sec. 2.3), in the oracle.

Pins: the projector is a Hermitian idempotent of rank N_bas - N_dropped and the identity
when the threshold lies below every eigenvalue of S(k); applied to the raw KS
coefficients it removes exactly the contamination the generator put along the dropped
directions; the transform equals explicit loops over (mu, nu) and, for an identity basis,
a plain selection of pair-fit coefficients; chi0 equals the fit-basis polarizability of
Sec. 2.2 written element by element from the pair expansion (which fixes which index
carries the conjugate); the resulting energy equals the plasmon closed form computed from
the generator's projected coefficients.
"""
import numpy as np

from oracle import rpa_oracle as orc
from paper_2505_06021_amd import inputs
from tests import pins


def tiny(nbas=12, nw=4, **kw):
    return inputs.make_ao_system("ao_tiny", (2, 2, 1), nbas, 2, 3, 6, nw, 5, **kw)


def test_projector_is_a_hermitian_idempotent_of_the_kept_rank():
    s = tiny()
    T = orc.projector(s.S_ao, s.eps_d)
    for t in T:
        assert np.abs(t - t.conj().T).max() < 1e-14
        assert np.abs(t @ t - t).max() < 1e-13
        assert abs(np.trace(t).real - (s.nbas - 4)) < 1e-12
    T0 = orc.projector(s.S_ao, 1e-12)          # below every eigenvalue: nothing removed
    for t in T0:
        assert np.abs(t - np.eye(s.nbas)).max() < 1e-12


def test_projector_removes_the_contamination():
    s = tiny()
    ct = orc.projected_coefficients(s)
    ref = np.concatenate([s.c_occ, s.c_virt], axis=2)
    assert np.abs(ct - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(s.c_raw - ref).max() > 1e-3          # the raw coefficients differ


def test_transform_matches_explicit_loops():
    s = tiny(nbas=6, n_lowdep=1)
    s.naux = 3
    ct = orc.projected_coefficients(s)
    iq, ik = 3, 1
    got = orc.ao_pair_coefficients(s, ct, iq, ik)
    assert np.array_equal(orc.ao_B_block(s, ct, iq, ik), got.conj())
    C = inputs.philox_C_block(s.seed, s.sigma, s.nk, iq, ik, s.nbas, s.naux)
    cv, co = ct[ik][:, s.nocc:], ct[s.kq[iq, ik]][:, :s.nocc]
    ref = np.zeros_like(got)
    for i in range(s.nocc):
        for a in range(s.nvirt):
            for g in range(s.naux):
                acc = 0j
                for mu in range(s.nbas):
                    for nu in range(s.nbas):
                        acc += np.conj(cv[mu, a]) * C[mu, nu, g] * co[nu, i]
                ref[i, a, g] = acc
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_identity_basis_selects_pair_fit_coefficients():
    s = tiny(nbas=5, n_lowdep=0)
    eye = np.eye(5, dtype=np.complex128)
    s.c_raw = np.repeat(eye[None], s.nk, axis=0)
    s.S_ao = np.repeat(eye[None], s.nk, axis=0)
    ct = orc.projected_coefficients(s)
    for iq in range(s.nq):
        for ik in range(s.nk):
            C = inputs.philox_C_block(s.seed, s.sigma, s.nk, iq, ik, s.nbas, s.naux)
            B = orc.ao_B_block(s, ct, iq, ik)
            for i in range(s.nocc):
                for a in range(s.nvirt):
                    assert np.array_equal(B[i, a], C[s.nocc + a, i].conj())


def test_chi0_is_the_fit_basis_polarizability_element_by_element():
    """P_{g g'}(q, i w) = -2 sum_k zeta_k sum_ia C^{ai}_g C*^{ai}_{g'} / (Delta - i w) + c.c.
    (the c.c. taken of the resonant denominator), with C^{ai}_g(k+q, k) the coefficient of
    f_g in the expansion of psi*_a(k) psi_i(k+q): psi_n(k) = sum_mu c~_{mu n}(k) chi_mu(k)
    and chi*_mu(k) chi_nu(k+q) = sum_g C^{mu nu}_g(k+q, k) f_g.  Built by loops from the
    generator's projected coefficients; zeta_q stays outside chi0."""
    s = tiny(nbas=7, n_lowdep=1)
    s.naux = 4
    for iq, om in ((1, 0.0), (3, 0.61)):
        ref = np.zeros((s.naux, s.naux), dtype=complex)
        for ik in range(s.nk):
            C = inputs.philox_C_block(s.seed, s.sigma, s.nk, iq, ik, s.nbas, s.naux)
            kq = s.kq[iq, ik]
            for i in range(s.nocc):
                for a in range(s.nvirt):
                    pair = [0j] * s.naux
                    for g in range(s.naux):
                        for mu in range(s.nbas):
                            for nu in range(s.nbas):
                                pair[g] += (np.conj(s.c_virt[ik, mu, a]) * s.c_occ[kq, nu, i]
                                            * C[mu, nu, g])
                    dl = s.eps_virt[ik, a] - s.eps_occ[kq, i]
                    res = 1.0 / (dl - 1j * om)
                    den = res + np.conj(res)
                    for g in range(s.naux):
                        for gp in range(s.naux):
                            ref[g, gp] += -2.0 * s.zeta_k[ik] * pair[g] * np.conj(pair[gp]) * den
        got = orc.chi0(s, iq, om)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
        # the index order matters here: the transpose is a different matrix
        assert np.abs(ref - ref.T).max() > 1e-2 * np.abs(ref).max()


def test_ao_energy_matches_plasmon_closed_form():
    s = tiny(nbas=10, nw=48, n_lowdep=2)
    e = orc.energy(s)[0]
    ex = pins.plasmon_energy(s)
    assert abs(e - ex) <= 1e-9 * abs(ex)
