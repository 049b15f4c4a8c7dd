"""Plain FP64 CPU oracle of the periodic RPA correlation energy hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import, call or link this
module; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP path: its inputs come from the
seeded input generators, and it computes every step of the method itself, slowly
and in the order the paper states it.

Steps (the paper's notation; "the paper" is arXiv:2505.06021):

1. transition energies  Delta_ia(k,q) = eps_a(k) - eps_i(k (+) q)
   (polarizability in the fit basis, Sec. 2.2, the equation for P^(0)_{gamma gamma'}).
2. frequency weight     w_ia(omega) = -4 Delta / (Delta^2 + omega^2): the factor -2 of
   the closed-shell occupations times the resonant term 1/(Delta - i omega) plus its
   complex conjugate (same equation).
3. polarizability       chi0_PQ(q, i omega) = sum_k zeta_k sum_ia conj(B^P_ia) w_ia B^Q_ia
   (same equation).  The paper writes P_{gamma gamma'} with C^{ai}_gamma C^{*ai}_{gamma'},
   C^{ai}_gamma(k+q,k) being the coefficient of f_gamma in the pair expansion of
   psi*_a(k) psi_i(k+q) (Sec. 2.2); B is the complex conjugate of that coefficient,
   B^P_ia = conj(C^{ai}_P), so that conj(B^P) B^Q = C^{ai}_P conj(C^{ai}_Q) keeps the
   paper's index order.  For synthetic coefficients B is the input itself.
4. Pi = V^(1/2) chi0 V^(1/2)   (the symmetrised response of the working equation;
   Algorithm 1, sandwich step).
5. eps(q, omega) = ln det(1 - Pi) + Re Tr Pi, with ln det from the Cholesky factor of the
   Hermitian positive definite 1 - Pi: ln det = 2 sum ln L_ii.  The sign follows Eq. 1
   (sum_n Z^n/n = -ln(1 - Z)); Algorithm 1 prints the term with the opposite sign, which
   would leave a first-order term in the energy.
6. E = sum_q zeta_q sum_j W_j eps(q, omega_j) / (2 pi)   (Eq. 1 with the q-sum of the
   working equation and the quadrature of the main-loop equation).

For systems given in an atomic-orbital basis the coefficients B of step 3 are built
first (Sec. 2.2 and the periodic projector method of Sec. 2.3):

0a. projector  S(k) = U D U^H; R(k) keeps the eigen-directions with D_ii >= eps_d; the
    cumulative mask is the product of the R(k) over all k (eigenvalues in ascending
    order); T(k) = U R U^H and the KS coefficients become c~ = T c.
0b. MO transform  C^{ai}_gamma(k+q,k) = sum_{mu nu} conj(c~_{mu a}(k)) C^{mu nu}_gamma(k,q)
    c~_{nu i}(k (+) q): the pair-fit expansion of psi*_a(k) psi_i(k+q) from that of the
    basis-function products; B^gamma_ia(k,q) = conj(C^{ai}_gamma) (step 3).

Every function here is pinned by tests against closed forms and library routines
(plasmon formula, second-order ring limit, eigenvalue route of Tr ln, invariants).
"""
from __future__ import annotations

import math

import numpy as np


def projector(S, eps_d):
    """T(k) for every k from the overlaps S[k] and the threshold eps_d  (step 0a)."""
    vals, vecs = [], []
    for Sk in S:
        d, U = np.linalg.eigh(Sk)
        vals.append(d)
        vecs.append(U)
    keep = np.ones(len(vals[0]), dtype=bool)
    for d in vals:
        keep &= d >= eps_d
    return [(U * keep[None, :]) @ U.conj().T for U in vecs]


def projected_coefficients(system):
    """c~(k) = T(k) c(k) for all bands, [nk][nbas][nocc + nvirt]  (step 0a)."""
    T = projector(system.S_ao, system.eps_d)
    return np.array([T[k] @ system.c_raw[k] for k in range(len(T))])


def ao_pair_coefficients(system, ct, iq, ik):
    """C^{ai}_gamma(k+q, k) of block (q, k), as [i][a][gamma]: the MO transform of the
    pair-fit coefficients  (step 0b)."""
    C = system.C_block(iq, ik)
    cv = ct[ik][:, system.nocc:]
    co = ct[system.kq[iq, ik]][:, :system.nocc]
    return np.einsum("ma,mng,ni->iag", cv.conj(), C, co, optimize=True)


def ao_B_block(system, ct, iq, ik):
    """B[i][a][gamma] of block (q, k) = conj(C^{ai}_gamma)  (steps 0b and 3)."""
    return ao_pair_coefficients(system, ct, iq, ik).conj()


def transition_energies(eps_occ, eps_virt, kq, iq):
    """Delta[k, i, a] = eps_virt[k, a] - eps_occ[k (+) q, i]  (step 1)."""
    return eps_virt[:, None, :] - eps_occ[kq[iq]][:, :, None]


def frequency_weight(delta, omega):
    """w = -4 Delta / (Delta^2 + omega^2)  (step 2)."""
    return -4.0 * delta / (delta * delta + omega * omega)


def chi0(system, iq, omega, row_block=None):
    """chi0(q, i omega) as an [naux, naux] matrix, accumulated k by k  (step 3).

    B is taken from the system row block by row block, so that large systems never
    hold more than one block of coefficients.
    """
    n = system.naux
    dt = np.complex128 if system.is_complex else np.float64
    out = np.zeros((n, n), dtype=dt)
    delta = transition_energies(system.eps_occ, system.eps_virt, system.kq, iq)
    w = frequency_weight(delta, omega)
    rb = system.nocc if row_block is None else row_block
    ct = projected_coefficients(system) if system.nbas > 0 else None
    for ik in range(system.nk):
        blk = ao_B_block(system, ct, iq, ik) if ct is not None else None
        for i0 in range(0, system.nocc, rb):
            i1 = min(system.nocc, i0 + rb)
            Bk = (blk[i0:i1] if blk is not None else system.B_rows(iq, ik, i0, i1)).reshape(-1, n)
            wk = system.zeta_k[ik] * w[ik, i0:i1].reshape(-1)
            out += Bk.conj().T @ (wk[:, None] * Bk)
    return out


def pi_matrix(vhalf_q, chi0_q):
    """Pi = V^(1/2) chi0 V^(1/2)  (step 4)."""
    return vhalf_q @ chi0_q @ vhalf_q


def trace_log(pi):
    """ln det(1 - Pi) + Re Tr Pi via Cholesky of 1 - Pi  (step 5)."""
    n = pi.shape[0]
    L = np.linalg.cholesky(np.eye(n, dtype=pi.dtype) - pi)
    return 2.0 * float(np.sum(np.log(np.real(np.diagonal(L))))) + float(np.real(np.trace(pi)))


def point(system, iq, j, row_block=None):
    """eps(q, omega_j) of one (q, omega) point (steps 1-5)."""
    c = chi0(system, iq, system.omega[j], row_block)
    return trace_log(pi_matrix(system.vhalf[iq], c))


def eps_grid(system, points=None):
    """eps[q][j] on all points (or on the listed (q, j) pairs, others NaN)."""
    out = np.full((system.nq, system.nw), np.nan)
    if points is None:
        points = [(iq, j) for iq in range(system.nq) for j in range(system.nw)]
    for iq, j in points:
        out[iq, j] = point(system, iq, j)
    return out


def quadrature(eps_qw, zeta_q, weight):
    """E = sum_q zeta_q sum_j W_j eps(q, omega_j) / (2 pi), summed exactly  (step 6)."""
    terms = []
    for iq in range(eps_qw.shape[0]):
        for j in range(eps_qw.shape[1]):
            terms.append(zeta_q[iq] * weight[j] * eps_qw[iq, j] / (2.0 * math.pi))
    return math.fsum(terms)


def energy(system):
    """RPA correlation energy per cell and the eps[q][omega] grid."""
    g = eps_grid(system)
    return quadrature(g, system.zeta_q, system.weight), g
