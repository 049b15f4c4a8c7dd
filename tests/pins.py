"""Independent closed forms that pin the oracle (test code, not part of the oracle).

None of these routes goes through the frequency integral, the Cholesky factor or the
sandwich V^(1/2) chi0 V^(1/2) that the oracle uses, so a dropped term, a wrong sign or
index, or a transposed operand in the oracle shows up as a mismatch.

Notation: x = (k, i, a) runs over the M transitions of one q; Delta_x as in the
polarizability equation of the paper (Sec. 2.2); c_x = 2 zeta_k so that
w_x(omega) zeta_k = -c_x * 2 Delta_x / (Delta_x^2 + omega^2); Ktilde = B V B^H with
V = (V^(1/2))^2 and B the M x N_aux coefficient matrix.  By Sylvester's identity
det(1 - V^(1/2) chi0 V^(1/2)) = det(1 - W Ktilde), which turns the q-integrand into a
function of the M x M matrix Ktilde only.
"""
from __future__ import annotations

import math

import numpy as np


def ao_block(system, iq, ik):
    """B[i][a][gamma] of an atomic-orbital system, one gamma at a time as the conjugate of
    the matrix product (c_virt(k)^H C_gamma c_occ(k (+) q))^T (the pair coefficient
    C^{ai}_gamma of Sec. 2.2; B is its conjugate), from the generator's projected
    coefficients."""
    from paper_2505_06021_amd import inputs
    C = inputs.philox_C_block(system.seed, system.sigma, system.nk, iq, ik, system.nbas, system.naux)
    cv = system.c_virt[ik]
    co = system.c_occ[system.kq[iq, ik]]
    out = np.empty((system.nocc, system.nvirt, system.naux), dtype=np.complex128)
    for g in range(system.naux):
        out[:, :, g] = (cv.conj().T @ C[:, :, g] @ co).T
    return out.conj()


def transitions(system, iq):
    """Delta_x, c_x and the [M, N_aux] coefficient matrix B of one q, built directly."""
    rows, deltas, cs = [], [], []
    for ik in range(system.nk):
        kq = system.kq[iq, ik]
        for i in range(system.nocc):
            for a in range(system.nvirt):
                deltas.append(system.eps_virt[ik, a] - system.eps_occ[kq, i])
                cs.append(2.0 * system.zeta_k[ik])
        blk = ao_block(system, iq, ik) if system.nbas > 0 else system.B_block(iq, ik)
        rows.append(blk.reshape(-1, system.naux))
    return np.array(deltas), np.array(cs), np.concatenate(rows, axis=0)


def coupling(system, iq):
    d, c, B = transitions(system, iq)
    V = system.vhalf[iq] @ system.vhalf[iq]
    Kt = B @ V @ B.conj().T
    return d, c, Kt


def plasmon_energy(system, vscale=1.0):
    """Exact frequency integral (dRPA plasmon formula, Furche 2008).

    Per q: E_q = 1/2 [sum_n Omega_n - sum_x Delta_x - Tr K] with
    K = C^(1/2) Ktilde C^(1/2) and Omega_n^2 the eigenvalues of D^2 + 2 D^(1/2) K D^(1/2);
    E = sum_q zeta_q E_q.  Follows from int_0^inf ln(1 + c/(Delta^2 + w^2)) dw
    = pi (sqrt(Delta^2 + c) - Delta) in the eigenbasis.
    """
    total = []
    for iq in range(system.nq):
        d, c, Kt = coupling(system, iq)
        K = vscale * np.sqrt(c)[:, None] * Kt * np.sqrt(c)[None, :]
        sd = np.sqrt(d)
        A = np.diag(d * d) + 2.0 * sd[:, None] * K * sd[None, :]
        om2 = np.linalg.eigvalsh(0.5 * (A + A.conj().T))
        Eq = 0.5 * (np.sum(np.sqrt(om2)) - np.sum(d) - float(np.real(np.trace(K))))
        total.append(system.zeta_q[iq] * Eq)
    return math.fsum(total)


def ring_mp2_energy(system):
    """Second-order (direct ring) limit: E2 = -1/2 sum_xy c_x c_y |Ktilde_xy|^2/(Delta_x+Delta_y).

    Equal to -(1/4 pi) int_0^inf Tr Pi^2 d omega, using
    int_0^inf 4 Dx Dy / ((Dx^2+w^2)(Dy^2+w^2)) dw = 2 pi / (Dx + Dy).
    At Gamma with zeta = 1 this is -2 sum |(ia|jb)|^2 / (Delta_ia + Delta_jb).
    """
    total = []
    for iq in range(system.nq):
        d, c, Kt = coupling(system, iq)
        num = (c[:, None] * c[None, :]) * np.abs(Kt) ** 2
        total.append(system.zeta_q[iq] * (-0.5) * np.sum(num / (d[:, None] + d[None, :])))
    return math.fsum(total)


def trace_log_eig(pi):
    """sum_i ln(1 - lambda_i) + lambda_i from the eigenvalues of the Hermitian Pi."""
    lam = np.linalg.eigvalsh(0.5 * (pi + pi.conj().T))
    return float(np.sum(np.log1p(-lam) + lam))


def chi0_bruteforce(system, iq, omega):
    """chi0_PQ = sum_k zeta_k sum_ia conj(B^P_ia) w_ia B^Q_ia by explicit loops (tiny sizes)."""
    n = system.naux
    out = [[0j] * n for _ in range(n)]
    for ik in range(system.nk):
        Bk = system.B_block(iq, ik)
        kq = system.kq[iq, ik]
        for i in range(system.nocc):
            for a in range(system.nvirt):
                dl = system.eps_virt[ik, a] - system.eps_occ[kq, i]
                w = -4.0 * dl / (dl * dl + omega * omega)
                for P in range(n):
                    bp = complex(Bk[i, a, P]).conjugate()
                    for Q in range(n):
                        out[P][Q] += system.zeta_k[ik] * bp * w * complex(Bk[i, a, Q])
    return np.array(out)
