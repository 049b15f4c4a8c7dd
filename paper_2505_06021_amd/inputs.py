"""Seeded synthetic inputs for the periodic RPA hot path.

This module is the one place that both the HIP path (through its tests and the
benchmark) and the CPU oracle draw their inputs from.  It contains no step of the
RPA method itself: it only produces the data the method consumes, i.e. band
energies, the k (+) q index map, the integration weights, the square root of the
Coulomb matrix V(q), the imaginary-frequency grid and the density-fitted
transition coefficients B^P_ia(k,q).

Input recipe (the paper's physical systems need DFT data that is not available,
so slab-shaped synthetic systems of the paper's sizes stand in for them):

* k-grids are regular n1 x n2 x n3 grids in reduced coordinates kappa_d = n_d/N_d,
  and Q_G equals K_G (regular grids, Sec. "Dual grids", the regular-grid case);
  k (+) q is index addition modulo the grid in every direction.  make_dual_system
  builds the dual grids of that section instead: Gamma removed from the q-grid, 2^D
  points sum_i (+-d_i) b_i added around it (D directions with more than one point,
  d_i = frac/N_i), and K_G = {k_j + q}; the occupied energies are then given on K_G.
* Band energies: eps0_i ~ U[-1.0,-0.3] Ha (occupied), eps0_a ~ U[0.05,3.0] Ha
  (virtual), plus a band-independent dispersion 0.1*cos(2 pi (k1+k2+k3)) for
  periodic systems, so every transition energy is >= 0.15 Ha (insulator, as the
  polarizability section of the paper assumes).
* V(q) = Q Lambda Q^H with Q Haar-distributed (QR of a Gaussian matrix with the
  diagonal phase of R moved into Q) and Lambda = 10^U[-2,1] * f(q); f(q) = 1 for a
  Gamma-only system, else f(q) = 1 + 1/|q|^2 with |q|^2 = (2 pi)^2 sum kappa_d^2
  (kappa folded into [-1/2,1/2)), and f(0) = 1 + 1/|q_min|^2 (regularised head).
  Only V^(1/2) = Q Lambda^(1/2) Q^H is handed over.
* B^P_ia(k,q) is drawn from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
  followed by a Box-Muller transform; CN(0, sigma^2) for complex systems
  (real and imaginary parts each N(0, sigma^2/2)), N(0, sigma^2) for real ones.
  Stream layout: key = (seed mod 2^32, (seed >> 32) + q*N_k + k mod 2^32),
  counter = (e mod 2^32, e >> 32, 0, 0) with e = (i*N_virt + a)*N_aux + P.
  The four output words w0..w3 give two uniforms
  u = ((w_even >> 6) * 2^26 + (w_odd >> 6) + 1/2) * 2^-52 in (0,1), exactly
  representable in binary64; r = sqrt(-2 ln u1), theta = 2 pi u2 and
  B = sigma/sqrt(2) * r * (cos theta + i sin theta) (complex) or
  B = sigma * r * cos theta (real).  The device generator follows the same
  definition; the 32-bit words agree bit for bit, the transcendental functions
  may differ in the last ulp.
* Frequencies: n-point Gauss-Legendre on x in [0,1], mapped by omega = x/(1-x);
  the weight carries the Jacobian d omega/dx = 1/(1-x)^2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Philox4x32 constants from the published definition (SC'11): round multipliers
# and the Weyl key increments.
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on arrays.

    ctr: tuple of four uint64 arrays holding 32-bit counter words.
    key: tuple of two uint64 arrays (or scalars) holding 32-bit key words.
    Returns four uint64 arrays holding the 32-bit output words.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    k0 = np.asarray(key[0], dtype=np.uint64) & _MASK32
    k1 = np.asarray(key[1], dtype=np.uint64) & _MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    w0 = np.uint64(PHILOX_W0)
    w1 = np.uint64(PHILOX_W1)
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            k0 = (k0 + w0) & _MASK32
            k1 = (k1 + w1) & _MASK32
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & _MASK32
        hi1, lo1 = p1 >> s32, p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox_key(seed: int, nk: int, iq: int, ik: int):
    """Key words of the B stream of block (q, k)."""
    k0 = seed & 0xFFFFFFFF
    k1 = ((seed >> 32) + iq * nk + ik) & 0xFFFFFFFF
    return k0, k1


def _uniform_pair(wa, wb):
    x = ((wa >> np.uint64(6)) << np.uint64(26)) | (wb >> np.uint64(6))
    return (x.astype(np.float64) + 0.5) * 2.0 ** -52


def philox_words(seed: int, nk: int, iq: int, ik: int, e0: int, count: int):
    """Raw Philox words for elements e0..e0+count-1 of block (q, k); shape [count, 4]."""
    e = np.arange(e0, e0 + count, dtype=np.uint64)
    k0, k1 = philox_key(seed, nk, iq, ik)
    zero = np.zeros_like(e)
    w = philox4x32_10((e & _MASK32, e >> np.uint64(32), zero, zero),
                      (np.uint64(k0), np.uint64(k1)))
    return np.stack(w, axis=-1).astype(np.uint32)


def philox_normals(seed: int, sigma: float, nk: int, iq: int, ik: int, e0: int, e1: int,
                   is_complex: bool, stream: int = 0):
    """Elements e0 <= e < e1 of the normal stream of block (q, k): CN(0, sigma^2) or
    N(0, sigma^2).  The third counter word selects the stream (0: B, 1: pair-fit C)."""
    e = np.arange(e0, e1, dtype=np.uint64)
    k0, k1 = philox_key(seed, nk, iq, ik)
    zero = np.zeros_like(e)
    third = np.full_like(e, np.uint64(stream))
    w0, w1, w2, w3 = philox4x32_10((e & _MASK32, e >> np.uint64(32), third, zero),
                                   (np.uint64(k0), np.uint64(k1)))
    del e, zero, third
    u1 = _uniform_pair(w0, w1)
    u2 = _uniform_pair(w2, w3)
    del w0, w1, w2, w3
    r = np.sqrt(-2.0 * np.log(u1))
    theta = 2.0 * np.pi * u2
    if is_complex:
        s = sigma / math.sqrt(2.0)
        out = np.empty(r.shape, dtype=np.complex128)
        out.real = s * r * np.cos(theta)
        out.imag = s * r * np.sin(theta)
    else:
        out = sigma * r * np.cos(theta)
    return out


def philox_B_rows(seed: int, sigma: float, nk: int, iq: int, ik: int,
                  nvirt: int, naux: int, is_complex: bool, i0: int, i1: int):
    """B^P_ia(k,q) for occupied rows i0 <= i < i1 of block (q, k).

    Returns an array of shape [i1-i0, nvirt, naux], complex128 or float64.
    """
    per_i = nvirt * naux
    out = philox_normals(seed, sigma, nk, iq, ik, i0 * per_i, i1 * per_i, is_complex, 0)
    return out.reshape(i1 - i0, nvirt, naux)


def philox_C_block(seed: int, sigma: float, nk: int, iq: int, ik: int, nbas: int, naux: int):
    """Pair-fit coefficients C^{mu nu}_gamma(k, q) of block (q, k), complex [nbas, nbas, naux]
    (mu pairs with the band at k, nu with the band at k (+) q): stream 1 of the same
    Philox key, element e = (mu * nbas + nu) * naux + gamma."""
    n = nbas * nbas * naux
    return philox_normals(seed, sigma, nk, iq, ik, 0, n, True, 1).reshape(nbas, nbas, naux)


def philox_B_block(seed, sigma, nk, iq, ik, nocc, nvirt, naux, is_complex):
    """Whole block B[k][i][a][P] of one (q, k) pair."""
    return philox_B_rows(seed, sigma, nk, iq, ik, nvirt, naux, is_complex, 0, nocc)


# ----------------------------------------------------------------------------
# grids, band energies, Coulomb square roots, frequencies


def kgrid(grid):
    """Reduced coordinates [N_k, 3] of a regular grid and the k (+) q map [N_q, N_k]."""
    n1, n2, n3 = grid
    idx = np.array([(a, b, c) for a in range(n1) for b in range(n2) for c in range(n3)],
                   dtype=np.int64)
    dims = np.array([n1, n2, n3], dtype=np.int64)
    kappa = idx / dims
    nk = len(idx)
    kq = np.empty((nk, nk), dtype=np.int32)
    for q in range(nk):
        s = (idx + idx[q]) % dims
        kq[q] = s[:, 0] * n2 * n3 + s[:, 1] * n3 + s[:, 2]
    return kappa, kq


def dual_grids(grid, frac=0.1):
    """Dual k/q grids (Sec. 3.2, enhanced sampling around Gamma).

    K_reg is the regular grid.  Q_G is the regular q-grid without Gamma plus N_add = 2^D
    points sum_i (+-d_i) b_i, D the number of directions with more than one point and
    d_i = frac / N_i (frac = 0.1 is the one-tenth spacing the paper uses).  K_G holds every
    k_j + q with k_j in K_reg and q in Q_G (the travel relation k_j + q = k_i), K_reg first:
    for regular grids that is (N_add + 1) |K_reg| points.

    Returns (kappa_reg [N_k, 3], kappa_q [N_q, 3], kappa_g [N_G, 3], kq [N_q, N_k] rows of
    kappa_g, zeta_q [N_q]).  Weights: 1/N_k for each regular q and 1/(N_k N_add) for each
    displaced one, i.e. Gamma's weight shared evenly among the points that replace it (the
    paper gives no weights; this keeps sum zeta_q = 1).
    """
    n = np.array(grid, dtype=np.int64)
    kappa_reg, _ = kgrid(grid)
    nk = len(kappa_reg)
    dirs = [d for d in range(3) if n[d] > 1]
    if not dirs:
        raise ValueError("a dual grid needs at least one direction with more than one k-point")
    disp = []
    for signs in range(1 << len(dirs)):
        x = np.zeros(3)
        for b, d in enumerate(dirs):
            x[d] = (-1.0 if (signs >> b) & 1 else 1.0) * frac / n[d]
        disp.append(x)
    kappa_q = np.concatenate([kappa_reg[1:], np.array(disp)], axis=0)   # row 0 of kgrid is Gamma
    nadd = len(disp)
    zeta_q = np.concatenate([np.full(nk - 1, 1.0 / nk), np.full(nadd, 1.0 / (nk * nadd))])

    def key(x):
        f = np.mod(x, 1.0)
        f = np.where(np.abs(f - 1.0) < 1e-12, 0.0, f)
        return tuple(np.round(f, 10))

    pts = [np.mod(k, 1.0) for k in kappa_reg]
    index = {key(k): i for i, k in enumerate(pts)}
    kq = np.empty((len(kappa_q), nk), dtype=np.int32)
    for iq, q in enumerate(kappa_q):
        for ik, k in enumerate(kappa_reg):
            t = key(k + q)
            if t not in index:
                index[t] = len(pts)
                pts.append(np.array(t))
            kq[iq, ik] = index[t]
    return kappa_reg, kappa_q, np.array(pts), kq, zeta_q


def qnorm2(kappa):
    """|q|^2 with the reduced coordinates folded into [-1/2, 1/2) (lattice constant 1)."""
    f = (kappa + 0.5) % 1.0 - 0.5
    return (2.0 * np.pi) ** 2 * np.sum(f * f, axis=-1)


def haar_unitary(rng, n, is_complex):
    """Haar-distributed orthogonal / unitary matrix (Mezzadri's QR recipe)."""
    if is_complex:
        z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    else:
        z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    ph = d / np.abs(d)
    return q * ph[None, :]


def coulomb_sqrt(rng, naux, kappa, is_complex, periodic):
    """V^(1/2)(q) for every q of the grid: [N_q, naux, naux]."""
    nq = len(kappa)
    if periodic:
        q2 = qnorm2(kappa)
        nz = q2[q2 > 0]
        q2min = nz.min() if len(nz) else 1.0
        q2 = np.where(q2 > 0, q2, q2min)
        f = 1.0 + 1.0 / q2
    else:
        f = np.ones(nq)
    dt = np.complex128 if is_complex else np.float64
    out = np.empty((nq, naux, naux), dtype=dt)
    for iq in range(nq):
        Q = haar_unitary(rng, naux, is_complex)
        lam = 10.0 ** rng.uniform(-2.0, 1.0, size=naux) * f[iq]
        vh = (Q * np.sqrt(lam)[None, :]) @ Q.conj().T
        out[iq] = 0.5 * (vh + vh.conj().T)
    return out


def frequency_grid(nw):
    """Gauss-Legendre nodes on [0,1] mapped to omega = x/(1-x); weights include d omega/dx."""
    t, g = np.polynomial.legendre.leggauss(nw)
    x = 0.5 * (1.0 + t)
    omega = x / (1.0 - x)
    weight = 0.5 * g / (1.0 - x) ** 2
    return omega.astype(np.float64), weight.astype(np.float64)


@dataclasses.dataclass
class System:
    """One synthetic periodic system plus its frequency grid."""
    name: str
    grid: tuple
    nk: int
    nq: int
    nocc: int
    nvirt: int
    naux: int
    is_complex: bool
    kq: np.ndarray          # int32 [nq][nk], rows of eps_occ
    eps_occ: np.ndarray     # f64 [nk_occ][nocc] (nk_occ = nk on regular grids)
    eps_virt: np.ndarray    # f64 [nk][nvirt]
    zeta_k: np.ndarray      # f64 [nk]
    zeta_q: np.ndarray      # f64 [nq]
    vhalf: np.ndarray       # [nq][naux][naux]
    omega: np.ndarray       # f64 [nw]
    weight: np.ndarray      # f64 [nw]
    seed: int
    sigma: float
    B: Optional[np.ndarray] = None   # explicit [nq][nk][nocc][nvirt][naux] or None (Philox)
    # atomic-orbital data (nbas > 0): B is then the MO transform of Philox pair-fit
    # coefficients C(k, q) with the projected KS coefficients (see make_ao_system)
    nbas: int = 0
    c_occ: Optional[np.ndarray] = None    # projected, [nk_occ][nbas][nocc] (at every k (+) q)
    c_virt: Optional[np.ndarray] = None   # projected, [nk][nbas][nvirt]
    S_ao: Optional[np.ndarray] = None     # overlap S(k), [nk][nbas][nbas]
    c_raw: Optional[np.ndarray] = None    # KS coefficients before the projector, [nk][nbas][nocc+nvirt]
    eps_d: float = 0.0                    # projector threshold on the eigenvalues of S(k)

    @property
    def nw(self):
        return len(self.omega)

    @property
    def nk_occ(self):
        return int(self.eps_occ.shape[0])

    @property
    def M(self):
        return self.nk * self.nocc * self.nvirt

    def B_rows(self, iq, ik, i0, i1):
        """B[q][k][i0:i1] from the explicit array or the Philox stream."""
        if self.nbas > 0:
            raise ValueError("the B of an atomic-orbital system is the MO transform of its pair-fit "
                             "coefficients; it is not an input")
        if self.B is not None:
            return self.B[iq, ik, i0:i1]
        return philox_B_rows(self.seed, self.sigma, self.nk, iq, ik, self.nvirt,
                             self.naux, self.is_complex, i0, i1)

    def B_block(self, iq, ik):
        return self.B_rows(iq, ik, 0, self.nocc)

    def C_block(self, iq, ik):
        """Pair-fit coefficients C^{mu nu}_gamma(k, q) of an atomic-orbital system."""
        return philox_C_block(self.seed, self.sigma, self.nk, iq, ik, self.nbas, self.naux)

    def materialize_B(self):
        """Attach the explicit B array (small systems only)."""
        dt = np.complex128 if self.is_complex else np.float64
        B = np.empty((self.nq, self.nk, self.nocc, self.nvirt, self.naux), dtype=dt)
        for iq in range(self.nq):
            for ik in range(self.nk):
                B[iq, ik] = philox_B_block(self.seed, self.sigma, self.nk, iq, ik,
                                           self.nocc, self.nvirt, self.naux, self.is_complex)
        self.B = B
        return self


def make_system(name, grid, nocc, nvirt, naux, nw, seed, is_complex=True, sigma=None,
                periodic=None, vhalf_seed=None):
    """Build a seeded synthetic system.

    sigma defaults to sqrt(1.61/(nocc*nvirt)), which keeps sigma^2*nocc*nvirt at the value
    of the 3x3x1, N_aux = 384 system (0.03^2 * 16 * 112) for every size.
    """
    kappa, kq = kgrid(grid)
    nk = len(kappa)
    if periodic is None:
        periodic = nk > 1
    if sigma is None:
        sigma = math.sqrt(1.61 / (nocc * nvirt))
    rng = np.random.default_rng(seed)
    e0_occ = rng.uniform(-1.0, -0.3, size=nocc)
    e0_virt = rng.uniform(0.05, 3.0, size=nvirt)
    if periodic:
        disp = 0.1 * np.cos(2.0 * np.pi * kappa.sum(axis=1))
    else:
        disp = np.zeros(nk)
    eps_occ = e0_occ[None, :] + disp[:, None]
    eps_virt = e0_virt[None, :] + disp[:, None]
    vrng = np.random.default_rng(seed + 7919 if vhalf_seed is None else vhalf_seed)
    vhalf = coulomb_sqrt(vrng, naux, kappa, is_complex, periodic)
    omega, weight = frequency_grid(nw)
    return System(name=name, grid=tuple(grid), nk=nk, nq=nk, nocc=nocc, nvirt=nvirt,
                  naux=naux, is_complex=bool(is_complex), kq=kq,
                  eps_occ=np.ascontiguousarray(eps_occ), eps_virt=np.ascontiguousarray(eps_virt),
                  zeta_k=np.full(nk, 1.0 / nk), zeta_q=np.full(nk, 1.0 / nk),
                  vhalf=vhalf, omega=omega, weight=weight, seed=int(seed), sigma=float(sigma))


def make_ao_system(name, grid, nbas, nocc, nvirt, naux, nw, seed, n_lowdep=4, eps_d=1e-4, sigma=None):
    """A seeded synthetic system given in an atomic-orbital basis.

    Per k: an overlap S(k) = U diag(d) U^H (U Haar unitary) whose n_lowdep lowest
    eigenvalues are 10^U[-8,-6] (near-linear dependencies, below eps_d) and the rest
    U[0.5, 2]; KS coefficients c = U_keep d_keep^(-1/2) Q (Q Haar, so c^H S c = 1 on the
    retained subspace) for the nocc + nvirt bands, handed over with a contamination along
    the dropped directions (c_raw = c + U_low N, N ~ 0.1 N(0,1)).  The projector of the
    paper's periodic projector method removes exactly that contamination, so the projected
    coefficients are c itself; they are stored as c_occ and c_virt.  Band energies follow
    make_system's recipe; the pair-fit coefficients are Philox stream 1 (philox_C_block).
    """
    kappa, kq = kgrid(grid)
    nk = len(kappa)
    nkeep = nbas - n_lowdep
    nband = nocc + nvirt
    if nkeep < nband:
        raise ValueError("nbas - n_lowdep must be at least nocc + nvirt")
    if sigma is None:
        sigma = math.sqrt(1.61 / (nocc * nvirt))
    rng = np.random.default_rng(seed)
    e0_occ = rng.uniform(-1.0, -0.3, size=nocc)
    e0_virt = rng.uniform(0.05, 3.0, size=nvirt)
    disp = 0.1 * np.cos(2.0 * np.pi * kappa.sum(axis=1)) if nk > 1 else np.zeros(nk)
    eps_occ = e0_occ[None, :] + disp[:, None]
    eps_virt = e0_virt[None, :] + disp[:, None]
    arng = np.random.default_rng(seed + 104729)
    S = np.empty((nk, nbas, nbas), dtype=np.complex128)
    c_clean = np.empty((nk, nbas, nband), dtype=np.complex128)
    c_raw = np.empty_like(c_clean)
    for ik in range(nk):
        U = haar_unitary(arng, nbas, True)
        d = np.concatenate([np.sort(10.0 ** arng.uniform(-8.0, -6.0, size=n_lowdep)),
                            np.sort(arng.uniform(0.5, 2.0, size=nkeep))])
        Sk = (U * d[None, :]) @ U.conj().T
        S[ik] = 0.5 * (Sk + Sk.conj().T)
        Q = haar_unitary(arng, nkeep, True)[:, :nband]
        c = (U[:, n_lowdep:] * (1.0 / np.sqrt(d[n_lowdep:]))[None, :]) @ Q
        noise = 0.1 * (arng.standard_normal((n_lowdep, nband)) + 1j * arng.standard_normal((n_lowdep, nband)))
        c_clean[ik] = c
        c_raw[ik] = c + U[:, :n_lowdep] @ noise
    vrng = np.random.default_rng(seed + 7919)
    vhalf = coulomb_sqrt(vrng, naux, kappa, True, nk > 1)
    omega, weight = frequency_grid(nw)
    return System(name=name, grid=tuple(grid), nk=nk, nq=nk, nocc=nocc, nvirt=nvirt,
                  naux=naux, is_complex=True, kq=kq,
                  eps_occ=np.ascontiguousarray(eps_occ), eps_virt=np.ascontiguousarray(eps_virt),
                  zeta_k=np.full(nk, 1.0 / nk), zeta_q=np.full(nk, 1.0 / nk),
                  vhalf=vhalf, omega=omega, weight=weight, seed=int(seed), sigma=float(sigma),
                  nbas=int(nbas), c_occ=np.ascontiguousarray(c_clean[:, :, :nocc]),
                  c_virt=np.ascontiguousarray(c_clean[:, :, nocc:]), S_ao=S, c_raw=c_raw,
                  eps_d=float(eps_d))


def make_dual_system(name, grid, nocc, nvirt, naux, nw, seed, frac=0.1, is_complex=True, sigma=None,
                     vhalf_seed=None):
    """A seeded synthetic system on the dual grids of dual_grids(grid, frac).

    Band energies follow make_system's recipe (the dispersion evaluated at K_G for the
    occupied bands, at K_reg for the virtual ones), V^(1/2)(q) is drawn for every q of
    Q_G with f(q) = 1 + 1/|q|^2 (no Gamma head: Gamma is not in Q_G), and B^P_ia(k,q)
    comes from the same Philox stream keyed by the Q_G index q and the K_reg index k.
    """
    kappa_reg, kappa_q, kappa_g, kq, zeta_q = dual_grids(grid, frac)
    nk, nq = len(kappa_reg), len(kappa_q)
    if sigma is None:
        sigma = math.sqrt(1.61 / (nocc * nvirt))
    rng = np.random.default_rng(seed)
    e0_occ = rng.uniform(-1.0, -0.3, size=nocc)
    e0_virt = rng.uniform(0.05, 3.0, size=nvirt)
    eps_occ = e0_occ[None, :] + 0.1 * np.cos(2.0 * np.pi * kappa_g.sum(axis=1))[:, None]
    eps_virt = e0_virt[None, :] + 0.1 * np.cos(2.0 * np.pi * kappa_reg.sum(axis=1))[:, None]
    vrng = np.random.default_rng(seed + 7919 if vhalf_seed is None else vhalf_seed)
    vhalf = coulomb_sqrt(vrng, naux, kappa_q, is_complex, True)
    omega, weight = frequency_grid(nw)
    return System(name=name, grid=tuple(grid), nk=nk, nq=nq, nocc=nocc, nvirt=nvirt,
                  naux=naux, is_complex=bool(is_complex), kq=kq,
                  eps_occ=np.ascontiguousarray(eps_occ), eps_virt=np.ascontiguousarray(eps_virt),
                  zeta_k=np.full(nk, 1.0 / nk), zeta_q=zeta_q,
                  vhalf=vhalf, omega=omega, weight=weight, seed=int(seed), sigma=float(sigma))


# The five workloads of the benchmark plan, by what they are.
def gamma_real_128(seed=1234):
    """Gamma-only real system: N_occ 8, N_virt 56, N_aux 128, 8 frequencies, B ~ N(0, 0.05^2)."""
    return make_system("gamma_real_naux128", (1, 1, 1), 8, 56, 128, 8, seed,
                       is_complex=False, sigma=0.05, periodic=False)


def slab_3x3_384(seed=2025):
    """3x3x1 slab, N_occ 16, N_virt 112, N_aux 384, 12 frequencies, B ~ CN(0, 0.03^2)."""
    return make_system("slab3x3_naux384", (3, 3, 1), 16, 112, 384, 12, seed,
                       is_complex=True, sigma=0.03)


def slab_6x6_1200(seed=4242):
    """6x6x1 slab, N_occ 48, N_virt 400, N_aux 1200, 16 frequencies (B streamed)."""
    return make_system("slab6x6_naux1200", (6, 6, 1), 48, 400, 1200, 16, seed)


def slab_3x3_2400(seed=9001):
    """3x3x1 slab, N_occ 96, N_virt 900, N_aux 2400, 16 frequencies (B streamed)."""
    return make_system("slab3x3_naux2400", (3, 3, 1), 96, 900, 2400, 16, seed)


def slab_3x3_dual_384(seed=3031):
    """The 3x3x1 N_aux 384 slab on dual grids (Gamma replaced by 4 points at 1/10 of the
    grid step): 12 q-points, 45 k-points for the occupied bands, 12 frequencies."""
    return make_dual_system("slab3x3_dual_naux384", (3, 3, 1), 16, 112, 384, 12, seed, frac=0.1,
                            is_complex=True, sigma=0.03)


def slab_3x3_ao_384(seed=5050):
    """The 3x3x1 N_aux 384 slab given in an atomic-orbital basis of 144 functions (4 of them
    near-linearly dependent): B is built on the fly from Philox pair-fit coefficients."""
    return make_ao_system("slab3x3_ao_naux384", (3, 3, 1), 144, 16, 112, 384, 12, seed, n_lowdep=4,
                          eps_d=1e-4, sigma=0.03)


def serving_jobs(njobs=256, rate=4.0, seed=77, naux_range=(200, 1500)):
    """Job stream of the serving workload: Poisson arrivals, log-uniform N_aux.

    Returns a list of dicts with arrival time (s) and the job's sizes and seed;
    call make_job_system(job) to build its inputs.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    grids = [(1, 1, 1), (2, 2, 1), (3, 3, 1)]
    for j in range(njobs):
        t += rng.exponential(1.0 / rate)
        naux = int(round(math.exp(rng.uniform(math.log(naux_range[0]), math.log(naux_range[1])))))
        g = grids[int(rng.integers(0, 3))]
        nw = int(rng.integers(8, 17))
        jobs.append(dict(id=j, arrival=t, naux=naux, nocc=max(1, round(naux / 12)),
                         nvirt=max(1, round(naux / 1.5)), grid=g, nw=nw,
                         seed=int(rng.integers(1, 2 ** 31))))
    return jobs


def make_job_system(job):
    return make_system(f"job{job['id']}", job["grid"], job["nocc"], job["nvirt"], job["naux"],
                       job["nw"], job["seed"], is_complex=True)
