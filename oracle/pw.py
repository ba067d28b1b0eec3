"""Dense plane-wave Hamiltonian, written out from its definition.

Sec. 2.1 expands each wave-function over plane waves e^{i(k+G).r} and projects
the Kohn-Sham operator onto them; with a norm-conserving (identity) overlap the
projected problem is H c = eps c with

    H_ij = 1/2 |k+G_i|^2 delta_ij                                  (kinetic)
         + Vt(n_i - n_j)                                           (local, v_loc)
         + sum_{a,p} D_ap beta_ap(k+G_i) conj(beta_ap(k+G_j))      (non-local, v_nl)

where G = b-vectors times integer Miller indices n, Vt is the discrete Fourier
coefficient of the local potential sampled on the FFT grid,

    Vt(m) = N^-3 sum_j V(r_j) exp(-2 pi i m.j / N),

and beta are separable Kleinman-Bylander projectors
beta_{a,lm}(q) = Omega^-1/2 c exp(-|q|^2/2) Y_lm(q^) exp(-i q.R_a) with
c = (32 pi^(5/2))^(1/2) (so that sum_G |beta|^2 -> 1 in the continuum limit).

Everything is float64 / complex128 and written for clarity, not speed.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

C_KB = np.sqrt(32.0 * np.pi ** 2.5)   # projector normalisation constant


def reciprocal(cell: np.ndarray) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij (a_i = rows of `cell`)."""
    return 2.0 * np.pi * np.linalg.inv(cell).T


def sphere(cell, kfrac, ecut):
    """Miller indices n with 1/2 |b(n + k)|^2 <= ecut (inclusive, FP64).

    Sec. 2.1 (plane-wave expansion).  Returns int64 [npw, 3] in lexicographic
    (n_x, n_y, n_z) order.  The box bound per axis follows from
    |n_i + k_i| = |a_i . q| / 2pi <= |a_i| sqrt(2 ecut) / 2pi.
    """
    cell = np.asarray(cell, float)
    kfrac = np.asarray(kfrac, float)
    B = reciprocal(cell)
    qmax = np.sqrt(2.0 * ecut)
    lim = [int(np.ceil(np.linalg.norm(cell[i]) * qmax / (2 * np.pi)
                       + abs(kfrac[i]))) + 1 for i in range(3)]
    r = [np.arange(-lim[i], lim[i] + 1) for i in range(3)]
    n = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    q = (n + kfrac) @ B
    keep = 0.5 * np.einsum("ij,ij->i", q, q) <= ecut
    return n[keep].astype(np.int64)


def kvectors(cell, kfrac, miller):
    """q = k + G for each Miller index (bohr^-1), [npw, 3]."""
    return (np.asarray(miller, float) + np.asarray(kfrac, float)) @ reciprocal(cell)


def kinetic(cell, kfrac, miller):
    """Kinetic diagonal 1/2 |k+G|^2 (Ha)."""
    q = kvectors(cell, kfrac, miller)
    return 0.5 * np.einsum("ij,ij->i", q, q)


def vtilde_table(vgrid, mrange):
    """Vt(m) for every m in mrange^3, by the DFT definition.

    Vt(m) = N^-3 sum_j V_j exp(-2 pi i m.j/N), evaluated as three successive
    one-axis DFT-matrix contractions (the definition written axis by axis; no
    FFT).  `mrange` = (lo, hi) inclusive signed range per axis.  Returns the
    table indexed [m_x - lo, m_y - lo, m_z - lo].
    """
    v = np.asarray(vgrid, float)
    n0, n1, n2 = v.shape
    lo, hi = mrange
    m = np.arange(lo, hi + 1)
    F = [np.exp(-2j * np.pi * np.outer(m, np.arange(nn)) / nn) for nn in (n0, n1, n2)]
    t = np.tensordot(F[0], v, axes=([1], [0]))            # [mx, j1, j2]
    t = np.tensordot(t, F[1], axes=([1], [1]))            # [mx, j2, my]
    t = np.tensordot(t, F[2], axes=([1], [1]))            # [mx, my, mz]
    return t / (n0 * n1 * n2)


def real_ylm(l, m, q):
    """Real spherical harmonics for l = 0, 1 evaluated at directions of q.

    Y00 = 1/(2 sqrt(pi)); (Y1,-1, Y1,0, Y1,1) = sqrt(3/4pi) (y, z, x)/|q|.
    At q = 0 the l = 1 harmonics are defined as 0.
    """
    q = np.asarray(q, float)
    if l == 0:
        return np.full(q.shape[0], 0.5 / np.sqrt(np.pi))
    if l != 1:
        raise ValueError("only l = 0, 1")
    qn = np.linalg.norm(q, axis=1)
    comp = {-1: 1, 0: 2, 1: 0}[m]
    out = np.zeros(q.shape[0])
    nz = qn > 0
    out[nz] = np.sqrt(3.0 / (4.0 * np.pi)) * q[nz, comp] / qn[nz]
    return out


def projectors(cell, kfrac, miller, pos, lm):
    """Projector matrix B[g, a*len(lm) + p] = beta_{a,p}(k+G_g).

    Sec. 2.2 (iv) / sec. 4.3: the non-local part of the potential acts in
    reciprocal space through separable projectors.
    """
    cell = np.asarray(cell, float)
    omega = abs(np.linalg.det(cell))
    q = kvectors(cell, kfrac, miller)
    radial = C_KB / np.sqrt(omega) * np.exp(-0.5 * np.einsum("ij,ij->i", q, q))
    cols = []
    for a in range(np.asarray(pos).shape[0]):
        phase = np.exp(-1j * (q @ np.asarray(pos[a], float)))
        for (l, mm) in lm:
            cols.append(radial * real_ylm(l, mm, q) * phase)
    if not cols:
        return np.zeros((q.shape[0], 0), complex)
    return np.stack(cols, axis=1)


def dense_hamiltonian(cell, kfrac, miller, vgrid, pos=None, lm=(), D=None):
    """Dense Galerkin matrix H_ij of sec. 2.1 (identity overlap), complex128.

    Kinetic + local (Vt of the same grid the device receives, indexed by the
    Miller-index difference) + non-local sum_p D_p beta_p beta_p^H.  Built
    Hermitian by construction: the local block uses Vt(n_i - n_j), and
    Vt(-m) = conj(Vt(m)) holds exactly for the real table entries used.
    """
    miller = np.asarray(miller, np.int64)
    npw = miller.shape[0]
    span = int(np.abs(miller).max()) if npw else 0
    table = vtilde_table(vgrid, (-2 * span, 2 * span))
    d = miller[:, None, :] - miller[None, :, :] + 2 * span
    H = table[d[..., 0], d[..., 1], d[..., 2]]
    # exact Hermitian symmetrisation (the two triangles differ only by rounding
    # of the DFT sums; use the upper one on both sides)
    H = np.triu(H, 1) + np.triu(H, 1).conj().T + np.diag(np.real(np.diag(H)))
    H = H + np.diag(kinetic(cell, kfrac, miller))
    if lm and pos is not None and len(pos):
        B = projectors(cell, kfrac, miller, pos, lm)
        H = H + (B * np.asarray(D, float)[None, :]) @ B.conj().T
        H = 0.5 * (H + H.conj().T)
    return H


def overlap_dense(B, q):
    """Overlap operator O = I + sum_p q_p beta_p beta_p^H, complex128.

    Sec. 2.1 puts an overlap operator O on the right-hand side of the
    Kohn-Sham equations (H psi = eps O psi) for ultrasoft / PAW projectors and
    gives no formula; the Vanderbilt form I + sum_ij |beta_i> q_ij <beta_j| is
    used with q diagonal in the projector index, over the same projector
    table B as the non-local potential.  q >= 0 makes O >= I (positive
    definite)."""
    B = np.asarray(B, complex)
    O = np.eye(B.shape[0], dtype=complex)
    if B.shape[1]:
        O = O + (B * np.asarray(q, float)[None, :]) @ B.conj().T
        O = 0.5 * (O + O.conj().T)
    return O


def generalized_to_standard(H, O):
    """The pencil (H, O) as one Hermitian matrix with the same eigenvalues:
    O = L L^H (Cholesky), A = L^-1 H L^-H; an eigenvector y of A gives the
    pencil's eigenvector x = L^-H y (x^H O x = y^H y).  Returns (A, L)."""
    L = scipy.linalg.cholesky(O, lower=True)
    Y = scipy.linalg.solve_triangular(L, H, lower=True)
    A = scipy.linalg.solve_triangular(L, Y.conj().T, lower=True).conj().T
    return 0.5 * (A + A.conj().T), L


def density(cell, kfrac, miller, n, C, occ):
    """Electron density on the n^3 grid from the band coefficients (sec. 4.1: the
    density is formed from the bands with the FFT): rho(r_j) = sum_b occ_b
    |psi_b(r_j)|^2, psi_b(r) = Omega^-1/2 sum_G C[G, b] e^{i(k+G).r},
    r_j = cell^T j / n, C order [j0][j1][j2].  The phase e^{ik.r} has unit
    modulus and drops out.  numpy's inverse FFT evaluates the sum over G."""
    cell = np.asarray(cell, dtype=float)
    omega = abs(np.linalg.det(cell))
    idx = np.mod(np.asarray(miller), n)
    rho = np.zeros((n, n, n))
    for b in range(C.shape[1]):
        g = np.zeros((n, n, n), dtype=complex)
        g[idx[:, 0], idx[:, 1], idx[:, 2]] = C[:, b]
        psi = np.fft.ifftn(g) * n ** 3          # sum_G C e^{+2 pi i n.j / n}
        rho += occ[b] * (psi.real ** 2 + psi.imag ** 2)
    return rho / omega
