"""Matrix-free CPU reference: H.X by FFTs and the block LOBPCG of sec. 3.

TEST INFRASTRUCTURE ONLY (oracle).  Plain numpy/scipy, FP64/complex128.

* `MatFreeH.apply` -- the Hamiltonian apply that sec. 2.2 (iii) and sec. 4.1
  describe: place the plane-wave coefficients on the FFT grid (zero padding
  outside the sphere), transform to real space, multiply by the local potential,
  transform back, add the kinetic diagonal, add the non-local projector term in
  reciprocal space.  Full (unpruned) library FFTs; equal to the dense matrix of
  oracle.pw.dense_hamiltonian in exact arithmetic.
* `MatFreeH.apply_O` -- the overlap operator O = I + sum_p q_p |beta_p><beta_p|
  of the generalized form (sec. 2.1; see oracle.pw.overlap_dense), identity
  when no q is given.
* `lobpcg_block` -- block LOBPCG (sec. 3.2) for one block: each iteration
  is a Rayleigh-Ritz projection of the pencil (H, O) onto the span of the
  current Ritz vectors, their preconditioned residuals (K of sec. 3.1) and the
  previous search direction, with the block kept O-orthogonal to the bands of
  earlier blocks.
* `solve` -- the multiband-by-multiband sweep over M/m blocks followed by the
  final Rayleigh-Ritz over all M bands (end of sec. 3.2; the subspace diagonalisation of sec. 2.1).
* `certificate` -- residual-based eigenvalue error bounds for Hermitian H.

The preconditioner K is called "PW optimized" in sec. 3.1 without a formula;
the Teter-Payne-Allan rational function in T_g / E_kin is used.  K changes the
iteration count, never the fixed point.
"""
from __future__ import annotations

import time

import numpy as np
import scipy.fft
import scipy.linalg

from . import pw


class MatFreeH:
    """H = T + V_loc + sum_p D_p |beta_p><beta_p| on one sphere (sec. 2.1, 2.2)."""

    def __init__(self, cell, kfrac, miller, vgrid, pos=None, lm=(), D=None,
                 workers: int = -1, q=None):
        self.miller = np.asarray(miller, np.int64)
        self.vgrid = np.asarray(vgrid, float)
        self.shape = self.vgrid.shape
        self.idx = tuple(np.mod(self.miller[:, a], self.shape[a]) for a in range(3))
        self.T = pw.kinetic(cell, kfrac, self.miller)
        self.npw = self.miller.shape[0]
        self.workers = workers
        if lm and pos is not None and len(pos):
            self.B = pw.projectors(cell, kfrac, self.miller, pos, lm)
            self.D = np.asarray(D, float)
        else:
            self.B = None
            self.D = None
        # overlap coefficients per projector (None: O = I)
        self.q = None if q is None or self.B is None else np.asarray(q, float)
        self.napply = 0

    def apply_local(self, X, chunk: int = 8):
        """Kinetic + local part: T X + FFT^-1[ V . FFT[X on grid] ] restricted to the sphere."""
        X = np.asarray(X, np.complex128)
        Y = self.T[:, None] * X
        N3 = float(np.prod(self.shape))
        for c0 in range(0, X.shape[1], chunk):
            c1 = min(X.shape[1], c0 + chunk)
            grid = np.zeros((c1 - c0,) + self.shape, np.complex128)
            grid[(slice(None),) + self.idx] = X[:, c0:c1].T
            # psi(r_j) = sum_n c(n) exp(+2 pi i n.j / N)   (no normalisation)
            psi = scipy.fft.ifftn(grid, axes=(1, 2, 3), workers=self.workers) * N3
            psi *= self.vgrid[None]
            # (V psi)(n) = N^-3 sum_j (V psi)(r_j) exp(-2 pi i n.j / N)
            out = scipy.fft.fftn(psi, axes=(1, 2, 3), workers=self.workers) / N3
            Y[:, c0:c1] += out[(slice(None),) + self.idx].T
        return Y

    def apply(self, X):
        Y = self.apply_local(X)
        if self.B is not None:
            Y += self.B @ (self.D[:, None] * (self.B.conj().T @ X))
        self.napply += X.shape[1]
        return Y


    def apply_O(self, X):
        """O X = X + B (q . (B^H X)); X itself (no copy) when O = I."""
        X = np.asarray(X, np.complex128)
        if self.q is None:
            return X
        return X + self.B @ (self.q[:, None] * (self.B.conj().T @ X))


def tpa_precondition(T, X, R, ekin_floor: float = 1e-3):
    """W = K(R), K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4), x = T_g/E_kin,n.

    E_kin,n = <x_n| -1/2 Laplacian |x_n> / <x_n|x_n> per band, floored at ekin_floor.
    """
    ekin = np.einsum("g,gn->n", T, np.abs(X) ** 2) / np.einsum("gn->n", np.abs(X) ** 2)
    ekin = np.maximum(ekin, ekin_floor)
    x = T[:, None] / ekin[None, :]
    num = 27 + 18 * x + 12 * x ** 2 + 8 * x ** 3
    return (num / (num + 16 * x ** 4)) * R


def rayleigh_ritz(Z, HZ, nwant: int, drop_rel: float = 1e-14, OZ=None):
    """Rayleigh-Ritz on span(Z): lowest `nwant` Ritz pairs as coefficients C.

    The Gram pair A = Z^H H Z, B = Z^H O Z (O Z given as OZ; Z^H Z without
    it) is reduced through a B-orthonormal basis of span(Z) taken from the
    eigenvectors of B (directions with eigenvalue below drop_rel * max are
    outside the numerically spanned space), then A is diagonalised.  Returns
    (theta[nwant], C[ncol, nwant]) with C^H B C = I.
    """
    A = Z.conj().T @ HZ
    B = Z.conj().T @ (Z if OZ is None else OZ)
    A = 0.5 * (A + A.conj().T)
    B = 0.5 * (B + B.conj().T)
    bv, bu = scipy.linalg.eigh(B)
    keep = bv > drop_rel * bv.max()
    S = bu[:, keep] / np.sqrt(bv[keep])[None, :]
    Ah = S.conj().T @ A @ S
    Ah = 0.5 * (Ah + Ah.conj().T)
    theta, U = scipy.linalg.eigh(Ah)
    return theta[:nwant], S @ U[:, :nwant]


def _orth_against(V, Y, OY=None):
    """V - Y (Y^H O V): the O-orthogonal complement of span(Y), O Y given as OY."""
    if Y is None or Y.shape[1] == 0:
        return V
    return V - Y @ ((Y if OY is None else OY).conj().T @ V)


class _Images:
    """A block V together with H V and O V (kept together through every linear
    combination, so no operator is applied twice to the same vectors)."""

    def __init__(self, V, HV, OV):
        self.V, self.HV, self.OV = V, HV, OV

    @classmethod
    def of(cls, H: MatFreeH, V):
        return cls(V, H.apply(V), H.apply_O(V))

    @classmethod
    def join(cls, parts):
        return cls(*(np.hstack([getattr(p, a) for p in parts]) for a in ("V", "HV", "OV")))

    @property
    def width(self):
        return self.V.shape[1]

    def times(self, C):
        return _Images(self.V @ C, self.HV @ C, self.OV @ C)

    def scaled(self, s):
        return _Images(self.V * s[None, :], self.HV * s[None, :], self.OV * s[None, :])

    def ritz(self, nwant):
        return rayleigh_ritz(self.V, self.HV, nwant, OZ=self.OV)


def lobpcg_block(H: MatFreeH, Psi0, Y=None, tol=1e-8, maxit=300, history=None, nconv=None,
                 OY=None, out=None):
    """Block LOBPCG for one block of m bands (sec. 3.2), O-orthogonal to Y (O Y given as OY).

    The method is a locally optimal three-term recurrence: every iteration
    replaces the block by the lowest m Ritz vectors of the pencil (H, O)
    restricted to a trial space of three parts --
      * the current Ritz vectors x_j,
      * their residuals H x_j - theta_j O x_j (theta_j the Rayleigh quotient,
        Eq. 1) after the preconditioner K (sec. 3.1) and the O-orthogonal
        projection away from the bands of earlier blocks,
      * the previous search direction, i.e. the part of the last update that
        came from outside the old block (a stable basis of span{x^(i-1), x^(i)}).
    Columns are scaled to unit length before the projection (the scale of a
    basis vector does not change the trial space).

    Iterates all m columns of Psi0; stops when the lowest `nconv` (default m)
    residual norms are <= tol.  Returns (eps[m], Psi[npw, m], HPsi, res[m],
    iterations); with `out` (a dict) also out["OPsi"] = O Psi.
    """
    m = Psi0.shape[1]
    nconv = m if nconv is None else nconv
    x = _Images.of(H, _orth_against(np.asarray(Psi0, np.complex128), Y, OY))
    eps, C = x.ritz(m)
    x = x.times(C)
    direction = None
    res = None
    iters = 0
    while True:
        norm2 = np.einsum("gn,gn->n", x.V.conj(), x.OV).real
        eps = np.einsum("gn,gn->n", x.V.conj(), x.HV).real / norm2
        R = x.HV - x.OV * eps[None, :]
        res = np.linalg.norm(R, axis=0) / np.sqrt(norm2)
        if history is not None:
            history.append(eps.copy())
        if np.all(res[:nconv] <= tol) or iters == maxit:
            break
        iters += 1
        S = _orth_against(tpa_precondition(H.T, x.V, R), Y, OY)
        s = _Images.of(H, S / np.linalg.norm(S, axis=0)[None, :])
        parts = [x, s]
        if direction is not None:
            lens = np.linalg.norm(direction.V, axis=0)
            lens[lens == 0] = 1.0
            parts.append(direction.scaled(1.0 / lens))
        trial = _Images.join(parts)
        eps, C = trial.ritz(m)
        # the new block, and the step it took outside span(x)
        outside = _Images.join(parts[1:]).times(C[m:])
        x = _Images(x.V @ C[:m] + outside.V, x.HV @ C[:m] + outside.HV, x.OV @ C[:m] + outside.OV)
        direction = outside
    nrm = np.sqrt(np.einsum("gn,gn->n", x.V.conj(), x.OV).real)
    x = x.scaled(1.0 / nrm)
    if out is not None:
        out["OPsi"] = x.OV
    return eps, x.V, x.HV, res, iters


def guard_count(block: int) -> int:
    """Guard columns per block: iterated but neither required to converge nor kept."""
    return block // 8


def solve(H: MatFreeH, nbands: int, block: int, tol=1e-8, maxit=300, seed=0,
          start=None, final_rr=True, log=None, guard=None):
    """Multiband-by-multiband LOBPCG over the M bands, then a final Rayleigh-Ritz.

    Each block iterates `block` columns; the lowest block - guard of them must
    converge and are kept (the top `guard` columns only shield them from a
    near-degenerate neighbour above the block); the last block keeps the rest.
    `start(b, npw, m)` returns the starting block of block b (default: the
    seeded complex normal blocks of workloads.start_block).  Returns a dict
    with eigenvalues (ascending), vectors, residual norms and per-block
    iteration counts.
    """
    g = guard_count(block) if guard is None else guard
    if start is None:
        from workloads import start_block

        def start(b, npw, m):
            return start_block(seed * 1000 + b, npw, m)
    npw = H.npw
    Xs, HXs, OXs, iters = [], [], [], []
    t0 = time.perf_counter()
    b, ib = 0, 0
    while b < nbands:
        keep = min(block - g, nbands - b)
        width = min(block, keep + g, npw - b)
        Y = np.hstack(Xs) if Xs else None
        OY = np.hstack(OXs) if OXs else None
        extra = {}
        eps, Psi, HPsi, res, it = lobpcg_block(H, start(ib, npw, width), Y,
                                               tol=tol, maxit=maxit, nconv=keep, OY=OY,
                                               out=extra)
        Xs.append(Psi[:, :keep])
        HXs.append(HPsi[:, :keep])
        OXs.append(extra["OPsi"][:, :keep])
        iters.append(it)
        if log:
            log(f"block {ib}: {it} iterations, max res {res[:keep].max():.2e}, "
                f"{time.perf_counter() - t0:.1f}s")
        b += keep
        ib += 1
    X = np.hstack(Xs)
    HX = np.hstack(HXs)
    OX = np.hstack(OXs)
    if final_rr:
        eps, C = rayleigh_ritz(X, HX, nbands, OZ=OX)
        X, HX, OX = X @ C, HX @ C, OX @ C
    nrm2 = np.einsum("gn,gn->n", X.conj(), OX).real
    eps = np.einsum("gn,gn->n", X.conj(), HX).real / nrm2
    order = np.argsort(eps)
    X, HX, OX, eps, nrm2 = X[:, order], HX[:, order], OX[:, order], eps[order], nrm2[order]
    R = HX - OX * eps[None, :]
    res = np.linalg.norm(R, axis=0) / np.sqrt(nrm2)
    return dict(eig=eps, X=X, HX=HX, res=res, iters=iters,
                seconds=time.perf_counter() - t0)


def certificate(theta, res):
    """Per-eigenvalue error bounds for Ritz pairs (theta_j, x_j), ||x_j|| = 1, of a
    Hermitian operator, given the residual norms res_j = ||H x_j - theta_j x_j||.

    * Krylov-Bogolyubov (Weinstein): some eigenvalue lies within res_j of theta_j.
      Always valid.
    * Kato-Temple: if the open interval (a, b) around theta_j holds exactly one
      eigenvalue lambda, then |lambda - theta_j| <= res_j^2 / min(theta_j - a, b - theta_j).
      The interval is bounded by the neighbouring Ritz intervals
      [theta_i - res_i, theta_i + res_i]; that reading takes the computed values to be
      the lowest eigenvalues with none missed between them (what the dense oracle
      checks on the small cells).  Below the lowest value a = -inf.  Above the top
      value nothing computed bounds the next eigenvalue from below, so the top band
      keeps the Krylov-Bogolyubov bound.
    Returns the smaller valid bound per band (input order).
    """
    theta = np.asarray(theta, float)
    res = np.asarray(res, float)
    n = theta.size
    out = res.copy()
    order = np.argsort(theta, kind="stable")
    for pos in range(n - 1):              # the top band (pos = n - 1) keeps res
        j = order[pos]
        above = theta[order[pos + 1]] - res[order[pos + 1]] - theta[j]
        below = np.inf if pos == 0 else theta[j] - (theta[order[pos - 1]] + res[order[pos - 1]])
        delta = min(above, below)
        if delta > 0:
            out[j] = min(out[j], res[j] ** 2 / delta)
    return out
