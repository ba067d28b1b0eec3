"""Convenience set-up of one plane-wave problem on a Context (marshalling only)."""
from __future__ import annotations

import numpy as np

from ._binding import Context, PW_PREC_FP64


class PlaneWaveProblem:
    """Basis, potential, projectors and workspace of one cell at one k-point.

    `cell`: 3x3 rows = lattice vectors (bohr); `kfrac`: reduced k; `ecut`: Ha;
    `n`: cubic FFT size; `vgrid`: V(r) on the n^3 grid (Ha, C order);
    `pos`/`lm`/`D`: Kleinman-Bylander projector data (optional); `q`: overlap
    coefficients per projector (generalized form H psi = eps O psi; optional).
    """

    def __init__(self, cell, kfrac, ecut, n, vgrid, pos=None, lm=(), D=None, nbands=1,
                 block=1, device=0, stream=None, prec=PW_PREC_FP64, q=None):
        import torch
        self.torch = torch
        self.ctx = Context(device, stream)
        self.npw = self.ctx.init_basis(cell, kfrac, ecut, (n, n, n))
        self.ctx.set_local_potential(np.asarray(vgrid, np.float64))
        if pos is not None and len(lm):
            self.ctx.set_projectors(pos, lm, D)
        if q is not None:
            self.ctx.set_overlap(q)
        self.nbands, self.block = nbands, min(block, nbands)
        self.prec = prec
        self.ws = self.ctx.alloc_workspace(nbands, self.block, prec)
        self.device = device

    @classmethod
    def from_workload(cls, w, device=0, stream=None, nbands=None, block=None, prec=PW_PREC_FP64,
                      q=None):
        return cls(w.cell, w.kfrac, w.ecut, w.n, w.vgrid, w.pos if w.lm else None, w.lm, w.D,
                   nbands=w.nbands if nbands is None else nbands,
                   block=w.block if block is None else block, device=device, stream=stream,
                   prec=prec, q=q)

    def empty_block(self, nb):
        return self.torch.zeros((nb, self.npw), dtype=self.torch.complex128,
                                device=f"cuda:{self.device}")

    def apply_H(self, X):
        Y = self.torch.empty_like(X)
        self.ctx.apply_H(X, Y)
        return Y

    def apply_O(self, X):
        Y = self.torch.empty_like(X)
        self.ctx.apply_O(X, Y)
        return Y

    def solve(self, tol, max_iter=300, X=None, allow_not_converged=False, prec=None):
        if X is None:
            X = self.empty_block(self.nbands)
            use_guess = False
        else:
            use_guess = True
        eig, status = self.ctx.lobpcg_solve(self.nbands, self.block, tol, max_iter, X,
                                            use_guess=use_guess,
                                            prec=self.prec if prec is None else prec,
                                            allow_not_converged=allow_not_converged)
        return eig, X, status


def solve_batch(problems, tol, max_iter=300, Xs=None, prec=None, allow_not_converged=False):
    """Concurrent solves of several problems (e.g. the k-points of one cell) through
    pw_lobpcg_solve_batch: one host thread and one stream per problem.

    Every problem must share nbands and block.  Returns (eigs, Xs, statuses)."""
    import ctypes
    from ._binding import PWError, PW_OK, PW_ERR_NOT_CONVERGED, _ptr, _ld
    n = len(problems)
    nb, blk = problems[0].nbands, problems[0].block
    if any(p.nbands != nb or p.block != blk for p in problems):
        raise ValueError("solve_batch needs one (nbands, block) for every problem")
    prec = problems[0].prec if prec is None else prec
    use_guess = Xs is not None
    if Xs is None:
        Xs = [p.empty_block(nb) for p in problems]
    eigs = [np.zeros(nb, np.float64) for _ in problems]
    ctxs = (ctypes.c_void_p * n)(*[p.ctx.h for p in problems])
    xp = (ctypes.c_void_p * n)(*[_ptr(x).value for x in Xs])
    ld = (ctypes.c_int64 * n)(*[_ld(x) for x in Xs])
    ep = (ctypes.c_void_p * n)(*[e.ctypes.data for e in eigs])
    st = (ctypes.c_int * n)()
    lib = problems[0].ctx.lib
    rc = lib.pw_lobpcg_solve_batch(ctxs, n, nb, blk, float(tol), max_iter, prec, xp, ld,
                                   int(use_guess), ep, st)
    statuses = list(st)
    if rc != PW_OK and not (allow_not_converged and rc == PW_ERR_NOT_CONVERGED):
        bad = next(i for i, s in enumerate(statuses) if s != PW_OK)
        raise PWError(rc, f"problem {bad}: " + lib.pw_last_error(problems[bad].ctx.h).decode())
    return eigs, Xs, statuses
