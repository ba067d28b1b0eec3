"""Convenience set-up of one plane-wave problem on a Context (marshalling only)."""
from __future__ import annotations

import numpy as np

from ._binding import Context, PW_PREC_FP64


class PlaneWaveProblem:
    """Basis, potential, projectors and workspace of one cell at one k-point.

    `cell`: 3x3 rows = lattice vectors (bohr); `kfrac`: reduced k; `ecut`: Ha;
    `n`: cubic FFT size; `vgrid`: V(r) on the n^3 grid (Ha, C order);
    `pos`/`lm`/`D`: Kleinman-Bylander projector data (optional).
    """

    def __init__(self, cell, kfrac, ecut, n, vgrid, pos=None, lm=(), D=None, nbands=1,
                 block=1, device=0, stream=None, prec=PW_PREC_FP64):
        import torch
        self.torch = torch
        self.ctx = Context(device, stream)
        self.npw = self.ctx.init_basis(cell, kfrac, ecut, (n, n, n))
        self.ctx.set_local_potential(np.asarray(vgrid, np.float64))
        if pos is not None and len(lm):
            self.ctx.set_projectors(pos, lm, D)
        self.nbands, self.block = nbands, min(block, nbands)
        self.prec = prec
        self.ws = self.ctx.alloc_workspace(nbands, self.block, prec)
        self.device = device

    @classmethod
    def from_workload(cls, w, device=0, stream=None, nbands=None, block=None, prec=PW_PREC_FP64):
        return cls(w.cell, w.kfrac, w.ecut, w.n, w.vgrid, w.pos if w.lm else None, w.lm, w.D,
                   nbands=w.nbands if nbands is None else nbands,
                   block=w.block if block is None else block, device=device, stream=stream,
                   prec=prec)

    def empty_block(self, nb):
        return self.torch.zeros((nb, self.npw), dtype=self.torch.complex128,
                                device=f"cuda:{self.device}")

    def apply_H(self, X):
        Y = self.torch.empty_like(X)
        self.ctx.apply_H(X, Y)
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
