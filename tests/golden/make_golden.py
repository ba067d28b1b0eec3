"""Write the stored expected eigenvalues under tests/golden/.

Calls only `oracle/` (and the seeded input generators in `workloads/`):

  gamma_l10   dense H (oracle.pw) diagonalised by the oracle's C Jacobi.
  mid_nl      dense H diagonalised by the oracle's C Jacobi.
  fcc32_l12   oracle.matfree.solve (block LOBPCG + final Rayleigh-Ritz), tol 1e-9.
  fcc108_l20  oracle.matfree.solve, tol 1e-8 (34181 plane waves: no dense H).
  kpts_l16_k0, kpts_l16_k1, kpts_l16_k5, kpts_l16_k9
              oracle.matfree.solve, tol 1e-8, at k-points 0, 1, 5 and 9 of the
              ten-k-point batch cell (workloads.make_kpoint_workloads; k5 has
              the most plane waves, 11416, k9 the fewest, 11296).
  max_l24_lo128
              the lowest 128 bands of the largest served cell (max_l24: 82561
              plane waves, 748 projectors, 120^3 grid): oracle.matfree.solve with
              128 bands in blocks of 64, tol 1e-8.
  request2, request6
              requests 2 (5680 plane waves, 224 bands) and 6 (8049 plane waves,
              192 bands) of the served stream (workloads.make_request, base seed
              1000): oracle.matfree.solve, tol 1e-8.
  mid_nl_ovl  generalized form H c = eps O c on the mid_nl cell with the overlap
              coefficients of workloads.overlap_coefficients: dense H and O
              (oracle.pw), Cholesky reduction, the oracle's C Jacobi.
  fcc32_l12_ovl
              the same overlap on fcc32_l12: oracle.matfree.solve in the
              O-metric, tol 1e-9 (its error bound holds because O >= I makes
              the residual 2-norm an upper bound of its O^-1-norm).

Each file lists index, eigenvalue (Ha) and, for the matrix-free runs, the
residual norm and the residual certificate (oracle.matfree.certificate).

Usage:  python tests/golden/make_golden.py [name ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pw, matfree                      # noqa: E402
from oracle.jacobi import eigh_jacobi              # noqa: E402
from workloads import (make_workload, make_kpoint_workloads, make_request,   # noqa: E402
                       overlap_coefficients)


def dense_case(name):
    w = make_workload(name)
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    ev, _, sweeps = eigh_jacobi(H)
    path = os.path.join(HERE, f"{name}_eig.txt")
    with open(path, "w") as f:
        f.write(f"# {name}: npw={len(mil)}, dense H diagonalised by cyclic Jacobi "
                f"({sweeps} sweeps), all {len(ev)} eigenvalues in Ha\n")
        f.write("# written by tests/golden/make_golden.py (oracle only)\n")
        for i, e in enumerate(ev):
            f.write(f"{i} {e:.17e}\n")
    print("wrote", path)


def dense_pencil_case(base):
    w = make_workload(base)
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    O = pw.overlap_dense(pw.projectors(w.cell, w.kfrac, mil, w.pos, w.lm), overlap_coefficients(w))
    A, _ = pw.generalized_to_standard(H, O)
    ev, _, sweeps = eigh_jacobi(A)
    path = os.path.join(HERE, f"{base}_ovl_eig.txt")
    with open(path, "w") as f:
        f.write(f"# {base}_ovl: npw={len(mil)}, pencil (H, O) with O = I + B diag(q) B^H, "
                f"Cholesky reduction diagonalised by cyclic Jacobi ({sweeps} sweeps), "
                f"all {len(ev)} eigenvalues in Ha\n")
        f.write("# written by tests/golden/make_golden.py (oracle only)\n")
        for i, e in enumerate(np.sort(ev)):
            f.write(f"{i} {e:.17e}\n")
    print("wrote", path)


def matfree_case(name, tol, w=None, overlap=False, nbands=None):
    w = make_workload(name) if w is None else w
    nbands = w.nbands if nbands is None else nbands
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    q = overlap_coefficients(w) if overlap else None
    H = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D, q=q)
    if overlap:
        name = name + "_ovl"
    t0 = time.time()
    r = matfree.solve(H, nbands, w.block, tol=tol, seed=w.seed,
                      log=lambda s: print(name, s, flush=True))
    cert = matfree.certificate(r["eig"], r["res"])
    path = os.path.join(HERE, f"{name}_eig.txt")
    with open(path, "w") as f:
        f.write(f"# {name}: npw={len(mil)}, M={nbands}, m={w.block}, oracle block "
                f"LOBPCG tol={tol:g} + final Rayleigh-Ritz, iterations per block "
                f"{r['iters']}, {time.time() - t0:.0f} s\n")
        f.write("# written by tests/golden/make_golden.py (oracle only)\n")
        f.write("# columns: index, eigenvalue (Ha), residual norm, error bound\n")
        for i, (e, s, c) in enumerate(zip(r["eig"], r["res"], cert)):
            f.write(f"{i} {e:.17e} {s:.3e} {c:.3e}\n")
    print("wrote", path)


CASES = {
    "gamma_l10": lambda: dense_case("gamma_l10"),
    "mid_nl": lambda: dense_case("mid_nl"),
    "fcc32_l12": lambda: matfree_case("fcc32_l12", 1e-9),
    "fcc108_l20": lambda: matfree_case("fcc108_l20", 1e-8),
    "kpts_l16_k0": lambda: matfree_case("kpts_l16_k0", 1e-8, make_kpoint_workloads()[0]),
    "kpts_l16_k1": lambda: matfree_case("kpts_l16_k1", 1e-8, make_kpoint_workloads()[1]),
    "kpts_l16_k5": lambda: matfree_case("kpts_l16_k5", 1e-8, make_kpoint_workloads()[5]),
    "kpts_l16_k9": lambda: matfree_case("kpts_l16_k9", 1e-8, make_kpoint_workloads()[9]),
    "max_l24_lo128": lambda: matfree_case("max_l24_lo128", 1e-8, make_workload("max_l24"), nbands=128),
    "request2": lambda: matfree_case("request2", 1e-8, make_request(2)[0]),
    "request6": lambda: matfree_case("request6", 1e-8, make_request(6)[0]),
    "mid_nl_ovl": lambda: dense_pencil_case("mid_nl"),
    "fcc32_l12_ovl": lambda: matfree_case("fcc32_l12", 1e-9, overlap=True),
}

if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        CASES[n]()
