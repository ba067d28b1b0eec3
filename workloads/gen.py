"""Synthetic Gaussian-well cells (seeded, numpy PCG64).

Every workload is a cubic cell of side L (bohr) holding Gaussian wells of depth
2 Ha and width 1 bohr, periodically repeated:

    V(r) = sum_a  -2 exp(-|r - R_a - T|^2 / 2),  T in L Z^3,

sampled on the FFT grid r_j = L j / N (C order [x][y][z]).  The image sum is
separable: each well contributes -2 g_x (x) g_y (x) g_z with
g(x) = sum_{t=-3..3} exp(-(x - X_a - tL)^2 / 2); images farther than 3L are
below 1e-40 of the peak for L >= 8 and are dropped.

Kleinman-Bylander projector data (positions, (l, m) list, couplings D) is also
drawn here; how a projector acts is the method's business and lives elsewhere.

Random draws follow one fixed order per workload: positions (uniform, or fcc
sites), fcc jitter, couplings D.  Starting blocks come from their own stream
(`start_block`).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

# (l, m) of the four projectors per atom: one s and three real p harmonics.
LM4 = ((0, 0), (1, -1), (1, 0), (1, 1))


@dataclass
class Workload:
    name: str
    seed: int
    L: float                 # cubic cell side, bohr
    ecut: float              # plane-wave cutoff, Ha
    n: int                   # FFT grid points per axis
    kfrac: tuple             # k in units of 2*pi/L
    pos: np.ndarray          # [natom, 3] well centres, bohr
    nbands: int              # M
    block: int               # m
    tol: float               # residual tolerance
    lm: tuple = ()           # projector (l, m) list per atom (empty: local only)
    D: np.ndarray | None = None   # [natom * len(lm)] couplings, Ha
    vgrid: np.ndarray = field(default=None, repr=False)   # [n, n, n] float64

    @property
    def cell(self) -> np.ndarray:
        return np.eye(3) * self.L

    @property
    def natom(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nproj(self) -> int:
        return self.natom * len(self.lm)


def well_potential(L: float, n: int, pos: np.ndarray, depth: float = 2.0,
                   images: int = 3) -> np.ndarray:
    """Periodic sum of Gaussian wells sampled on the n^3 grid, C order [x][y][z]."""
    x = L * np.arange(n) / n
    t = np.arange(-images, images + 1) * L
    v = np.zeros((n, n, n))
    for a in range(pos.shape[0]):
        g = []
        for ax in range(3):
            d = x[:, None] - pos[a, ax] - t[None, :]
            g.append(np.exp(-0.5 * d * d).sum(axis=1))
        v -= depth * np.einsum("i,j,k->ijk", g[0], g[1], g[2])
    return v


def _fcc_sites(L: float, reps: int) -> np.ndarray:
    a = L / reps
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    sites = []
    for i in range(reps):
        for j in range(reps):
            for k in range(reps):
                for b in basis:
                    sites.append(a * (np.array([i, j, k]) + b))
    return np.array(sites)


def make_workload(name: str) -> Workload:
    spec = WORKLOADS[name]
    rng = np.random.default_rng(spec["seed"])
    L = spec["L"]
    if spec.get("fcc"):
        pos = _fcc_sites(L, spec["fcc"])
        pos = pos + rng.uniform(-0.2, 0.2, pos.shape)
        pos = np.mod(pos, L)
    else:
        pos = rng.uniform(0.0, L, (spec["natom"], 3))
    lm = LM4 if spec.get("proj") else ()
    D = rng.uniform(0.5, 1.5, pos.shape[0] * len(lm)) if lm else None
    w = Workload(name=name, seed=spec["seed"], L=L, ecut=spec["ecut"],
                 n=spec["n"], kfrac=tuple(spec["k"]), pos=pos,
                 nbands=spec["M"], block=spec["m"], tol=spec["tol"],
                 lm=lm, D=D)
    w.vgrid = well_potential(L, w.n, pos)
    return w


KPTS_4X4X4_IRREDUCIBLE = ((0, 0, 0), (0, 0, .25), (0, 0, .5), (0, .25, .25), (0, .25, .5),
                          (0, .5, .5), (.25, .25, .25), (.25, .25, .5), (.25, .5, .5), (.5, .5, .5))


def make_kpoint_workloads(name: str = "kpts_l16", kpts=KPTS_4X4X4_IRREDUCIBLE) -> list:
    """One workload per k-point, all sharing the cell, wells, projectors and V(r)."""
    base = make_workload(name)
    out = []
    for k in kpts:
        w = Workload(name=f"{name}@{k}", seed=base.seed, L=base.L, ecut=base.ecut, n=base.n,
                     kfrac=tuple(float(x) for x in k), pos=base.pos, nbands=base.nbands,
                     block=base.block, tol=base.tol, lm=base.lm, D=base.D)
        w.vgrid = base.vgrid
        out.append(w)
    return out


# grid sizes a served request may use (products of 2, 3, 5 with both factors of
# a two-factor split <= 16)
SERVE_FFT_SIZES = (16, 20, 24, 32, 36, 40, 48, 60, 64, 72, 80, 96, 108, 120, 128)


def make_request(i: int, base_seed: int = 1000, L_range=(8.0, 24.0), ecut_range=(5.0, 25.0)):
    """Request i of a served stream: a cubic cell with L ~ U(L_range), Ecut ~ U(ecut_range),
    round(0.0135 L^3) Gaussian wells at uniform positions with 4 projectors each,
    k ~ U[0,1)^3, nbands = 32 round(5.5 natom / 32) clamped to [32, 1024], block
    min(64, nbands), tol 1e-6, and a precision flag (mixed with probability 1/2).
    The grid is the smallest listed size >= 4 nmax + 1 with nmax = ceil(L sqrt(2 Ecut) / 2 pi + 1)
    (products of two bands are then resolved without wrap-around).
    Returns (Workload, mixed)."""
    rng = np.random.default_rng(base_seed + i)
    L = float(rng.uniform(*L_range))
    ecut = float(rng.uniform(*ecut_range))
    natom = max(1, int(round(0.0135 * L ** 3)))
    kfrac = tuple(float(x) for x in rng.uniform(0.0, 1.0, 3))
    mixed = bool(rng.uniform() < 0.5)
    pos = rng.uniform(0.0, L, (natom, 3))
    D = rng.uniform(0.5, 1.5, natom * len(LM4))
    nbands = int(min(1024, max(32, 32 * round(5.5 * natom / 32))))
    nmax = int(np.ceil(L * np.sqrt(2.0 * ecut) / (2 * np.pi) + 1.0))
    n = next(s for s in SERVE_FFT_SIZES if s >= 4 * nmax + 1)
    w = Workload(name=f"request{i}", seed=base_seed + i, L=L, ecut=ecut, n=n, kfrac=kfrac,
                 pos=pos, nbands=nbands, block=min(64, nbands), tol=1e-6, lm=LM4, D=D)
    w.vgrid = well_potential(L, n, pos)
    return w, mixed


def overlap_coefficients(w: Workload, lo: float = 0.2, hi: float = 0.8) -> np.ndarray:
    """Overlap coefficients q_p ~ U(lo, hi) per projector of w (the generalized
    form's O = I + sum_p q_p |beta_p><beta_p|), from their own PCG64 stream.
    q >= 0 keeps O positive definite."""
    rng = np.random.default_rng(20_000 + w.seed)
    return rng.uniform(lo, hi, w.nproj)


def start_block(seed: int, npw: int, ncol: int) -> np.ndarray:
    """Complex standard-normal block [npw, ncol] from its own PCG64 stream."""
    rng = np.random.default_rng(10_000 + seed)
    return (rng.standard_normal((npw, ncol))
            + 1j * rng.standard_normal((npw, ncol))) / np.sqrt(2.0)


# Workload table.  `gamma_l10` is the small Gamma-point FP64 case, `fcc108_l20`
# the paper-scale single-k case (108 wells at jittered fcc sites, 432
# projectors, 512 bands in blocks of 64).  The others are test cells.
WORKLOADS = {
    "gamma_l10": dict(seed=0, L=10.0, ecut=5.0, n=24, k=(0, 0, 0), natom=8,
                      M=16, m=16, tol=1e-8),
    "fcc108_l20": dict(seed=1, L=20.0, ecut=20.0, n=96, k=(0.25, 0.25, 0.25),
                       fcc=3, proj=True, M=512, m=64, tol=1e-6),
    "tiny_nl": dict(seed=7, L=8.0, ecut=4.0, n=20, k=(0.1, 0.2, 0.3), natom=2,
                    proj=True, M=12, m=4, tol=1e-8),
    "mid_nl": dict(seed=11, L=12.0, ecut=8.0, n=36, k=(0.25, 0.0, 0.5),
                   natom=6, proj=True, M=48, m=16, tol=1e-7),
    # ten k-points of one cell (the irreducible Gamma-centred 4x4x4 set under
    # cubic symmetry), solved as a batch; `k` is replaced per k-point
    "kpts_l16": dict(seed=3, L=16.0, ecut=15.0, n=72, k=(0, 0, 0), natom=64,
                     proj=True, M=256, m=32, tol=1e-6),
    "fcc32_l12": dict(seed=5, L=12.0, ecut=12.0, n=48, k=(0.25, 0.25, 0.25),
                      fcc=2, proj=True, M=128, m=32, tol=1e-6),
    # the largest request of the served stream (L = 24 bohr, Ecut = 25 Ha,
    # round(0.0135 L^3) = 187 wells with 748 projectors, 1024 bands) on the
    # 120^3 grid the serving rule picks, and on the largest supported grid
    "max_l24": dict(seed=4, L=24.0, ecut=25.0, n=120, k=(0.3, 0.1, 0.7), natom=187,
                    proj=True, M=1024, m=64, tol=1e-6),
    "max_l24_n128": dict(seed=4, L=24.0, ecut=25.0, n=128, k=(0.3, 0.1, 0.7), natom=187,
                         proj=True, M=1024, m=64, tol=1e-6),
}
