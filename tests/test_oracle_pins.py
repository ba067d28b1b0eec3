"""Pins of the CPU oracle against facts it does not compute itself.

Each test ties one oracle function to a closed form, an integer brute force,
a lattice-sum table, a textbook special case or a library routine, chosen so
that a dropped term, a sign error, a wrong index or a transposed operand in
the oracle fails at least one of them.
"""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg

from conftest import GOLDEN
from oracle import matfree, pw
from oracle.jacobi import eigh_jacobi
from workloads import make_workload, well_potential, start_block


def _load_r3():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "r3_sum_of_three_squares.txt"))
            if l.strip() and not l.startswith("#")]
    return {int(a): int(b) for a, b in rows}


# ---- plane-wave sphere (sec. 2.1 expansion) ---------------------------------------

def test_sphere_count_integer_brute_force():
    """Gamma, cubic L=10, Ecut=5: |n|^2 <= floor(2 Ecut L^2 / (2pi)^2) = 25 by integer loops."""
    w = make_workload("gamma_l10")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    lim = int(np.floor(2 * w.ecut * w.L ** 2 / (2 * np.pi) ** 2))
    assert lim == 25
    count = sum(1 for a in range(-6, 7) for b in range(-6, 7) for c in range(-6, 7)
                if a * a + b * b + c * c <= lim)
    assert mil.shape[0] == count == 515


def test_sphere_shells_match_sum_of_three_squares():
    """Shell populations at Gamma equal r3(s), the number of representations of s
    as a sum of three squares (table in tests/golden, OEIS A005875)."""
    r3 = _load_r3()
    w = make_workload("gamma_l10")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    s = (mil ** 2).sum(axis=1)
    for k in range(26):
        assert (s == k).sum() == r3[k], k
    # Legendre: s = 4^a (8b + 7) is never a sum of three squares
    assert r3[7] == r3[15] == r3[23] == 0


def test_sphere_paper_scale_counts():
    """Lattice counts recorded independently of this code (survey-time brute force):
    34181 plane waves for L=20, Ecut=20, k=(1/4,1/4,1/4)."""
    w = make_workload("fcc108_l20")
    assert pw.sphere(w.cell, w.kfrac, w.ecut).shape[0] == 34181
    cell = np.eye(3) * 16.0
    kpts = [(0, 0, 0), (0, 0, .25), (0, 0, .5), (0, .25, .25), (0, .25, .5), (0, .5, .5),
            (.25, .25, .25), (.25, .25, .5), (.25, .5, .5), (.5, .5, .5)]
    expect = [11363, 11320, 11380, 11350, 11368, 11416, 11371, 11382, 11348, 11296]
    got = [pw.sphere(cell, k, 15.0).shape[0] for k in kpts]
    assert got == expect


def test_sphere_symmetric_at_gamma_and_inclusive():
    w = make_workload("gamma_l10")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    assert {tuple(x) for x in mil} == {tuple(-x) for x in mil}
    # inclusive boundary: a cutoff exactly at a shell keeps that shell
    b2 = (2 * np.pi / w.L) ** 2
    assert pw.sphere(w.cell, (0, 0, 0), 0.5 * b2 * 2).shape[0] == 1 + 6 + 12


# ---- local potential (DFT of the sampled grid) ----------------------------------------

def test_vtilde_zero_is_closed_form_mean():
    """Vt(0) = mean V = -2 natom (2 pi)^(3/2) / L^3 for unit-width Gaussian wells."""
    w = make_workload("gamma_l10")
    t = pw.vtilde_table(w.vgrid, (0, 0))
    closed = -2 * w.natom * (2 * np.pi) ** 1.5 / w.L ** 3
    assert abs(t[0, 0, 0] - closed) <= 1e-14
    assert abs(closed - (-0.2519938)) < 1e-7


def test_vtilde_matches_continuum_fourier_coefficients():
    """Vt(m) = -2 (2pi)^(3/2)/Omega sum_a exp(-|G|^2/2) exp(-i G.R_a), G = 2 pi m / L
    (aliasing of the sampled Gaussian is below 1e-40 on these grids)."""
    w = make_workload("gamma_l10")
    t = pw.vtilde_table(w.vgrid, (-3, 3))
    for m in [(1, 0, 0), (0, -2, 1), (3, 3, -3), (-1, 2, 0)]:
        G = 2 * np.pi * np.array(m) / w.L
        closed = (-2 * (2 * np.pi) ** 1.5 / w.L ** 3 * np.exp(-0.5 * G @ G)
                  * np.exp(-1j * (w.pos @ G)).sum())
        assert abs(t[m[0] + 3, m[1] + 3, m[2] + 3] - closed) <= 1e-15, m


def test_well_potential_is_image_sum():
    """Separable generator equals the direct periodic image sum at sample points."""
    L, n = 8.0, 10
    pos = np.array([[1.0, 7.5, 3.3], [4.0, 0.2, 6.9]])
    v = well_potential(L, n, pos)
    rng = np.random.default_rng(0)
    for _ in range(5):
        j = rng.integers(0, n, 3)
        r = L * j / n
        direct = 0.0
        for a in range(2):
            for t in np.ndindex(7, 7, 7):
                d = r - pos[a] - L * (np.array(t) - 3)
                direct += -2 * np.exp(-0.5 * d @ d)
        assert abs(v[tuple(j)] - direct) <= 1e-13


# ---- dense Hamiltonian ------------------------------------------------------------------

def _dense(name, **over):
    w = make_workload(name)
    for k, v in over.items():
        setattr(w, k, v)
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    return w, mil, H


def test_dense_hermitian_and_trace_identities():
    w, mil, H = _dense("tiny_nl")
    assert np.array_equal(H, H.conj().T)
    ev = np.linalg.eigvalsh(H)
    assert abs(np.trace(H).real - ev.sum()) <= 1e-11
    assert abs(np.linalg.norm(H) ** 2 - (ev ** 2).sum()) <= 1e-9


def test_free_electrons_at_zero_potential():
    w = make_workload("gamma_l10")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, np.zeros_like(w.vgrid))
    ev = np.linalg.eigvalsh(H)
    b2 = (2 * np.pi / w.L) ** 2
    exact = np.sort(0.5 * b2 * (mil ** 2).sum(axis=1))
    assert np.abs(ev - exact).max() <= 1e-13
    # shells 0, 6 x 0.197392, 12 x 0.394784
    assert abs(ev[0]) < 1e-14 and np.allclose(ev[1:7], 0.5 * b2) and np.allclose(ev[7:19], b2)


def test_constant_potential_shifts_spectrum():
    w = make_workload("tiny_nl")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    H0 = pw.dense_hamiltonian(w.cell, w.kfrac, mil, np.zeros_like(w.vgrid))
    H1 = pw.dense_hamiltonian(w.cell, w.kfrac, mil, np.full_like(w.vgrid, -0.7))
    assert np.abs(np.linalg.eigvalsh(H1) - (np.linalg.eigvalsh(H0) - 0.7)).max() <= 1e-13


def test_cosine_potential_reduces_to_tridiagonal_chains():
    """V = A cos(2 pi x / L) couples only n and n +- (1,0,0) with A/2: the spectrum is
    the union of the tridiagonal chains along x (scipy eigvalsh_tridiagonal)."""
    w = make_workload("tiny_nl")
    A = 0.9
    x = w.L * np.arange(w.n) / w.n
    v = np.broadcast_to(A * np.cos(2 * np.pi * x / w.L)[:, None, None], (w.n,) * 3).copy()
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, v)
    kin = pw.kinetic(w.cell, w.kfrac, mil)
    chains = {}
    for g, (a, b, c) in enumerate(mil):
        chains.setdefault((b, c), []).append((a, g))
    parts = []
    for key, lst in chains.items():
        lst.sort()
        xs = [a for a, _ in lst]
        assert xs == list(range(xs[0], xs[0] + len(xs)))   # contiguous along x
        d = np.array([kin[g] for _, g in lst])
        e = np.full(len(lst) - 1, A / 2)
        parts.append(scipy.linalg.eigvalsh_tridiagonal(d, e) if len(lst) > 1 else d)
    ref = np.sort(np.concatenate(parts))
    assert np.abs(np.linalg.eigvalsh(H) - ref).max() <= 1e-13


def test_single_projector_secular_equation():
    """H = T + D |b><b| with one s projector and V = 0: eigenvalues below min(T) solve
    1 + D sum_g |b_g|^2 / (T_g - lam) = 0 (rank-one update of a diagonal)."""
    w = make_workload("tiny_nl")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    D = np.array([-1.3])
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, np.zeros_like(w.vgrid),
                             pos=w.pos[:1], lm=((0, 0),), D=D)
    T = pw.kinetic(w.cell, w.kfrac, mil)
    b2 = np.abs(pw.projectors(w.cell, w.kfrac, mil, w.pos[:1], ((0, 0),))[:, 0]) ** 2
    f = lambda lam: 1 + D[0] * np.sum(b2 / (T - lam))
    lo, hi = T.min() - 10.0, T.min() - 1e-12
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            lo = mid
        else:
            hi = mid
    lam0 = 0.5 * (lo + hi)
    assert lam0 < T.min()
    assert abs(np.linalg.eigvalsh(H)[0] - lam0) <= 1e-12


def test_projector_normalisation():
    """s projector: sum_G |beta|^2 = 1 (the lattice sum of a Gaussian equals its
    integral up to exp(-L^2/4) by Poisson summation; c = sqrt(32 pi^(5/2))).
    p projectors: sum_m |Y_1m|^2 = 3/(4 pi) = 3 |Y_00|^2 (addition theorem), so the
    three p norms add up to three s norms exactly when q = 0 is not on the lattice."""
    cell = np.eye(3) * 10.0
    mil = pw.sphere(cell, (0.1, 0, 0), 40.0)
    B = pw.projectors(cell, (0.1, 0, 0), mil, np.array([[1.0, 2.0, 3.0]]),
                      ((0, 0), (1, -1), (1, 0), (1, 1)))
    n2 = np.linalg.norm(B, axis=0) ** 2
    assert abs(n2[0] - 1) < 1e-10
    assert abs(n2[1:].sum() - 3 * n2[0]) < 1e-12
    # y and z are equivalent for k along x; the x-like harmonic differs
    assert abs(n2[1] - n2[2]) < 1e-12


def test_time_reversal_and_rigid_shift():
    w, mil, H = _dense("tiny_nl")
    wk = make_workload("tiny_nl")
    kneg = tuple(-np.array(wk.kfrac))
    mil2 = pw.sphere(wk.cell, kneg, wk.ecut)
    H2 = pw.dense_hamiltonian(wk.cell, kneg, mil2, wk.vgrid, wk.pos, wk.lm, wk.D)
    assert np.abs(np.linalg.eigvalsh(H) - np.linalg.eigvalsh(H2)).max() <= 1e-12
    # shift every atom by a whole grid step: same spectrum
    shift = np.array([2, -1, 3]) * wk.L / wk.n
    pos3 = np.mod(wk.pos + shift, wk.L)
    v3 = well_potential(wk.L, wk.n, pos3)
    H3 = pw.dense_hamiltonian(wk.cell, wk.kfrac, mil, v3, pos3, wk.lm, wk.D)
    assert np.abs(np.linalg.eigvalsh(H) - np.linalg.eigvalsh(H3)).max() <= 1e-12


# ---- Jacobi -----------------------------------------------------------------------------

def test_jacobi_against_lapack():
    rng = np.random.default_rng(2)
    for n in (1, 2, 7, 40):
        M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        A = M + M.conj().T
        w, V, _ = eigh_jacobi(A)
        nrm = max(1.0, np.abs(w).max())
        assert np.abs(w - np.linalg.eigvalsh(A)).max() <= 1e-12 * nrm
        assert np.abs(A @ V - V * w).max() <= 1e-12 * nrm
        assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-13


def test_jacobi_on_hamiltonian():
    w, mil, H = _dense("tiny_nl")
    ev, V, _ = eigh_jacobi(H)
    assert np.abs(ev - np.linalg.eigvalsh(H)).max() <= 1e-12 * np.abs(ev).max()
    from conftest import load_golden
    g = load_golden("gamma_l10")[0]
    w0 = make_workload("gamma_l10")
    H0 = pw.dense_hamiltonian(w0.cell, w0.kfrac, pw.sphere(w0.cell, w0.kfrac, w0.ecut), w0.vgrid)
    assert np.abs(g[:16] - np.linalg.eigvalsh(H0)[:16]).max() <= 1e-12


# ---- matrix-free apply and LOBPCG --------------------------------------------------------

@pytest.mark.parametrize("name", ["gamma_l10", "tiny_nl"])
def test_matfree_apply_equals_dense(name):
    w, mil, H = _dense(name)
    mf = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    X = start_block(1, mil.shape[0], 6)
    assert np.abs(mf.apply(X) - H @ X).max() <= 1e-13 * np.abs(H).sum(axis=1).max()


def test_library_fft_against_naive_dft():
    """The FFT convention used by the matrix-free apply, on a 6^3 grid, against
    explicit DFT sums."""
    rng = np.random.default_rng(4)
    n = 6
    c = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    j = np.arange(n)
    E = np.exp(2j * np.pi * np.outer(j, j) / n)
    naive = np.einsum("ai,bj,ck,ijk->abc", E, E, E, c)
    import scipy.fft
    assert np.abs(scipy.fft.ifftn(c) * n ** 3 - naive).max() <= 1e-12


@pytest.mark.parametrize("name", ["gamma_l10", "tiny_nl"])
def test_oracle_lobpcg_matches_dense(name):
    w, mil, H = _dense(name)
    mf = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    r = matfree.solve(mf, w.nbands, w.block, tol=w.tol, seed=w.seed)
    ref = np.linalg.eigvalsh(H)[:w.nbands]
    assert np.abs(r["eig"] - ref).max() <= 1e-10
    assert r["res"].max() <= w.tol
    cert = matfree.certificate(r["eig"], r["res"])
    assert np.all(np.abs(r["eig"] - ref) <= cert + 1e-13)


def test_oracle_lobpcg_matches_scipy_lobpcg():
    """Same lowest eigenvalues as scipy.sparse.linalg.lobpcg on the matrix-free operator."""
    w = make_workload("mid_nl")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    mf = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    r = matfree.solve(mf, 12, 12, tol=1e-8, seed=3)
    op = scipy.sparse.linalg.LinearOperator((mil.shape[0],) * 2, matvec=lambda x: mf.apply(np.asarray(x).reshape(-1, 1))[:, 0],
                                            matmat=lambda x: mf.apply(np.asarray(x)), dtype=np.complex128)
    X0 = start_block(9, mil.shape[0], 16)
    ev, _ = scipy.sparse.linalg.lobpcg(op, X0, largest=False, tol=1e-9, maxiter=500)
    assert np.abs(np.sort(ev)[:12] - r["eig"]).max() <= 1e-8


def test_final_rayleigh_ritz_is_variational():
    """Ritz values after the final Rayleigh-Ritz never lie below the exact eigenvalues."""
    w, mil, H = _dense("tiny_nl")
    mf = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    r = matfree.solve(mf, w.nbands, w.block, tol=1e-4, seed=1)
    ref = np.linalg.eigvalsh(H)[:w.nbands]
    assert np.all(r["eig"] >= ref - 1e-13)


def test_density_pins():
    """oracle.pw.density: Parseval (the grid sum equals sum occ ||c||^2 N^3 / Omega),
    a single plane wave gives the uniform occ / Omega, and grid points evaluated by
    direct summation over the sphere (no FFT) agree."""
    from workloads import make_workload
    w = make_workload("tiny_nl")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    rng = np.random.default_rng(3)
    C = rng.standard_normal((mil.shape[0], 3)) + 1j * rng.standard_normal((mil.shape[0], 3))
    occ = np.array([2.0, 1.0, 0.5])
    rho = pw.density(w.cell, w.kfrac, mil, w.n, C, occ)
    omega = abs(np.linalg.det(w.cell))
    total = rho.sum() * omega / w.n ** 3
    expect = sum(occ[b] * np.vdot(C[:, b], C[:, b]).real for b in range(3))
    assert abs(total - expect) <= 1e-12 * expect
    one = np.zeros((mil.shape[0], 1), complex)
    one[5, 0] = 1.0
    r1 = pw.density(w.cell, w.kfrac, mil, w.n, one, [1.5])
    assert np.allclose(r1, 1.5 / omega, rtol=0, atol=1e-14 / omega)
    for j in [(0, 0, 0), (1, 2, 3), (w.n - 1, 7, 11), (4, w.n // 2, 9)]:
        ph = np.exp(2j * np.pi * (mil @ np.array(j)) / w.n)
        direct = sum(occ[b] * abs(np.sum(C[:, b] * ph)) ** 2 for b in range(3)) / omega
        assert abs(rho[j] - direct) <= 1e-12 * direct


# ---- generalized form (overlap operator O != I) --------------------------------------

def _overlap_case(name):
    from workloads import overlap_coefficients
    w = make_workload(name)
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    q = overlap_coefficients(w)
    B = pw.projectors(w.cell, w.kfrac, mil, w.pos, w.lm)
    return w, mil, q, B


def test_overlap_operator_properties():
    """O = I + B diag(q) B^H: the matrix-free apply equals the dense matrix; O >= I
    for q >= 0 with exactly nproj eigenvalues above 1, and those equal the
    eigenvalues of 1 + diag(q)^1/2 B^H B diag(q)^1/2 (same nonzero spectrum of
    M M^H and M^H M); trace(O - I) = sum_p q_p |beta_p|^2."""
    w, mil, q, B = _overlap_case("tiny_nl")
    O = pw.overlap_dense(B, q)
    mf = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D, q=q)
    X = start_block(4, mil.shape[0], 5)
    assert np.abs(mf.apply_O(X) - O @ X).max() <= 1e-13
    ev = np.linalg.eigvalsh(O)
    assert ev.min() >= 1 - 1e-13
    above = np.sort(ev[ev > 1 + 1e-10])
    assert above.size == w.nproj
    sq = np.sqrt(q)
    small = np.linalg.eigvalsh(np.eye(w.nproj) + sq[:, None] * (B.conj().T @ B) * sq[None, :])
    assert np.abs(above - np.sort(small)).max() <= 1e-12
    assert abs(np.trace(O).real - mil.shape[0] - np.sum(q * np.linalg.norm(B, axis=0) ** 2)) <= 1e-11


def test_overlap_pencil_secular_equation():
    """H = T (V = 0, no non-local term), O = I + q |b><b| with one s projector: the
    pencil T c = lam O c has, per distinct kinetic value t of multiplicity d,
    d - 1 eigenvalues equal to t, and one root of 1 = lam q sum_t w_t / (t - lam)
    (w_t = sum of |b_g|^2 over that value) between consecutive values t and
    below the smallest.  Against the oracle's dense route (Cholesky reduction +
    Jacobi)."""
    from scipy.optimize import brentq
    w = make_workload("tiny_nl")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    T = pw.kinetic(w.cell, w.kfrac, mil)
    b = pw.projectors(w.cell, w.kfrac, mil, w.pos[:1], ((0, 0),))
    qv = 0.7
    O = pw.overlap_dense(b, [qv])
    A, _ = pw.generalized_to_standard(np.diag(T).astype(complex), O)
    got = np.sort(eigh_jacobi(A)[0])
    # group equal kinetic values (equal up to rounding)
    order = np.argsort(T)
    ts, ws, mult = [], [], []
    for i in order:
        if ts and abs(T[i] - ts[-1]) <= 1e-9 * max(1.0, ts[-1]):
            ws[-1] += abs(b[i, 0]) ** 2
            mult[-1] += 1
        else:
            ts.append(T[i])
            ws.append(abs(b[i, 0]) ** 2)
            mult.append(1)
    ts, ws = np.array(ts), np.array(ws)
    assert ts[0] > 0 and np.all(ws > 0)
    f = lambda lam: lam * qv * np.sum(ws / (ts - lam)) - 1.0
    roots = [brentq(f, 1e-14, ts[0] * (1 - 1e-14), xtol=1e-15, rtol=1e-15, maxiter=500)]
    for i in range(len(ts) - 1):
        gap = ts[i + 1] - ts[i]
        roots.append(brentq(f, ts[i] + 1e-12 * gap, ts[i + 1] - 1e-12 * gap,
                            xtol=1e-15, rtol=1e-15, maxiter=500))
    ref = np.sort(np.concatenate([roots, np.repeat(ts, np.array(mult) - 1)]))
    assert ref.size == got.size
    assert np.abs(got[:60] - ref[:60]).max() <= 1e-10
    assert np.all(got[:60] < np.sort(T)[:60] + 1e-12)   # O >= I lowers a positive spectrum


def test_generalized_reduction_matches_lapack_pencil():
    """Cholesky reduction + the oracle's Jacobi against LAPACK's Hermitian-definite
    pencil solver (zhegvd) on the full Hamiltonian and overlap."""
    w, mil, q, B = _overlap_case("tiny_nl")
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    O = pw.overlap_dense(B, q)
    A, L = pw.generalized_to_standard(H, O)
    ev, V, _ = eigh_jacobi(A)
    ref = scipy.linalg.eigh(H, O, eigvals_only=True, driver="gvd")
    assert np.abs(np.sort(ev) - ref).max() <= 1e-12
    # eigenvectors map back to O-orthonormal pencil eigenvectors
    X = scipy.linalg.solve_triangular(L.conj().T, V, lower=False)
    assert np.abs(X.conj().T @ O @ X - np.eye(X.shape[1])).max() <= 1e-11
    assert np.abs(H @ X - O @ X * ev[None, :]).max() <= 1e-10


@pytest.mark.parametrize("name", ["tiny_nl", "mid_nl"])
def test_oracle_generalized_lobpcg_matches_dense(name):
    """The matrix-free block LOBPCG in the O-metric against the dense pencil."""
    w, mil, q, B = _overlap_case(name)
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
    O = pw.overlap_dense(B, q)
    ref = scipy.linalg.eigh(H, O, eigvals_only=True, driver="gvd")[:w.nbands]
    mf = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D, q=q)
    r = matfree.solve(mf, w.nbands, w.block, tol=1e-9, seed=w.seed)
    assert np.abs(r["eig"] - ref).max() <= 1e-10, np.abs(r["eig"] - ref).max()
    assert r["res"].max() <= 1e-9
    # the overlap moves the spectrum: the standard problem is far away
    assert np.abs(np.linalg.eigvalsh(H)[:w.nbands] - ref).max() > 1e-3


def test_oracle_generalized_with_zero_overlap_is_standard():
    w = make_workload("tiny_nl")
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    a = matfree.solve(matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D),
                      w.nbands, w.block, tol=1e-9, seed=1)
    b = matfree.solve(matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D,
                                       q=np.zeros(w.nproj)), w.nbands, w.block, tol=1e-9, seed=1)
    assert np.abs(a["eig"] - b["eig"]).max() <= 1e-12


# ---- preconditioner and residual certificates ----------------------------------------

def _tpa_factor(T, ekin):
    """K at x = T / ekin, read off oracle.matfree.tpa_precondition with R = 1 and a
    one-plane-wave block whose kinetic energy is ekin."""
    T = np.asarray(T, float)
    X = np.zeros((T.size + 1, 1), complex)
    X[-1, 0] = 1.0
    Tall = np.concatenate([T, [ekin]])
    return matfree.tpa_precondition(Tall, X, np.ones((T.size + 1, 1), complex))[:-1, 0].real


def test_tpa_preconditioner_values():
    """The Teter-Payne-Allan factor (Phys. Rev. B 40, 12255), fixed by its published
    polynomial independently of any implementation: K(0) = 1, K(1) = 65/81,
    K(2) = 175/431, K(x) -> 1/(2x) for large x, and K = 1 - (16/27) x^4 + O(x^5)
    near 0 (the first three derivatives vanish)."""
    e = 0.7
    x = np.array([0.0, 1.0, 2.0, 1e4, 1e-2])
    K = _tpa_factor(x * e, e)
    assert K[0] == 1.0
    assert abs(K[1] - 65.0 / 81.0) <= 1e-15
    assert abs(K[2] - 175.0 / 431.0) <= 1e-15
    assert abs(K[3] * 2 * x[3] - 1.0) <= 1e-3
    # 1 - K = 16 x^4 / (27 + 18 x + ...): within 2 (18/27) x of 16 x^4 / 27 at x = 0.01
    assert abs((1.0 - K[4]) / x[4] ** 4 * 27.0 / 16.0 - 1.0) <= 2 * (18.0 / 27.0) * x[4]
    # monotone and in (0, 1]
    xs = np.linspace(0, 50, 2001)
    Ks = _tpa_factor(xs * e, e)
    assert np.all(np.diff(Ks) <= 0) and np.all(Ks > 0) and np.all(Ks <= 1)


def test_tpa_preconditioner_band_energy_and_floor():
    """x = T_g / E_kin,n with E_kin,n = <x_n|T|x_n> / <x_n|x_n> per band, floored at 1e-3 Ha:
    a band spread evenly over T = 1 and T = 3 has E_kin = 2, so the T = 2 row gets
    K(1) = 65/81; a band on the T = 0 plane wave alone gets the floor, so a row with
    T = 1e-3 gets K(1) too; R is scaled row by row and column by column."""
    T = np.array([1.0, 3.0, 2.0, 0.0, 1e-3])
    X = np.zeros((5, 2), complex)
    X[0, 0] = X[1, 0] = 1.0 / np.sqrt(2.0)
    X[3, 1] = 1j
    R = np.arange(1, 11).reshape(5, 2) * (1 + 2j)
    W = matfree.tpa_precondition(T, X, R)
    assert abs(W[2, 0] / R[2, 0] - 65.0 / 81.0) <= 1e-15
    assert abs(W[4, 1] / R[4, 1] - 65.0 / 81.0) <= 1e-15
    assert abs(W[3, 1] / R[3, 1] - 1.0) <= 1e-15


def test_certificate_bounds_hold_for_the_top_band():
    """H = diag(0, 1, 1 + eps): the second Ritz pair from x = (0, cos t, sin t) has
    theta - 1 = eps sin^2 t and residual eps sin t cos t.  The only computed value
    below it sits at 0, so a gap taken from the computed values alone would claim
    res^2 / 1, far below the true error; no computed value bounds lambda_3 from
    below, so the bound must not fall under the true error."""
    eps, t = 1e-3, 0.3
    H = np.diag([0.0, 1.0, 1.0 + eps])
    x1 = np.array([1.0, 0.0, 0.0])
    x2 = np.array([0.0, np.cos(t), np.sin(t)])
    theta = np.array([x1 @ H @ x1, x2 @ H @ x2])
    res = np.array([np.linalg.norm(H @ x1 - theta[0] * x1), np.linalg.norm(H @ x2 - theta[1] * x2)])
    cert = matfree.certificate(theta, res)
    true_err = theta[1] - 1.0
    assert cert[1] >= true_err
    assert abs(cert[1] - res[1]) <= 1e-18          # the Krylov-Bogolyubov bound
    # below the top, Kato-Temple on a well separated spectrum is valid and sharp
    rng = np.random.default_rng(5)
    lam = np.array([0.0, 1.0, 2.0, 3.0])
    Q = np.linalg.qr(rng.standard_normal((4, 4)))[0]
    A = Q @ np.diag(lam) @ Q.T
    V = Q[:, :3] + 1e-4 * rng.standard_normal((4, 3))
    V = V / np.linalg.norm(V, axis=0)
    th = np.einsum("gi,gh,hi->i", V, A, V)
    r = np.linalg.norm(A @ V - V * th, axis=0)
    c = matfree.certificate(th, r)
    assert np.all(np.abs(th - lam[:3]) <= c)
    assert np.all(c[:2] < r[:2]) and c[2] == r[2]
