"""H.X on the GPU (rows a2-a7) against the oracle.

Small cells: the dense Galerkin matrix of oracle.pw (kinetic + DFT of the
local potential + projectors) times X.  Paper-scale cell (34181 plane waves,
96^3 grid, 432 projectors) at the 64-column block the solver applies: the
oracle's matrix-free numpy-FFT apply, plus rows recomputed one by one from the
dense definition.  Tolerance: FP64, |dY| <= 1e-13 * ||H|| * ||x_j|| per
column (a few ulps per FFT stage times log N stages).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _setup(torch, oracle_problem, name, dense=True, nbands=None, block=None):
    from paper_0707_3405_amd import PlaneWaveProblem
    w, mil, H, mf = oracle_problem(name, dense=dense)
    prob = PlaneWaveProblem.from_workload(w, device=0, nbands=nbands, block=block)
    assert prob.npw == mil.shape[0]
    assert (prob.ctx.get_miller() == mil).all()
    return w, mil, H, mf, prob


def _run(torch, prob, X):
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")
    Y = prob.apply_H(Xd)
    torch.cuda.synchronize()
    return Y.cpu().numpy().T


@pytest.mark.parametrize("name,nb", [("gamma_l10", 16), ("gamma_l10", 5), ("tiny_nl", 12),
                                     ("tiny_nl", 1), ("mid_nl", 48), ("mid_nl", 37)])
def test_apply_matches_dense(torch_cuda, oracle_problem, name, nb):
    torch = torch_cuda
    from workloads import start_block
    w, mil, H, mf, prob = _setup(torch, oracle_problem, name, nbands=max(nb, 16), block=16)
    X = start_block(3, mil.shape[0], nb)
    Y = _run(torch, prob, X)
    ref = H @ X
    hn = np.abs(np.linalg.eigvalsh(H)).max()
    err = np.linalg.norm(Y - ref, axis=0) / (hn * np.linalg.norm(X, axis=0))
    assert err.max() <= 1e-13, err.max()


def test_apply_paper_scale(torch_cuda, oracle_problem):
    """fcc108_l20 at one 64-band block (the solver's launch shape)."""
    torch = torch_cuda
    from oracle import pw
    from workloads import start_block
    w, mil, _, mf, prob = _setup(torch, oracle_problem, "fcc108_l20", dense=False)
    X = start_block(11, mil.shape[0], 64)
    Y = _run(torch, prob, X)
    ref = mf.apply(X)
    # ||H|| bounded by Ecut + max|V| + sum_p D_p ||beta_p||^2
    hn = w.ecut + np.abs(w.vgrid).max() + np.abs(w.D).sum()
    err = np.linalg.norm(Y - ref, axis=0) / (hn * np.linalg.norm(X, axis=0))
    assert err.max() <= 1e-13, err.max()
    # sampled rows from the dense definition, computed one by one
    rng = np.random.default_rng(0)
    rows = rng.choice(mil.shape[0], 6, replace=False)
    span = int(np.abs(mil).max())
    table = pw.vtilde_table(w.vgrid, (-2 * span, 2 * span))
    kin = pw.kinetic(w.cell, w.kfrac, mil)
    B = mf.B
    for i in rows:
        d = mil[i][None, :] - mil + 2 * span
        hrow = table[d[:, 0], d[:, 1], d[:, 2]].copy()
        hrow[i] += kin[i]
        hrow += (B[i] * w.D) @ B.conj().T
        yi = hrow @ X
        assert np.abs(yi - Y[i]).max() <= 1e-12 * hn * np.abs(X).max() * np.sqrt(mil.shape[0])


def test_apply_is_hermitian(torch_cuda, oracle_problem):
    """<y, H x> = conj(<x, H y>) at paper scale (property at any size)."""
    torch = torch_cuda
    from workloads import start_block
    w, mil, _, mf, prob = _setup(torch, oracle_problem, "fcc108_l20", dense=False)
    X = start_block(21, mil.shape[0], 2)
    Y = _run(torch, prob, X)
    a = np.vdot(X[:, 1], Y[:, 0])
    b = np.vdot(X[:, 0], Y[:, 1])
    assert abs(a - np.conj(b)) <= 1e-12 * abs(a)


def test_apply_potential_on_device(torch_cuda, oracle_problem):
    torch = torch_cuda
    from workloads import start_block
    w, mil, H, mf, prob = _setup(torch, oracle_problem, "gamma_l10", nbands=16, block=16)
    prob.ctx.set_local_potential(torch.from_numpy(w.vgrid).to("cuda"))
    X = start_block(4, mil.shape[0], 3)
    Y = _run(torch, prob, X)
    assert np.abs(Y - H @ X).max() <= 1e-12


@pytest.mark.parametrize("N", [16, 20, 24, 32, 36, 40, 48, 60, 64, 72, 80, 96, 108, 120, 128])
def test_every_fft_size(torch_cuda, N):
    """Every supported grid size (each has its own compile-time radix split):
    the wells, projectors and k-point of tiny_nl sampled on an N^3 grid; H.X of
    five bands (a ragged block) against the dense Galerkin matrix of that same
    V grid in FP64 and complex64, and the density against the oracle's."""
    torch = torch_cuda
    from oracle import pw
    from paper_0707_3405_amd import PlaneWaveProblem, PW_PREC_MIXED, fft_sizes
    from workloads import make_workload, well_potential, start_block
    assert N in fft_sizes()
    w = make_workload("tiny_nl")
    v = well_potential(w.L, N, w.pos)
    prob = PlaneWaveProblem(w.cell, w.kfrac, w.ecut, N, v, w.pos, w.lm, w.D, nbands=8, block=4, device=0,
                            prec=PW_PREC_MIXED)
    mil = prob.ctx.get_miller()
    H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, v, w.pos, w.lm, w.D)
    hn = np.abs(np.linalg.eigvalsh(H)).max()
    X = start_block(17, mil.shape[0], 5)
    xn = np.linalg.norm(X, axis=0)
    Y = _run(torch, prob, X)
    err = np.linalg.norm(Y - H @ X, axis=0) / (hn * xn)
    X32 = X.astype(np.complex64)
    Xd32 = torch.from_numpy(np.ascontiguousarray(X32.T)).to("cuda")
    Yd32 = torch.empty_like(Xd32)
    prob.ctx.apply_H(Xd32, Yd32, prec=PW_PREC_MIXED)
    occ = np.array([2.0, 1.5, 1.0, 0.5, 0.25])
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")
    rho = torch.empty((N, N, N), dtype=torch.float64, device="cuda")
    prob.ctx.density(Xd, occ, rho)
    torch.cuda.synchronize()
    err32 = (np.linalg.norm(Yd32.cpu().numpy().T - H @ X32.astype(np.complex128), axis=0)
             / (hn * np.linalg.norm(X32, axis=0)))
    ref = pw.density(w.cell, w.kfrac, mil, N, X, occ)
    rerr = np.abs(rho.cpu().numpy() - ref).max() / ref.max()
    print(f"N={N}: FP64 {err.max():.2e}, complex64 {err32.max():.2e}, density {rerr:.2e}")
    assert err.max() <= 1e-13, err.max()
    assert err32.max() <= 1e-6, err32.max()
    assert rerr <= 1e-12, rerr


def test_general_cell(torch_cuda):
    """A triclinic cell (the basis takes any 3x3 lattice): H.X against the dense
    Galerkin matrix of the same cell and V grid, and a 12-band solve against
    its exact eigenvalues.  V is input data; a well grid of another cell serves."""
    torch = torch_cuda
    from oracle import pw
    from paper_0707_3405_amd import PlaneWaveProblem
    from workloads import well_potential, start_block
    cell = np.array([[7.0, 0.0, 0.0], [1.5, 8.0, 0.0], [0.3, -0.7, 9.0]])
    kfrac, ecut, N = (0.2, -0.1, 0.05), 6.0, 40
    rng = np.random.default_rng(77)
    pos = rng.uniform(0.0, 7.0, (3, 3))
    lm = ((0, 0), (1, -1), (1, 0), (1, 1))
    D = rng.uniform(0.5, 1.5, 3 * len(lm))
    v = well_potential(8.0, N, pos)
    prob = PlaneWaveProblem(cell, kfrac, ecut, N, v, pos, lm, D, nbands=12, block=4, device=0)
    mil = prob.ctx.get_miller()
    assert (mil == pw.sphere(cell, kfrac, ecut)).all()
    H = pw.dense_hamiltonian(cell, kfrac, mil, v, pos, lm, D)
    hn = np.abs(np.linalg.eigvalsh(H)).max()
    X = start_block(23, mil.shape[0], 6)
    Y = _run(torch, prob, X)
    err = np.linalg.norm(Y - H @ X, axis=0) / (hn * np.linalg.norm(X, axis=0))
    eig, Xs, _ = prob.solve(1e-8, max_iter=300)
    torch.cuda.synchronize()
    ref = np.linalg.eigvalsh(H)[:12]
    print(f"triclinic cell (npw {mil.shape[0]}): apply err {err.max():.2e}, "
          f"max |eig - dense| {np.abs(eig - ref).max():.2e}")
    assert err.max() <= 1e-13, err.max()
    assert np.abs(eig - ref).max() <= 1e-8
