"""Per-step parity of the HIP building blocks against their plain definitions.

Gram blocks and block updates (the Rayleigh-Ritz and block update of sec. 3.2, Algorithm 1; sec. 4.1 zgemm) against
numpy products; the small Hermitian eigensolver (Rayleigh-Ritz, sec. 3.2 /
4.2) against LAPACK through numpy; residuals and the preconditioner (Eq. (1),
Rayleigh quotients, residuals and preconditioning of sec. 3.2) against their formulas.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _ctx(torch, npw_case="tiny_nl"):
    from paper_0707_3405_amd import PlaneWaveProblem
    from workloads import make_workload
    w = make_workload(npw_case)
    return PlaneWaveProblem.from_workload(w, device=0, nbands=64, block=16)


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("K,p,q", [(1, 1, 1), (17, 3, 5), (515, 16, 16), (1000, 70, 33),
                                   (4099, 128, 64), (34181, 192, 192), (2000, 200, 130)])
def test_gram_matches_definition(torch_cuda, K, p, q):
    torch = torch_cuda
    prob = _ctx(torch)
    # workspace large enough for the partials of the biggest case
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    prob.ctx.set_workspace(ws[(-ws.data_ptr()) % 256:])
    rng = np.random.default_rng(K + 7 * p + 13 * q)
    A = _crandn(rng, p, K)          # (ncol, ld) = column-major [K x p]
    B = _crandn(rng, q, K)
    C = torch.zeros((q, p), dtype=torch.complex128, device="cuda")
    prob.ctx.gram(_dev(torch, A), _dev(torch, B), C)
    ref = (A.conj() @ B.T)           # [p x q] = A^H B
    got = C.cpu().numpy().T
    scale = np.sqrt(K) * 2.0
    assert np.abs(got - ref).max() <= 1e-13 * scale * np.sqrt(K), np.abs(got - ref).max()
    # determinism: a second call is bitwise identical
    C2 = torch.zeros_like(C)
    prob.ctx.gram(_dev(torch, A), _dev(torch, B), C2)
    assert torch.equal(C, C2)


@pytest.mark.parametrize("K,p,q,alpha,beta", [(1, 1, 1, 1.0, 0.0), (515, 16, 16, 1.0, 0.0),
                                              (1000, 48, 33, -1.0, 1.0), (34181, 192, 128, 1.0, 0.0),
                                              (4097, 512, 512, 1.0, 0.0), (333, 7, 64, 0.5, 1.0)])
def test_block_update_matches_definition(torch_cuda, K, p, q, alpha, beta):
    torch = torch_cuda
    prob = _ctx(torch)
    rng = np.random.default_rng(K + p + q)
    A = _crandn(rng, p, K)
    Cm = _crandn(rng, q, p)
    Y0 = _crandn(rng, q, K)
    Y = _dev(torch, Y0)
    prob.ctx.block_update(_dev(torch, A), _dev(torch, Cm), Y, alpha=alpha, beta=beta)
    ref = alpha * (A.T @ Cm.T) + beta * Y0.T
    got = Y.cpu().numpy().T
    assert np.abs(got - ref).max() <= 1e-13 * np.sqrt(p) * 4, np.abs(got - ref).max()


def test_block_update_in_place(torch_cuda):
    torch = torch_cuda
    prob = _ctx(torch)
    rng = np.random.default_rng(3)
    K, q = 3001, 64
    A = _crandn(rng, q, K)
    Cm = _crandn(rng, q, q)
    X = _dev(torch, A)
    prob.ctx.block_update(X, _dev(torch, Cm), X)
    ref = A.T @ Cm.T
    assert np.abs(X.cpu().numpy().T - ref).max() <= 1e-12


# sizes straddle the kernel variants: register-resident reduction (n <= 192),
# LDS CholQR2 of the eigenvectors (k <= 64, n <= 219), one-wave back-transform
# (n <= 256) and the general forms above those sizes, up to the largest
# Rayleigh-Ritz (n = 1024, where the back-transform also shrinks its LDS staging)
@pytest.mark.parametrize("n,k,kind", [(1, 1, "rand"), (2, 2, "rand"), (5, 3, "rand"), (33, 7, "rand"),
                                      (48, 16, "rand"), (64, 64, "rand"), (100, 1, "rand"),
                                      (130, 40, "rand"), (192, 64, "rand"), (192, 64, "degenerate"),
                                      (128, 64, "graded"), (193, 64, "rand"), (230, 70, "rand"),
                                      (300, 32, "degenerate"), (512, 512, "rand"),
                                      (1000, 64, "degenerate"), (1024, 1024, "rand")])
def test_small_eigh(torch_cuda, n, k, kind):
    torch = torch_cuda
    prob = _ctx(torch)
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    prob.ctx.set_workspace(ws[(-ws.data_ptr()) % 256:])
    rng = np.random.default_rng(n * 31 + k)
    if kind == "rand":
        M = _crandn(rng, n, n)
        A = M + M.conj().T
    else:
        Q, _ = np.linalg.qr(_crandn(rng, n, n))
        if kind == "degenerate":
            lam = np.repeat(np.arange(n // 4), 4)[:n].astype(float)
            lam = np.concatenate([lam, np.arange(n - lam.size)])
        else:
            lam = np.logspace(-8, 2, n) * np.where(np.arange(n) % 2, 1, -1)
        A = (Q * lam) @ Q.conj().T
        A = 0.5 * (A + A.conj().T)
    Ad = _dev(torch, A.T)            # column-major storage of A
    w = torch.zeros(k, dtype=torch.float64, device="cuda")
    V = torch.zeros((k, n), dtype=torch.complex128, device="cuda")
    prob.ctx.small_eigh(Ad, n, k, w, V)
    ref = np.linalg.eigvalsh(A)[:k]
    wn = w.cpu().numpy()
    Vn = V.cpu().numpy().T
    nrm = np.abs(np.linalg.eigvalsh(A)).max()
    assert np.abs(wn - ref).max() <= 1e-13 * nrm * max(1, np.sqrt(n) / 4), np.abs(wn - ref).max()
    assert np.abs(A @ Vn - Vn * wn).max() <= 1e-12 * nrm
    # eigenvectors of separated clusters come from inverse iteration alone once
    # n k is too large for a full re-orthogonalisation in LDS: their overlaps are
    # bounded by the solve's backward error over the gap, ~ n eps ||T|| / gap
    # (gap = 1 between the clusters of the degenerate matrices)
    orth = 1e-12 if kind != "degenerate" else max(1e-12, n * np.finfo(float).eps * nrm / 1.0)
    assert np.abs(Vn.conj().T @ Vn - np.eye(k)).max() <= orth


def test_residuals_and_preconditioner(torch_cuda, oracle_problem):
    torch = torch_cuda
    from oracle import matfree
    w, mil, H, mf = oracle_problem("gamma_l10")
    prob = _ctx(torch, "gamma_l10")
    rng = np.random.default_rng(5)
    X = _crandn(rng, mil.shape[0], 16)
    X /= np.linalg.norm(X, axis=0)
    HX = H @ X
    theta = torch.zeros(16, dtype=torch.float64, device="cuda")
    res = torch.zeros(16, dtype=torch.float64, device="cuda")
    W = torch.zeros((16, mil.shape[0]), dtype=torch.complex128, device="cuda")
    prob.ctx.residuals(_dev(torch, X.T), _dev(torch, HX.T), 16, theta, res, W)
    th_ref = np.einsum("gn,gn->n", X.conj(), HX).real
    R = HX - X * th_ref
    assert np.abs(theta.cpu().numpy() - th_ref).max() <= 1e-13
    assert np.abs(res.cpu().numpy() - np.linalg.norm(R, axis=0)).max() <= 1e-13
    Wref = matfree.tpa_precondition(mf.T, X, R)
    assert np.abs(W.cpu().numpy().T - Wref).max() <= 1e-13


@pytest.mark.parametrize("n,cond", [(1, 1.0), (7, 10.0), (16, 1e3), (33, 1e2), (63, 1e4), (64, 1e6)])
def test_chol_inv(torch_cuda, n, cond):
    """R^-1 of G = R^H R (R upper, positive real diagonal: unique) against the
    definition computed by numpy; bar from the conditioning: the relative error
    of R^-1 grows like cond(G)^1/2 times the roundoff."""
    torch = torch_cuda
    prob = _ctx(torch)
    rng = np.random.default_rng(n * 7 + int(np.log10(cond)))
    Q, _ = np.linalg.qr(_crandn(rng, n, n))
    lam = np.logspace(0, np.log10(cond), n)
    G = (Q * lam) @ Q.conj().T
    G = 0.5 * (G + G.conj().T)
    Gd = _dev(torch, G.T)
    Rd = torch.full((n, n), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    prob.ctx.chol_inv(Gd, n, Rd)
    Rinv = Rd.cpu().numpy().T
    # the documented diagonal shift is part of the definition
    shift = 1e-15 * n * np.max(np.diag(G).real)
    R = np.linalg.cholesky(G + shift * np.eye(n)).conj().T
    ref = np.linalg.inv(R)
    err = np.abs(Rinv - ref).max() / np.abs(ref).max()
    assert err <= 1e-14 * np.sqrt(cond) * n, err
    assert np.all(np.tril(Rinv, -1) == 0)
    assert np.all(np.abs(np.diag(Rinv).imag) == 0) and np.all(np.diag(Rinv).real > 0)
    # W R^-1 is orthonormal for W^H W = G (up to the shift)
    assert np.abs(Rinv.conj().T @ G @ Rinv - np.eye(n)).max() <= 1e-13 * cond + 2 * shift


def test_chol_inv_breakdown(torch_cuda):
    torch = torch_cuda
    from paper_0707_3405_amd import PWError, PW_ERR_NUMERIC
    prob = _ctx(torch)
    G = np.eye(8, dtype=complex)
    G[5, 5] = -1.0
    Rd = torch.zeros((8, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(PWError) as e:
        prob.ctx.chol_inv(_dev(torch, G.T), 8, Rd)
    assert e.value.status == PW_ERR_NUMERIC
