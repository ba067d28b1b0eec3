"""Batched k-points: independent solves run concurrently (pw_lobpcg_solve_batch).

Sec. 5.2: k-points are independent inside the eigensolve.  Each problem has
its own context and stream; the library drives them from separate host
threads.  Checks: every batched result is bitwise the result of the same
problem solved alone (the kernels are deterministic and share nothing), the
eigenvalues match the oracle (dense H at small cells; the oracle's block
LOBPCG, stored in tests/golden/, at two k-points of the ten-k-point cell), and
every residual is within tol.
"""
import numpy as np
import pytest

from conftest import load_golden

pytestmark = pytest.mark.gpu


def _problems(torch, wl, prec):
    from paper_0707_3405_amd import PlaneWaveProblem
    return [PlaneWaveProblem.from_workload(w, device=0, stream=torch.cuda.Stream(), prec=prec)
            for w in wl]


def test_batch_small_cells_match_solo_and_dense(torch_cuda):
    torch = torch_cuda
    from oracle import pw
    from paper_0707_3405_amd import solve_batch, PW_PREC_FP64
    from workloads import make_kpoint_workloads
    wl = make_kpoint_workloads("mid_nl", kpts=[(0, 0, 0), (0.25, 0, 0.5), (0.5, 0.5, 0.5)])
    probs = _problems(torch, wl, PW_PREC_FP64)
    assert len({p.npw for p in probs}) > 1          # uneven plane-wave counts
    eigs, Xs, st = solve_batch(probs, wl[0].tol)
    torch.cuda.synchronize()
    for w, p, e in zip(wl, probs, eigs):
        res = p.ctx.get_residuals(p.nbands)
        assert res.max() <= w.tol
        mil = pw.sphere(w.cell, w.kfrac, w.ecut)
        H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
        ref = np.linalg.eigvalsh(H)[:w.nbands]
        assert np.abs(e - ref).max() <= 1e-8, np.abs(e - ref).max()
        solo, _, _ = p.solve(w.tol)
        torch.cuda.synchronize()
        assert np.array_equal(solo, e)


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_batch_ten_kpoints(torch_cuda, prec_name):
    """The ten irreducible k-points of the 4x4x4 grid of the L = 16 bohr cell (256 bands each)."""
    torch = torch_cuda
    import time
    from paper_0707_3405_amd import solve_batch, PW_PREC_FP64, PW_PREC_MIXED
    from workloads import make_kpoint_workloads
    prec = PW_PREC_FP64 if prec_name == "fp64" else PW_PREC_MIXED
    wl = make_kpoint_workloads()
    probs = _problems(torch, wl, prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eigs, Xs, st = solve_batch(probs, wl[0].tol)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    for w, p in zip(wl, probs):
        assert p.ctx.get_residuals(p.nbands).max() <= w.tol
    for idx in (0, 1, 5, 9):   # Gamma, k1, the most (k5: 11416) and the fewest (k9: 11296) plane waves
        ref = load_golden(f"kpts_l16_k{idx}")[0][:wl[idx].nbands]
        err = np.abs(eigs[idx] - ref)
        print(f"{prec_name} k{idx}: max |eig - oracle| = {err.max():.3e}")
        assert err.max() <= (1e-8 if prec == PW_PREC_FP64 else 1e-6), err.max()
    t0 = time.perf_counter()
    solo, _, _ = probs[1].solve(wl[1].tol)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    assert np.array_equal(solo, eigs[1])
    print(f"{prec_name}: batch of 10 k-points {t_batch:.2f} s, one k-point alone {t_solo:.2f} s, "
          f"{10 * 256 / t_batch:.1f} eigenpairs/s batched")


def _batch_setup(torch, wl, prec, nb):
    from paper_0707_3405_amd import PlaneWaveProblem, PW_PREC_FP64
    from workloads import start_block
    s = torch.cuda.Stream()   # one stream for every context of the batched apply
    probs = [PlaneWaveProblem.from_workload(w, device=0, stream=s, prec=prec) for w in wl]
    dt = torch.complex128 if prec == PW_PREC_FP64 else torch.complex64
    Xs = [torch.from_numpy(np.ascontiguousarray(start_block(40 + k, p.npw, nb).T)).to("cuda").to(dt)
          for k, p in enumerate(probs)]
    return s, probs, Xs


@pytest.mark.parametrize("prec_name,nb", [("fp64", 40), ("mixed", 32), ("fp64", 7)])
def test_apply_batch_matches_per_context(torch_cuda, prec_name, nb):
    """pw_apply_H_batch over the ten k-points of the L = 16 bohr cell (uneven npw,
    one launch per FFT pass for every (k-point, band) item, the potential of the
    first context shared) gives every context's pw_apply_H result bitwise; 40
    columns are two chunks of the 32-band workspace."""
    torch = torch_cuda
    from paper_0707_3405_amd import apply_H_batch, PW_PREC_FP64, PW_PREC_MIXED
    from workloads import make_kpoint_workloads
    prec = PW_PREC_FP64 if prec_name == "fp64" else PW_PREC_MIXED
    wl = make_kpoint_workloads()
    s, probs, Xs = _batch_setup(torch, wl, prec, nb)
    assert len({p.npw for p in probs}) > 1
    Ys = [torch.empty_like(X) for X in Xs]
    Yr = [torch.empty_like(X) for X in Xs]
    with torch.cuda.stream(s):
        apply_H_batch([p.ctx for p in probs], Xs, Ys, prec=prec)
        for p, X, Y in zip(probs, Xs, Yr):
            p.ctx.apply_H(X, Y, prec=prec)
    s.synchronize()
    for k, (Y, R) in enumerate(zip(Ys, Yr)):
        assert torch.equal(Y, R), k


def test_apply_batch_matches_oracle(torch_cuda):
    """The batched apply against the oracle's dense H at three k-points of the
    mid-size cell: 1e-13 ||H|| ||x|| per column."""
    torch = torch_cuda
    from oracle import pw
    from paper_0707_3405_amd import apply_H_batch, PW_PREC_FP64
    from workloads import make_kpoint_workloads
    wl = make_kpoint_workloads("mid_nl", kpts=[(0, 0, 0), (0.25, 0, 0.5), (0.5, 0.5, 0.5)])
    s, probs, Xs = _batch_setup(torch, wl, PW_PREC_FP64, 12)
    Ys = [torch.empty_like(X) for X in Xs]
    with torch.cuda.stream(s):
        apply_H_batch([p.ctx for p in probs], Xs, Ys)
    s.synchronize()
    for w, p, X, Y in zip(wl, probs, Xs, Ys):
        mil = pw.sphere(w.cell, w.kfrac, w.ecut)
        H = pw.dense_hamiltonian(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D)
        x = X.cpu().numpy().T
        err = np.linalg.norm(Y.cpu().numpy().T - H @ x, axis=0) / (np.linalg.norm(H, 2) * np.linalg.norm(x, axis=0))
        assert err.max() <= 1e-13, err.max()


def test_apply_batch_graph_replay(torch_cuda):
    """The batched apply recorded into a graph (kernel launches only) replays to
    the eager result bitwise, three times, with eager work and synchronisations
    between the replays."""
    torch = torch_cuda
    from paper_0707_3405_amd import apply_H_batch, PW_PREC_FP64
    from workloads import make_kpoint_workloads
    wl = make_kpoint_workloads()[:4]
    s, probs, Xs = _batch_setup(torch, wl, PW_PREC_FP64, 32)
    ctxs = [p.ctx for p in probs]
    Ys = [torch.empty_like(X) for X in Xs]
    with torch.cuda.stream(s):
        apply_H_batch(ctxs, Xs, Ys)   # eager: also sets the kernels' LDS limits
    s.synchronize()
    ref = [Y.clone() for Y in Ys]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        apply_H_batch(ctxs, Xs, Ys)
    scratch = [torch.empty_like(X) for X in Xs]
    for rep in range(3):
        with torch.cuda.stream(s):
            for Y in Ys:
                Y.zero_()
            for p, X, Z in zip(probs, Xs, scratch):   # eager work between the replays
                p.ctx.apply_H(X, Z)
        s.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (Y, R) in enumerate(zip(Ys, ref)):
            assert torch.equal(Y, R), (rep, k)
