"""Autotuner of the FFT tiles and the split-K GEMM target (pw_autotune / pw_set_tuning).

The tuned parameters only repartition the work: the local H.X (no projectors)
must be bitwise the same under every FFT tiling, a solve after tuning must
still match the oracle's goldens, and two contexts given the same parameters
must give bitwise the same solve.
"""
import numpy as np
import pytest

from conftest import load_golden

pytestmark = pytest.mark.gpu


def test_autotune_choices_and_timings(torch_cuda):
    torch = torch_cuda
    from paper_0707_3405_amd import PlaneWaveProblem
    from workloads import make_workload
    w = make_workload("fcc32_l12")
    prob = PlaneWaveProblem.from_workload(w, device=0)
    t = prob.ctx.autotune(w.block)
    print("fcc32_l12 tuning:", t)
    assert t["fft_sticks_per_block"] in (0, 16, 32, 64)
    assert t["fft_plane_rows"] in (0, 16, 32, 48, 96)
    assert t["gemm_split_workgroups"] in (0, 384, 512, 768, 1024)
    assert 0 < t["apply_ms_tuned"] <= t["apply_ms_default"]
    assert 0 < t["gemm_ms_tuned"] <= t["gemm_ms_default"]
    eig, X, status = prob.solve(w.tol, max_iter=300)
    torch.cuda.synchronize()
    ref = load_golden("fcc32_l12")[0][:w.nbands]
    assert np.abs(eig - ref).max() <= 1e-8


@pytest.mark.parametrize("spb,rb", [(16, 8), (64, 16), (32, 32), (16, 48), (32, 96), (1, 1)])
def test_fft_tiling_is_bitwise_neutral(torch_cuda, spb, rb):
    torch = torch_cuda
    from paper_0707_3405_amd import PlaneWaveProblem
    from workloads import make_workload, start_block
    w = make_workload("fcc32_l12")
    loc = PlaneWaveProblem(w.cell, w.kfrac, w.ecut, w.n, w.vgrid, None, (), None, nbands=32, block=32,
                           device=0)
    X = torch.from_numpy(np.ascontiguousarray(start_block(4, loc.npw, 32).T)).cuda()
    Y0, Y1 = torch.empty_like(X), torch.empty_like(X)
    loc.ctx.apply_H(X, Y0)
    loc.ctx.set_tuning(fft_sticks_per_block=spb, fft_plane_rows=rb)
    loc.ctx.apply_H(X, Y1)
    torch.cuda.synchronize()
    assert torch.equal(Y0, Y1)


def test_same_tuning_same_result(torch_cuda):
    torch = torch_cuda
    from paper_0707_3405_amd import PlaneWaveProblem, PWError, PW_ERR_ARG
    from workloads import make_workload
    w = make_workload("mid_nl")
    out = []
    for _ in range(2):
        prob = PlaneWaveProblem.from_workload(w, device=0)
        prob.ctx.set_tuning(fft_sticks_per_block=16, fft_plane_rows=8, gemm_split_workgroups=384)
        eig, X, _ = prob.solve(w.tol, max_iter=300)
        torch.cuda.synchronize()
        out.append((eig, X.clone()))
    assert np.array_equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
    ref = load_golden("mid_nl")[0][:w.nbands]
    assert np.abs(out[0][0] - ref).max() <= 1e-8
    with pytest.raises(PWError) as e:
        prob.ctx.set_tuning(fft_sticks_per_block=65)
    assert e.value.status == PW_ERR_ARG
    prob.ctx.set_tuning(reset=True)
