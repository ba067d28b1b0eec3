"""Benchmark: block-LOBPCG eigenpairs/s on the paper-scale synthetic cell.

Workload (one "step" = one full pw_lobpcg_solve from a ready context to
eigenvalues on the host, final Rayleigh-Ritz included): 108 Gaussian wells at
jittered fcc sites in a 20 bohr cube, Ecut 20 Ha (34181 plane waves), k =
(1/4,1/4,1/4), 96^3 grid, 432 KB projectors, 512 bands in blocks of 64,
residual tolerance 1e-6, FP64.

Prints ONE JSON line (rank 0).  Besides the headline value (FP64) it reports
the same solve in the mixed-precision forms (complex64 iteration + FP64
refinement; FP32 products, split-bf16 projector products, split-bf16 projector
and Gram products) with their per-eigenvalue differences from the FP64 result, the H.X
FFT throughput in both precisions, the roofline of the dominant phase and of
the other two (each timed with HIP events on the stream it runs on at its
canonical launch shape), solve-latency percentiles, and the CPU oracle timed on
a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu] [--mixed-steps 2]
    python bench.py --roofline-only      # the roofline launches alone (profiling)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by a plain-copy
# calibration; profiles/hbm_bytes_fcc108_l20.txt) for the kernels as they were profiled,
# over the same kernels as the launch time (the Grams include k_reduce_parts);
# set an entry to None when its kernels change.
TRAFFIC_MEASURED = {"apply": 6.15e8, "gemm": 3.63e8, "gemm_complex64": 1.84e8, "dense": 5.43e6}
FP64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3       # MI355X dense FP32 (matrix)
WORKLOAD = "fcc108_l20"


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def event_time_ms(torch, stream, fn, reps):
    """Average duration of fn() over reps launches, HIP events on `stream`."""
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def cpu_model_name():
    """The host CPU's model string (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def cpu_baseline(w, gpu_iterations, cores, sample_iters=6, full_block=True):
    """The oracle on the host cores, three ways:
    * the paper-scale cell: block 0 of the oracle's block LOBPCG, `sample_iters`
      iterations timed and extrapolated to the GPU solve's iteration count (the
      headline value), and -- with full_block -- block 0 iterated to the GPU's
      tolerance, extrapolated over the ten blocks;
    * the small Gamma-point cell (515 plane waves, 16 bands): dense H built and
      diagonalised by the oracle's plain C Jacobi on one core, with
      numpy.linalg.eigh on all cores as context."""
    from oracle import matfree, pw
    from oracle.jacobi import eigh_jacobi
    from workloads import start_block, make_workload
    mil = pw.sphere(w.cell, w.kfrac, w.ecut)
    mf = matfree.MatFreeH(w.cell, w.kfrac, mil, w.vgrid, w.pos, w.lm, w.D, workers=cores)
    X0 = start_block(0, mil.shape[0], w.block)
    t0 = time.perf_counter()
    matfree.lobpcg_block(mf, X0, None, tol=0.0, maxit=1)
    t1 = time.perf_counter()
    matfree.lobpcg_block(mf, X0, None, tol=0.0, maxit=1 + sample_iters)
    t2 = time.perf_counter()
    t_iter = ((t2 - t1) - (t1 - t0)) / sample_iters
    est = t_iter * gpu_iterations
    out = dict(value=w.nbands / est, unit="eigenpairs/s", cores=cores, kind="oracle",
               cpu_model=cpu_model_name(), affinity_cpus=len(os.sched_getaffinity(0)),
               sample=(f"oracle block LOBPCG ({WORKLOAD}, block 0, {w.block} bands), "
                       f"{sample_iters} iterations timed ({t_iter:.2f} s/iteration), "
                       f"extrapolated to the GPU solve's {gpu_iterations} iterations"),
               seconds_per_iteration=t_iter, sample_seconds=t2 - t0)
    # H.X throughput of the oracle on the same byte model as the GPU apply
    Xh = start_block(1, mil.shape[0], w.block)
    t3 = time.perf_counter()
    mf.apply_local(Xh)
    t_apply = time.perf_counter() - t3
    out["hx_local_seconds_per_64_bands"] = t_apply
    if full_block:
        guard = w.block // 8
        t4 = time.perf_counter()
        _, _, _, res, iters = matfree.lobpcg_block(mf, X0, None, tol=w.tol, maxit=300,
                                                    nconv=w.block - guard)
        t_block = time.perf_counter() - t4
        nblocks = -(-w.nbands // (w.block - guard))
        out["full_block0"] = dict(
            seconds=t_block, iterations=iters, max_residual=float(res[:w.block - guard].max()),
            eigenpairs_per_s_extrapolated=w.nbands / (t_block * nblocks),
            sample=(f"block 0 of {WORKLOAD} iterated to tol {w.tol:g} ({w.block} columns, "
                    f"{w.block - guard} kept), time x {nblocks} blocks"))
    # the small cell: dense build + plain C Jacobi on one core; LAPACK as context
    w0 = make_workload("gamma_l10")
    t5 = time.perf_counter()
    mil0 = pw.sphere(w0.cell, w0.kfrac, w0.ecut)
    H0 = pw.dense_hamiltonian(w0.cell, w0.kfrac, mil0, w0.vgrid)
    t6 = time.perf_counter()
    ev, _, sweeps = eigh_jacobi(H0)
    t7 = time.perf_counter()
    np.linalg.eigh(H0)
    t8 = time.perf_counter()
    out["gamma_l10"] = dict(
        npw=int(mil0.shape[0]), nbands=w0.nbands, build_seconds=t6 - t5, jacobi_seconds=t7 - t6,
        jacobi_sweeps=int(sweeps), eigenpairs_per_s=w0.nbands / (t7 - t5), jacobi_cores=1,
        numpy_eigh_seconds=t8 - t7, numpy_eigh_cores=cores,
        sample="dense H of the 8-well Gamma-point cell built by the oracle and fully diagonalised "
               "by its cyclic Jacobi (plain C, one thread); numpy.linalg.eigh of the same H on all "
               "cores as context")
    return out


def eig_error_quantiles(eig, ref):
    """Per-eigenvalue |eig - ref| summarised (Ha): quantiles over the bands."""
    err = np.abs(np.asarray(eig) - np.asarray(ref))
    return {"max": float(err.max()), "p99": float(np.percentile(err, 99)),
            "p90": float(np.percentile(err, 90)), "p50": float(np.percentile(err, 50)),
            "mean": float(err.mean()), "bands": int(err.size)}


def load_oracle_golden(name):
    """Eigenvalues the oracle wrote under tests/golden/ (index, eigenvalue, ...)."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_eig.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return np.array([float(r[1]) for r in rows])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=15)
    ap.add_argument("--mixed-steps", type=int, default=2, help="timed solves in the mixed form")
    ap.add_argument("--autotune", type=int, default=1,
                    help="also run the autotuner on a fresh context and time one solve with its choice")
    ap.add_argument("--overlap-steps", type=int, default=1,
                    help="timed solves of the same cell in the generalized form (O != I)")
    ap.add_argument("--batch-steps", type=int, default=1,
                    help="timed batches of the ten-k-point cell (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests in the narrowed served-stream sample (0: skip)")
    ap.add_argument("--serve-full-requests", type=int, default=60,
                    help="requests of the full-range served stream (L 8-24 bohr, Ecut 5-25 Ha; 0: skip)")
    ap.add_argument("--serve-full-cap-s", type=float, default=220.0,
                    help="cap on the full-range served stream's arrival span (seconds)")
    ap.add_argument("--cpu-full-block", type=int, default=1,
                    help="also time one complete oracle block of the paper-scale cell on the CPU")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the per-kernel roofline timings (for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0707_3405_amd import (PlaneWaveProblem, PW_PREC_FP64, PW_PREC_MIXED,
                                     PW_PREC_MIXED_BF16, PW_PREC_MIXED_BF16_GRAM, PW_PREC_MIXED_FP32_RR,
                                     solve_batch)
    from workloads import make_workload, make_kpoint_workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = make_workload(WORKLOAD)
    log(f"workload {WORKLOAD}: L={w.L} ecut={w.ecut} n={w.n} M={w.nbands} m={w.block}")
    # the workspace is sized for the mixed form, which also covers FP64
    prob = PlaneWaveProblem.from_workload(w, device=0, prec=PW_PREC_MIXED)
    npw = prob.npw
    X = prob.empty_block(w.nbands)

    def solve(prec=PW_PREC_FP64):
        eig, st = prob.ctx.lobpcg_solve(w.nbands, w.block, w.tol, 300, X, use_guess=False, prec=prec)
        return eig

    if not args.roofline_only:
        for i in range(args.warmup):
            solve()
            log(f"warmup {i + 1}/{args.warmup} done")
        torch.cuda.synchronize()
        lat = []
        iters = []
        t_start = time.perf_counter()
        for i in range(args.steps):
            t0 = time.perf_counter()
            eig = solve()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            st = prob.ctx.get_stats()
            iters.append(st["iterations"])
            log(f"step {i + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms, {st['iterations']} iterations")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        ms_per_step = 1e3 * elapsed / args.steps
        value = w.nbands / (elapsed / args.steps)
        res = prob.ctx.get_residuals(w.nbands)
        stats = prob.ctx.get_stats()
        eig64 = eig.copy()

        # the phase split comes from one more (untimed) solve with per-phase HIP
        # events: each is a marker between kernels and they cost ~5 % of a solve,
        # so the timed solves run without them
        def phase_split(ctx, run):
            ctx.set_phase_timing(True)
            run()
            torch.cuda.synchronize()
            ctx.set_phase_timing(False)
            pst = ctx.get_stats()
            return {k: pst[k] for k in ("ms_apply", "ms_gemm", "ms_dense", "ms_vec", "ms_final_rr")}
        phases = phase_split(prob.ctx, solve)
        # the oracle's eigenvalues of the same cell (block LOBPCG to 1e-8, tests/golden)
        golden = load_oracle_golden(WORKLOAD)[:w.nbands]
        fp64_err = eig_error_quantiles(eig64, golden)

        # ---- the same cell in the mixed forms (complex64 iteration + FP64 refinement;
        # the BF16 forms also run the projector products, and the second one the
        # Rayleigh-Ritz Gram, on split-bf16 matrix cores; the FP32-RR form reduces the
        # complex64 stage's Rayleigh-Ritz problems to tridiagonal form in FP32)
        def run_mixed(prec, label):
            solve(prec)
            torch.cuda.synchronize()
            mlat = []
            for i in range(args.mixed_steps):
                t0 = time.perf_counter()
                eigm = solve(prec)
                torch.cuda.synchronize()
                mlat.append(time.perf_counter() - t0)
                log(f"{label} step {i + 1}/{args.mixed_steps}: {mlat[-1] * 1e3:.1f} ms")
            mst = prob.ctx.get_stats()
            mres = prob.ctx.get_residuals(w.nbands)
            err = np.abs(eigm - eig64)
            per_eig = eig_error_quantiles(eigm, golden)
            return {"value": w.nbands / float(np.mean(mlat)), "unit": "eigenpairs/s",
                    "ms_per_solve": 1e3 * float(np.mean(mlat)),
                    "latency_p50_ms": float(np.percentile(np.array(mlat) * 1e3, 50)),
                    "latency_p99_ms": float(np.percentile(np.array(mlat) * 1e3, 99)),
                    "speedup_vs_fp64": (w.nbands / float(np.mean(mlat))) / value,
                    "max_abs_eig_diff_vs_fp64_ha": float(err.max()),
                    "mean_abs_eig_diff_vs_fp64_ha": float(err.mean()),
                    "abs_eig_err_vs_oracle_ha": per_eig,
                    "max_residual": float(mres.max()),
                    "iterations": mst["iterations"], "complex64_iterations": mst["mixed_iterations"],
                    "phase_ms": phase_split(prob.ctx, lambda: solve(prec))}

        mixed = mixed_bf16 = mixed_bf16_gram = mixed_fp32_rr = None
        if args.mixed_steps > 0:
            mixed = run_mixed(PW_PREC_MIXED, "mixed")
            mixed_bf16 = run_mixed(PW_PREC_MIXED_BF16, "mixed-bf16")
            mixed_bf16_gram = run_mixed(PW_PREC_MIXED_BF16_GRAM, "mixed-bf16-gram")
            mixed_fp32_rr = run_mixed(PW_PREC_MIXED_FP32_RR, "mixed-fp32-rr")

        # ---- the same cell as the pencil (H, O), O = I + sum_p q_p |beta_p><beta_p|
        generalized = None
        if args.overlap_steps > 0:
            from workloads import overlap_coefficients
            gprob = PlaneWaveProblem.from_workload(w, device=0, q=overlap_coefficients(w))
            Xg = gprob.empty_block(w.nbands)
            glat = []
            for i in range(args.overlap_steps + 1):
                t0 = time.perf_counter()
                gprob.ctx.lobpcg_solve(w.nbands, w.block, w.tol, 300, Xg)
                torch.cuda.synchronize()
                if i > 0:
                    glat.append(time.perf_counter() - t0)
                log(f"generalized step {i}/{args.overlap_steps}: {(time.perf_counter() - t0) * 1e3:.1f} ms")
            gst = gprob.ctx.get_stats()
            generalized = {"value": w.nbands / float(np.mean(glat)), "unit": "eigenpairs/s",
                           "ms_per_solve": 1e3 * float(np.mean(glat)),
                           "max_residual": float(gprob.ctx.get_residuals(w.nbands).max()),
                           "iterations": gst["iterations"],
                           "overlap": "q_p ~ U(0.2, 0.8) per projector",
                           "phase_ms": phase_split(gprob.ctx, lambda: gprob.ctx.lobpcg_solve(
                               w.nbands, w.block, w.tol, 300, Xg))}
            del gprob, Xg

        # ---- autotuner on a fresh context of the same cell (FFT tiles, split-K target),
        # and one FP64 solve with its choice
        tuned = None
        if args.autotune:
            tprob = PlaneWaveProblem.from_workload(w, device=0)
            tchoice = tprob.ctx.autotune(w.block)
            Xt = tprob.empty_block(w.nbands)
            tprob.ctx.lobpcg_solve(w.nbands, w.block, w.tol, 300, Xt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eigt, _ = tprob.ctx.lobpcg_solve(w.nbands, w.block, w.tol, 300, Xt)
            torch.cuda.synchronize()
            tdt = time.perf_counter() - t0
            tuned = {"choice": tchoice, "value": w.nbands / tdt, "unit": "eigenpairs/s",
                     "max_abs_eig_diff_vs_default_ha": float(np.abs(eigt - eig64).max())}
            log(f"autotuned: {tchoice}, {w.nbands / tdt:.1f} eigenpairs/s")
            del tprob, Xt

        # ---- full H.X (local + 432 projectors) per 64 bands in the three forms
        Xh = torch.randn((w.block, npw), dtype=torch.complex128, device="cuda")
        Yh = torch.empty_like(Xh)
        Xh32 = Xh.to(torch.complex64)
        Yh32 = torch.empty_like(Xh32)
        hx_full = {
            "fp64": event_time_ms(torch, prob.ctx.stream, lambda: prob.ctx.apply_H(Xh, Yh), 10),
            "complex64": event_time_ms(torch, prob.ctx.stream,
                                       lambda: prob.ctx.apply_H(Xh32, Yh32, prec=PW_PREC_MIXED), 10),
            "complex64_bf16_projectors": event_time_ms(
                torch, prob.ctx.stream, lambda: prob.ctx.apply_H(Xh32, Yh32, prec=PW_PREC_MIXED_BF16), 10)}

    # ---- H.X FFT apply (local part, 64 bands), its own context without projectors
    mil = prob.ctx.get_miller()
    nst = len({(a, b) for a, b, _ in mil})
    nb = w.block
    loc = PlaneWaveProblem(w.cell, w.kfrac, w.ecut, w.n, w.vgrid, None, (), None, nbands=nb,
                           block=nb, device=0, prec=PW_PREC_MIXED)
    Xa = torch.randn((nb, npw), dtype=torch.complex128, device="cuda")
    Ya = torch.empty_like(Xa)
    t_fft = event_time_ms(torch, loc.ctx.stream, lambda: loc.ctx.apply_H(Xa, Ya), 20)
    Xa32, Ya32 = Xa.to(torch.complex64), torch.empty((nb, npw), dtype=torch.complex64, device="cuda")
    t_fft32 = event_time_ms(torch, loc.ctx.stream,
                            lambda: loc.ctx.apply_H(Xa32, Ya32, prec=PW_PREC_MIXED), 20)
    bc = 16
    n3 = w.n ** 3
    nzp = 2 * int(np.abs(mil).max()) + 1          # kept z-planes of the plane-first model
    b_alg_survey = nb * (2 * npw * bc + 4 * nzp * w.n ** 2 * bc) + n3 * 8
    b_alg_design = nb * (3 * npw * bc + 4 * nst * w.n * bc) + n3 * 8
    fft_gbs = b_alg_design / (t_fft * 1e-3) / 1e9
    b_alg_design32 = nb * (3 * npw * 8 + 4 * nst * w.n * 8) + n3 * 4
    fft_gbs32 = b_alg_design32 / (t_fft32 * 1e-3) / 1e9

    # ---- Gram GEMM at the Rayleigh-Ritz shape: [X P W]^H [HX HP HW], 192 x 192, K = npw
    ncol = 3 * w.block
    Z = torch.randn((ncol, npw), dtype=torch.complex128, device="cuda")
    HZ = torch.randn((ncol, npw), dtype=torch.complex128, device="cuda")
    G = torch.empty((ncol, ncol), dtype=torch.complex128, device="cuda")
    t_gram = event_time_ms(torch, prob.ctx.stream, lambda: prob.ctx.gram(Z, HZ, G), 20)
    gram_flops = 8.0 * ncol * ncol * npw
    gram_tflops = gram_flops / (t_gram * 1e-3) / 1e12
    # the same Gram on complex64 blocks (the mixed form's Rayleigh-Ritz; FP32 MFMA)
    Z32, HZ32 = Z.to(torch.complex64), HZ.to(torch.complex64)
    t_gram32 = event_time_ms(torch, prob.ctx.stream, lambda: prob.ctx.gram(Z32, HZ32, G), 20)
    gram32_tflops = gram_flops / (t_gram32 * 1e-3) / 1e12

    # ---- small dense eigensolver at the Rayleigh-Ritz shape (192 x 192, lowest 64)
    rng = np.random.default_rng(0)
    Mh = rng.standard_normal((ncol, ncol)) + 1j * rng.standard_normal((ncol, ncol))
    Ah = torch.from_numpy(np.ascontiguousarray((Mh + Mh.conj().T).T)).to("cuda")
    Aw = torch.empty_like(Ah)
    wv = torch.empty(w.block, dtype=torch.float64, device="cuda")
    Vv = torch.empty((w.block, ncol), dtype=torch.complex128, device="cuda")

    def eig_once():
        Aw.copy_(Ah)
        prob.ctx.small_eigh(Aw, ncol, w.block, wv, Vv)
    t_eig = event_time_ms(torch, prob.ctx.stream, eig_once, 10)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    # Householder reduction 16/3 n^3 + back-transform 8 n^2 k real FLOPs
    eig_flops = 16.0 / 3.0 * ncol ** 3 + 8.0 * ncol ** 2 * w.block
    eig_tflops = eig_flops / (t_eig * 1e-3) / 1e12

    roofs = {
        "dense": dict(bound="alu", kernel="pw_small_eigh 192x192 lowest 64 (k_hetrd_la<6, double>, k_stebz_w<3>, "
                      "k_stein_w<3>, k_orth_chol2, k_unmtr_w<3>, k_check_w)", achieved=eig_tflops, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                      frac=eig_tflops / FP64_PEAK_TFLOPS, traffic=TRAFFIC_MEASURED["dense"],
                      algorithmic=f"{eig_flops:.3e} FLOP per call (16/3 n^3 + 8 n^2 k)", launch_ms=t_eig,
                      # the reduction is one workgroup, i.e. one CU, by construction
                      one_cu_peak=FP64_PEAK_TFLOPS / n_cu, one_cu_frac=eig_tflops / (FP64_PEAK_TFLOPS / n_cu)),
        "gemm": dict(bound="mfma", kernel="k_gemm_tn_lds (+k_reduce_parts), Rayleigh-Ritz Gram 192x192, "
                     "K=34181",
                     achieved=gram_tflops, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                     frac=gram_tflops / FP64_PEAK_TFLOPS, traffic=TRAFFIC_MEASURED["gemm"],
                     algorithmic=f"{gram_flops:.3e} FLOP per launch (8 p q K)", launch_ms=t_gram),
        "gemm_complex64": dict(bound="mfma", kernel="k_gemm_tn_lds<float> (+k_reduce_parts), Rayleigh-Ritz "
                               "Gram 192x192, K=34181, complex64 blocks on FP32 MFMA",
                               achieved=gram32_tflops, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                               frac=gram32_tflops / FP32_PEAK_TFLOPS,
                               traffic=TRAFFIC_MEASURED["gemm_complex64"],
                               algorithmic=f"{gram_flops:.3e} FLOP per launch (8 p q K)",
                               launch_ms=t_gram32),
        "apply": dict(bound="hbm", kernel="k_zinv + k_plane + k_zfwd (local H.X, 64 bands)",
                      achieved=fft_gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=fft_gbs / HBM_PEAK_GBS,
                      traffic=TRAFFIC_MEASURED["apply"], algorithmic=f"{b_alg_design:.3e} B per 64-band apply",
                      launch_ms=t_fft),
    }
    # ---- batched k-points: the ten irreducible k-points of the 4x4x4 grid of the
    # L = 16 bohr cell (256 bands each, blocks of 32), solved concurrently
    batched = None
    if args.batch_steps > 0 and not args.roofline_only:
        wk = make_kpoint_workloads()
        probs = [PlaneWaveProblem.from_workload(x, device=0, stream=torch.cuda.Stream(),
                                                prec=PW_PREC_MIXED) for x in wk]
        batched = {"workload": "kpts_l16: 10 k-points, L=16, Ecut=15, 72^3, 64 wells, 256 proj.",
                   "nbands_total": sum(x.nbands for x in wk),
                   "npw": [p.npw for p in probs]}
        res_eigs = {}
        for name, prec in (("fp64", PW_PREC_FP64), ("mixed", PW_PREC_MIXED)):
            solve_batch(probs[:2], wk[0].tol, prec=prec)       # first-call set-up
            torch.cuda.synchronize()
            ts = []
            for i in range(args.batch_steps):
                t0 = time.perf_counter()
                eigs, _, _ = solve_batch(probs, wk[0].tol, prec=prec)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            res_eigs[name] = np.concatenate(eigs)
            batched[name] = {"value": batched["nbands_total"] / float(np.mean(ts)),
                             "unit": "eigenpairs/s", "ms_per_batch": 1e3 * float(np.mean(ts)),
                             "max_residual": float(max(p.ctx.get_residuals(p.nbands).max()
                                                       for p in probs))}
            log(f"batched k-points {name}: {1e3 * np.mean(ts):.0f} ms")
        batched["max_abs_eig_diff_mixed_vs_fp64_ha"] = float(np.abs(res_eigs["mixed"] -
                                                                    res_eigs["fp64"]).max())
        del probs
        # multi-k-point H.X: the ten k-points' full H (local + projectors) on 32 bands in
        # one pw_apply_H_batch (one launch per FFT pass over all (k, band) items) against
        # ten pw_apply_H calls on the same stream
        from paper_0707_3405_amd import apply_H_batch
        sb = torch.cuda.Stream()
        probs = [PlaneWaveProblem.from_workload(x, device=0, stream=sb, prec=PW_PREC_MIXED) for x in wk]
        ctxs = [p.ctx for p in probs]
        nbk = wk[0].block
        batched["apply_batch"] = {"bands_per_kpoint": nbk}
        for name, prec, dt in (("fp64", PW_PREC_FP64, torch.complex128),
                               ("mixed", PW_PREC_MIXED, torch.complex64)):
            Xk = [torch.randn((nbk, p.npw), dtype=dt, device="cuda") for p in probs]
            Yk = [torch.empty_like(x) for x in Xk]
            t_b = event_time_ms(torch, sb, lambda: apply_H_batch(ctxs, Xk, Yk, prec=prec), 10)
            t_s = event_time_ms(torch, sb, lambda: [c.apply_H(x, y, prec=prec) for c, x, y in zip(ctxs, Xk, Yk)],
                                10)
            batched["apply_batch"][name] = {"batched_ms": t_b, "separate_ms": t_s}
            log(f"multi-k H.X {name}: batched {t_b:.3f} ms, separate {t_s:.3f} ms")
        del probs, ctxs

    # ---- served stream sample: Poisson arrivals (4/s) of cells with L in [8, 16] bohr,
    # Ecut in [5, 15] Ha, bands ~ atoms, random k, FP64 or mixed
    served = None
    if args.serve_requests > 0 and not args.roofline_only:
        from paper_0707_3405_amd.serve import Server, poisson_arrivals
        from workloads import make_request
        arr = poisson_arrivals(args.serve_requests, 4.0)
        reqs = []
        for i in range(args.serve_requests):
            wr, mixed_r = make_request(i, L_range=(8.0, 16.0), ecut_range=(5.0, 15.0))
            reqs.append((float(arr[i]), wr, PW_PREC_MIXED if mixed_r else PW_PREC_FP64))
        _, served = Server(max_active=8).run(reqs)
        served["sample"] = ("Poisson arrivals at 4/s; L ~ U[8,16] bohr, Ecut ~ U[5,15] Ha, "
                            "round(0.0135 L^3) wells with 4 projectors, bands 32 round(5.5 atoms/32), "
                            "k ~ U[0,1)^3, FP64 or mixed with p = 1/2")
        log(f"served stream: {served['solves_per_s']:.2f} solves/s, p99 {served['latency_p99_s']:.3f} s")

    # ---- served stream over the full request range (L ~ U[8, 24] bohr, Ecut ~ U[5, 25] Ha,
    # up to 1024 bands): capacity measured first on a closed-loop calibration set, then
    # Poisson arrivals at 0.7 x that capacity
    served_full = None
    if args.serve_full_requests > 0 and not args.roofline_only:
        from paper_0707_3405_amd.serve import Server, poisson_arrivals
        from workloads import make_request

        def reqs_of(ids, times):
            out = []
            for t, i in zip(times, ids):
                wr, mixed_r = make_request(i)
                out.append((float(t), wr, PW_PREC_MIXED if mixed_r else PW_PREC_FP64))
            return out
        calib_ids = list(range(500, 510))
        t0 = time.perf_counter()
        _, calib = Server(max_active=8).run(reqs_of(calib_ids, [0.0] * len(calib_ids)))
        capacity = calib["solves_per_s"]
        rate = 0.7 * capacity
        nreq = args.serve_full_requests
        arr = poisson_arrivals(nreq, rate)
        keep = int(np.searchsorted(arr, args.serve_full_cap_s, side="right"))
        results_f, served_full = Server(max_active=8).run(reqs_of(range(keep), arr[:keep]))
        served_full["capacity_solves_per_s"] = capacity
        served_full["capacity_sample"] = (f"{len(calib_ids)} requests (stream indices 500-509) admitted "
                                          f"at once, closed loop, {calib['eigenpairs_per_s']:.1f} eigenpairs/s")
        served_full["arrival_rate_per_s"] = rate
        served_full["npw_range"] = [int(min(r.get("npw", 0) for r in results_f)),
                                    int(max(r.get("npw", 0) for r in results_f))]
        served_full["nbands_range"] = [int(min(r["nbands"] for r in results_f)),
                                       int(max(r["nbands"] for r in results_f))]
        served_full["sample"] = (f"{keep} requests, Poisson arrivals at 0.7 x the measured capacity; "
                                 "L ~ U[8,24] bohr, Ecut ~ U[5,25] Ha, round(0.0135 L^3) wells with 4 "
                                 "projectors, bands 32 round(5.5 atoms/32) in [32, 1024], k ~ U[0,1)^3, "
                                 "FP64 or mixed with p = 1/2")
        served_full["leg_seconds"] = time.perf_counter() - t0
        log(f"served stream (full range): {served_full['solves_per_s']:.2f} solves/s, "
            f"p50 {served_full['latency_p50_s']:.2f} s, p99 {served_full['latency_p99_s']:.2f} s, "
            f"{keep} requests")

    if args.roofline_only:
        # plain device copy of known size: reference for HBM byte counters
        src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        t_copy = event_time_ms(torch, torch.cuda.current_stream(), lambda: dst.copy_(src), 5)
        print(json.dumps({"roofline_all": roofs, "copy_256MiB_ms": t_copy,
                          "copy_256MiB_gbs": 2 * (1 << 28) / (t_copy * 1e-3) / 1e9}), flush=True)
        return
    dominant = max(("dense", "gemm", "apply"), key=lambda k: phases["ms_" + k])
    roof = roofs[dominant]

    out = {
        "metric": "LOBPCG eigenpairs/s + H·X FFT GB/s, mixed vs FP64; p50/p99 solve latency",
        "value": value,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "npw": npw, "fft": w.n, "nbands": w.nbands,
                   "block": w.block, "nproj": w.nproj, "tol": w.tol, "precision": "fp64",
                   "k": list(w.kfrac)},
        "hx_fft_gbs": fft_gbs,
        "hx_fft_ms_per_64_bands": t_fft,
        "hx_fft_gbs_survey_byte_model": b_alg_survey / (t_fft * 1e-3) / 1e9,
        "hx_fft_gbs_complex64": fft_gbs32,
        "hx_fft_ms_per_64_bands_complex64": t_fft32,
        "gram_tflops": gram_tflops,
        "gram_ms": t_gram,
        "gram_complex64_tflops": gram32_tflops,
        "gram_complex64_ms": t_gram32,
        "latency_p50_ms": float(np.percentile(np.array(lat) * 1e3, 50)),
        "latency_p99_ms": float(np.percentile(np.array(lat) * 1e3, 99)),
        "iterations": stats["iterations"],
        "blocks": stats["blocks"],
        "phase_ms": phases,
        "max_residual": float(res.max()),
        "abs_eig_err_vs_oracle_ha": fp64_err,
        "roofline": roof,
        "roofline_all": roofs,
        "mixed": mixed,
        "mixed_bf16": mixed_bf16,
        "mixed_bf16_gram": mixed_bf16_gram,
        "mixed_fp32_rr": mixed_fp32_rr,
        "generalized": generalized,
        "autotuned": tuned,
        "hx_full_ms_per_64_bands": hx_full,
        "batched_kpoints": batched,
        "served": served,
        "served_full_range": served_full,
    }
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        omp = os.environ.get("OMP_NUM_THREADS")
        if omp and omp.isdigit():
            cores = min(cores, int(omp))
        log(f"cpu baseline on {cores} threads ...")
        out["cpu_baseline"] = cpu_baseline(w, stats["iterations"], cores, args.cpu_iters,
                                           full_block=bool(args.cpu_full_block))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
