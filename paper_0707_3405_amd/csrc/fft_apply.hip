// Plane-wave H.X apply, kinetic + local part (hot-path rows a2-a6).
//
// Sec. 2.2 (iii) and sec. 4.1: the local potential is applied by transforming
// each band to real space on the FFT grid (coefficients zero-padded outside
// the sphere), multiplying by V(r), and transforming back.  Here the 3-D
// transform is pruned to the sphere and split into three passes over a
// "stick" buffer S[band][z][stick] (a stick is one (n_x, n_y) column of the
// sphere):
//
//   pass 1 (k_zinv):  per (band, group of sticks): scatter the sphere
//                     coefficients of each stick into LDS, inverse z-FFT,
//                     write S (only sticks, not the full grid).
//   pass 2 (k_plane): per (band, z-plane): scatter the plane's sticks into the
//                     kept x-columns, inverse y-FFT on those columns, then row
//                     by row inverse x-FFT (its first stage reading the kept
//                     columns directly), multiply by V(r)/N^3, forward
//                     x-FFT (keeping only the kept columns), forward y-FFT,
//                     gather the sticks back into S.
//   pass 3 (k_zfwd):  per (band, group of sticks): forward z-FFT, gather the
//                     sphere points, add the kinetic term 1/2|k+G|^2 X.
//
// Sign convention: grid <- G uses exp(+2 pi i n.j/N) with no scale, G <- grid
// uses exp(-2 pi i n.j/N) with 1/N^3 (folded into the stored potential).
#include "fft_core.h"
#include "pw_internal.h"

namespace pw {
namespace {

using namespace fft;

constexpr int kThreads = 256;
// Workgroup size of the plane pass.  An FP64 plane (up to 150 KB of LDS) runs
// alone on its CU, so it takes 1024 threads (at most 128 VGPRs, no spills up to
// N = 120): twice the work items per phase to hide LDS and FP64 latency.  A
// complex64 plane takes 512 so that two workgroups share a CU.
template <int N, class T>
constexpr int plane_threads() {
    return (sizeof(T) == 8 && N <= 120) ? 1024 : 512;
}
// default row chunk of the plane pass (capped by LDS): 48 rows for FP64; 24
// for complex64, measured faster at N = 96 (0.251 -> 0.239 ms per 64 bands;
// 16, 32 and 48 rows all slower)
constexpr int kPlaneRb = 48;
constexpr int kPlaneRb32 = 24;
constexpr int kRhoThreads = 512;   // workgroup size of the density plane pass
constexpr int kRhoRb = 32;         // row chunk of the density plane pass

// the k-point items of one launch, passed by value (blockIdx.z picks one)
template <class T>
struct ApplyItems {
    FftApplyItem<T> it[kMaxApplyBatch];
};

template <class T>
__device__ __forceinline__ void load_twiddles(cpx<T> *tw_s, const double *tw_g, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        tw_s[i] = cpx<T>{T(tw_g[2 * i]), T(tw_g[2 * i + 1])};
}

// ---- pass 1: inverse z-FFT per stick ---------------------------------------
template <class P, class T>
__global__ void __launch_bounds__(kThreads) k_zinv(const ApplyItems<T> items, int spb) {
    const FftApplyItem<T> &item = items.it[blockIdx.z];
    const SphereDev &sp = item.sp;
    const cpx<T> *__restrict__ X = item.X;
    const int64_t ldx = item.ldx;
    cpx<T> *__restrict__ S = item.S;
    constexpr int N = P::N, LD = N + 1;
    constexpr int R1 = P::R1, R2 = P::R2;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *tw = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = tw + N;

    const int band = blockIdx.y;
    const int s0 = blockIdx.x * spb;
    const int ns = min(spb, sp.nst - s0);
    if (ns <= 0) return;
    const cpx<T> *Xb = X + (int64_t)band * ldx;

    load_twiddles(tw, sp.twid, N);
    for (int i = threadIdx.x; i < ns * LD; i += blockDim.x) buf[i] = cpx<T>{T(0), T(0)};
    __syncthreads();
    const int g0 = sp.st_start[s0];
    const int g1 = sp.st_start[s0 + ns - 1] + sp.st_len[s0 + ns - 1];
    for (int g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
        const int pos = sp.g_map[g];
        const int s = pos / N, z = pos - s * N;
        buf[(s - s0) * LD + z] = Xb[g];
    }
    __syncthreads();
    for (int it = threadIdx.x; it < ns * R2; it += blockDim.x) {
        const int seq = it % ns, n2 = it / ns;
        dit_a<P, +1>(buf + seq * LD, n2, tw);
    }
    __syncthreads();
    cpx<T> *Sb = S + (int64_t)band * N * sp.ldst + s0;
    for (int it = threadIdx.x; it < ns * R1; it += blockDim.x) {
        const int seq = it % ns, k1 = it / ns;
        cpx<T> out[R2];
        dit_b<P, +1>(buf + seq * LD, k1, out);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) Sb[(int64_t)(k1 + R1 * k2) * sp.ldst + seq] = out[k2];
    }
}

// ---- pass 2: per z-plane xy transforms with the potential in between -------
// XCD-aware mapping: consecutive hardware workgroup ids go round-robin over
// the 8 XCDs; each XCD is given a contiguous range of (plane, band) work so
// that all bands of one plane share that XCD's L2 copy of V(z, :, :).
__device__ __forceinline__ int xcd_logical(int lin, int total) {
    const int q = total / 8, r = total % 8;
    const int xcd = lin % 8, local = lin / 8;
    return xcd * q + min(xcd, r) + local;
}

template <class P, class T>
__global__ void __launch_bounds__((plane_threads<P::N, T>())) k_plane(const ApplyItems<T> items,
                                                                       const T *__restrict__ vperm, int nb, int rb) {
    const FftApplyItem<T> &item = items.it[blockIdx.z];
    const SphereDev &sp = item.sp;
    cpx<T> *__restrict__ S = item.S;
    constexpr int N = P::N, LD = N + 1;
    constexpr int R1 = P::R1, R2 = P::R2;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *tw = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *A = tw + N;                 // [ncx][LD], y along the row
    cpx<T> *R = A + sp.ncx * LD;        // [rb][LD], x along the row

    const int total = N * nb;
    const int lid = xcd_logical(blockIdx.x, total);
    const int z = lid / nb, band = lid % nb;
    const int ncx = sp.ncx;
    cpx<T> *Sp = S + ((int64_t)band * N + z) * sp.ldst;
    const T *Vz = vperm + (int64_t)z * N * N;

    load_twiddles(tw, sp.twid, N);
    for (int i = threadIdx.x; i < ncx * LD; i += blockDim.x) A[i] = cpx<T>{T(0), T(0)};
    __syncthreads();
    for (int s = threadIdx.x; s < sp.nst; s += blockDim.x) A[sp.st_xc[s] * LD + sp.st_y[s]] = Sp[s];
    __syncthreads();
    // inverse y-FFT on the kept columns (natural -> digit-reversed)
    for (int it = threadIdx.x; it < ncx * R2; it += blockDim.x) {
        const int c = it % ncx, n2 = it / ncx;
        dit_a<P, +1>(A + c * LD, n2, tw);
    }
    __syncthreads();
    for (int it = threadIdx.x; it < ncx * R1; it += blockDim.x) {
        const int c = it % ncx, k1 = it / ncx;
        cpx<T> out[R2];
        dit_b<P, +1>(A + c * LD, k1, out);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) A[c * LD + k1 * R2 + k2] = out[k2];
    }
    __syncthreads();
    // rows: x-iFFT, * V, x-FFT, in chunks of rb rows
    const int xmin_g = ((sp.xmin % N) + N) % N;
    for (int y0 = 0; y0 < N; y0 += rb) {
        const int nr = min(rb, N - y0);
        // first inverse x stage, its inputs read straight from the kept columns
        // of A (the other x are zero): no row buffer fill, no barrier for it
        // (n2 runs fastest over the lanes: the reads of A then step by whole
        // columns, conflict-free, where rows of one x stepped by R2 and collided)
        for (int it = threadIdx.x; it < nr * R2; it += blockDim.x) {
            const int n2 = it % R2, r = it / R2;
            const int ypos = digit_rev<P>(y0 + r);
            cpx<T> u[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) {
                int xc = n1 * R2 + n2 - xmin_g;
                xc += (xc < 0) ? N : 0;
                u[n1] = (xc < ncx) ? A[xc * LD + ypos] : cpx<T>{T(0), T(0)};
            }
            dit_a_regs<P, +1>(u, n2, tw);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) R[r * LD + k1 * R2 + n2] = u[k1];
        }
        __syncthreads();
        // second inverse stage, V multiply and first forward stage act on the
        // same R2 values of item k1: fused in registers
        for (int it = threadIdx.x; it < nr * R1; it += blockDim.x) {
            const int r = it % nr, k1 = it / nr;
            cpx<T> out[R2];
            dit_b<P, +1>(R + r * LD, k1, out);
            const T *vrow = Vz + (int64_t)(y0 + r) * N + k1 * R2;
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) out[k2] = cscale(out[k2], vrow[k2]);
            Dft<R2, -1, T>::run(out);
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) R[r * LD + k1 * R2 + n2] = out[n2];
        }
        __syncthreads();
        for (int it = threadIdx.x; it < nr * R2; it += blockDim.x) {   // n2 fastest, as above
            const int n2 = it % R2, r = it / R2;
            cpx<T> out[R1];
            dif_a<P, -1>(R + r * LD, n2, tw, out);
            const int ypos = digit_rev<P>(y0 + r);
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) {
                const int x = n1 * R2 + n2;
                int xc = x - xmin_g;
                xc += (xc < 0) ? N : 0;
                if (xc < ncx) A[xc * LD + ypos] = out[n1];
            }
        }
        __syncthreads();
    }
    // forward y-FFT on the kept columns (digit-reversed -> natural)
    for (int it = threadIdx.x; it < ncx * R1; it += blockDim.x) {
        const int c = it % ncx, k1 = it / ncx;
        dif_b<P, -1>(A + c * LD, k1);
    }
    __syncthreads();
    for (int it = threadIdx.x; it < ncx * R2; it += blockDim.x) {
        const int c = it % ncx, n2 = it / ncx;
        cpx<T> out[R1];
        dif_a<P, -1>(A + c * LD, n2, tw, out);
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) A[c * LD + n1 * R2 + n2] = out[n1];
    }
    __syncthreads();
    for (int s = threadIdx.x; s < sp.nst; s += blockDim.x) Sp[s] = A[sp.st_xc[s] * LD + sp.st_y[s]];
}

// ---- density: per z-plane inverse xy transforms, occ |psi|^2 accumulated -----
// rho_zyx[z][y][x] += sum_b occ[b] |psi_b(x, y, z)|^2 over the nb bands of the
// stick buffer (psi without the 1/sqrt(Omega) factor).  One workgroup owns one
// plane and adds the bands in order, so no two threads write one element and
// the sum is deterministic.
template <int N, class T>
__global__ void __launch_bounds__(kRhoThreads)
    k_plane_rho(SphereDev sp, const cpx<T> *__restrict__ S, int nb, const double *__restrict__ occ,
                double *__restrict__ rho_zyx, int rb) {
    using P = Split<N>;   // the density pass uses the default split (its output is in natural order)
    constexpr int LD = N + 1;
    constexpr int R1 = P::R1, R2 = P::R2;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *tw = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *A = tw + N;                 // [ncx][LD], y along the row
    cpx<T> *R = A + sp.ncx * LD;        // [rb][LD], x along the row
    const int z = blockIdx.x;
    const int ncx = sp.ncx;
    const int xmin_g = ((sp.xmin % N) + N) % N;
    double *rz = rho_zyx + (int64_t)z * N * N;
    load_twiddles(tw, sp.twid, N);
    for (int band = 0; band < nb; ++band) {
        const double f = occ[band];
        const cpx<T> *Sp = S + ((int64_t)band * N + z) * sp.ldst;
        __syncthreads();
        for (int i = threadIdx.x; i < ncx * LD; i += blockDim.x) A[i] = cpx<T>{T(0), T(0)};
        __syncthreads();
        for (int s = threadIdx.x; s < sp.nst; s += blockDim.x) A[sp.st_xc[s] * LD + sp.st_y[s]] = Sp[s];
        __syncthreads();
        for (int it = threadIdx.x; it < ncx * R2; it += blockDim.x) {
            const int c = it % ncx, n2 = it / ncx;
            dit_a<P, +1>(A + c * LD, n2, tw);
        }
        __syncthreads();
        for (int it = threadIdx.x; it < ncx * R1; it += blockDim.x) {
            const int c = it % ncx, k1 = it / ncx;
            cpx<T> out[R2];
            dit_b<P, +1>(A + c * LD, k1, out);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) A[c * LD + k1 * R2 + k2] = out[k2];
        }
        __syncthreads();
        for (int y0 = 0; y0 < N; y0 += rb) {
            const int nr = min(rb, N - y0);
            for (int i = threadIdx.x; i < nr * N; i += blockDim.x) {
                const int r = i / N, x = i - r * N;
                int xc = x - xmin_g;
                xc += (xc < 0) ? N : 0;
                R[r * LD + x] = (xc < ncx) ? A[xc * LD + digit_rev<P>(y0 + r)] : cpx<T>{T(0), T(0)};
            }
            __syncthreads();
            for (int it = threadIdx.x; it < nr * R2; it += blockDim.x) {
                const int r = it % nr, n2 = it / nr;
                dit_a<P, +1>(R + r * LD, n2, tw);
            }
            __syncthreads();
            for (int it = threadIdx.x; it < nr * R1; it += blockDim.x) {
                const int r = it % nr, k1 = it / nr;
                cpx<T> out[R2];
                dit_b<P, +1>(R + r * LD, k1, out);
                double *row = rz + (int64_t)(y0 + r) * N;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) {
                    const int x = freq_at<P>(k1 * R2 + k2);
                    const double a = (double)out[k2].x, b = (double)out[k2].y;
                    row[x] += f * (a * a + b * b);
                }
            }
            __syncthreads();
        }
    }
}

// rho[x][y][z] = rho_zyx[z][y][x] * scale
__global__ void k_rho_permute(const double *__restrict__ rho_zyx, int n, double scale,
                              double *__restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * n * n) return;
    const int z = (int)(i % n), y = (int)((i / n) % n), x = (int)(i / ((int64_t)n * n));
    rho[i] = rho_zyx[((int64_t)z * n + y) * n + x] * scale;
}

// ---- pass 3: forward z-FFT per stick, gather, kinetic -----------------------
template <class P, class T>
__global__ void __launch_bounds__(kThreads) k_zfwd(const ApplyItems<T> items, int spb) {
    const FftApplyItem<T> &item = items.it[blockIdx.z];
    const SphereDev &sp = item.sp;
    const cpx<T> *__restrict__ S = item.S;
    const cpx<T> *__restrict__ X = item.X;
    const int64_t ldx = item.ldx;
    cpx<T> *__restrict__ Y = item.Y;
    const int64_t ldy = item.ldy;
    constexpr int N = P::N, LD = N + 1;
    constexpr int R1 = P::R1, R2 = P::R2;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *tw = reinterpret_cast<cpx<T> *>(smem_raw);
    cpx<T> *buf = tw + N;

    const int band = blockIdx.y;
    const int s0 = blockIdx.x * spb;
    const int ns = min(spb, sp.nst - s0);
    if (ns <= 0) return;
    load_twiddles(tw, sp.twid, N);
    const cpx<T> *Sb = S + (int64_t)band * N * sp.ldst + s0;
    for (int i = threadIdx.x; i < ns * N; i += blockDim.x) {
        const int z = i / ns, seq = i - z * ns;
        buf[seq * LD + digit_rev<P>(z)] = Sb[(int64_t)z * sp.ldst + seq];
    }
    __syncthreads();
    for (int it = threadIdx.x; it < ns * R1; it += blockDim.x) {
        const int seq = it % ns, k1 = it / ns;
        dif_b<P, -1>(buf + seq * LD, k1);
    }
    __syncthreads();
    for (int it = threadIdx.x; it < ns * R2; it += blockDim.x) {
        const int seq = it % ns, n2 = it / ns;
        cpx<T> out[R1];
        dif_a<P, -1>(buf + seq * LD, n2, tw, out);
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) buf[seq * LD + n1 * R2 + n2] = out[n1];
    }
    __syncthreads();
    const int g0 = sp.st_start[s0];
    const int g1 = sp.st_start[s0 + ns - 1] + sp.st_len[s0 + ns - 1];
    const cpx<T> *Xb = X + (int64_t)band * ldx;
    cpx<T> *Yb = Y + (int64_t)band * ldy;
    for (int g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
        const int pos = sp.g_map[g];
        const int s = pos / N, zz = pos - s * N;
        const cpx<T> v = buf[(s - s0) * LD + zz];
        const cpx<T> x = Xb[g];
        const T t = T(sp.kin[g]);
        Yb[g] = cpx<T>{v.x + t * x.x, v.y + t * x.y};
    }
}

// ---- potential layout: vperm[z][y][p] = scale * V[x(p)][y][z] ---------------
// p is the digit-reversed x position produced by the inverse x-FFT of pass 2
// (it depends on the radix split P), so the multiply in pass 2 reads V
// contiguously.
template <class P>
__global__ void k_permute_v(const double *__restrict__ v, double scale, double *__restrict__ out,
                            int *bad) {
    constexpr int N = P::N;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * N * N) return;
    const int p = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / ((int64_t)N * N));
    const int x = freq_at<P>(p);
    const double val = v[((int64_t)x * N + y) * N + z];
    if (!isfinite(val)) atomicOr(bad, 1);
    out[i] = val * scale;
}

// the same potential moved from the layout of split PF to that of split PT
template <class PF, class PT>
__global__ void k_repermute_v(const double *__restrict__ in, double *__restrict__ out) {
    constexpr int N = PT::N;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * N * N) return;
    const int p = (int)(i % N);
    const int64_t row = i - p;
    out[i] = in[row + digit_rev<PF>(freq_at<PT>(p))];
}

// ---- dispatch ---------------------------------------------------------------
constexpr int kSticksPerBlock = 16;   // default sticks per workgroup of the z passes

template <class P, class T>
void run_apply_split(const ApplyItems<T> &items, int nk, const T *vperm, int nb, hipStream_t st) {
    constexpr int N = P::N;
    const Tuning &tune = thread_tuning();
    const int spb = tune.fft_spb > 0 ? tune.fft_spb : kSticksPerBlock;
    const size_t e = sizeof(cpx<T>);
    const size_t sm13 = (size_t)N * e + (size_t)spb * (N + 1) * e;
    int nst_max = 0, ncx_max = 0;
    for (int k = 0; k < nk; ++k) {
        nst_max = std::max(nst_max, items.it[k].sp.nst);
        ncx_max = std::max(ncx_max, items.it[k].sp.ncx);
    }
    dim3 g13((nst_max + spb - 1) / spb, nb, nk);
    // pass 2 LDS: twiddles + kept columns + row chunk; largest row chunk that
    // keeps the workgroup under 150 KB.
    const size_t base2 = (size_t)N * e + (size_t)ncx_max * (N + 1) * e;
    int rb = tune.fft_rb > 0 ? tune.fft_rb : (sizeof(T) == 4 ? kPlaneRb32 : kPlaneRb);
    auto sm2_of = [&](int r) { return base2 + (size_t)r * (N + 1) * e; };
    while (rb > 1 && sm2_of(rb) > 150 * 1024) rb /= 2;
    if (rb > N) rb = N;
    const size_t sm2 = sm2_of(rb);
    PW_REQUIRE(sm2 <= 160 * 1024, PW_ERR_ARG, "FFT plane does not fit in LDS");
    ensure_smem_limit((const void *)k_zinv<P, T>, sm13);
    ensure_smem_limit((const void *)k_plane<P, T>, sm2);
    ensure_smem_limit((const void *)k_zfwd<P, T>, sm13);
    hipLaunchKernelGGL((k_zinv<P, T>), g13, dim3(kThreads), sm13, st, items, spb);
    hipLaunchKernelGGL((k_plane<P, T>), dim3(N * nb, 1, nk), dim3(plane_threads<N, T>()), sm2, st, items, vperm,
                       nb, rb);
    hipLaunchKernelGGL((k_zfwd<P, T>), g13, dim3(kThreads), sm13, st, items, spb);
    PW_HIP(hipGetLastError());
}

// host-side compile-time loop over the candidate second factors 2..16
template <int B, int E, class F>
void host_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        host_for<B + 1, E>(static_cast<F &&>(f));
    }
}

// the split a context's tuning selects for length N (0: the default)
int effective_r2(int n, int r2) { return r2 > 0 ? r2 : choose_r2(n); }

template <int N, class T>
void run_apply(const ApplyItems<T> &items, int nk, const T *vperm, int nb, hipStream_t st) {
    const int r2 = effective_r2(N, thread_tuning().fft_r2);
    bool done = false;
    host_for<2, 17>([&](auto R) {
        constexpr int r = R;
        if constexpr (split_ok(N, r)) {
            if (!done && r == r2) {
                run_apply_split<Split<N, r>, T>(items, nk, vperm, nb, st);
                done = true;
            }
        }
    });
    PW_REQUIRE(done, PW_ERR_ARG, "radix split not available for this FFT length");
}

#define PW_FFT_SIZES(X) X(16) X(20) X(24) X(32) X(36) X(40) X(48) X(60) X(64) X(72) X(80) X(96) X(108) X(120) X(128)

}  // namespace

bool fft_size_supported(int n) {
#define PW_CASE(NN) if (n == NN) return true;
    PW_FFT_SIZES(PW_CASE)
#undef PW_CASE
    return false;
}

std::vector<int> fft_supported_sizes() {
    std::vector<int> v;
#define PW_CASE(NN) v.push_back(NN);
    PW_FFT_SIZES(PW_CASE)
#undef PW_CASE
    return v;
}

template <int N>
void permute_for(int r2, const double *v, double scale, double *v_zyx, int *bad, hipStream_t st) {
    const int64_t tot = (int64_t)N * N * N;
    const dim3 grid((unsigned)((tot + 255) / 256));
    bool done = false;
    host_for<2, 17>([&](auto R) {
        constexpr int r = R;
        if constexpr (split_ok(N, r)) {
            if (!done && r == r2) {
                hipLaunchKernelGGL((k_permute_v<Split<N, r>>), grid, dim3(256), 0, st, v, scale, v_zyx, bad);
                done = true;
            }
        }
    });
    PW_REQUIRE(done, PW_ERR_ARG, "radix split not available for this FFT length");
}

template <int N>
void repermute_for(int r2_from, int r2_to, const double *in, double *out, hipStream_t st) {
    const int64_t tot = (int64_t)N * N * N;
    const dim3 grid((unsigned)((tot + 255) / 256));
    bool done = false;
    host_for<2, 17>([&](auto RF) {
        constexpr int rf = RF;
        if constexpr (split_ok(N, rf)) {
            host_for<2, 17>([&](auto RT) {
                constexpr int rt = RT;
                if constexpr (split_ok(N, rt)) {
                    if (!done && rf == r2_from && rt == r2_to) {
                        hipLaunchKernelGGL((k_repermute_v<Split<N, rf>, Split<N, rt>>), grid, dim3(256), 0, st,
                                           in, out);
                        done = true;
                    }
                }
            });
        }
    });
    PW_REQUIRE(done, PW_ERR_ARG, "radix split not available for this FFT length");
}

void launch_permute_potential(const double *v, int n, double scale, double *v_zyx, int *bad, int r2,
                              hipStream_t st) {
    switch (n) {
#define PW_CASE(NN)                                                              \
    case NN:                                                                     \
        permute_for<NN>(effective_r2(NN, r2), v, scale, v_zyx, bad, st);        \
        break;
        PW_FFT_SIZES(PW_CASE)
#undef PW_CASE
        default:
            throw Error{PW_ERR_ARG, "unsupported FFT size"};
    }
    PW_HIP(hipGetLastError());
}

void launch_repermute_potential(const double *in, int n, int r2_from, int r2_to, double *out,
                                hipStream_t st) {
    switch (n) {
#define PW_CASE(NN)                                                                                 \
    case NN:                                                                                        \
        repermute_for<NN>(effective_r2(NN, r2_from), effective_r2(NN, r2_to), in, out, st);         \
        break;
        PW_FFT_SIZES(PW_CASE)
#undef PW_CASE
        default:
            throw Error{PW_ERR_ARG, "unsupported FFT size"};
    }
    PW_HIP(hipGetLastError());
}

std::vector<int> fft_radix_splits(int n) {
    std::vector<int> v;
    for (int r = 2; r <= 16; ++r)
        if (split_ok(n, r)) v.push_back(r);
    return v;
}

int fft_default_r2(int n) { return choose_r2(n); }

template <int N>
void run_density(const SphereDev &sp, const cd *X, int64_t ldx, int nb, const double *occ,
                 double *rho_zyx, cd *S, hipStream_t st) {
    const int spb = kSticksPerBlock;
    const size_t e = sizeof(cd);
    const size_t sm1 = (size_t)N * e + (size_t)spb * (N + 1) * e;
    const size_t base2 = (size_t)N * e + (size_t)sp.ncx * (N + 1) * e;
    int rb = kRhoRb;
    while (rb > 1 && base2 + (size_t)rb * (N + 1) * e > 150 * 1024) rb /= 2;
    if (rb > N) rb = N;
    const size_t sm2 = base2 + (size_t)rb * (N + 1) * e;
    PW_REQUIRE(sm2 <= 160 * 1024, PW_ERR_ARG, "FFT plane does not fit in LDS");
    ensure_smem_limit((const void *)k_zinv<Split<N>, double>, sm1);
    ensure_smem_limit((const void *)k_plane_rho<N, double>, sm2);
    ApplyItems<double> items{};
    items.it[0] = FftApplyItem<double>{sp, X, ldx, nullptr, 0, S};
    hipLaunchKernelGGL((k_zinv<Split<N>, double>), dim3((sp.nst + spb - 1) / spb, nb), dim3(kThreads), sm1, st,
                       items, spb);
    hipLaunchKernelGGL((k_plane_rho<N, double>), dim3(N), dim3(kRhoThreads), sm2, st, sp, S, nb, occ,
                       rho_zyx, rb);
    PW_HIP(hipGetLastError());
}

void launch_density_accumulate(const SphereDev &sp, const cd *X, int64_t ldx, int nb,
                               const double *occ, double *rho_zyx, cd *S, hipStream_t st) {
    if (nb <= 0) return;
    switch (sp.n) {
#define PW_CASE(NN)                                                         \
    case NN:                                                                \
        run_density<NN>(sp, X, ldx, nb, occ, rho_zyx, S, st);               \
        return;
        PW_FFT_SIZES(PW_CASE)
#undef PW_CASE
        default:
            throw Error{PW_ERR_ARG, "unsupported FFT size"};
    }
}

void launch_density_finish(const double *rho_zyx, int n, double scale, double *rho, hipStream_t st) {
    const int64_t tot = (int64_t)n * n * n;
    hipLaunchKernelGGL(k_rho_permute, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, rho_zyx, n,
                       scale, rho);
    PW_HIP(hipGetLastError());
}

template <class T>
void fft_apply_impl(const ApplyItems<T> &items, int nk, const T *v_zyx, int nb, hipStream_t st) {
    if (nb <= 0 || nk <= 0) return;
    const int n = items.it[0].sp.n;
    switch (n) {
#define PW_CASE(NN)                                     \
    case NN:                                            \
        run_apply<NN, T>(items, nk, v_zyx, nb, st);     \
        return;
        PW_FFT_SIZES(PW_CASE)
#undef PW_CASE
        default:
            throw Error{PW_ERR_ARG, "unsupported FFT size"};
    }
}

template <class T>
void fft_apply_batch(const FftApplyItem<T> *items, int nk, const T *v_zyx, int nb, hipStream_t st) {
    PW_REQUIRE(nk >= 1 && nk <= kMaxApplyBatch, PW_ERR_ARG, "k-points per batched apply must be in [1, 16]");
    ApplyItems<T> all{};
    for (int k = 0; k < nk; ++k) {
        PW_REQUIRE(items[k].sp.n == items[0].sp.n, PW_ERR_ARG, "batched apply needs one FFT grid");
        all.it[k] = items[k];
    }
    fft_apply_impl(all, nk, v_zyx, nb, st);
}

void launch_fft_apply(const SphereDev &sp, const double *v_zyx, const cd *X, int64_t ldx, cd *Y,
                      int64_t ldy, int nb, cd *S, hipStream_t st) {
    const FftApplyItem<double> it{sp, X, ldx, Y, ldy, S};
    fft_apply_batch(&it, 1, v_zyx, nb, st);
}
void launch_fft_apply(const SphereDev &sp, const float *v_zyx, const cf *X, int64_t ldx, cf *Y,
                      int64_t ldy, int nb, cf *S, hipStream_t st) {
    const FftApplyItem<float> it{sp, X, ldx, Y, ldy, S};
    fft_apply_batch(&it, 1, v_zyx, nb, st);
}
void launch_fft_apply_batch(const FftApplyItem<double> *items, int nk, const double *v_zyx, int nb,
                            hipStream_t st) {
    fft_apply_batch(items, nk, v_zyx, nb, st);
}
void launch_fft_apply_batch(const FftApplyItem<float> *items, int nk, const float *v_zyx, int nb,
                            hipStream_t st) {
    fft_apply_batch(items, nk, v_zyx, nb, st);
}

}  // namespace pw
