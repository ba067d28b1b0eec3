// Small dense FP64 steps of the iteration, each in one workgroup.
//
//  * k_chol_inv: Cholesky factor of a Gram matrix G = R^H R and R^-1, used to
//    orthonormalise a block (W <- W R^-1; BLOPEX-style LOBPCG, sec. 3.2).
//  * k_heev: lowest k eigenpairs of a Hermitian matrix -- the Rayleigh-Ritz
//    eigenproblem of the LOBPCG iteration (sec. 3.2, Algorithm 1; size 3m) and of the final
//    Rayleigh-Ritz over all bands (sec. 3.2, sec. 4.2).  Householder
//    reduction to real tridiagonal form, bisection with Sturm counts,
//    inverse iteration, classical Gram-Schmidt applied twice, back-transform.
#include <algorithm>
#include <cfloat>
#include <type_traits>

#include "pw_internal.h"

namespace pw {
namespace {

__device__ __forceinline__ cd cconj(cd a) { return {a.x, -a.y}; }
__device__ __forceinline__ cd cmulz(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cf cconj(cf a) { return {a.x, -a.y}; }
__device__ __forceinline__ cf cmulz(cf a, cf b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// 1 / d to within an ulp without the division sequence: the hardware
// reciprocal refined by two Newton steps (d finite and normal).  Measured on
// gfx950 over 4M samples: v_rcp_f64 alone is off by up to 4.6e-8 relative,
// one step leaves up to 14 ulp, two steps at most 1 ulp.
__device__ __forceinline__ double rcp_nr(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// FP32: the hardware reciprocal (within 1 ulp) and square root
__device__ __forceinline__ float rcp_nr(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_sqrtf(x); }

// value of v in lane `lane` (uniform), as a wave-uniform value
__device__ __forceinline__ double lane_read(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
__device__ __forceinline__ float lane_read(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Block-wide sum of one double per thread: wave shuffles, then the wave
// partials added in wave order by every thread (deterministic, 2 barriers).
__device__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q];
    __syncthreads();
    return s;
}

// ---- Cholesky + inverse of the factor (n <= 64, in registers) -----------------
// Gaussian elimination without pivoting on the augmented matrix [G | I]: the
// row operations that reduce G (Hermitian positive definite, G = L D L^H) to
// the upper triangle D L^H turn I into L^-1; scaling row j of both by d_j^-1/2
// gives [R | R^-H] with G = R^H R.  Step j subtracts conj(g_ja) / d_j times the
// (unscaled) pivot row from every row a > j, so the only communication is the
// pivot row, broadcast through LDS (double buffered: one barrier per step);
// rows stay unscaled (the augmented half ends as L^-1) and are scaled by
// d_a^-1/2 at the end.  1024 threads as a 32 x 32 grid; thread (ti, tj) holds the 2 x 2 tiles rows
// 2 ti .., columns 2 tj .. of G (upper part used) and of the augmented half.
// A wave covers rows 4w .. 4w + 3 and stops updating once they are all
// eliminated; waves of each SIMD cover rows spread over the matrix, so the
// work per SIMD shrinks with the step.  Rows and columns >= n are padded with
// the identity (inert pivots).
constexpr int kCholMax = 64;

__global__ void __launch_bounds__(1024) k_chol_inv(const cd *__restrict__ G, int64_t ldg, int n,
                                                   cd *__restrict__ Rinv, int64_t ldr, int *status) {
    // pivot rows j, j + 1 of a pair step, double buffered: [buffer][row of the pair][column]
    __shared__ cd pg[2][2][kCholMax];   // G part (columns >= j meaningful)
    __shared__ cd pu[2][2][kCholMax];   // augmented part (columns <= j + 1 meaningful)
    __shared__ double diag[kCholMax];
    const int t = threadIdx.x, ti = t >> 5, tj = t & 31;
    const int a0 = 2 * ti, b0 = 2 * tj;         // rows a0, a0 + 1 form one pivot pair
    const int wrow_last = 4 * (t >> 6) + 3;   // last row of this wave
    cd g[2][2], u[2][2];
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
            const int a = a0 + ia, b = b0 + ib;
            cd v = {a == b ? 1.0 : 0.0, 0.0};
            if (a < n && b < n) {   // Hermitian part of the stored Gram
                const cd x = G[(int64_t)b * ldg + a], y = G[(int64_t)a * ldg + b];
                v = cd{0.5 * (x.x + y.x), 0.5 * (x.y - y.y)};
                if (a == b) v.y = 0.0;
            }
            g[ia][ib] = v;
            u[ia][ib] = cd{a == b ? 1.0 : 0.0, 0.0};
            if (a == b) diag[a] = v.x;
            if (ti == 0) {
                pg[0][ia][b] = v;
                pu[0][ia][b] = u[ia][ib];
            }
        }
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) dmax = fmax(dmax, diag[i]);
    // a tiny diagonal shift keeps a numerically semi-definite Gram factorable
    const double shift = 1e-15 * dmax * n;
    bool fail = false;
    double dpiv[2] = {1.0, 1.0};   // pivots of this thread's rows (rows stay unscaled)
    // two pivots per barrier: every thread forms row j + 1 after pivot j itself
    // from the two broadcast rows (row j + 1 arrives without pivot j applied)
    for (int j = 0; j < n; j += 2) {
        const int bsel = (j >> 1) & 1;
        const cd *r0g = pg[bsel][0], *r1g = pg[bsel][1], *r0u = pu[bsel][0], *r1u = pu[bsel][1];
        double d0 = r0g[j].x + shift;
        if (!(d0 > 1e-300) || !isfinite(d0)) {
            fail = true;
            d0 = 1.0;
        }
        const double inv0 = rcp_nr(d0);
        const cd c01 = r0g[j + 1];
        const cd l = {c01.x * inv0, -c01.y * inv0};   // row j + 1 multiplier of pivot j
        auto r1gp = [&](int c) {                       // row j + 1 of G after pivot j
            const cd pr = cmulz(l, r0g[c]);
            const cd v = r1g[c];
            return cd{v.x - pr.x, v.y - pr.y};
        };
        double d1 = r1gp(j + 1).x + shift;
        if (j + 1 < n && (!(d1 > 1e-300) || !isfinite(d1))) {
            fail = true;
            d1 = 1.0;
        }
        if (j + 1 >= n) d1 = 1.0;
#pragma unroll
        for (int ia = 0; ia < 2; ++ia) {
            if (a0 + ia == j) dpiv[ia] = d0;
            if (a0 + ia == j + 1) dpiv[ia] = d1;
        }
        if (wrow_last > j) {   // rows below pivot j in this wave (uniform per wave)
            const double inv1 = rcp_nr(d1);
            cd m0[2], m1[2];
#pragma unroll
            for (int ia = 0; ia < 2; ++ia) {
                const int a = a0 + ia;
                const cd p0 = r0g[a], p1 = r1gp(a);
                m0[ia] = a > j ? cd{p0.x * inv0, -p0.y * inv0} : cd{0.0, 0.0};
                m1[ia] = a > j + 1 ? cd{p1.x * inv1, -p1.y * inv1} : cd{0.0, 0.0};
            }
            cd g0[2], g1[2], u0[2], u1[2];
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) {
                const int b = b0 + ib;
                g0[ib] = r0g[b];
                g1[ib] = r1gp(b);
                u0[ib] = r0u[b];
                const cd pr = cmulz(l, u0[ib]), v = r1u[b];
                u1[ib] = cd{v.x - pr.x, v.y - pr.y};
            }
#pragma unroll
            for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    const int a = a0 + ia, b = b0 + ib;
                    if (b >= a) {
                        const cd p0 = cmulz(m0[ia], g0[ib]), p1 = cmulz(m1[ia], g1[ib]);
                        g[ia][ib].x -= p0.x + p1.x;
                        g[ia][ib].y -= p0.y + p1.y;
                    }
                    const cd q0 = cmulz(m0[ia], u0[ib]), q1 = cmulz(m1[ia], u1[ib]);
                    u[ia][ib].x -= q0.x + q1.x;
                    u[ia][ib].y -= q0.y + q1.y;
                }
            // the next pair's rows (j + 2 after pivots <= j + 1, j + 3 likewise) to the other buffer
            if (j + 2 < n && a0 == j + 2) {
#pragma unroll
                for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib) {
                        pg[bsel ^ 1][ia][b0 + ib] = g[ia][ib];
                        pu[bsel ^ 1][ia][b0 + ib] = u[ia][ib];
                    }
            }
        }
        __syncthreads();
    }
    // R^-1 (upper) = (R^-H)^H with R^-H = D^-1/2 L^-1
#pragma unroll
    for (int ia = 0; ia < 2; ++ia) {
        const double isd = 1.0 / sqrt(dpiv[ia]);
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
            const int a = a0 + ia, c = b0 + ib;
            if (a < n && c < n) Rinv[(int64_t)a * ldr + c] = cd{u[ia][ib].x * isd, -u[ia][ib].y * isd};
        }
    }
    if (fail && t == 0) atomicOr(status, 1);
}

// ---- Hermitian eigensolver ---------------------------------------------------
// Five stages on the stream:
//   reduction  A = Q T Q^H, T real tridiagonal (lower Householder):
//              k_hetrd_la (1 workgroup, n <= 192) or k_trd_apply + k_trd_step
//   k_stebz_w / k_stebz (k groups)  lowest k eigenvalues of T by 512-point multisection
//   k_stein_w  (k waves)       eigenvectors of T by inverse iteration, in registers (n <= 256)
//   k_stein    (k/E groups)    the same with the LU in LDS (n > 256)
//   k_orth_chol2 / k_orth_chol / k_orth (1 workgroup)  re-orthogonalisation
//   k_unmtr_w / k_unmtr (k/cw groups)  back-transform V = Q Z
//
// ---- multi-workgroup reduction for n > 192 (the final Rayleigh-Ritz) --------
// H_j = I - tau_j v_j v_j^H, A <- H_j^H A H_j, w = tau y - (|tau|^2 / 2)
// Re(v^H y) v, A -= w v^H + v w^H, both triangles of the trailing square kept;
// one column step is two launches:
//   k_trd_apply (many workgroups): on the trailing square [j+1, n)^2 apply the
//     pending rank-2 update of step j-1 and accumulate y = A v_j; a workgroup
//     owns 64 rows (one per lane) and 64 columns (16 per wave), so every
//     partial of y is a plain per-lane sum; partials go to ypart[chunk][row].
//   k_trd_step (one workgroup): y = sum of the chunk partials (fixed order),
//     w_j = tau y - (|tau|^2 / 2) Re(v^H y) v, the pivot column j+1 with the
//     update of step j applied on the fly, d_{j+1}, and the reflector j+1
//     (stored below the subdiagonal of column j+1, beta on the subdiagonal).
// v of consecutive steps alternates between two buffers; rows outside a
// reflector's range are zero in its buffer.
struct TrdState {
    cd *v[2];      // [n] reflectors of even / odd steps
    cd *w;         // [n] w of the last step
    cd *ypart;     // [nchunk][n]
};

__global__ void k_herm_sym(cd *__restrict__ A, int64_t lda, int n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int r = (int)(idx % n), c = (int)(idx / n);
    if (r > c) {
        const cd a = A[(int64_t)c * lda + r], b = A[(int64_t)r * lda + c];
        const cd m = {0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
        A[(int64_t)c * lda + r] = m;
        A[(int64_t)r * lda + c] = cconj(m);
    } else if (r == c) {
        A[(int64_t)c * lda + r].y = 0.0;
    }
}

__global__ void __launch_bounds__(256)
    k_trd_apply(cd *__restrict__ A, int64_t lda, int n, int j, TrdState S) {
    __shared__ cd cvp[64], cwp[64], cv[64];
    __shared__ cd yw[4][64];
    const int r0 = j + 1;
    const int L = n - r0;
    const int nrb = (L + 63) / 64;
    const int rb = blockIdx.x % nrb, cc = blockIdx.x / nrb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const cd *vp = S.v[(j + 1) & 1];   // v_{j-1} (zero for j = 0)
    const cd *v = S.v[j & 1];
    const cd *wp = S.w;                // w_{j-1} (zero for j = 0)
    const int c0 = r0 + 64 * cc;
    if (threadIdx.x < 64) {
        const int c = c0 + threadIdx.x;
        const bool ok = c < n;
        cvp[threadIdx.x] = ok ? vp[c] : cd{0.0, 0.0};
        cwp[threadIdx.x] = ok ? wp[c] : cd{0.0, 0.0};
        cv[threadIdx.x] = ok ? v[c] : cd{0.0, 0.0};
    }
    __syncthreads();
    const int i = r0 + 64 * rb + lane;
    const bool rowok = i < n;
    const cd vpi = rowok ? vp[i] : cd{0.0, 0.0}, wpi = rowok ? wp[i] : cd{0.0, 0.0};
    double yr = 0.0, yi = 0.0;
    if (rowok) {
#pragma unroll 4
        for (int q = 16 * wave; q < 16 * wave + 16; ++q) {
            const int c = c0 + q;
            if (c >= n) break;
            cd a = A[(int64_t)c * lda + i];
            const cd u1 = cmulz(wpi, cconj(cvp[q])), u2 = cmulz(vpi, cconj(cwp[q]));
            a.x -= u1.x + u2.x;
            a.y -= u1.y + u2.y;
            A[(int64_t)c * lda + i] = a;
            const cd vc = cv[q];
            yr += a.x * vc.x - a.y * vc.y;
            yi += a.x * vc.y + a.y * vc.x;
        }
    }
    yw[wave][lane] = cd{yr, yi};
    __syncthreads();
    if (wave == 0 && rowok) {
        const double sr = ((yw[0][lane].x + yw[1][lane].x) + yw[2][lane].x) + yw[3][lane].x;
        const double si = ((yw[0][lane].y + yw[1][lane].y) + yw[2][lane].y) + yw[3][lane].y;
        S.ypart[(int64_t)cc * n + i] = cd{sr, si};
    }
}

// j = -1: no previous step (w = 0), pivot column 0 as stored
__global__ void __launch_bounds__(1024)
    k_trd_step(cd *__restrict__ A, int64_t lda, int n, int j, TrdState S, double *__restrict__ dd,
               double *__restrict__ ee, cd *__restrict__ tau_out) {
    __shared__ double red[16];
    __shared__ cd s_y[1024], s_wl[1024];   // y and w of this step (n <= 1024)
    __shared__ cd s_tau, s_scale;
    __shared__ double s_beta;
    const int t = threadIdx.x, nt = blockDim.x;
    const int p = j + 1;   // pivot column of the next reflector
    cd *v = S.v[j & 1];    // v_j (unused for j = -1)
    cd *vn = S.v[p & 1];   // receives v_{j+1}
    if (j >= 0) {
        const int L = n - p, nch = (L + 63) / 64;
        const cd tau = tau_out[j];
        double part = 0.0;
        for (int i = p + t; i < n; i += nt) {
            double sr = 0.0, si = 0.0;
            for (int q = 0; q < nch; ++q) {
                const cd y = S.ypart[(int64_t)q * n + i];
                sr += y.x;
                si += y.y;
            }
            s_y[i] = cd{sr, si};
            const cd vi = v[i];
            part += vi.x * sr + vi.y * si;
        }
        const double vhy = block_sum(part, red);
        const double nu = 0.5 * (tau.x * tau.x + tau.y * tau.y) * vhy;
        for (int i = t; i < n; i += nt) {
            cd wi = {0.0, 0.0};
            if (i >= p) {
                const cd y = s_y[i], vi = v[i];
                const cd ty = cmulz(tau, y);
                wi = cd{ty.x - nu * vi.x, ty.y - nu * vi.y};
            }
            S.w[i] = wi;
            s_wl[i] = wi;
        }
        __syncthreads();
    } else {
        for (int i = t; i < n; i += nt) {
            S.w[i] = cd{0.0, 0.0};
            s_wl[i] = cd{0.0, 0.0};
        }
        __syncthreads();
    }
    // pivot column p with the update of step j: A(i, p) - v_i conj(w_p) - w_i conj(v_p)
    const cd w1 = s_wl[p];
    const cd v1 = j >= 0 ? v[p] : cd{0.0, 0.0};
    auto col = [&](int i) -> cd {
        cd a = A[(int64_t)p * lda + i];
        if (j >= 0) {
            const cd vi = v[i], wi = s_wl[i];
            const cd u1 = cmulz(vi, cconj(w1)), u2 = cmulz(wi, cconj(v1));
            a.x -= u1.x + u2.x;
            a.y -= u1.y + u2.y;
        }
        return a;
    };
    if (t == 0) dd[p] = col(p).x;
    if (p == n - 1) return;
    double part = 0.0;
    for (int i = p + 2 + t; i < n; i += nt) {
        const cd a = col(i);
        part += a.x * a.x + a.y * a.y;
    }
    const double sigma = block_sum(part, red);
    if (t == 0) {
        const cd alpha = col(p + 1);
        if (sigma == 0.0 && alpha.y == 0.0) {
            s_tau = cd{0.0, 0.0};
            s_beta = alpha.x;
            s_scale = cd{0.0, 0.0};
        } else {
            const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sigma);
            const double beta = alpha.x >= 0.0 ? -nrm : nrm;
            const double dr = alpha.x - beta, di = alpha.y;
            const double ib = 1.0 / beta, iden = 1.0 / (dr * dr + di * di);
            s_tau = cd{-dr * ib, -alpha.y * ib};
            s_scale = cd{dr * iden, -di * iden};
            s_beta = beta;
        }
    }
    __syncthreads();
    const cd tau = s_tau, scale = s_scale;
    const bool reflect = !(tau.x == 0.0 && tau.y == 0.0);
    for (int i = t; i < n; i += nt) {
        cd vv = {0.0, 0.0};
        if (reflect && i == p + 1) vv = cd{1.0, 0.0};
        else if (reflect && i > p + 1) vv = cmulz(col(i), scale);
        vn[i] = vv;
        if (i > p + 1) A[(int64_t)p * lda + i] = vv;   // reflector kept for the back-transform
    }
    if (t == 0) {
        tau_out[p] = tau;
        ee[p] = s_beta;
        A[(int64_t)p * lda + p + 1] = cd{s_beta, 0.0};
    }
}

// ---- register-resident reduction for n <= 32 T (T <= 6) ----------------------
// The same Householder sequence as k_trd_apply / k_trd_step, but the whole
// matrix stays in registers: 1024 threads on a 32 x 32 grid, each holding one
// element of every tile b <= a (off-diagonal tiles are stored once and used
// for both triangles of y = A v; diagonal tiles are stored in full).  Tiles
// whose rows or columns are all finished are skipped.  All sums run in a fixed
// order (deterministic).  The kernel is k_hetrd_la below.
constexpr int kRfMaxT = 6;

template <int B, int E, class F>
__device__ __forceinline__ void unroll_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        unroll_for<B + 1, E>(static_cast<F &&>(f));
    }
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {   // one 32-bit move
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
// sum over the 16 lanes of a DPP row; every lane of the row gets the same value
template <class R>
__device__ __forceinline__ R row16_sum(R x) {
    x += dpp_mov<0xB1>(x);    // quad_perm [1,0,3,2]
    x += dpp_mov<0x4E>(x);    // quad_perm [2,3,0,1]
    x += dpp_mov<0x141>(x);   // row_half_mirror
    x += dpp_mov<0x140>(x);   // row_mirror
    return x;
}
template <class R>
__device__ __forceinline__ R quad_sum(R x) {
    x += dpp_mov<0xB1>(x);
    x += dpp_mov<0x4E>(x);
    return x;
}
// lanes whose DPP row is disabled by ROW_MASK read 0
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_rows(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_rows(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, false));
}
// Wave sum returned as a wave-uniform value, without LDS: the row sums, then
// row_bcast:15 adds row 0 into row 1 and row 2 into row 3, row_bcast:31 adds
// rows 0 + 1 into rows 2 and 3, and lane 63 holds the total (same order of
// additions in every wave).
template <class R>
__device__ __forceinline__ R wave_total(R x) {
    x = row16_sum(x);
    x += dpp_rows<0x142, 0xA>(x);   // row_bcast:15
    x += dpp_rows<0x143, 0xC>(x);   // row_bcast:31
    return lane_read(x, 63);
}

// Look-ahead form of the register-resident reduction (same Householder
// sequence and storage of the reflectors): thread (ti, tj) = (t % 32, t / 32)
// holds A(ti + 32a, tj + 32b) for tiles b <= a, so column c of the matrix is
// held by the 32 lanes of one half-wave.  Step j: every wave applies the rank-2
// update of step j - 1 to its live tiles; the wave holding column j does so
// with raised priority, then forms reflector j from its own registers (norm by
// DPP over the half-wave) and writes it to LDS while the other waves are still
// updating.  Then the partials of y = A v (row partials one per half-wave,
// column partials summed over lane quads by DPP, both in LDS) and w = tau y -
// nu v by four threads per row: three barriers per column instead of four.
// R is the arithmetic type: double, or float for the Rayleigh-Ritz problems of
// the complex64 stage of the mixed iteration (the input is rounded to float,
// the outputs are stored as double).
template <int T, class R>
__global__ void __launch_bounds__(1024)
    k_hetrd_la(cd *__restrict__ A, int64_t lda, int n, double *__restrict__ dd,
               double *__restrict__ ee, cd *__restrict__ tau_out) {
    using C = cpx<R>;
    constexpr int NR = 32 * T;
    constexpr int NE = T * (T + 1) / 2;
    __shared__ C vs[2][NR];          // reflectors of steps of both parities
    __shared__ C ws[NR];             // w of the last step, zero outside its live rows
    __shared__ C pr[32][NR + 1];     // row sums of y, one per half-wave (padded)
    __shared__ C pc[8][NR + 1];      // column sums of y, one per lane quad (padded)
    __shared__ R sv[16];             // per-wave partials of Re(v^H A v)
    __shared__ C s_tau[2];
    const int t = threadIdx.x, ti = t & 31, tj = t >> 5, wave = t >> 6, lane = t & 63;

    C E[NE];
    unroll_for<0, T>([&](auto a_) {
        constexpr int a = a_;
        unroll_for<0, a + 1>([&](auto b_) {
            constexpr int b = b_;
            const int i = ti + 32 * a, c = tj + 32 * b;
            C m = {R(0), R(0)};
            if (i < n && c < n) {   // exact Hermitian part (A + A^H) / 2
                const cd x = A[(int64_t)c * lda + i], y = A[(int64_t)i * lda + c];
                m = C{R(0.5 * (x.x + y.x)), R(0.5 * (x.y - y.y))};
                if (i == c) m.y = R(0);
            }
            E[a * (a + 1) / 2 + b] = m;
        });
    });
    for (int i = t; i < NR; i += 1024) vs[0][i] = vs[1][i] = ws[i] = C{R(0), R(0)};
    __syncthreads();
    // A -= w v^H + v w^H on the live tiles of step jm (v = vs[par], w = ws)
    auto update = [&](int jm, int par) {
        unroll_for<0, T>([&](auto a_) {
            constexpr int a = a_;
            if (32 * a + 31 <= jm) return;
            const C vi = vs[par][ti + 32 * a], wi = ws[ti + 32 * a];
            unroll_for<0, a + 1>([&](auto b_) {
                constexpr int b = b_;
                if (32 * b + 31 <= jm) return;
                const C vj = cconj(vs[par][tj + 32 * b]), wj = cconj(ws[tj + 32 * b]);
                const C u1 = cmulz(wi, vj), u2 = cmulz(vi, wj);
                // whole-element update (member-wise updates kept FP32 elements in scratch)
                const C e = E[a * (a + 1) / 2 + b];
                E[a * (a + 1) / 2 + b] = C{e.x - (u1.x + u2.x), e.y - (u1.y + u2.y)};
            });
        });
    };
    // entry (ti + 32 a, col) of this lane for the column tile jb (zero above it)
    auto col_entry = [&](auto a_, int jb) -> C {
        constexpr int a = decltype(a_)::value;
        // selects by component (an element-wise pick became a dynamically indexed
        // stack array in FP32)
        R xr = R(0), xi = R(0);
        unroll_for<0, a + 1>([&](auto b_) {
            constexpr int b = b_;
            const bool hit = b == jb;
            xr = hit ? E[a * (a + 1) / 2 + b].x : xr;
            xi = hit ? E[a * (a + 1) / 2 + b].y : xi;
        });
        return C{xr, xi};
    };
    for (int j = 0; j + 1 < n; ++j) {
        const int par = j & 1, own = j & 31, jb = j >> 5;
        const bool owner = wave == (own >> 1);   // uniform per wave
        if (owner) __builtin_amdgcn_s_setprio(2);
        if (j > 0) update(j - 1, par ^ 1);
        if (owner) {
            // ---- reflector j from column j, held by half-wave `own` ----
            const int base = (own & 1) * 32;
            R sg = R(0);
            unroll_for<0, T>([&](auto a_) {
                constexpr int a = a_;
                const int r = ti + 32 * a;
                if (r >= j + 2 && r < n) {
                    const C x = col_entry(a_, jb);
                    sg += x.x * x.x + x.y * x.y;
                }
            });
            sg = row16_sum(sg);
            sg += dpp_rows<0x142, 0xA>(sg);   // lanes 31 and 63: the two half-wave totals
            const R sigma = lane_read(sg, base + 31);
            const int a1 = (j + 1) >> 5;
            C xa = {R(0), R(0)}, xd = {R(0), R(0)};
            unroll_for<0, T>([&](auto a_) {
                constexpr int a = a_;
                if (a == a1) xa = col_entry(a_, jb);
                if (a == jb) xd = col_entry(a_, jb);
            });
            const C alpha = {lane_read(xa.x, base + ((j + 1) & 31)), lane_read(xa.y, base + ((j + 1) & 31))};
            const R djj = lane_read(xd.x, base + own);
            C tau, scale;
            R beta;
            if (sigma == R(0) && alpha.y == R(0)) {
                tau = C{R(0), R(0)};
                beta = alpha.x;
                scale = C{R(0), R(0)};
            } else {
                const R nrm = sqrt_r(alpha.x * alpha.x + alpha.y * alpha.y + sigma);
                beta = alpha.x >= R(0) ? -nrm : nrm;
                const R dr = alpha.x - beta, di = alpha.y;
                const R ib = rcp_nr(beta), iden = rcp_nr(dr * dr + di * di);
                tau = C{-dr * ib, -alpha.y * ib};
                scale = C{dr * iden, -di * iden};
            }
            const bool reflect = !(tau.x == R(0) && tau.y == R(0));
            if (tj == own) {   // the owning half-wave writes the whole reflector
                unroll_for<0, T>([&](auto a_) {
                    constexpr int a = a_;
                    const int r = ti + 32 * a;
                    C vv = {R(0), R(0)};
                    if (reflect && r > j && r < n) vv = r == j + 1 ? C{R(1), R(0)} : cmulz(col_entry(a_, jb), scale);
                    vs[par][r] = vv;
                    if (r > j + 1 && r < n) A[(int64_t)j * lda + r] = cd{vv.x, vv.y};   // kept for the back-transform
                });
                if (ti == own) {
                    dd[j] = djj;
                    ee[j] = beta;
                    tau_out[j] = cd{tau.x, tau.y};
                    A[(int64_t)j * lda + j + 1] = cd{beta, 0.0};
                    s_tau[par] = tau;
                }
            }
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        // ---- partials of y = A v ----
        {
            R vpart = R(0);
            unroll_for<0, T>([&](auto a_) {   // row sums over this lane's tiles of row ti + 32a
                constexpr int a = a_;
                if (32 * a + 31 <= j) return;
                R rr = R(0), ri = R(0);
                unroll_for<0, a + 1>([&](auto b_) {
                    constexpr int b = b_;
                    if (32 * b + 31 <= j) return;
                    const C e = E[a * (a + 1) / 2 + b];
                    const C vj = vs[par][tj + 32 * b];
                    rr += e.x * vj.x - e.y * vj.y;
                    ri += e.x * vj.y + e.y * vj.x;
                });
                const C vi = vs[par][ti + 32 * a];
                vpart += vi.x * rr + vi.y * ri;
                pr[tj][ti + 32 * a] = C{rr, ri};
            });
            unroll_for<0, T - 1>([&](auto b_) {   // conj(e) v_i into y_j, off-diagonal tiles
                constexpr int b = b_;
                if (32 * b + 31 <= j) return;
                R cr = R(0), ci = R(0);
                unroll_for<b + 1, T>([&](auto a_) {
                    constexpr int a = a_;
                    const C e = E[a * (a + 1) / 2 + b];
                    const C vi = vs[par][ti + 32 * a];
                    cr += e.x * vi.x + e.y * vi.y;
                    ci += e.x * vi.y - e.y * vi.x;
                });
                const C vj = vs[par][tj + 32 * b];
                vpart += vj.x * cr + vj.y * ci;
                cr = quad_sum(cr);   // the eight quad sums of a column are added in the w step
                ci = quad_sum(ci);
                if ((ti & 3) == 0) pc[ti >> 2][tj + 32 * b] = C{cr, ci};
            });
            vpart = wave_total(vpart);
            if (lane == 0) sv[wave] = vpart;
        }
        __syncthreads();
        // ---- w = tau y - nu v, four threads per row ----
        if (t < 4 * NR) {
            const int r = t >> 2, q = t & 3;
            const bool live = r > j && r < n;
            R sr = R(0), si = R(0);
            if (live) {
                R er = R(0), ei = R(0);
#pragma unroll
                for (int h = 0; h < 8; h += 2) {
                    sr += pr[8 * q + h][r].x;
                    si += pr[8 * q + h][r].y;
                    er += pr[8 * q + h + 1][r].x;
                    ei += pr[8 * q + h + 1][r].y;
                }
                if (r < 32 * (T - 1)) {   // the last column tile has no tile below the diagonal
                    sr += pc[2 * q][r].x;
                    si += pc[2 * q][r].y;
                    er += pc[2 * q + 1][r].x;
                    ei += pc[2 * q + 1][r].y;
                }
                sr += er;
                si += ei;
            }
            sr = quad_sum(sr);
            si = quad_sum(si);
            R vhy = (sv[4 * q] + sv[4 * q + 1]) + (sv[4 * q + 2] + sv[4 * q + 3]);
            vhy = quad_sum(vhy);
            const C tau = s_tau[par];
            const R nu = R(0.5) * (tau.x * tau.x + tau.y * tau.y) * vhy;
            if (q == 0) {
                C wr = {R(0), R(0)};
                if (live) {
                    const C ty = cmulz(tau, C{sr, si});
                    const C vr = vs[par][r];
                    wr = C{ty.x - nu * vr.x, ty.y - nu * vr.y};
                }
                ws[r] = wr;
            }
        }
        __syncthreads();
    }
    if (n >= 2) update(n - 2, (n - 2) & 1);
    {   // d_{n-1}: element (n-1, n-1) after the last update
        const int m = n - 1, mb = m >> 5;
        if (ti == (m & 31) && tj == (m & 31)) {
            unroll_for<0, T>([&](auto a_) {
                constexpr int a = a_;
                if (a == mb) dd[m] = E[a * (a + 1) / 2 + a].x;
            });
        }
    }
}

// Sturm counts (number of eigenvalues below x) at two shifts at once: the two
// recurrences are independent, so their division chains overlap.
__device__ void sturm_count2(const double *d, const double *e2, int n, double x1, double x2,
                             double pivmin, int &c1, int &c2) {
    c1 = c2 = 0;
    double q1 = d[0] - x1, q2 = d[0] - x2;
    if (fabs(q1) < pivmin) q1 = -pivmin;
    if (fabs(q2) < pivmin) q2 = -pivmin;
    c1 += q1 < 0;
    c2 += q2 < 0;
    for (int i = 1; i < n; ++i) {
        // e^2 / q by the refined hardware reciprocal (within an ulp, as the
        // count's backward-error argument needs; |q| >= pivmin keeps it finite)
        const double di = d[i], ei = e2[i - 1];
        q1 = di - x1 - ei * rcp_nr(q1);
        q2 = di - x2 - ei * rcp_nr(q2);
        if (fabs(q1) < pivmin) q1 = -pivmin;
        if (fabs(q2) < pivmin) q2 = -pivmin;
        c1 += q1 < 0;
        c2 += q2 < 0;
    }
}

struct TriBounds {
    double gl, gu, pivmin, tnorm;
};

__device__ TriBounds tri_bounds(const double *ds, const double *ee, int n) {
    double gl = ds[0], gu = ds[0], tnorm = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
        gl = fmin(gl, ds[i] - r);
        gu = fmax(gu, ds[i] + r);
        tnorm = fmax(tnorm, fabs(ds[i]) + r);
    }
    const double pivmin = DBL_MIN * fmax(1.0, tnorm * tnorm);
    const double span = fmax(gu - gl, DBL_EPSILON * fmax(1.0, tnorm));
    return {gl - 2.0 * DBL_EPSILON * span - 1e-300, gu + 2.0 * DBL_EPSILON * span + 1e-300, pivmin,
            tnorm};
}

// One workgroup of 256 threads per eigenvalue: each round evaluates 512
// interior points of the bracket (two interleaved Sturm chains per thread)
// and keeps the sub-interval where the count crosses the index, so a bracket
// shrinks by 513x (9 bits) per round, ~6-7 rounds from the Gershgorin
// interval to double precision.  The first point with count > idx is found
// by per-wave ballots and a minimum over the waves in LDS.
constexpr int kStebzThreads = 256;
__global__ void __launch_bounds__(kStebzThreads) k_stebz(const double *__restrict__ dd,
                                                          const double *__restrict__ ee, int n, int /*k*/,
                                                          double *__restrict__ w) {
    extern __shared__ unsigned char smem_raw[];
    double *ds = reinterpret_cast<double *>(smem_raw);
    double *e2 = ds + n;
    __shared__ TriBounds tb;
    __shared__ int wfirst[2][kStebzThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int NP = 2 * kStebzThreads;   // interior points per round
    for (int i = t; i < n; i += blockDim.x) {
        ds[i] = dd[i];
        e2[i] = (i + 1 < n) ? ee[i] * ee[i] : 0.0;
    }
    if (t == 0) tb = tri_bounds(dd, ee, n);
    __syncthreads();
    const int idx = blockIdx.x;
    double lo = tb.gl, hi = tb.gu;
    for (int round = 0; round < 16; ++round) {
        const double width = hi - lo;
        if (width <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + tb.pivmin) break;
        // thread t evaluates points t and t + 256 (1-based: point p at lo + width p / (NP + 1))
        const double x1 = lo + width * (double)(t + 1) / (double)(NP + 1);
        const double x2 = lo + width * (double)(t + 1 + kStebzThreads) / (double)(NP + 1);
        int c1, c2;
        sturm_count2(ds, e2, n, x1, x2, tb.pivmin, c1, c2);
        const uint64_t b1 = __ballot(c1 > idx), b2 = __ballot(c2 > idx);
        const int buf = round & 1;
        if (lane == 0) {
            wfirst[buf][wave] = b1 ? 64 * wave + __ffsll((unsigned long long)b1) - 1
                                   : (b2 ? kStebzThreads + 64 * wave + __ffsll((unsigned long long)b2) - 1
                                         : NP);
        }
        __syncthreads();
        // the first point (0-based) whose count exceeds idx; NP if none
        int first = NP;
        for (int q = 0; q < kStebzThreads / 64; ++q) {
            const int f = wfirst[buf][q];
            // points of the first half (< 256) come before every point of the second half
            first = min(first, f);
        }
        const double nlo = first == 0 ? lo : lo + width * (double)first / (double)(NP + 1);
        const double nhi = first == NP ? hi : lo + width * (double)(first + 1) / (double)(NP + 1);
        lo = nlo;
        hi = nhi;
    }
    if (t == 0) w[idx] = 0.5 * (lo + hi);
}

// The same multisection with d_i and e_{i-1}^2 held in registers of every wave
// (entry i in lane i % 64, slot i / 64) and read with readlane, so the Sturm
// chains never wait on LDS; the bounds come from wave reductions (min / max,
// exact in any order).  Same points, counts and rounds as k_stebz.  n <= 64 RPL.
// rel_tol: relative width at which a bracket stops (DBL_EPSILON; FLT_EPSILON
// for a tridiagonal matrix from the FP32 reduction, whose eigenvalues carry
// FP32 rounding anyway: 3 rounds instead of 6)
template <int RPL>
__global__ void __launch_bounds__(kStebzThreads) k_stebz_w(const double *__restrict__ dd,
                                                           const double *__restrict__ ee, int n, int /*k*/,
                                                           double *__restrict__ w, double rel_tol) {
    __shared__ int wfirst[2][kStebzThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int NP = 2 * kStebzThreads;
    double dreg[RPL], e2reg[RPL];
    double gl = DBL_MAX, gu = -DBL_MAX, tnorm = 0.0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int i = lane + 64 * q;
        dreg[q] = i < n ? dd[i] : 0.0;
        e2reg[q] = (i >= 1 && i < n) ? ee[i - 1] * ee[i - 1] : 0.0;
        if (i < n) {
            const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
            gl = fmin(gl, dd[i] - r);
            gu = fmax(gu, dd[i] + r);
            tnorm = fmax(tnorm, fabs(dd[i]) + r);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        gl = fmin(gl, __shfl_xor(gl, off));
        gu = fmax(gu, __shfl_xor(gu, off));
        tnorm = fmax(tnorm, __shfl_xor(tnorm, off));
    }
    const double pivmin = DBL_MIN * fmax(1.0, tnorm * tnorm);
    {
        const double span = fmax(gu - gl, DBL_EPSILON * fmax(1.0, tnorm));
        gl = gl - 2.0 * DBL_EPSILON * span - 1e-300;
        gu = gu + 2.0 * DBL_EPSILON * span + 1e-300;
    }
    const int idx = blockIdx.x;
    double lo = gl, hi = gu;
    for (int round = 0; round < 16; ++round) {
        const double width = hi - lo;
        if (width <= 2.0 * rel_tol * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        const double x1 = lo + width * (double)(t + 1) / (double)(NP + 1);
        const double x2 = lo + width * (double)(t + 1 + kStebzThreads) / (double)(NP + 1);
        // Sturm counts at x1 and x2 (the recurrence of sturm_count2)
        int c1 = 0, c2 = 0;
        double q1 = lane_read(dreg[0], 0) - x1, q2 = lane_read(dreg[0], 0) - x2;
        if (fabs(q1) < pivmin) q1 = -pivmin;
        if (fabs(q2) < pivmin) q2 = -pivmin;
        c1 += q1 < 0;
        c2 += q2 < 0;
        unroll_for<0, RPL>([&](auto q_) {
            constexpr int q = q_;
            const int lim = min(64, n - 64 * q);
            for (int l = q == 0 ? 1 : 0; l < lim; ++l) {
                const double di = lane_read(dreg[q], l), ei = lane_read(e2reg[q], l);
                q1 = di - x1 - ei * rcp_nr(q1);
                q2 = di - x2 - ei * rcp_nr(q2);
                if (fabs(q1) < pivmin) q1 = -pivmin;
                if (fabs(q2) < pivmin) q2 = -pivmin;
                c1 += q1 < 0;
                c2 += q2 < 0;
            }
        });
        const uint64_t b1 = __ballot(c1 > idx), b2 = __ballot(c2 > idx);
        const int buf = round & 1;
        if (lane == 0) {
            wfirst[buf][wave] = b1 ? 64 * wave + __ffsll((unsigned long long)b1) - 1
                                   : (b2 ? kStebzThreads + 64 * wave + __ffsll((unsigned long long)b2) - 1
                                         : NP);
        }
        __syncthreads();
        int first = NP;
        for (int q = 0; q < kStebzThreads / 64; ++q) first = min(first, wfirst[buf][q]);
        const double nlo = first == 0 ? lo : lo + width * (double)first / (double)(NP + 1);
        const double nhi = first == NP ? hi : lo + width * (double)(first + 1) / (double)(NP + 1);
        lo = nlo;
        hi = nhi;
    }
    if (t == 0) w[idx] = 0.5 * (lo + hi);
}

// Inverse iteration: one thread per eigenvalue, E eigenvalues per workgroup,
// the LU factors of T - lambda I and the iterate in LDS, interleaved [i][e].
__global__ void __launch_bounds__(64) k_stein(const double *__restrict__ dd,
                                              const double *__restrict__ ee, int n, int k, int E,
                                              const double *__restrict__ w, double *__restrict__ Z) {
    extern __shared__ unsigned char smem_raw[];
    double *ds = reinterpret_cast<double *>(smem_raw);   // [n]
    double *es = ds + n;                                  // [n]
    double *lu = es + n;                                  // [6][n][E]
    __shared__ double s_tnorm;
    const int t = threadIdx.x;
    for (int i = t; i < n; i += blockDim.x) {
        ds[i] = dd[i];
        es[i] = (i + 1 < n) ? ee[i] : 0.0;
    }
    if (t == 0) s_tnorm = tri_bounds(dd, ee, n).tnorm;
    __syncthreads();
    const int idx = blockIdx.x * E + t;
    if (t >= E || idx >= k) return;
    auto at = [&](int arr, int i) -> double & { return lu[((size_t)arr * n + i) * E + t]; };
    enum { DL = 0, DD, DU, DU2, PIV, ZZ };
    const double lam = w[idx];
    const double eps_t = DBL_EPSILON * fmax(s_tnorm, 1e-300);
    // LU with partial pivoting of T - lambda I (LAPACK dlagtf order).  The
    // entries that the next step modifies (diagonal d and superdiagonal u of
    // row i) are carried in registers and the untouched inputs of step i + 1
    // are loaded during step i, so the serial chain never waits on LDS.  DD
    // keeps the reciprocal pivot, the same refined reciprocal that forms the
    // multiplier.
    double d_cur = ds[0] - lam, u_cur = es[0];
    double sub = es[0];
    double d_nx = n > 1 ? ds[1] - lam : 0.0, u_nx = n > 1 ? es[1] : 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        const double sub_n = es[i + 1];   // es holds n entries, the last one zero
        const double d_nx_n = i + 2 < n ? ds[i + 2] - lam : 0.0;
        const double u_nx_n = i + 2 < n ? es[i + 2] : 0.0;
        if (fabs(d_cur) >= fabs(sub)) {
            const double dp = fabs(d_cur) < eps_t ? (d_cur < 0 ? -eps_t : eps_t) : d_cur;
            const double r = rcp_nr(dp);
            const double m = sub * r;
            at(DD, i) = r;
            at(DL, i) = m;
            at(DU, i) = u_cur;
            at(DU2, i) = 0.0;
            at(PIV, i) = 0.0;
            d_cur = d_nx - m * u_cur;
            u_cur = u_nx;
        } else {
            const double r = rcp_nr(sub);
            const double m = d_cur * r;
            at(DD, i) = r;
            at(DL, i) = m;
            at(DU, i) = d_nx;
            at(PIV, i) = 1.0;
            at(DU2, i) = i + 2 < n ? u_nx : 0.0;
            d_cur = u_cur - m * d_nx;
            u_cur = i + 2 < n ? -m * u_nx : u_nx;
        }
        sub = sub_n;
        d_nx = d_nx_n;
        u_nx = u_nx_n;
    }
    at(DD, n - 1) = 1.0 / (fabs(d_cur) < eps_t ? eps_t : d_cur);
    at(DU, n - 1) = 0.0;
    at(DU2, n - 1) = 0.0;
    at(PIV, n - 1) = 0.0;
    for (int i = 0; i < n; ++i) {
        uint64_t h = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull ^ (uint64_t)(idx + 7) * 0xD1B54A32D192ED03ull;
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        at(ZZ, i) = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    // two solves; the iterate stays unscaled in LDS and the 1 / max-norm of the
    // first solve is applied as the second one reads it; inputs of the next
    // step are again loaded one step ahead
    double scale = 1.0, n2 = 0.0;
    for (int iter = 0; iter < 2; ++iter) {
        // L solve with the row interchanges; z carries the running entry
        double z = at(ZZ, 0) * scale;
        double znx = n > 1 ? at(ZZ, 1) * scale : 0.0, l = at(DL, 0), piv = at(PIV, 0);
        for (int i = 0; i + 1 < n; ++i) {
            const double znx_n = i + 2 < n ? at(ZZ, i + 2) * scale : 0.0;   // not yet overwritten
            const double l_n = at(DL, i + 1), piv_n = at(PIV, i + 1);
            if (piv != 0.0) {
                at(ZZ, i) = znx;
                z = z - l * znx;
            } else {
                at(ZZ, i) = z;
                z = znx - l * z;
            }
            znx = znx_n;
            l = l_n;
            piv = piv_n;
        }
        at(ZZ, n - 1) = z;
        // U solve from the bottom; z1, z2 carry the two entries below
        double nrm = 0.0, z1 = 0.0, z2 = 0.0;
        n2 = 0.0;
        double zz = at(ZZ, n - 1), du = at(DU, n - 1), du2 = at(DU2, n - 1), rd = at(DD, n - 1);
        for (int i = n - 1; i >= 0; --i) {
            double zz_n = 0.0, du_n = 0.0, du2_n = 0.0, rd_n = 0.0;
            if (i > 0) {   // row i - 1: L-solve output, not yet overwritten
                zz_n = at(ZZ, i - 1);
                du_n = at(DU, i - 1);
                du2_n = at(DU2, i - 1);
                rd_n = at(DD, i - 1);
            }
            const double sv = (zz - du * z1 - du2 * z2) * rd;
            at(ZZ, i) = sv;
            nrm = fmax(nrm, fabs(sv));
            n2 += sv * sv;
            z2 = z1;
            z1 = sv;
            zz = zz_n;
            du = du_n;
            du2 = du2_n;
            rd = rd_n;
        }
        scale = nrm > 0 ? 1.0 / nrm : 1.0;
    }
    // unit 2-norm (the second solve's result is at most ~1 / eps_t in size,
    // so its squares stay far from overflow)
    const double inv = n2 > 0 ? 1.0 / sqrt(n2) : 1.0;
    for (int i = 0; i < n; ++i) Z[(int64_t)i * k + idx] = at(ZZ, i) * inv;
}

// Inverse iteration, one eigenvalue per wave, with no memory access inside the
// recurrences: every lane runs the same (wave-uniform) LU factorisation and
// solves, entry i of each per-step array (the LU factors, the iterate, d and e)
// is kept by lane i % 64 in register slot i / 64, written with a lane select and
// read back with readlane.  The arithmetic and its order are those of k_stein
// (LU with partial pivoting of T - lambda I in dlagtf order, two solves from a
// hashed start vector, unit 2-norm), with the pivot choice taken by selects.
// n <= 64 RPL.
template <int RPL>
__global__ void __launch_bounds__(64) k_stein_w(const double *__restrict__ dd,
                                                const double *__restrict__ ee, int n, int k,
                                                const double *__restrict__ w, double *__restrict__ Z) {
    const int L = threadIdx.x;
    const int idx = blockIdx.x;
    double dv[RPL], ev[RPL];   // d_i and e_i (e_{n-1} = 0) of entry i = L + 64 q
    double tn = 0.0;           // max_i |d_i| + |e_{i-1}| + |e_i|, as in tri_bounds
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int i = L + 64 * q;
        dv[q] = i < n ? dd[i] : 0.0;
        ev[q] = i + 1 < n ? ee[i] : 0.0;
        if (i < n) {
            const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
            tn = fmax(tn, fabs(dd[i]) + r);
        }
    }
    for (int off = 32; off > 0; off >>= 1) tn = fmax(tn, __shfl_xor(tn, off));
    const double lam = w[idx];
    const double eps_t = DBL_EPSILON * fmax(tn, 1e-300);
    double fdd[RPL], fdl[RPL], fdu[RPL], fdu2[RPL], zz[RPL];
    int fpiv[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        fdd[q] = fdl[q] = fdu[q] = fdu2[q] = 0.0;
        fpiv[q] = 0;
        const int i = L + 64 * q;
        uint64_t h = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull ^ (uint64_t)(idx + 7) * 0xD1B54A32D192ED03ull;
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        zz[q] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    // ---- LU of T - lambda I: step i eliminates row i + 1 ----
    double d_cur = lane_read(dv[0], 0) - lam, u_cur = lane_read(ev[0], 0), sub = u_cur;
    // step i (slot Q, lane l) with the entries i + 1 read from slot QN, lane ln
    auto lu_step = [&](auto Q_, auto QN_, int l, int ln) {
        constexpr int Q = decltype(Q_)::value, QN = decltype(QN_)::value;
        double d_nx = 0.0, u_nx = 0.0;
        if constexpr (QN < RPL) {
            d_nx = lane_read(dv[QN], ln) - lam;
            u_nx = lane_read(ev[QN], ln);
        }
        const bool piv = fabs(d_cur) < fabs(sub);
        const double dp = fabs(d_cur) < eps_t ? (d_cur < 0 ? -eps_t : eps_t) : d_cur;
        const double r = rcp_nr(piv ? sub : dp);
        const double m = (piv ? d_cur : sub) * r;
        const double du = piv ? d_nx : u_cur;
        const bool me = L == l;
        fdd[Q] = me ? r : fdd[Q];
        fdl[Q] = me ? m : fdl[Q];
        fdu[Q] = me ? du : fdu[Q];
        fdu2[Q] = me ? (piv ? u_nx : 0.0) : fdu2[Q];
        fpiv[Q] = me ? (int)piv : fpiv[Q];
        d_cur = fma(-m, du, piv ? u_cur : d_nx);
        u_cur = piv ? -m * u_nx : u_nx;
        sub = u_nx;
    };
    unroll_for<0, RPL>([&](auto q_) {
        constexpr int q = q_;
        const int lim = min(63, n - 1 - 64 * q);   // steps i = 64 q + l <= n - 2 with i + 1 in slot q
        for (int l = 0; l < lim; ++l) lu_step(std::integral_constant<int, q>{}, std::integral_constant<int, q>{}, l, l + 1);
        if (64 * q + 63 < n - 1)
            lu_step(std::integral_constant<int, q>{}, std::integral_constant<int, q + 1>{}, 63, 0);
    });
    {   // row n - 1
        const int qn = (n - 1) >> 6, ln = (n - 1) & 63;
        const double r = 1.0 / (fabs(d_cur) < eps_t ? eps_t : d_cur);
        const bool me = L == ln;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            if (q != qn) continue;
            fdd[q] = me ? r : fdd[q];
            fdu[q] = me ? 0.0 : fdu[q];
            fdu2[q] = me ? 0.0 : fdu2[q];
            fpiv[q] = me ? 0 : fpiv[q];
        }
    }
    // ---- two solves; the first one's 1 / max-norm is applied as the second reads it ----
    double scale = 1.0, n2 = 0.0;
    for (int iter = 0; iter < 2; ++iter) {
        // L solve with the row interchanges: z is the running entry of row i
        double z = lane_read(zz[0], 0) * scale;
        auto l_step = [&](auto Q_, auto QN_, int l, int ln) {
            constexpr int Q = decltype(Q_)::value, QN = decltype(QN_)::value;
            double znx = 0.0;
            if constexpr (QN < RPL) znx = lane_read(zz[QN], ln) * scale;
            const double lm = lane_read(fdl[Q], l);
            const bool piv = __builtin_amdgcn_readlane(fpiv[Q], l) != 0;
            const double out = piv ? znx : z;
            zz[Q] = L == l ? out : zz[Q];
            z = fma(-lm, out, piv ? z : znx);
        };
        unroll_for<0, RPL>([&](auto q_) {
            constexpr int q = q_;
            const int lim = min(63, n - 1 - 64 * q);
            for (int l = 0; l < lim; ++l) l_step(std::integral_constant<int, q>{}, std::integral_constant<int, q>{}, l, l + 1);
            if (64 * q + 63 < n - 1)
                l_step(std::integral_constant<int, q>{}, std::integral_constant<int, q + 1>{}, 63, 0);
        });
        {
            const int qn = (n - 1) >> 6, ln = (n - 1) & 63;
#pragma unroll
            for (int q = 0; q < RPL; ++q)
                if (q == qn) zz[q] = L == ln ? z : zz[q];
        }
        // U solve from the bottom; z1, z2 are the two entries below
        double nrm = 0.0, z1 = 0.0, z2 = 0.0;
        n2 = 0.0;
        unroll_for<0, RPL>([&](auto qr_) {
            constexpr int q = RPL - 1 - decltype(qr_)::value;
            const int top = min(63, n - 1 - 64 * q);
            for (int l = top; l >= 0; --l) {
                const double zi = lane_read(zz[q], l), du = lane_read(fdu[q], l), du2 = lane_read(fdu2[q], l),
                             rd = lane_read(fdd[q], l);
                const double sv = (zi - du * z1 - du2 * z2) * rd;
                zz[q] = L == l ? sv : zz[q];
                nrm = fmax(nrm, fabs(sv));
                n2 += sv * sv;
                z2 = z1;
                z1 = sv;
            }
        });
        scale = nrm > 0 ? 1.0 / nrm : 1.0;
    }
    const double inv = n2 > 0 ? 1.0 / sqrt(n2) : 1.0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int i = L + 64 * q;
        if (i < n) Z[(int64_t)i * k + idx] = zz[q] * inv;
    }
}

// Gram-Schmidt (twice) of the columns of Z [n][k] in eigenvalue order.  In
// LDS when it fits; otherwise only within clusters of eigenvalues closer than
// ctol (vectors of separated eigenvalues are already orthogonal to ~n eps ||T|| / gap,
// the backward error of the inverse-iteration solves over the gap).
__global__ void __launch_bounds__(1024) k_orth(double *__restrict__ Zg, int n, int k, int in_lds,
                                               const double *__restrict__ w, double ctol_rel,
                                               const double *__restrict__ dd,
                                               const double *__restrict__ ee) {
    extern __shared__ unsigned char smem_raw[];
    double *coef = reinterpret_cast<double *>(smem_raw);   // [k]
    double *red = coef + k;                                 // [blockDim]
    double *Zl = red + blockDim.x;                          // [n][k] if in_lds
    const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wave = t >> 6, nw = nt >> 6;
    const int ldz = in_lds ? k + 1 : k;   // padded rows in LDS (no bank conflicts)
    double *Z = in_lds ? Zl : Zg;
    __shared__ double s_ctol;
    if (t == 0) s_ctol = ctol_rel * fmax(tri_bounds(dd, ee, n).tnorm, 1e-300);
    __syncthreads();
    const double ctol = s_ctol;
    if (in_lds) {
        for (int i = t; i < n * k; i += nt) Zl[(i / k) * ldz + i % k] = Zg[i];
        __syncthreads();
    }
    int cstart = 0;
    for (int j = 0; j < k; ++j) {
        if (!in_lds && j > 0 && !(w[j] - w[j - 1] <= ctol)) cstart = j;
        const int i0 = in_lds ? 0 : cstart;
        for (int pass = 0; pass < 2; ++pass) {
            if (j > i0) {
                // coef[i] = z_i . z_j, one wave per i, lanes over rows
                for (int i = i0 + wave; i < j; i += nw) {
                    double sacc = 0.0;
                    for (int r = lane; r < n; r += 64) sacc += Z[(int64_t)r * ldz + i] * Z[(int64_t)r * ldz + j];
                    for (int off = 32; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off);
                    if (lane == 0) coef[i] = sacc;
                }
                __syncthreads();
                for (int r = t; r < n; r += nt) {
                    double sv = Z[(int64_t)r * ldz + j];
                    for (int i = i0; i < j; ++i) sv -= coef[i] * Z[(int64_t)r * ldz + i];
                    Z[(int64_t)r * ldz + j] = sv;
                }
                __syncthreads();
            }
            double pn = 0.0;
            for (int r = t; r < n; r += nt) {
                const double vv = Z[(int64_t)r * ldz + j];
                pn += vv * vv;
            }
            const double nn = block_sum(pn, red);
            const double inv = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
            for (int r = t; r < n; r += nt) Z[(int64_t)r * ldz + j] *= inv;
            __syncthreads();
        }
    }
    if (in_lds)
        for (int i = t; i < n * k; i += nt) Zg[i] = Zl[(i / k) * ldz + i % k];
}

// CholQR, twice, of the columns of Z [n][k] (k <= 64, n <= 256, all in LDS):
// G = Z^T Z, G = R^T R, Z <- Z R^-1.  Equivalent to Gram-Schmidt in column
// (eigenvalue) order; one thread per row for the triangular multiply.
constexpr int kOrthMaxK = 64;
__global__ void __launch_bounds__(256) k_orth_chol(double *__restrict__ Zg, int n, int k,
                                                   int *__restrict__ status) {
    extern __shared__ unsigned char smem_raw[];
    const int ldz = k + 1, ldg = k + 1;
    double *Z = reinterpret_cast<double *>(smem_raw);   // [n][k+1]
    double *G = Z + (size_t)n * ldz;                     // [k][k+1]: G, then R, then R^-1
    double *rowt = G + (size_t)k * ldg;                  // [k]
    const int t = threadIdx.x, nt = blockDim.x;
    for (int i = t; i < n * k; i += nt) Z[(i / k) * ldz + i % k] = Zg[i];
    __syncthreads();
    bool fail = false;
    for (int pass = 0; pass < 2; ++pass) {
        // G = Z^T Z (upper triangle), four independent partial sums per dot
        const int npair = k * (k + 1) / 2;
        for (int pidx = t; pidx < npair; pidx += nt) {
            int a = 0, rem = pidx;
            while (rem >= k - a) {
                rem -= k - a;
                ++a;
            }
            const int b = a + rem;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int r = 0;
            for (; r + 3 < n; r += 4) {
                s0 += Z[r * ldz + a] * Z[r * ldz + b];
                s1 += Z[(r + 1) * ldz + a] * Z[(r + 1) * ldz + b];
                s2 += Z[(r + 2) * ldz + a] * Z[(r + 2) * ldz + b];
                s3 += Z[(r + 3) * ldz + a] * Z[(r + 3) * ldz + b];
            }
            for (; r < n; ++r) s0 += Z[r * ldz + a] * Z[r * ldz + b];
            G[a * ldg + b] = (s0 + s1) + (s2 + s3);
        }
        __syncthreads();
        // Cholesky G = R^T R (upper); the trailing update uses the unscaled pivot row
        for (int j = 0; j < k; ++j) {
            double d = G[j * ldg + j];
            if (!(d > 1e-300)) {
                fail = true;
                d = 1.0;
            }
            const double inv_d = 1.0 / d;
            const int m = k - j - 1;
            for (int i = t; i < m * m; i += nt) {
                const int a = j + 1 + i % m, b = j + 1 + i / m;
                if (b >= a) G[a * ldg + b] -= G[j * ldg + a] * G[j * ldg + b] * inv_d;
            }
            __syncthreads();
            const double isd = 1.0 / sqrt(d);
            for (int c = j + 1 + t; c < k; c += nt) G[j * ldg + c] *= isd;
            if (t == 0) G[j * ldg + j] = d * isd;
        }
        __syncthreads();
        // R^-1 in place, rows from the bottom: X_ic = (delta_ic - sum_{q=i+1..c} R_iq X_qc) / R_ii
        for (int i = k - 1; i >= 0; --i) {
            for (int c = i + t; c < k; c += nt) rowt[c] = G[i * ldg + c];
            __syncthreads();
            for (int c = i + t; c < k; c += nt) {
                double sacc = (c == i) ? 1.0 : 0.0;
                for (int q = i + 1; q <= c; ++q) sacc -= rowt[q] * G[q * ldg + c];
                G[i * ldg + c] = sacc / rowt[i];
            }
            __syncthreads();
        }
        // Z <- Z R^-1, one thread per row (row in registers)
        for (int r = t; r < n; r += nt) {
            double z[kOrthMaxK];
#pragma unroll
            for (int i = 0; i < kOrthMaxK; ++i) z[i] = i < k ? Z[r * ldz + i] : 0.0;
            for (int j = 0; j < k; ++j) {
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int i = 0; i < kOrthMaxK; i += 2) {
                    if (i <= j) s0 += z[i] * G[i * ldg + j];
                    if (i + 1 <= j) s1 += z[i + 1] * G[(i + 1) * ldg + j];
                }
                Z[r * ldz + j] = s0 + s1;
            }
        }
        __syncthreads();
    }
    for (int i = t; i < n * k; i += nt) Zg[i] = Z[(i / k) * ldz + i % k];
    if (t == 0 && fail) atomicOr(status, 2);
}

// V[:, c] = H_0 ... H_{n-2} Z[:, c] for a chunk of cw columns held in LDS.
// Reflectors are staged into LDS nrefl at a time (the host picks cw and nrefl
// so that both fit; the staging depth does not change the arithmetic).
__global__ void __launch_bounds__(256) k_unmtr(const cd *__restrict__ A, int64_t lda, int n, int k,
                                               int cw, int nrefl, const cd *__restrict__ tau,
                                               const double *__restrict__ Z, cd *__restrict__ V,
                                               int64_t ldv) {
    extern __shared__ unsigned char smem_raw[];
    cd *Vs = reinterpret_cast<cd *>(smem_raw);   // [n][cw + 1]
    cd *vb = Vs + (size_t)n * (cw + 1);          // [nrefl][n] staged reflectors
    cd *sp = vb + (size_t)nrefl * n;             // [blockDim] partial dots
    cd *sc = sp + blockDim.x;                    // [cw]
    const int t = threadIdx.x, nt = blockDim.x;
    const int c0 = blockIdx.x * cw;
    const int ncol = min(cw, k - c0);
    const int LD = cw + 1;
    for (int i = t; i < n * cw; i += nt) {
        const int r = i / cw, c = i % cw;
        Vs[r * LD + c] = cd{c < ncol ? Z[(int64_t)r * k + c0 + c] : 0.0, 0.0};
    }
    const int parts = nt / cw;   // threads per column in the dot products
    for (int jhi = n - 2; jhi >= 0; jhi -= nrefl) {
        const int jlo = max(0, jhi - nrefl + 1);
        __syncthreads();
        // stage reflectors jhi..jlo: slot q holds reflector jhi - q, rows j+1..n-1
        for (int idx = t; idx < nrefl * n; idx += nt) {
            const int q = idx / n, i = idx % n;
            const int j = jhi - q;
            if (j >= jlo) {
                const int L = n - j - 1;
                vb[q * n + i] = (i >= L) ? cd{0.0, 0.0} : (i == 0) ? cd{1.0, 0.0} : A[(int64_t)j * lda + j + 1 + i];
            }
        }
        __syncthreads();
        for (int j = jhi; j >= jlo; --j) {
            const cd tj = tau[j];
            if (tj.x == 0.0 && tj.y == 0.0) continue;
            const cd *vv = vb + (jhi - j) * n;
            const int L = n - j - 1;
            {
                const int c = t % cw, p = t / cw;
                double sr0 = 0.0, si0 = 0.0, sr1 = 0.0, si1 = 0.0;
                if (p < parts) {
                    int i = p;
                    for (; i + parts < L; i += 2 * parts) {
                        const cd a0 = vv[i], x0 = Vs[(j + 1 + i) * LD + c];
                        const cd a1 = vv[i + parts], x1 = Vs[(j + 1 + i + parts) * LD + c];
                        sr0 += a0.x * x0.x + a0.y * x0.y;
                        si0 += a0.x * x0.y - a0.y * x0.x;
                        sr1 += a1.x * x1.x + a1.y * x1.y;
                        si1 += a1.x * x1.y - a1.y * x1.x;
                    }
                    for (; i < L; i += parts) {
                        const cd a0 = vv[i], x0 = Vs[(j + 1 + i) * LD + c];
                        sr0 += a0.x * x0.x + a0.y * x0.y;
                        si0 += a0.x * x0.y - a0.y * x0.x;
                    }
                }
                sp[t] = cd{sr0 + sr1, si0 + si1};
            }
            __syncthreads();
            if (t < cw) {
                double sr = 0.0, si = 0.0;
                for (int p = 0; p < parts; ++p) {
                    sr += sp[p * cw + t].x;
                    si += sp[p * cw + t].y;
                }
                sc[t] = cmulz(tj, cd{sr, si});
            }
            __syncthreads();
            for (int i = t; i < L * cw; i += nt) {
                const int r = i / cw, c = i % cw;
                const cd pr = cmulz(vv[r], sc[c]);
                cd &x = Vs[(j + 1 + r) * LD + c];
                x.x -= pr.x;
                x.y -= pr.y;
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int i = t; i < n * ncol; i += nt) {
        const int c = i / n, r = i % n;
        V[(int64_t)(c0 + c) * ldv + r] = Vs[r * LD + c];
    }
}

// CholQR applied twice to the real eigenvector block Z [n x k] (k <= 64,
// n <= 217), in LDS, 1024 threads.  G = Z^T Z and Z R^-1 run on the FP64
// matrix cores (16 x 16 output tiles, one to three per wave).  The factor
// comes from elimination on [G | I] as in k_chol_inv (pivot row broadcast
// through LDS, one barrier per step, rows kept unscaled until the end: the
// augmented half becomes L^-1 and R^-T = D^-1/2 L^-1), with 2 x 2 tiles per
// thread on a 32 x 32 grid.  Columns >= k carry an identity block of G.
constexpr int kOc2Ld = 68;   // LDS row stride of Z (doubles)
constexpr int kOc2Lr = 65;   // LDS row stride of G and of R^-1
__host__ __device__ constexpr size_t orth_chol2_lds(int n) {
    return ((size_t)((n + 15) / 16 * 16) * kOc2Ld + 64 * kOc2Lr + 8 * 64) * sizeof(double);
}
__global__ void __launch_bounds__(1024) k_orth_chol2(double *__restrict__ Zg, int n, int k,
                                                     int *__restrict__ status) {
    typedef double v4d __attribute__((ext_vector_type(4)));
    extern __shared__ double smd[];
    const int n16 = (n + 15) / 16 * 16;     // rows padded with zeros to whole tiles
    double *Z = smd;                        // [n16][kOc2Ld], columns >= k zero
    double *Gs = Z + (size_t)n16 * kOc2Ld;  // [64][kOc2Lr]: G, then R^-1
    double *pg = Gs + 64 * kOc2Lr;          // [2][2][64] pivot row pairs of G
    double *pu = pg + 4 * 64;               // [2][2][64] pivot row pairs of the augmented half
    const int t = threadIdx.x, nt = blockDim.x;
    const int ti = t >> 5, tj = t & 31, a0 = 2 * ti, b0 = 2 * tj;
    const int wave = t >> 6, lane = t & 63, li = lane & 15, lg = lane >> 4;
    const int wrow_last = 4 * wave + 3;
    for (int i = t; i < n16 * kOc2Ld; i += nt) {
        const int r = i / kOc2Ld, c = i % kOc2Ld;
        Z[i] = (r < n && c < k) ? Zg[(size_t)r * k + c] : 0.0;
    }
    __syncthreads();
    bool fail = false;
    for (int pass = 0; pass < 2; ++pass) {
        {   // G = Z^T Z: wave w computes the 16 x 16 tile (w / 4, w % 4)
            const int ra = 16 * (wave >> 2), cb = 16 * (wave & 3);
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < n16; k0 += 4) {
                const double *zr = Z + (size_t)(k0 + lg) * kOc2Ld;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(zr[ra + li], zr[cb + li], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) Gs[(ra + lg + 4 * r) * kOc2Lr + cb + li] = acc[r];
        }
        __syncthreads();
        double g[2][2], u[2][2], dpiv[2] = {1.0, 1.0};
#pragma unroll
        for (int ia = 0; ia < 2; ++ia)
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) {
                const int a = a0 + ia, b = b0 + ib;
                g[ia][ib] = (a == b && a >= k) ? 1.0 : Gs[a * kOc2Lr + b];
                u[ia][ib] = a == b ? 1.0 : 0.0;
                if (ti == 0) {   // rows 0 and 1: the first pivot pair
                    pg[64 * ia + b] = g[ia][ib];
                    pu[64 * ia + b] = u[ia][ib];
                }
            }
        __syncthreads();
        // two pivots per barrier (as in k_chol_inv): rows j, j + 1 arrive with
        // the pivots < j applied; row j + 1 after pivot j is formed locally
        for (int j = 0; j < 64; j += 2) {
            const int bsel = (j >> 1) & 1;
            const double *r0g = pg + 128 * bsel, *r1g = r0g + 64, *r0u = pu + 128 * bsel, *r1u = r0u + 64;
            double d0 = r0g[j];
            if (!(d0 > 1e-300) || !isfinite(d0)) {
                fail = true;
                d0 = 1.0;
            }
            const double inv0 = rcp_nr(d0);
            const double l = r0g[j + 1] * inv0;
            double d1 = r1g[j + 1] - l * r0g[j + 1];
            if (!(d1 > 1e-300) || !isfinite(d1)) {
                fail = true;
                d1 = 1.0;
            }
#pragma unroll
            for (int ia = 0; ia < 2; ++ia) {
                if (a0 + ia == j) dpiv[ia] = d0;
                if (a0 + ia == j + 1) dpiv[ia] = d1;
            }
            if (wrow_last > j) {   // rows below pivot j in this wave (uniform per wave)
                const double inv1 = rcp_nr(d1);
                double m0[2], m1[2];
#pragma unroll
                for (int ia = 0; ia < 2; ++ia) {
                    const int a = a0 + ia;
                    m0[ia] = a > j ? r0g[a] * inv0 : 0.0;
                    m1[ia] = a > j + 1 ? (r1g[a] - l * r0g[a]) * inv1 : 0.0;
                }
                double g0[2], g1[2], u0[2], u1[2];
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    const int b = b0 + ib;
                    g0[ib] = r0g[b];
                    g1[ib] = r1g[b] - l * g0[ib];
                    u0[ib] = r0u[b];
                    u1[ib] = r1u[b] - l * u0[ib];
                }
#pragma unroll
                for (int ia = 0; ia < 2; ++ia) {
                    const int a = a0 + ia;
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib) {
                        if (b0 + ib >= a) g[ia][ib] -= m0[ia] * g0[ib] + m1[ia] * g1[ib];
                        u[ia][ib] -= m0[ia] * u0[ib] + m1[ia] * u1[ib];
                    }
                }
                if (j + 2 < 64 && a0 == j + 2) {
                    double *ng = pg + 128 * (bsel ^ 1), *nu = pu + 128 * (bsel ^ 1);
#pragma unroll
                    for (int ia = 0; ia < 2; ++ia) {
                        ng[64 * ia + b0] = g[ia][0];
                        ng[64 * ia + b0 + 1] = g[ia][1];
                        nu[64 * ia + b0] = u[ia][0];
                        nu[64 * ia + b0 + 1] = u[ia][1];
                    }
                }
            }
            __syncthreads();
        }
        // R^-1 (c, a) = (D^-1/2 L^-1)(a, c)
#pragma unroll
        for (int ia = 0; ia < 2; ++ia) {
            const double isd = 1.0 / sqrt(dpiv[ia]);
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) Gs[(b0 + ib) * kOc2Lr + a0 + ia] = u[ia][ib] * isd;
        }
        __syncthreads();
        {   // Z <- Z R^-1: wave w computes column tile w % 4 of row tiles w / 4 + 4 i
            const int cb = 16 * (wave & 3);
            v4d acc[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < 64; k0 += 4) {
                const double b = Gs[(k0 + lg) * kOc2Lr + cb + li];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int rt = 16 * ((wave >> 2) + 4 * i);
                    if (rt < n16)
                        acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(Z[(size_t)(rt + li) * kOc2Ld + k0 + lg], b,
                                                                      acc[i], 0, 0, 0);
                }
            }
            __syncthreads();   // every read of Z done before it is overwritten
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rt = 16 * ((wave >> 2) + 4 * i);
                if (rt < n16)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = rt + lg + 4 * r, col = cb + li;
                        Z[(size_t)row * kOc2Ld + col] = (row < n && col < k) ? acc[i][r] : 0.0;
                    }
            }
        }
        __syncthreads();
    }
    for (int i = t; i < n * k; i += nt) Zg[i] = Z[(i / k) * kOc2Ld + i % k];
    if (t == 0 && fail) atomicOr(status, 2);
}

// V[:, c] = H_0 ... H_{n-2} Z[:, c] for n <= 64 RPL: one wave per kUwCols
// columns, RPL rows per lane, column sums by DPP alone (wave_total), no barriers.
// Reflectors are applied in groups of kUwRing with a ring of kUwRing
// reflectors loaded ahead, so the loads of one group overlap the work of the
// previous one.
constexpr int kUwCols = 1;
constexpr int kUwRing = 8;
template <int RPL>
__global__ void __launch_bounds__(64) k_unmtr_w(const cd *__restrict__ A, int64_t lda, int n, int k,
                                                const cd *__restrict__ tau,
                                                const double *__restrict__ Z, cd *__restrict__ V,
                                                int64_t ldv) {
    const int l = threadIdx.x;
    const int c0 = blockIdx.x * kUwCols;
    cd x[RPL][kUwCols];
#pragma unroll
    for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int c = 0; c < kUwCols; ++c) {
            const int r = l + 64 * q;
            x[q][c] = cd{(r < n && c0 + c < k) ? Z[(int64_t)r * k + c0 + c] : 0.0, 0.0};
        }
    cd ring[kUwRing][RPL];
    cd rtau[kUwRing];
    // reflector j (0 <= j <= n-2): rows j+1..n-1, v_{j+1} = 1; j < 0 is a no-op
    auto load = [&](int slot_j, cd (&v)[RPL], cd &tj) {
        const int j = slot_j;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int r = l + 64 * q;
            v[q] = (j >= 0 && r == j + 1) ? cd{1.0, 0.0}
                                          : ((j >= 0 && r > j + 1 && r < n) ? A[(int64_t)j * lda + r]
                                                                            : cd{0.0, 0.0});
        }
        tj = j >= 0 ? tau[j] : cd{0.0, 0.0};
    };
    const int jtop = n - 2;
#pragma unroll
    for (int s = 0; s < kUwRing; ++s) load(jtop - s, ring[s], rtau[s]);
    for (int jg = jtop; jg >= 0; jg -= kUwRing) {
#pragma unroll
        for (int s = 0; s < kUwRing; ++s) {
            const cd tj = rtau[s];
            cd v[RPL];
#pragma unroll
            for (int q = 0; q < RPL; ++q) v[q] = ring[s][q];
            load(jg - s - kUwRing, ring[s], rtau[s]);   // refill the slot for the next group
            if (tj.x == 0.0 && tj.y == 0.0) continue;
#pragma unroll
            for (int c = 0; c < kUwCols; ++c) {
                double dr = 0.0, di = 0.0;   // v^H x_c
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    dr += v[q].x * x[q][c].x + v[q].y * x[q][c].y;
                    di += v[q].x * x[q][c].y - v[q].y * x[q][c].x;
                }
                dr = wave_total(dr);
                di = wave_total(di);
                const cd sc = cmulz(tj, cd{dr, di});
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    const cd u = cmulz(v[q], sc);
                    x[q][c].x -= u.x;
                    x[q][c].y -= u.y;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kUwCols; ++c) {
        if (c0 + c >= k) break;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int r = l + 64 * q;
            if (r < n) V[(int64_t)(c0 + c) * ldv + r] = x[q][c];
        }
    }
}

__global__ void k_check_w(const double *w, int k, int *status) {
    for (int i = threadIdx.x; i < k; i += blockDim.x)
        if (!isfinite(w[i])) atomicOr(status, 4);
}

}  // namespace

void launch_chol_inv_f64(const cd *G, int64_t ldg, int n, cd *Rinv, int64_t ldr, int *status,
                         hipStream_t st) {
    PW_REQUIRE(n >= 1 && n <= kCholMax, PW_ERR_ARG, "block size must be in [1, 64]");
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(1024), 0, st, G, ldg, n, Rinv, ldr, status);
    PW_HIP(hipGetLastError());
}

size_t heev_scratch_bytes(int n, int k) {
    const size_t nch = (size_t)(n + 63) / 64;
    return 8 * 256 + (size_t)n * 16 + 2 * (size_t)n * 8 + (size_t)n * k * 8 +
           (3 + nch) * (size_t)n * 16;   // reflector pair, w and the y partials (n > 192)
}

void launch_heev_f64(cd *A, int64_t lda, int n, int k, double *w, cd *V, int64_t ldv, void *scratch,
                     int *status, hipStream_t st, bool fp32_reduction) {
    PW_REQUIRE(n >= 1 && n <= 1024 && k >= 1 && k <= n, PW_ERR_ARG, "heev: need 1 <= k <= n <= 1024");
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    char *p = static_cast<char *>(scratch);
    cd *tau = reinterpret_cast<cd *>(p);
    p += align((size_t)n * 16);
    double *d = reinterpret_cast<double *>(p);
    p += align((size_t)n * 8);
    double *e = reinterpret_cast<double *>(p);
    p += align((size_t)n * 8);
    double *Z = reinterpret_cast<double *>(p);
    p += align((size_t)n * k * 8);
    // 1. tridiagonalisation (the trailing block of A is overwritten in both triangles)
    if (n <= 32 * kRfMaxT) {
        const int T = (n + 31) / 32;
        auto go = [&](auto r_) {
            using R = decltype(r_);
            switch (T) {
                case 1: hipLaunchKernelGGL((k_hetrd_la<1, R>), dim3(1), dim3(1024), 0, st, A, lda, n, d, e, tau); break;
                case 2: hipLaunchKernelGGL((k_hetrd_la<2, R>), dim3(1), dim3(1024), 0, st, A, lda, n, d, e, tau); break;
                case 3: hipLaunchKernelGGL((k_hetrd_la<3, R>), dim3(1), dim3(1024), 0, st, A, lda, n, d, e, tau); break;
                case 4: hipLaunchKernelGGL((k_hetrd_la<4, R>), dim3(1), dim3(1024), 0, st, A, lda, n, d, e, tau); break;
                case 5: hipLaunchKernelGGL((k_hetrd_la<5, R>), dim3(1), dim3(1024), 0, st, A, lda, n, d, e, tau); break;
                default: hipLaunchKernelGGL((k_hetrd_la<6, R>), dim3(1), dim3(1024), 0, st, A, lda, n, d, e, tau); break;
            }
        };
        if (fp32_reduction)
            go(0.0f);
        else
            go(0.0);
    } else {
        TrdState S;
        S.v[0] = reinterpret_cast<cd *>(p);
        p += align((size_t)n * 16);
        S.v[1] = reinterpret_cast<cd *>(p);
        p += align((size_t)n * 16);
        S.w = reinterpret_cast<cd *>(p);
        p += align((size_t)n * 16);
        S.ypart = reinterpret_cast<cd *>(p);
        hipLaunchKernelGGL(k_herm_sym, dim3((unsigned)(((int64_t)n * n + 255) / 256)), dim3(256), 0, st, A, lda,
                           n);
        launch_zero(S.v[0], n, n, 1, st);
        launch_zero(S.v[1], n, n, 1, st);
        hipLaunchKernelGGL(k_trd_step, dim3(1), dim3(1024), 0, st, A, lda, n, -1, S, d, e, tau);
        for (int j = 0; j + 1 < n; ++j) {
            const int L = n - 1 - j, nb = (L + 63) / 64;
            hipLaunchKernelGGL(k_trd_apply, dim3(nb * nb), dim3(256), 0, st, A, lda, n, j, S);
            hipLaunchKernelGGL(k_trd_step, dim3(1), dim3(1024), 0, st, A, lda, n, j, S, d, e, tau);
        }
    }
    // 2. eigenvalues
    const size_t sm2 = 2 * (size_t)n * 8;
    // one workgroup per eigenvalue, spread over k CUs
    const bool lowp = fp32_reduction && n <= 32 * kRfMaxT;
    const double tol = lowp ? (double)FLT_EPSILON : DBL_EPSILON;
    switch ((n + 63) / 64) {
        case 1: hipLaunchKernelGGL(k_stebz_w<1>, dim3(k), dim3(kStebzThreads), 0, st, d, e, n, k, w, tol); break;
        case 2: hipLaunchKernelGGL(k_stebz_w<2>, dim3(k), dim3(kStebzThreads), 0, st, d, e, n, k, w, tol); break;
        case 3: hipLaunchKernelGGL(k_stebz_w<3>, dim3(k), dim3(kStebzThreads), 0, st, d, e, n, k, w, tol); break;
        case 4: hipLaunchKernelGGL(k_stebz_w<4>, dim3(k), dim3(kStebzThreads), 0, st, d, e, n, k, w, tol); break;
        default: hipLaunchKernelGGL(k_stebz, dim3(k), dim3(kStebzThreads), sm2, st, d, e, n, k, w); break;
    }
    // 3. inverse iteration
    if (n <= 256) {
        switch ((n + 63) / 64) {
            case 1: hipLaunchKernelGGL(k_stein_w<1>, dim3(k), dim3(64), 0, st, d, e, n, k, w, Z); break;
            case 2: hipLaunchKernelGGL(k_stein_w<2>, dim3(k), dim3(64), 0, st, d, e, n, k, w, Z); break;
            case 3: hipLaunchKernelGGL(k_stein_w<3>, dim3(k), dim3(64), 0, st, d, e, n, k, w, Z); break;
            default: hipLaunchKernelGGL(k_stein_w<4>, dim3(k), dim3(64), 0, st, d, e, n, k, w, Z); break;
        }
    } else {
    const size_t budget = 150 * 1024;
    int E = (int)((budget - 16 * (size_t)n) / (48 * (size_t)n));
    E = std::max(1, std::min(4, E));   // few eigenvalues per workgroup: spread over CUs
    const size_t sm3 = 16 * (size_t)n + 48 * (size_t)n * E;
    ensure_smem_limit((const void *)k_stein, sm3);
    hipLaunchKernelGGL(k_stein, dim3((k + E - 1) / E), dim3(64), sm3, st, d, e, n, k, E, w, Z);
    }
    // 4. orthogonalisation
    const size_t smc = ((size_t)n * (k + 1) + (size_t)k * (k + 1) + k) * 8;
    if (k <= 64 && orth_chol2_lds(n) <= 150 * 1024) {
        const size_t sm = orth_chol2_lds(n);
        ensure_smem_limit((const void *)k_orth_chol2, sm);
        hipLaunchKernelGGL(k_orth_chol2, dim3(1), dim3(1024), sm, st, Z, n, k, status);
    } else if (k <= kOrthMaxK && n <= 256 && smc <= 150 * 1024) {
        ensure_smem_limit((const void *)k_orth_chol, smc);
        hipLaunchKernelGGL(k_orth_chol, dim3(1), dim3(256), smc, st, Z, n, k, status);
    } else {
    const bool in_lds = (size_t)n * (k + 1) * 8 + (size_t)(k + 1024) * 8 <= 140 * 1024;
    const size_t sm4 = (size_t)(k + 1024) * 8 + (in_lds ? (size_t)n * (k + 1) * 8 : 0);
    ensure_smem_limit((const void *)k_orth, sm4);
    hipLaunchKernelGGL(k_orth, dim3(1), dim3(1024), sm4, st, Z, n, k, in_lds ? 1 : 0, w, 2e-5, d, e);
    }
    // 5. back-transform
    if (n <= 256) {
        const dim3 g((k + kUwCols - 1) / kUwCols);
        switch ((n + 63) / 64) {
            case 1: hipLaunchKernelGGL(k_unmtr_w<1>, g, dim3(64), 0, st, A, lda, n, k, tau, Z, V, ldv); break;
            case 2: hipLaunchKernelGGL(k_unmtr_w<2>, g, dim3(64), 0, st, A, lda, n, k, tau, Z, V, ldv); break;
            case 3: hipLaunchKernelGGL(k_unmtr_w<3>, g, dim3(64), 0, st, A, lda, n, k, tau, Z, V, ldv); break;
            default: hipLaunchKernelGGL(k_unmtr_w<4>, g, dim3(64), 0, st, A, lda, n, k, tau, Z, V, ldv); break;
        }
        hipLaunchKernelGGL(k_check_w, dim3(1), dim3(256), 0, st, w, k, status);
        PW_HIP(hipGetLastError());
        return;
    }
    // columns per workgroup and staged reflectors: up to 32 and 8; past n ~ 930
    // both shrink (columns down to 4 first, then the staging depth) to fit LDS
    int cw = 32, nrefl = 8;
    auto sm5_of = [&](int w_, int r_) {
        return (size_t)n * (w_ + 1) * 16 + (size_t)r_ * n * 16 + 256 * 16 + (size_t)w_ * 16;
    };
    while (sm5_of(cw, nrefl) > 150 * 1024) {
        if (cw > 4) cw /= 2;
        else if (nrefl > 1) nrefl /= 2;
        else if (cw > 1) cw /= 2;
        else break;
    }
    const size_t sm5 = sm5_of(cw, nrefl);
    PW_REQUIRE(sm5 <= 150 * 1024, PW_ERR_ARG, "eigenproblem too large for the back-transform");
    ensure_smem_limit((const void *)k_unmtr, sm5);
    hipLaunchKernelGGL(k_unmtr, dim3((k + cw - 1) / cw), dim3(256), sm5, st, A, lda, n, k, cw, nrefl, tau,
                       Z, V, ldv);
    hipLaunchKernelGGL(k_check_w, dim3(1), dim3(256), 0, st, w, k, status);
    PW_HIP(hipGetLastError());
}

}  // namespace pw
