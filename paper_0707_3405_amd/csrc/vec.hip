// Streaming kernels over [npw x nb] blocks: Rayleigh quotients, residuals,
// preconditioner, projector table, and small helpers.
//
// Per-band reductions are two-level: each workgroup reduces a chunk of rows
// of one band in a fixed tree order, and a one-workgroup kernel sums the
// chunk partials in chunk order, so every result is bitwise reproducible.
#include <cfloat>

#include "pw_internal.h"

namespace pw {
namespace {

constexpr int kChunk = 2048;   // rows per reduction workgroup
constexpr int kThreads = 256;

// Blocks are stored as complex128 (cd) or complex64 (cf); arithmetic and every
// reduction run in double.
__device__ __forceinline__ cd widen(cd v) { return v; }
__device__ __forceinline__ cd widen(cf v) { return cd{(double)v.x, (double)v.y}; }
template <class S>
__device__ __forceinline__ S narrow(double x, double y) {
    return S{(decltype(S::x))x, (decltype(S::y))y};
}

template <int NV>
__device__ void wg_reduce(double (&v)[NV], double *red) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q * kThreads + t] = v[q];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int q = 0; q < NV; ++q) red[q * kThreads + t] += red[q * kThreads + t + s];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = red[q * kThreads];
}

// Rayleigh quotient pieces per (chunk, band): Re(x^H Hx), sum T|x|^2 and the
// norm: |x|^2, or Re(x^H Ox) in the generalized form (OX given).
template <class S>
__global__ void __launch_bounds__(kThreads)
    k_band_dots(const S *__restrict__ X, int64_t ldx, const S *__restrict__ HX, int64_t ldhx,
                const double *__restrict__ kin, int64_t npw, int nb, double *__restrict__ part,
                const S *__restrict__ OX, int64_t ldox) {
    __shared__ double red[3 * kThreads];
    const int c = blockIdx.x, b = blockIdx.y;
    const int64_t r0 = (int64_t)c * kChunk, r1 = min(npw, r0 + kChunk);
    const S *x = X + (int64_t)b * ldx;
    const S *h = HX + (int64_t)b * ldhx;
    const S *o = OX ? OX + (int64_t)b * ldox : nullptr;
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kThreads) {
        const cd a = widen(x[r]), hb = widen(h[r]);
        const double n2 = a.x * a.x + a.y * a.y;
        v[0] += a.x * hb.x + a.y * hb.y;
        v[1] += kin[r] * n2;
        if (o) {
            const cd ob = widen(o[r]);
            v[2] += a.x * ob.x + a.y * ob.y;
        } else {
            v[2] += n2;
        }
    }
    wg_reduce<3>(v, red);
    if (threadIdx.x == 0) {
        double *p = part + ((int64_t)c * nb + b) * 3;
        p[0] = v[0];
        p[1] = v[1];
        p[2] = v[2];
    }
}

// out[0..nb): theta, out[nb..2nb): E_kin, out[2nb..3nb): |x|^2
__global__ void k_band_dots_final(const double *__restrict__ part, int nchunk, int nb,
                                  double *__restrict__ theta, double *__restrict__ ekin_nrm) {
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            const double *p = part + ((int64_t)c * nb + b) * 3;
            s0 += p[0];
            s1 += p[1];
            s2 += p[2];
        }
        const double inv = s2 > 0 ? 1.0 / s2 : 0.0;
        theta[b] = s0 * inv;
        ekin_nrm[b] = s1 * inv;
        ekin_nrm[nb + b] = s2;
    }
}

// R = HX - theta X; W = K(T / E_kin) R (if W); partial |R|^2 per (chunk, band).
template <class S>
__global__ void __launch_bounds__(kThreads)
    k_resid(const S *__restrict__ X, int64_t ldx, const S *__restrict__ HX, int64_t ldhx,
            const double *__restrict__ kin, int64_t npw, int nb, const double *__restrict__ theta,
            const double *__restrict__ ekin, S *__restrict__ W, int64_t ldw,
            double *__restrict__ part) {
    __shared__ double red[kThreads];
    const int c = blockIdx.x, b = blockIdx.y;
    const int64_t r0 = (int64_t)c * kChunk, r1 = min(npw, r0 + kChunk);
    const S *x = X + (int64_t)b * ldx;
    const S *h = HX + (int64_t)b * ldhx;
    const double th = theta[b];
    const double ek = fmax(ekin[b], 1e-3);
    const double iek = 1.0 / ek;
    double v[1] = {0.0};
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kThreads) {
        const cd a = widen(x[r]), hb = widen(h[r]);
        const cd rr = {hb.x - th * a.x, hb.y - th * a.y};
        v[0] += rr.x * rr.x + rr.y * rr.y;
        if (W) {
            const double xx = kin[r] * iek;
            const double num = 27.0 + xx * (18.0 + xx * (12.0 + xx * 8.0));
            const double k = num / (num + 16.0 * xx * xx * xx * xx);
            W[(int64_t)b * ldw + r] = narrow<S>(k * rr.x, k * rr.y);
        }
    }
    wg_reduce<1>(v, red);
    if (threadIdx.x == 0) part[(int64_t)c * nb + b] = v[0];
}

// W[:, jj] = K(T / E_kin) (HX - theta X)[:, act[jj]] for the active columns.
template <class S>
__global__ void __launch_bounds__(kThreads)
    k_precond_map(const S *__restrict__ X, int64_t ldx, const S *__restrict__ HX, int64_t ldhx,
                  const double *__restrict__ kin, int64_t npw, const double *__restrict__ theta,
                  const double *__restrict__ ekin, const int *__restrict__ act, S *__restrict__ W,
                  int64_t ldw) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int jj = blockIdx.y;
    if (r >= npw) return;
    const int b = act[jj];
    const cd a = widen(X[(int64_t)b * ldx + r]), hb = widen(HX[(int64_t)b * ldhx + r]);
    const double th = theta[b];
    const double xx = kin[r] / fmax(ekin[b], 1e-3);
    const double num = 27.0 + xx * (18.0 + xx * (12.0 + xx * 8.0));
    const double k = num / (num + 16.0 * xx * xx * xx * xx);
    W[(int64_t)jj * ldw + r] = narrow<S>(k * (hb.x - th * a.x), k * (hb.y - th * a.y));
}

// status (optional): the context's status word, appended as res[nb] so that one
// copy brings the norms and the breakdown flags to the host
__global__ void k_resid_final(const double *__restrict__ part, int nchunk, int nb,
                              const double *__restrict__ nrm2, double *__restrict__ res,
                              const int *__restrict__ status) {
    if (status && threadIdx.x == 0) res[nb] = (double)*status;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * nb + b];
        const double n2 = nrm2 ? nrm2[b] : 1.0;
        res[b] = sqrt(s / (n2 > 0 ? n2 : 1.0));
    }
}

// beta_{a,lm}(q) = pref exp(-|q|^2/2) Y_lm(q^) exp(-i q.R_a)
__global__ void k_build_projectors(const double *__restrict__ qvec, int64_t npw, int /*natom*/,
                                   const double *__restrict__ pos, int nlm,
                                   const int *__restrict__ lm, double pref, cd *__restrict__ B,
                                   int64_t ldb) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (g >= npw) return;
    const int a = col / nlm, p = col % nlm;
    const double qx = qvec[3 * g], qy = qvec[3 * g + 1], qz = qvec[3 * g + 2];
    const double q2 = qx * qx + qy * qy + qz * qz;
    const double qn = sqrt(q2);
    const int l = lm[2 * p], m = lm[2 * p + 1];
    double ylm;
    if (l == 0) {
        ylm = 0.28209479177387814347403972578038630;   // 1 / (2 sqrt(pi))
    } else {
        const double c1 = 0.48860251190291992158638462283834700;   // sqrt(3 / (4 pi))
        const double comp = (m == -1) ? qy : (m == 0) ? qz : qx;
        ylm = qn > 0.0 ? c1 * comp / qn : 0.0;
    }
    const double rad = pref * exp(-0.5 * q2) * ylm;
    const double ph = qx * pos[3 * a] + qy * pos[3 * a + 1] + qz * pos[3 * a + 2];
    double s, c;
    sincos(ph, &s, &c);
    B[(int64_t)col * ldb + g] = cd{rad * c, -rad * s};
}

// copy with conversion between storage precisions (round to nearest)
template <class SA, class SB>
__global__ void k_copy_cols(const SA *__restrict__ A, int64_t lda, SB *__restrict__ B, int64_t ldb,
                            int64_t rows) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (r < rows) {
        const cd v = widen(A[(int64_t)c * lda + r]);
        B[(int64_t)c * ldb + r] = narrow<SB>(v.x, v.y);
    }
}

template <class S>
__global__ void k_zero(S *X, int64_t ldx, int64_t rows) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (r < rows) X[(int64_t)c * ldx + r] = narrow<S>(0.0, 0.0);
}

// Counter-based starting block: uniform(-1,1)^2 from a splitmix64 hash of
// (seed, row, column), damped by 1/(1 + T_g) towards low kinetic energy.
template <class S>
__global__ void k_random_block(S *X, int64_t ldx, int64_t rows, uint64_t seed,
                               const double *__restrict__ kin) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (r >= rows) return;
    auto mix = [](uint64_t z) {
        z += 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    const uint64_t h1 = mix(seed ^ mix((uint64_t)r * 0x100000001B3ull + (uint64_t)c));
    const uint64_t h2 = mix(h1);
    const double u1 = (double)(h1 >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    const double u2 = (double)(h2 >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    const double d = 1.0 / (1.0 + kin[r]);
    X[(int64_t)c * ldx + r] = narrow<S>(u1 * d, u2 * d);
}

__global__ void k_pcoef(const cd *__restrict__ Cf, int64_t ldc, int n, int m, cd *__restrict__ Cp,
                        int64_t ldp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= n) return;
    Cp[(int64_t)j * ldp + i] = (i < m) ? cd{0.0, 0.0} : Cf[(int64_t)j * ldc + i];
}

__global__ void k_pcoef_map(const cd *__restrict__ Cf, int64_t ldc, int n, int m,
                            const int *__restrict__ act, cd *__restrict__ Cp, int64_t ldp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int jj = blockIdx.y;
    if (i >= n) return;
    Cp[(int64_t)jj * ldp + i] = (i < m) ? cd{0.0, 0.0} : Cf[(int64_t)act[jj] * ldc + i];
}

__global__ void k_convert_f64_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ void k_check_finite(const double *a, int64_t n, int *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) atomicOr(status, 4);
}

}  // namespace

size_t resid_part_elems(int64_t npw, int nb) {
    const int64_t nchunk = (npw + kChunk - 1) / kChunk;
    return (size_t)nchunk * nb * 3;
}

template <class S>
void band_dots_impl(const S *X, int64_t ldx, const S *HX, int64_t ldhx, const double *kin,
                    int64_t npw, int nb, double *part, double *theta, double *ekin, hipStream_t st,
                    const S *OX, int64_t ldox) {
    const int nchunk = (int)((npw + kChunk - 1) / kChunk);
    hipLaunchKernelGGL(k_band_dots<S>, dim3(nchunk, nb), dim3(kThreads), 0, st, X, ldx, HX, ldhx, kin,
                       npw, nb, part, OX, ldox);
    hipLaunchKernelGGL(k_band_dots_final, dim3(1), dim3(256), 0, st, part, nchunk, nb, theta, ekin);
    PW_HIP(hipGetLastError());
}
void launch_band_dots(const cd *X, int64_t ldx, const cd *HX, int64_t ldhx, const double *kin,
                      int64_t npw, int nb, double *part, double *theta, double *ekin, hipStream_t st,
                      const cd *OX, int64_t ldox) {
    band_dots_impl(X, ldx, HX, ldhx, kin, npw, nb, part, theta, ekin, st, OX, ldox);
}
void launch_band_dots(const cf *X, int64_t ldx, const cf *HX, int64_t ldhx, const double *kin,
                      int64_t npw, int nb, double *part, double *theta, double *ekin, hipStream_t st,
                      const cf *OX, int64_t ldox) {
    band_dots_impl(X, ldx, HX, ldhx, kin, npw, nb, part, theta, ekin, st, OX, ldox);
}

template <class S>
void resid_impl(const S *X, int64_t ldx, const S *HX, int64_t ldhx, const double *kin, int64_t npw,
                int nb, const double *theta, const double *ekin, S *W, int64_t ldw, double *part,
                double *res, hipStream_t st, const int *status) {
    const int nchunk = (int)((npw + kChunk - 1) / kChunk);
    hipLaunchKernelGGL(k_resid<S>, dim3(nchunk, nb), dim3(kThreads), 0, st, X, ldx, HX, ldhx, kin, npw,
                       nb, theta, ekin, W, ldw, part);
    // ekin array carries |x|^2 in its second half (see k_band_dots_final)
    hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(256), 0, st, part, nchunk, nb, ekin + nb, res, status);
    PW_HIP(hipGetLastError());
}
void launch_resid_precond(const cd *X, int64_t ldx, const cd *HX, int64_t ldhx, const double *kin,
                          int64_t npw, int nb, const double *theta, const double *ekin, cd *W,
                          int64_t ldw, double *part, double *res, hipStream_t st, const int *status) {
    resid_impl(X, ldx, HX, ldhx, kin, npw, nb, theta, ekin, W, ldw, part, res, st, status);
}
void launch_resid_precond(const cf *X, int64_t ldx, const cf *HX, int64_t ldhx, const double *kin,
                          int64_t npw, int nb, const double *theta, const double *ekin, cf *W,
                          int64_t ldw, double *part, double *res, hipStream_t st, const int *status) {
    resid_impl(X, ldx, HX, ldhx, kin, npw, nb, theta, ekin, W, ldw, part, res, st, status);
}

void launch_build_projectors_f64(const double *qvec, int64_t npw, int natom, const double *pos,
                                 int nlm, const int *lm, double pref, cd *B, int64_t ldb,
                                 hipStream_t st) {
    if (natom * nlm == 0) return;
    hipLaunchKernelGGL(k_build_projectors, dim3((unsigned)((npw + 255) / 256), natom * nlm),
                       dim3(256), 0, st, qvec, npw, natom, pos, nlm, lm, pref, B, ldb);
    PW_HIP(hipGetLastError());
}

template <class SA, class SB>
void copy_impl(const SA *A, int64_t lda, SB *B, int64_t ldb, int64_t rows, int cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL((k_copy_cols<SA, SB>), dim3((unsigned)((rows + 255) / 256), cols), dim3(256), 0,
                       st, A, lda, B, ldb, rows);
    PW_HIP(hipGetLastError());
}
void launch_copy_cols(const cd *A, int64_t lda, cd *B, int64_t ldb, int64_t rows, int cols, hipStream_t st) {
    copy_impl(A, lda, B, ldb, rows, cols, st);
}
void launch_copy_cols(const cf *A, int64_t lda, cf *B, int64_t ldb, int64_t rows, int cols, hipStream_t st) {
    copy_impl(A, lda, B, ldb, rows, cols, st);
}
void launch_copy_cols(const cd *A, int64_t lda, cf *B, int64_t ldb, int64_t rows, int cols, hipStream_t st) {
    copy_impl(A, lda, B, ldb, rows, cols, st);
}
void launch_copy_cols(const cf *A, int64_t lda, cd *B, int64_t ldb, int64_t rows, int cols, hipStream_t st) {
    copy_impl(A, lda, B, ldb, rows, cols, st);
}

template <class S>
void zero_impl(S *X, int64_t ldx, int64_t rows, int cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(k_zero<S>, dim3((unsigned)((rows + 255) / 256), cols), dim3(256), 0, st, X, ldx,
                       rows);
    PW_HIP(hipGetLastError());
}
void launch_zero(cd *X, int64_t ldx, int64_t rows, int cols, hipStream_t st) { zero_impl(X, ldx, rows, cols, st); }
void launch_zero(cf *X, int64_t ldx, int64_t rows, int cols, hipStream_t st) { zero_impl(X, ldx, rows, cols, st); }

template <class S>
void random_impl(S *X, int64_t ldx, int64_t rows, int cols, uint64_t seed, const double *kin,
                 hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(k_random_block<S>, dim3((unsigned)((rows + 255) / 256), cols), dim3(256), 0, st,
                       X, ldx, rows, seed, kin);
    PW_HIP(hipGetLastError());
}
void launch_random_block(cd *X, int64_t ldx, int64_t rows, int cols, uint64_t seed, const double *kin,
                         hipStream_t st) {
    random_impl(X, ldx, rows, cols, seed, kin, st);
}
void launch_random_block(cf *X, int64_t ldx, int64_t rows, int cols, uint64_t seed, const double *kin,
                         hipStream_t st) {
    random_impl(X, ldx, rows, cols, seed, kin, st);
}

void launch_pcoef_f64(const cd *Cfull, int64_t ldc, int n, int m, cd *Cp, int64_t ldp,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_pcoef, dim3((n + 255) / 256, m), dim3(256), 0, st, Cfull, ldc, n, m, Cp,
                       ldp);
    PW_HIP(hipGetLastError());
}

template <class S>
void precond_map_impl(const S *X, int64_t ldx, const S *HX, int64_t ldhx, const double *kin,
                      int64_t npw, const double *theta, const double *ekin_nrm, const int *act, int na,
                      S *W, int64_t ldw, hipStream_t st) {
    if (na <= 0) return;
    hipLaunchKernelGGL(k_precond_map<S>, dim3((unsigned)((npw + kThreads - 1) / kThreads), na),
                       dim3(kThreads), 0, st, X, ldx, HX, ldhx, kin, npw, theta, ekin_nrm, act, W, ldw);
    PW_HIP(hipGetLastError());
}
void launch_precond_map(const cd *X, int64_t ldx, const cd *HX, int64_t ldhx, const double *kin,
                        int64_t npw, const double *theta, const double *ekin_nrm, const int *act, int na,
                        cd *W, int64_t ldw, hipStream_t st) {
    precond_map_impl(X, ldx, HX, ldhx, kin, npw, theta, ekin_nrm, act, na, W, ldw, st);
}
void launch_precond_map(const cf *X, int64_t ldx, const cf *HX, int64_t ldhx, const double *kin,
                        int64_t npw, const double *theta, const double *ekin_nrm, const int *act, int na,
                        cf *W, int64_t ldw, hipStream_t st) {
    precond_map_impl(X, ldx, HX, ldhx, kin, npw, theta, ekin_nrm, act, na, W, ldw, st);
}

void launch_pcoef_map_f64(const cd *Cfull, int64_t ldc, int n, int m, const int *act, int na, cd *Cp,
                          int64_t ldp, hipStream_t st) {
    if (na <= 0) return;
    hipLaunchKernelGGL(k_pcoef_map, dim3((n + 255) / 256, na), dim3(256), 0, st, Cfull, ldc, n, m, act,
                       Cp, ldp);
    PW_HIP(hipGetLastError());
}

void launch_convert_f64_f32(const double *a, float *b, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_convert_f64_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
    PW_HIP(hipGetLastError());
}

void launch_check_finite_f64(const double *a, int64_t n, int *status, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n,
                       status);
    PW_HIP(hipGetLastError());
}

}  // namespace pw
