// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "pwlobpcg.h"

namespace pw {

// Interleaved complex with natural alignment (16 B for double, 8 B for float).
template <class T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};
using cd = cpx<double>;
using cf = cpx<float>;

// Error carrier used inside the runtime; converted to pw_status at the ABI.
struct Error {
    pw_status code;
    std::string msg;
};

#define PW_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::pw::Error{PW_ERR_DEVICE, std::string(#call) + ": " +              \
                                                 hipGetErrorString(e_)};              \
    } while (0)

#define PW_REQUIRE(cond, code, text)                                                  \
    do {                                                                              \
        if (!(cond)) throw ::pw::Error{code, text};                                   \
    } while (0)

// Device-side description of the plane-wave sphere and its z-sticks.
// Sphere order is lexicographic (n_x, n_y, n_z): stick s holds the contiguous
// range [st_start[s], st_start[s] + st_len[s]) with n_z = st_z0[s] + j.
struct SphereDev {
    int64_t npw = 0;
    int32_t n = 0;            // cubic FFT size
    int32_t nst = 0;          // number of sticks
    int32_t ldst = 0;         // padded stick count (leading dim of stick buffers)
    int32_t ncx = 0;          // kept x columns (n_x in [xmin, xmin + ncx))
    int32_t xmin = 0;
    int32_t *st_start = nullptr;  // [nst]
    int32_t *st_len = nullptr;    // [nst]
    int32_t *st_z0 = nullptr;     // [nst] signed n_z of the first element
    int32_t *st_y = nullptr;      // [nst] grid y index (n_y mod n)
    int32_t *st_xc = nullptr;     // [nst] kept-column index n_x - xmin
    int32_t *g_map = nullptr;     // [npw] (stick * n + (n_z mod n))
    double *kin = nullptr;        // [npw] 1/2 |k+G|^2
    double *twid = nullptr;       // [n] exp(+2 pi i j / n), interleaved
};

// Dynamic LDS limit of a kernel: raised through the runtime only when a launch
// needs more than the largest limit already set for that kernel on the current
// device, and never lowered, so launches of one kernel from several call sites
// or host threads cannot undercut each other (and the runtime call is not paid
// on every launch).
void ensure_smem_limit(const void *kernel, size_t bytes);

// ---- kernel launchers (implemented in the .hip files) ----------------------

// FFT apply (rows a2-a6): Y = T X + (V psi)(G) for nb columns.  S is the stick
// buffer [nb][n][ldst] complex.  v_zyx is V / n^3 in [z][y][x] order.
void launch_fft_apply(const SphereDev &sp, const double *v_zyx, const cd *X, int64_t ldx,
                      cd *Y, int64_t ldy, int nb, cd *S, hipStream_t st);
// complex64 form: v_zyx as float
void launch_fft_apply(const SphereDev &sp, const float *v_zyx, const cf *X, int64_t ldx,
                      cf *Y, int64_t ldy, int nb, cf *S, hipStream_t st);
// Density: rho_zyx[z][y][x] += sum_b occ[b] |psi_b|^2 for nb columns of X (psi
// = inverse transform of the sphere coefficients, no 1/sqrt(Omega)); then
// rho[x][y][z] = scale * rho_zyx[z][y][x].
void launch_density_accumulate(const SphereDev &sp, const cd *X, int64_t ldx, int nb,
                               const double *occ, double *rho_zyx, cd *S, hipStream_t st);
void launch_density_finish(const double *rho_zyx, int n, double scale, double *rho, hipStream_t st);
bool fft_size_supported(int n);
std::vector<int> fft_supported_sizes();
// One k-point of a multi-k-point apply: its sphere, X and Y, its stick buffer.
// All items share the FFT grid, the radix split and the potential.
template <class T>
struct FftApplyItem {
    SphereDev sp;
    const cpx<T> *X;
    int64_t ldx;
    cpx<T> *Y;
    int64_t ldy;
    cpx<T> *S;
};
constexpr int kMaxApplyBatch = 16;   // k-points per launch (the items travel as kernel arguments)
// Y_k = T_k X_k + (V psi_k)(G) for nb columns of every item: each pass is one
// launch over all (k-point, band) work items.
void launch_fft_apply_batch(const FftApplyItem<double> *items, int nk, const double *v_zyx, int nb,
                            hipStream_t st);
void launch_fft_apply_batch(const FftApplyItem<float> *items, int nk, const float *v_zyx, int nb,
                            hipStream_t st);

// Launch parameters of the FFT passes and the split-K GEMM chosen per context
// (pw_autotune / pw_set_tuning; 0 = built-in default).  The launchers read the
// record of the context whose API call is running on this host thread.
struct Tuning {
    int fft_spb = 0;        // sticks per workgroup of the z passes
    int fft_rb = 0;         // row chunk of the plane pass (capped by LDS)
    int tn_split_wgs = 0;   // target workgroup count of a split-K TN launch
    int fft_r2 = 0;         // second factor R2 of the radix split N = R1 R2 (0: default)
};
// radix splits N = R1 R2 available for length n (R2 values) and the default R2
std::vector<int> fft_radix_splits(int n);
int fft_default_r2(int n);
const Tuning &thread_tuning();
const Tuning *set_thread_tuning(const Tuning *t);   // returns the previous record
constexpr int kTnSplitMax = 1024;   // largest split target; partial buffers are sized for it

// Complex GEMMs on MFMA over complex128 (cd) or complex64 (cf) blocks;
// small outputs and coefficient matrices are always complex128.
//   tn: part[s] = A^H B over K-chunk s; reduce: C = scale_row * sum_s part[s] (+ beta C)
size_t gemm_tn_part_elems(int64_t K, int p, int q, int *nsplit_out);
void launch_gemm_tn(const cd *A, int64_t lda, const cd *B, int64_t ldb, int64_t K, int p, int q,
                    cd *C, int64_t ldc, const double *scale_row, double beta, cd *part,
                    size_t part_elems, hipStream_t st);
void launch_gemm_tn(const cf *A, int64_t lda, const cf *B, int64_t ldb, int64_t K, int p, int q,
                    cd *C, int64_t ldc, const double *scale_row, double beta, cd *part,
                    size_t part_elems, hipStream_t st);
//   nn: Y = alpha A C + beta Y
void launch_gemm_nn(const cd *A, int64_t lda, const cd *C, int64_t ldc, int64_t K, int p, int q,
                    double alpha, double beta, cd *Y, int64_t ldy, hipStream_t st);
void launch_gemm_nn(const cf *A, int64_t lda, const cd *C, int64_t ldc, int64_t K, int p, int q,
                    double alpha, double beta, cf *Y, int64_t ldy, hipStream_t st);
//   the same two products on complex64 blocks with split-bf16 MFMA products
void launch_gemm_tn_bf16(const cf *A, int64_t lda, const cf *B, int64_t ldb, int64_t K, int p, int q,
                         cd *C, int64_t ldc, const double *scale_row, double beta, cd *part,
                         size_t part_elems, hipStream_t st, bool herm = false);
// A^H B for a Hermitian product (B = H A, H Hermitian): the p x p result with
// only the tiles on and above the diagonal formed, the others mirrored
void launch_gemm_herm(const cd *A, int64_t lda, const cd *B, int64_t ldb, int64_t K, int p, cd *C,
                      int64_t ldc, cd *part, size_t part_elems, hipStream_t st);
void launch_gemm_herm(const cf *A, int64_t lda, const cf *B, int64_t ldb, int64_t K, int p, cd *C,
                      int64_t ldc, cd *part, size_t part_elems, hipStream_t st);
void launch_gemm_nn_bf16(const cf *A, int64_t lda, const cd *C, int64_t ldc, int64_t K, int p, int q,
                         double alpha, double beta, cf *Y, int64_t ldy, hipStream_t st);

// Small dense FP64 (single workgroup).  fp32_reduction: the Householder
// reduction (n <= 192) runs in FP32 on the input rounded to float (the
// Rayleigh-Ritz problems of the complex64 stage of the mixed iteration); the
// eigenvalues, inverse iteration, orthogonalisation and back-transform stay
// FP64.
size_t heev_scratch_bytes(int n, int k);
void launch_heev_f64(cd *A, int64_t lda, int n, int k, double *w, cd *V, int64_t ldv,
                     void *scratch, int *status, hipStream_t st, bool fp32_reduction = false);
// Library-owned device scratch of the entry point that allocates nothing
// (noalloc.hip): a fixed array per GPU.  static_scratch_setup resolves its
// device address with `device` current (once per device, from pw_create);
// static_scratch returns that address (null until then).
size_t static_scratch_bytes();
hipError_t static_scratch_setup(int device);
void *static_scratch(int device);
void launch_clear_ints(int *p, int count, hipStream_t st);   // fill kernel, no memset node
// CholQR factor: G (n x n, Hermitian PD) -> Rinv (upper, G = R^H R, Rinv = R^-1)
// with a diagonal shift for robustness; status[0] |= 1 on breakdown.
void launch_chol_inv_f64(const cd *G, int64_t ldg, int n, cd *Rinv, int64_t ldr, int *status,
                         hipStream_t st);

// Vector kernels.
size_t resid_part_elems(int64_t npw, int nb);
// Blocks are complex128 (cd) or complex64 (cf); every reduction is in double.
// theta[nb]; ekin_nrm[2 nb] = (E_kin per band, |x|^2 per band); with OX (the
// generalized form) the norm is Re(x^H O x) and theta = x^H H x / x^H O x
void launch_band_dots(const cd *X, int64_t ldx, const cd *HX, int64_t ldhx, const double *kin,
                      int64_t npw, int nb, double *part, double *theta, double *ekin_nrm, hipStream_t st,
                      const cd *OX = nullptr, int64_t ldox = 0);
void launch_band_dots(const cf *X, int64_t ldx, const cf *HX, int64_t ldhx, const double *kin,
                      int64_t npw, int nb, double *part, double *theta, double *ekin_nrm, hipStream_t st,
                      const cf *OX = nullptr, int64_t ldox = 0);
void launch_resid_precond(const cd *X, int64_t ldx, const cd *HX, int64_t ldhx, const double *kin,
                          int64_t npw, int nb, const double *theta, const double *ekin_nrm, cd *W,
                          int64_t ldw, double *part, double *res, hipStream_t st,
                          const int *status = nullptr);   // status: also stored as res[nb]
void launch_resid_precond(const cf *X, int64_t ldx, const cf *HX, int64_t ldhx, const double *kin,
                          int64_t npw, int nb, const double *theta, const double *ekin_nrm, cf *W,
                          int64_t ldw, double *part, double *res, hipStream_t st,
                          const int *status = nullptr);   // status: also stored as res[nb]
void launch_build_projectors_f64(const double *qvec, int64_t npw, int natom, const double *pos,
                                 int nlm, const int *lm, double pref, cd *B, int64_t ldb,
                                 hipStream_t st);
// v_zyx in the layout of radix split r2 (0: the default split)
void launch_permute_potential(const double *v, int n, double scale, double *v_zyx,
                              int *bad, int r2, hipStream_t st);
// a permuted potential moved from the layout of split r2_from to that of r2_to
void launch_repermute_potential(const double *in, int n, int r2_from, int r2_to, double *out,
                                hipStream_t st);
// column copy, with conversion when the storage types differ
void launch_copy_cols(const cd *A, int64_t lda, cd *B, int64_t ldb, int64_t rows, int cols, hipStream_t st);
void launch_copy_cols(const cf *A, int64_t lda, cf *B, int64_t ldb, int64_t rows, int cols, hipStream_t st);
void launch_copy_cols(const cd *A, int64_t lda, cf *B, int64_t ldb, int64_t rows, int cols, hipStream_t st);
void launch_copy_cols(const cf *A, int64_t lda, cd *B, int64_t ldb, int64_t rows, int cols, hipStream_t st);
void launch_random_block(cd *X, int64_t ldx, int64_t rows, int cols, uint64_t seed, const double *kin,
                         hipStream_t st);
void launch_random_block(cf *X, int64_t ldx, int64_t rows, int cols, uint64_t seed, const double *kin,
                         hipStream_t st);
void launch_zero(cd *X, int64_t ldx, int64_t rows, int cols, hipStream_t st);
void launch_zero(cf *X, int64_t ldx, int64_t rows, int cols, hipStream_t st);
// P-coefficient block: rows [0, m) of Cfull set to zero (the X rows), others copied.
void launch_pcoef_f64(const cd *Cfull, int64_t ldc, int n, int m, cd *Cp, int64_t ldp,
                      hipStream_t st);
// Active-set variants: column jj of the output takes input column act[jj].
void launch_precond_map(const cd *X, int64_t ldx, const cd *HX, int64_t ldhx, const double *kin,
                        int64_t npw, const double *theta, const double *ekin_nrm, const int *act, int na,
                        cd *W, int64_t ldw, hipStream_t st);
void launch_precond_map(const cf *X, int64_t ldx, const cf *HX, int64_t ldhx, const double *kin,
                        int64_t npw, const double *theta, const double *ekin_nrm, const int *act, int na,
                        cf *W, int64_t ldw, hipStream_t st);
void launch_pcoef_map_f64(const cd *Cfull, int64_t ldc, int n, int m, const int *act, int na, cd *Cp,
                          int64_t ldp, hipStream_t st);
void launch_check_finite_f64(const double *a, int64_t n, int *status, hipStream_t st);
void launch_convert_f64_f32(const double *a, float *b, int64_t n, hipStream_t st);

}  // namespace pw
