// Small dense FP64 steps of the iteration, each in one workgroup.
//
//  * k_chol_inv: Cholesky factor of a Gram matrix G = R^H R and R^-1, used to
//    orthonormalise a block (W <- W R^-1; BLOPEX-style LOBPCG, sec. 3.2).
//  * k_heev: lowest k eigenpairs of a Hermitian matrix -- the Rayleigh-Ritz
//    eigenproblem of Algorithm 1 step 4 (size 3m) and of the final
//    Rayleigh-Ritz over all bands (sec. 3.2, sec. 4.2).  Householder
//    reduction to real tridiagonal form, bisection with Sturm counts,
//    inverse iteration, classical Gram-Schmidt applied twice, back-transform.
#include <cfloat>

#include "pw_internal.h"

namespace pw {
namespace {

constexpr int kDenseThreads = 512;

__device__ __forceinline__ cd cconj(cd a) { return {a.x, -a.y}; }
__device__ __forceinline__ cd cmulz(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// Block-wide sum of one double per thread (fixed order: deterministic).
__device__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// ---- Cholesky + inverse of the factor (n <= 64, in LDS) ---------------------
constexpr int kCholMax = 64;

__global__ void __launch_bounds__(256) k_chol_inv(const cd *__restrict__ G, int64_t ldg, int n,
                                                  cd *__restrict__ Rinv, int64_t ldr, int *status) {
    __shared__ cd Rs[kCholMax][kCholMax + 1];   // R (upper), row-major [row][col]
    __shared__ cd Xs[kCholMax][kCholMax + 1];   // R^-1
    __shared__ double dmax;
    __shared__ int fail;
    const int t = threadIdx.x;
    for (int i = t; i < n * n; i += blockDim.x) {
        const int r = i % n, c = i / n;
        Rs[r][c] = G[(int64_t)c * ldg + r];
    }
    if (t == 0) fail = 0;
    __syncthreads();
    if (t == 0) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, Rs[i][i].x);
        dmax = m;
    }
    __syncthreads();
    // a tiny diagonal shift keeps a numerically semi-definite Gram factorable
    const double shift = 1e-15 * dmax * n;
    for (int j = 0; j < n; ++j) {
        if (t == 0) {
            double d = Rs[j][j].x + shift;
            if (!(d > 1e-300) || !isfinite(d)) {
                fail = 1;
                d = 1.0;
            }
            Rs[j][j] = cd{sqrt(d), 0.0};
        }
        __syncthreads();
        const double inv = 1.0 / Rs[j][j].x;
        for (int c = j + 1 + t; c < n; c += blockDim.x) Rs[j][c] = cd{Rs[j][c].x * inv, Rs[j][c].y * inv};
        __syncthreads();
        const int m = n - j - 1;
        for (int i = t; i < m * m; i += blockDim.x) {
            const int a = j + 1 + i % m, b = j + 1 + i / m;
            if (b >= a) {
                const cd u = cconj(Rs[j][a]), v = Rs[j][b];
                const cd pr = cmulz(u, v);
                Rs[a][b].x -= pr.x;
                Rs[a][b].y -= pr.y;
            }
        }
        __syncthreads();
    }
    // R^-1 column by column: X_cc = 1/R_cc, X_ic = -(sum_{k=i+1..c} R_ik X_kc) / R_ii
    for (int c = t; c < n; c += blockDim.x) {
        for (int i = 0; i < n; ++i) Xs[i][c] = cd{0.0, 0.0};
        Xs[c][c] = cd{1.0 / Rs[c][c].x, 0.0};
        for (int i = c - 1; i >= 0; --i) {
            double sr = 0.0, si = 0.0;
            for (int k = i + 1; k <= c; ++k) {
                const cd pr = cmulz(Rs[i][k], Xs[k][c]);
                sr += pr.x;
                si += pr.y;
            }
            const double inv = 1.0 / Rs[i][i].x;
            Xs[i][c] = cd{-sr * inv, -si * inv};
        }
    }
    __syncthreads();
    for (int i = t; i < n * n; i += blockDim.x) {
        const int r = i % n, c = i / n;
        Rinv[(int64_t)c * ldr + r] = Xs[r][c];
    }
    if (t == 0 && fail) atomicOr(status, 1);
}

// ---- Hermitian eigensolver ---------------------------------------------------
struct HeevScratch {
    cd *tau;        // [n]
    double *d;      // [n]
    double *e;      // [n]
    double *Z;      // [n][k] tridiagonal eigenvectors, row i at Z + i*k
    double *lu;     // [5][n][k] per-eigenvalue LU factors, interleaved by eigenvalue
};

__device__ int sturm_count(const double *d, const double *e2, int n, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
        q = d[i] - x - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++cnt;
    }
    return cnt;
}

__global__ void __launch_bounds__(kDenseThreads)
    k_heev(cd *__restrict__ A, int64_t lda, int n, int k, double *__restrict__ w,
           cd *__restrict__ V, int64_t ldv, HeevScratch sc, int *status) {
    extern __shared__ unsigned char smem_raw[];
    cd *vs = reinterpret_cast<cd *>(smem_raw);   // [n]
    cd *ys = vs + n;                              // [n]
    cd *ws = ys + n;                              // [n]
    cd *ps = ws + n;                              // [blockDim] matvec partials
    double *red = reinterpret_cast<double *>(ps + blockDim.x);   // [blockDim]
    double *ds = red + blockDim.x;                // [n]
    double *e2 = ds + n;                          // [n]
    __shared__ cd tau_s;
    __shared__ double beta_s;

    const int t = threadIdx.x, nt = blockDim.x;
    auto Aat = [&](int r, int c) -> cd & { return A[(int64_t)c * lda + r]; };

    // ---- 1. Householder reduction to real tridiagonal (lower) ----
    for (int j = 0; j + 1 < n; ++j) {
        const int L = n - j - 1;
        // norm of x[1:] where x = A[j+1:, j]
        double part = 0.0;
        for (int i = 1 + t; i < L; i += nt) {
            const cd x = Aat(j + 1 + i, j);
            part += x.x * x.x + x.y * x.y;
        }
        const double sigma = block_sum(part, red);
        if (t == 0) {
            const cd alpha = Aat(j + 1, j);
            if (sigma == 0.0 && alpha.y == 0.0) {
                tau_s = cd{0.0, 0.0};
                beta_s = alpha.x;
            } else {
                const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sigma);
                const double beta = alpha.x >= 0.0 ? -nrm : nrm;
                tau_s = cd{(beta - alpha.x) / beta, -alpha.y / beta};
                // scale = 1 / (alpha - beta)
                const double dr = alpha.x - beta, di = alpha.y;
                const double den = dr * dr + di * di;
                ys[0] = cd{dr / den, -di / den};
                beta_s = beta;
            }
        }
        __syncthreads();
        const cd tau = tau_s;
        const bool reflect = !(tau.x == 0.0 && tau.y == 0.0);
        if (reflect) {
            const cd scale = ys[0];
            for (int i = t; i < L; i += nt) {
                if (i == 0) {
                    vs[0] = cd{1.0, 0.0};
                } else {
                    const cd x = Aat(j + 1 + i, j);
                    const cd v = cmulz(x, scale);
                    vs[i] = v;
                    Aat(j + 1 + i, j) = v;
                }
            }
        }
        if (t == 0) {
            sc.tau[j] = tau;
            sc.e[j] = beta_s;
            Aat(j + 1, j) = cd{beta_s, 0.0};
            sc.d[j] = Aat(j, j).x;
        }
        __syncthreads();
        if (reflect) {
            // y = A_sub v, A_sub = A[j+1:, j+1:] (full Hermitian storage)
            const int groups = max(1, nt / L);
            for (int r0 = 0; r0 < L; r0 += nt) {
                // generic path: one thread per row when L >= nt, else column groups
                if (groups == 1) {
                    const int i = r0 + t;
                    if (i < L) {
                        double sr = 0.0, si = 0.0;
                        for (int c = 0; c < L; ++c) {
                            const cd a = Aat(j + 1 + i, j + 1 + c);
                            const cd v = vs[c];
                            sr += a.x * v.x - a.y * v.y;
                            si += a.x * v.y + a.y * v.x;
                        }
                        ys[i] = cd{sr, si};
                    }
                } else {
                    const int i = t % L, cg = t / L;
                    double sr = 0.0, si = 0.0;
                    if (cg < groups) {
                        const int cb = (int)((int64_t)cg * L / groups);
                        const int ce = (int)((int64_t)(cg + 1) * L / groups);
                        for (int c = cb; c < ce; ++c) {
                            const cd a = Aat(j + 1 + i, j + 1 + c);
                            const cd v = vs[c];
                            sr += a.x * v.x - a.y * v.y;
                            si += a.x * v.y + a.y * v.x;
                        }
                    }
                    // partials in ps[cg * L + i] (groups * L <= nt)
                    if (cg < groups) ps[cg * L + i] = cd{sr, si};
                    __syncthreads();
                    if (t < L) {
                        double ar = 0.0, ai = 0.0;
                        for (int q2 = 0; q2 < groups; ++q2) {
                            ar += ps[q2 * L + t].x;
                            ai += ps[q2 * L + t].y;
                        }
                        ys[t] = cd{ar, ai};
                    }
                    break;
                }
            }
            __syncthreads();
            // alpha = |tau|^2 / 2 * Re(v^H y);  w = tau y - alpha v
            double pv = 0.0;
            for (int i = t; i < L; i += nt) pv += vs[i].x * ys[i].x + vs[i].y * ys[i].y;
            const double vhy = block_sum(pv, red);
            const double alpha = 0.5 * (tau.x * tau.x + tau.y * tau.y) * vhy;
            for (int i = t; i < L; i += nt) {
                const cd ty = cmulz(tau, ys[i]);
                ws[i] = cd{ty.x - alpha * vs[i].x, ty.y - alpha * vs[i].y};
            }
            __syncthreads();
            // A_sub -= w v^H + v w^H
            const int64_t tot = (int64_t)L * L;
            for (int64_t idx = t; idx < tot; idx += nt) {
                const int i = (int)(idx % L), c = (int)(idx / L);
                const cd a1 = cmulz(ws[i], cconj(vs[c]));
                const cd a2 = cmulz(vs[i], cconj(ws[c]));
                cd &a = Aat(j + 1 + i, j + 1 + c);
                a.x -= a1.x + a2.x;
                a.y -= a1.y + a2.y;
            }
            __syncthreads();
        }
    }
    if (t == 0) {
        sc.d[n - 1] = Aat(n - 1, n - 1).x;
        if (n >= 1) sc.e[n - 1] = 0.0;
    }
    __syncthreads();
    for (int i = t; i < n; i += nt) {
        ds[i] = sc.d[i];
        e2[i] = (i + 1 < n) ? sc.e[i] * sc.e[i] : 0.0;
    }
    __syncthreads();

    // ---- 2. bisection for eigenvalues 0..k-1 of T ----
    double gl = ds[0], gu = ds[0], tnorm = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(sc.e[i - 1]) : 0.0) + (i + 1 < n ? fabs(sc.e[i]) : 0.0);
        gl = fmin(gl, ds[i] - r);
        gu = fmax(gu, ds[i] + r);
        tnorm = fmax(tnorm, fabs(ds[i]) + r);
    }
    const double pivmin = DBL_MIN * fmax(1.0, tnorm * tnorm);
    const double span = fmax(gu - gl, DBL_EPSILON * fmax(1.0, tnorm));
    gl -= 2.0 * DBL_EPSILON * span + 1e-300;
    gu += 2.0 * DBL_EPSILON * span + 1e-300;
    for (int idx = t; idx < k; idx += nt) {
        double lo = gl, hi = gu;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) break;
            if (sturm_count(ds, e2, n, mid, pivmin) <= idx) lo = mid;
            else hi = mid;
        }
        w[idx] = 0.5 * (lo + hi);
    }
    __syncthreads();

    // ---- 3. inverse iteration on T for each eigenvalue ----
    // (T - lambda I) = P L U, tridiagonal LU with partial pivoting; arrays
    // interleaved [i][idx] so that threads access consecutive addresses.
    double *dl = sc.lu;                   // multipliers
    double *dd = sc.lu + (int64_t)n * k;  // U diagonal
    double *du = sc.lu + 2 * (int64_t)n * k;   // U first superdiagonal
    double *du2 = sc.lu + 3 * (int64_t)n * k;  // U second superdiagonal (fill)
    double *piv = sc.lu + 4 * (int64_t)n * k;  // 1 if rows swapped
    const double eps_t = DBL_EPSILON * fmax(tnorm, 1e-300);
    for (int idx = t; idx < k; idx += nt) {
        const double lam = w[idx];
        auto at = [&](double *arr, int i) -> double & { return arr[(int64_t)i * k + idx]; };
        // factor
        for (int i = 0; i < n; ++i) {
            at(dd, i) = ds[i] - lam;
            at(du, i) = (i + 1 < n) ? sc.e[i] : 0.0;
            at(du2, i) = 0.0;
            at(piv, i) = 0.0;
        }
        for (int i = 0; i + 1 < n; ++i) {
            const double sub = sc.e[i];   // A[i+1][i]
            if (fabs(at(dd, i)) >= fabs(sub)) {
                double di = at(dd, i);
                if (fabs(di) < eps_t) di = (di < 0 ? -eps_t : eps_t);
                at(dd, i) = di;
                const double m = sub / di;
                at(dl, i) = m;
                at(dd, i + 1) -= m * at(du, i);
            } else {
                // swap rows i and i+1
                const double m = at(dd, i) / sub;
                at(dl, i) = m;
                at(piv, i) = 1.0;
                at(dd, i) = sub;
                const double tmp = at(du, i);
                at(du, i) = at(dd, i + 1);
                at(dd, i + 1) = tmp - m * at(dd, i + 1);
                if (i + 2 < n) {
                    at(du2, i) = at(du, i + 1);
                    at(du, i + 1) = -m * at(du, i + 1);
                }
            }
        }
        if (fabs(at(dd, n - 1)) < eps_t) at(dd, n - 1) = eps_t;
        // starting vector: deterministic pseudo-random in (-1, 1)
        double *z = sc.Z;
        auto zat = [&](int i) -> double & { return z[(int64_t)i * k + idx]; };
        for (int i = 0; i < n; ++i) {
            uint64_t h = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull ^ (uint64_t)(idx + 7) * 0xD1B54A32D192ED03ull;
            h ^= h >> 31;
            h *= 0xBF58476D1CE4E5B9ull;
            h ^= h >> 29;
            zat(i) = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        }
        for (int iter = 0; iter < 3; ++iter) {
            // apply L^-1 P
            for (int i = 0; i + 1 < n; ++i) {
                if (at(piv, i) != 0.0) {
                    const double tmp = zat(i);
                    zat(i) = zat(i + 1);
                    zat(i + 1) = tmp - at(dl, i) * zat(i + 1);
                } else {
                    zat(i + 1) -= at(dl, i) * zat(i);
                }
            }
            // U^-1
            double nrm = 0.0;
            for (int i = n - 1; i >= 0; --i) {
                double s = zat(i);
                if (i + 1 < n) s -= at(du, i) * zat(i + 1);
                if (i + 2 < n) s -= at(du2, i) * zat(i + 2);
                zat(i) = s / at(dd, i);
            }
            for (int i = 0; i < n; ++i) nrm = fmax(nrm, fabs(zat(i)));
            const double inv = nrm > 0 ? 1.0 / nrm : 1.0;
            for (int i = 0; i < n; ++i) zat(i) *= inv;
        }
    }
    __syncthreads();

    // ---- 4. classical Gram-Schmidt, twice, in eigenvalue order ----
    double *Z = sc.Z;
    for (int j = 0; j < k; ++j) {
        for (int pass = 0; pass < 2; ++pass) {
            // coefficients c_i = z_i . z_j for i < j (one thread per i)
            // red[] holds up to nt coefficients; process in chunks of nt.
            for (int ib = 0; ib < j; ib += nt) {
                const int i = ib + t;
                double c = 0.0;
                if (i < j)
                    for (int r = 0; r < n; ++r) c += Z[(int64_t)r * k + i] * Z[(int64_t)r * k + j];
                __syncthreads();
                red[t] = c;
                __syncthreads();
                const int cnt = min(nt, j - ib);
                for (int r = t; r < n; r += nt) {
                    double s = Z[(int64_t)r * k + j];
                    for (int q2 = 0; q2 < cnt; ++q2) s -= red[q2] * Z[(int64_t)r * k + ib + q2];
                    Z[(int64_t)r * k + j] = s;
                }
                __syncthreads();
            }
            double pn = 0.0;
            for (int r = t; r < n; r += nt) {
                const double v = Z[(int64_t)r * k + j];
                pn += v * v;
            }
            const double nn = block_sum(pn, red);
            const double inv = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
            if (!(nn > 0) && t == 0) atomicOr(status, 2);
            for (int r = t; r < n; r += nt) Z[(int64_t)r * k + j] *= inv;
            __syncthreads();
        }
    }

    // ---- 5. back-transform V = H_0 ... H_{n-2} Z ----
    for (int idx = t; idx < n * k; idx += nt) {
        const int r = idx % n, c = idx / n;
        V[(int64_t)c * ldv + r] = cd{Z[(int64_t)r * k + c], 0.0};
    }
    __syncthreads();
    for (int j = n - 2; j >= 0; --j) {
        const cd tau = sc.tau[j];
        if (tau.x == 0.0 && tau.y == 0.0) continue;
        const int L = n - j - 1;
        // s_c = v^H V[j+1:, c]
        for (int c = t; c < k; c += nt) {
            double sr = 0.0, si = 0.0;
            for (int i = 0; i < L; ++i) {
                const cd v = (i == 0) ? cd{1.0, 0.0} : Aat(j + 1 + i, j);
                const cd x = V[(int64_t)c * ldv + j + 1 + i];
                sr += v.x * x.x + v.y * x.y;
                si += v.x * x.y - v.y * x.x;
            }
            const cd s = cmulz(tau, cd{sr, si});
            for (int i = 0; i < L; ++i) {
                const cd v = (i == 0) ? cd{1.0, 0.0} : Aat(j + 1 + i, j);
                cd &x = V[(int64_t)c * ldv + j + 1 + i];
                const cd pr = cmulz(v, s);
                x.x -= pr.x;
                x.y -= pr.y;
            }
        }
        __syncthreads();
    }
    for (int idx = t; idx < k; idx += nt)
        if (!isfinite(w[idx])) atomicOr(status, 4);
}

}  // namespace

void launch_chol_inv_f64(const cd *G, int64_t ldg, int n, cd *Rinv, int64_t ldr, int *status,
                         hipStream_t st) {
    PW_REQUIRE(n >= 1 && n <= kCholMax, PW_ERR_ARG, "block size must be in [1, 64]");
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, st, G, ldg, n, Rinv, ldr, status);
    PW_HIP(hipGetLastError());
}

size_t heev_scratch_bytes(int n, int k) {
    return 256 + (size_t)n * 16 + 2 * (size_t)n * 8 + 6 * (size_t)n * k * 8 + 4 * 256;
}

void launch_heev_f64(cd *A, int64_t lda, int n, int k, double *w, cd *V, int64_t ldv, void *scratch,
                     int *status, hipStream_t st) {
    PW_REQUIRE(n >= 1 && n <= 1024 && k >= 1 && k <= n, PW_ERR_ARG, "heev: need 1 <= k <= n <= 1024");
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    char *p = static_cast<char *>(scratch);
    HeevScratch sc;
    sc.tau = reinterpret_cast<cd *>(p);
    p += align((size_t)n * 16);
    sc.d = reinterpret_cast<double *>(p);
    p += align((size_t)n * 8);
    sc.e = reinterpret_cast<double *>(p);
    p += align((size_t)n * 8);
    sc.Z = reinterpret_cast<double *>(p);
    p += align((size_t)n * k * 8);
    sc.lu = reinterpret_cast<double *>(p);
    const size_t smem = 3 * (size_t)n * sizeof(cd) + (size_t)kDenseThreads * (sizeof(cd) + 8) +
                        2 * (size_t)n * 8;
    PW_HIP(hipFuncSetAttribute((const void *)k_heev, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)smem));
    hipLaunchKernelGGL(k_heev, dim3(1), dim3(kDenseThreads), smem, st, A, lda, n, k, w, V, ldv, sc,
                       status);
    PW_HIP(hipGetLastError());
}

}  // namespace pw
