// Complex FP64 GEMMs on the gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
// Sec. 4.1: the Gram blocks of LOBPCG and the block updates are dense complex
// matrix products over the plane-wave coefficients ("zgemm"), and sec. 5.1
// finds them to dominate the run time.  Two shapes occur:
//
//   tn:  C[p x q] = A^H B   with A [K x p], B [K x q], K = npw large
//        (Gram blocks, projector overlaps B^H X, constraint overlaps Y^H W).
//        Split over K into chunks; each workgroup writes its partial tile,
//        and a second kernel sums the partials in a fixed order, so results
//        are bitwise reproducible (no floating-point atomics).
//   nn:  Y[K x q] = alpha A C + beta Y   with C [p x q] small
//        (block updates Psi Delta + W Lambda + P Gamma, projector add-back,
//        orthonormalisation W <- W R^-1).
//
// A complex product is four real MFMAs (re.re, im.im, re.im, im.re).  The
// MFMA contraction index is mapped so that lane group g = lane/16 consumes
// k = kb + 4g + s in step s: each lane then reads four consecutive complex
// elements of one column (64 contiguous bytes), and lanes 16 apart read the
// neighbouring 64 bytes.
//
// MFMA operand layout (16x16x4, wave64): A operand lane l holds
// A[i = l%16][k = l/16]; B operand lane l holds B[k = l/16][j = l%16].  Result
// register r of lane l holds D[i][j = l%16] with i = l/16 + 4r for the f64
// form and i = 4(l/16) + r for the f32 form (both measured on gfx950).
//
// The same kernels serve complex128 blocks (v_mfma_f64_16x16x4f64) and the
// complex64 blocks of the mixed-precision form (v_mfma_f32_16x16x4f32, FP32
// products and accumulation within a K chunk; the chunk partials are summed
// in double).  Small coefficient matrices are always complex128 and are
// rounded to the block type as they are loaded.
//
// A third form serves the projector products of the BF16 mixed iteration:
// complex64 operands are split into bf16 pairs (x = hi + lo, hi = bf16(x),
// lo = bf16(x - hi)) and each real product is hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x16_bf16 with FP32 accumulation (the split-bfloat16
// scheme of Henry, Tang and Heinecke, ARITH 2019); the dropped lo*lo term and
// the rounding of lo leave a relative error near 2^-16 per product.
#include <atomic>
#include <type_traits>

#include "pw_internal.h"

namespace pw {
namespace {

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

constexpr int kTile = 64;      // workgroup tile (complex elements) per dimension
constexpr int kThreads = 256;  // 4 waves in a 2 x 2 arrangement, 32 x 32 each


// Loading operand tiles.  complex64: the loads carry no condition, their
// addresses are clamped into the operand, and values outside it are replaced
// by zero only where they are written to LDS (a load under a branch is waited
// on inside that branch, which turned the prefetch of the next k-block into a
// stall: the complex64 Gram 138 -> 89 us).  FP64 keeps the zero chosen at the
// load, which measured 2-7 % faster there (its MFMA takes twice the cycles, so
// the loads are off the critical path).
template <class T>
constexpr bool kZeroAtLoad = sizeof(T) == 8;
template <class T>
__device__ __forceinline__ cpx<T> tile_load(const cpx<T> *p, bool ok) {
    if constexpr (kZeroAtLoad<T>) return ok ? *p : cpx<T>{T(0), T(0)};
    return *p;
}
template <class T>
__device__ __forceinline__ cpx<T> tile_keep(const cpx<T> &v, bool ok) {
    if constexpr (kZeroAtLoad<T>) return v;
    return cpx<T>{ok ? v.x : T(0), ok ? v.y : T(0)};
}
// coefficient elements (complex128), rounded to the block type at the store
template <class T>
__device__ __forceinline__ cd coef_load(const cd *p, bool ok) {
    if constexpr (kZeroAtLoad<T>) return ok ? *p : cd{0.0, 0.0};
    return *p;
}
template <class T>
__device__ __forceinline__ cpx<T> coef_keep(const cd &v, bool ok) {
    if constexpr (kZeroAtLoad<T>) return cpx<T>{T(v.x), T(v.y)};
    return cpx<T>{ok ? T(v.x) : T(0), ok ? T(v.y) : T(0)};
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
struct Bf16Pair {
    s16x4 hi, lo;
};
// four FP32 values (consecutive k of one MFMA operand) as a hi/lo bf16 pair
__device__ __forceinline__ Bf16Pair split_bf16(float v0, float v1, float v2, float v3) {
    const f32x4 v = {v0, v1, v2, v3};
    const bf16x4 h = __builtin_convertvector(v, bf16x4);
    const bf16x4 l = __builtin_convertvector(v - __builtin_convertvector(h, f32x4), bf16x4);
    return {__builtin_bit_cast(s16x4, h), __builtin_bit_cast(s16x4, l)};
}
// c += a b over 16 k with the three split products, small terms first
__device__ __forceinline__ f32x4 mma_split(const Bf16Pair &a, const Bf16Pair &b, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, c, 0, 0, 0);
}

// Map a hardware workgroup id to a logical id so that each XCD (ids are
// dealt round-robin over 8 XCDs) receives a contiguous range.
__device__ __forceinline__ int xcd_logical(int lin, int total) {
    const int q = total / 8, r = total % 8;
    const int xcd = lin % 8, local = lin / 8;
    return xcd * q + min(xcd, r) + local;
}

// One k-block of the 3-multiplication complex product in split-bf16 form.
// SIGN = -1 forms t3 from (ar - ai)(br + bi) (TN, conj(a) b), SIGN = +1 from
// (ar + ai)(br + bi) (NN, a b); a, b hold k = 4g + s, s = 0..3.
template <int SIGN>
__device__ __forceinline__ void mma_bf16(const cpx<float> (&a)[2][4], const cpx<float> (&b)[2][4],
                                         const bool (&live)[2][2], f32x4 (&t1)[2][2],
                                         f32x4 (&t2)[2][2], f32x4 (&t3)[2][2]) {
    Bf16Pair ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        ar[t] = split_bf16(a[t][0].x, a[t][1].x, a[t][2].x, a[t][3].x);
        ai[t] = split_bf16(a[t][0].y, a[t][1].y, a[t][2].y, a[t][3].y);
        as[t] = split_bf16(a[t][0].x + SIGN * a[t][0].y, a[t][1].x + SIGN * a[t][1].y,
                           a[t][2].x + SIGN * a[t][2].y, a[t][3].x + SIGN * a[t][3].y);
        br[t] = split_bf16(b[t][0].x, b[t][1].x, b[t][2].x, b[t][3].x);
        bi[t] = split_bf16(b[t][0].y, b[t][1].y, b[t][2].y, b[t][3].y);
        bs[t] = split_bf16(b[t][0].x + b[t][0].y, b[t][1].x + b[t][1].y, b[t][2].x + b[t][2].y,
                           b[t][3].x + b[t][3].y);
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            if (!live[mi][nj]) continue;
            t1[mi][nj] = mma_split(ar[mi], br[nj], t1[mi][nj]);
            t2[mi][nj] = mma_split(ai[mi], bi[nj], t2[mi][nj]);
            t3[mi][nj] = mma_split(as[mi], bs[nj], t3[mi][nj]);
        }
}

// TN: the k-blocks are staged through LDS: each k-block of A and B
// (16 rows x 64 columns each) is read from HBM once per workgroup with loads
// that cover 4 columns x 256 contiguous bytes per wave instruction, written
// to LDS (column stride padded to 17 elements), and the MFMA operands are read
// from there.  The next block's global loads are in flight during the current
// block's MFMAs (two LDS buffers, one barrier per block).  BF selects the
// split-bf16 products (complex64 only): one 16x16x16 MFMA per product covers a
// whole k-block, lane group g holding k = 4g .. 4g + 3 in both operands.
template <class T, bool BF>
__global__ void __launch_bounds__(kThreads)
    k_gemm_tn_lds(const cpx<T> *__restrict__ A, int64_t lda, const cpx<T> *__restrict__ B,
                  int64_t ldb, int64_t K, int p, int q, int64_t kchunk, int tiles_m, int tiles_n,
                  int nsplit, cpx<T> *__restrict__ part, int herm) {
    using M = Mfma<T>;
    using v4 = typename M::v4;
    constexpr int KB = 16, LDC = KB + 1;
    __shared__ cpx<T> sA[2][kTile * LDC], sB[2][kTile * LDC];
    // herm: the product is Hermitian (A^H B with p = q), only the tiles on and
    // above the diagonal are formed, column by column, and the partials are
    // packed per tile (64 x 64 each)
    const int ntile = herm ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
    const int total = ntile * nsplit;
    const int lid = xcd_logical(blockIdx.x, total);
    const int split = lid / ntile;
    const int tile = lid % ntile;
    int tm, tn;
    if (herm) {
        int t = tile;
        tn = 0;
        while (t > tn) t -= ++tn;
        tm = t;
    } else {
        tm = tile % tiles_m;
        tn = tile / tiles_m;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, g = lane >> 4;
    const int64_t kbeg = (int64_t)split * kchunk;
    const int64_t kend = min(K, kbeg + kchunk);

    // global -> LDS assignment: instruction u covers columns 16 wave + 4u + g, rows li
    const cpx<T> *Ag[4];
    const cpx<T> *Bg[4];
    bool aok[4], bok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = 16 * wave + 4 * u + g;
        const int ca = tm * kTile + c, cb = tn * kTile + c;
        aok[u] = ca < p;
        bok[u] = cb < q;
        Ag[u] = A + (int64_t)(aok[u] ? ca : 0) * lda;
        Bg[u] = B + (int64_t)(bok[u] ? cb : 0) * ldb;
    }
    cpx<T> ra[4], rb[4];
    auto gload = [&](int64_t kb) {   // clamped addresses
        const int64_t k = min(kb + li, kend - 1);
        const bool kin = kb + li < kend;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ra[u] = tile_load(Ag[u] + k, kin && aok[u]);
            rb[u] = tile_load(Bg[u] + k, kin && bok[u]);
        }
    };
    auto lstore = [&](int buf, int64_t kb) {
        const bool kin = kb + li < kend;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = 16 * wave + 4 * u + g;
            sA[buf][c * LDC + li] = tile_keep(ra[u], kin && aok[u]);
            sB[buf][c * LDC + li] = tile_keep(rb[u], kin && bok[u]);
        }
    };

    // 3-multiplication complex product per 16x16 sub-tile: with
    // t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar - ai)(br + bi),
    // conj(a) b = (t1 + t2) + i (t3 - t1 + t2)
    v4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) t1[a][b] = t2[a][b] = t3[a][b] = v4{0, 0, 0, 0};
    const int ia = (wave & 1) * 32, jb = (wave >> 1) * 32;
    // sub-tiles wholly outside p x q are skipped (uniform per wave)
    bool live[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
            live[mi][nj] = tm * kTile + ia + 16 * mi < p && tn * kTile + jb + 16 * nj < q;
    // FULL: every sub-tile of the wave lies inside p x q (all but edge tiles),
    // so the MFMAs run without the per-sub-tile branches
    auto mma_t = [&](int buf, auto full) {
        constexpr bool FULL = decltype(full)::value;
        cpx<T> a[2][4], b[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                a[t][s] = sA[buf][(ia + 16 * t + li) * LDC + 4 * g + s];
                b[t][s] = sB[buf][(jb + 16 * t + li) * LDC + 4 * g + s];
            }
        if constexpr (BF) {
            constexpr bool kAll[2][2] = {{true, true}, {true, true}};
            mma_bf16<-1>(a, b, FULL ? kAll : live, t1, t2, t3);
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int nj = 0; nj < 2; ++nj) {
                        if (!FULL && !live[mi][nj]) continue;
                        t1[mi][nj] = M::op(a[mi][s].x, b[nj][s].x, t1[mi][nj]);
                        t2[mi][nj] = M::op(a[mi][s].y, b[nj][s].y, t2[mi][nj]);
                        t3[mi][nj] = M::op(a[mi][s].x - a[mi][s].y, b[nj][s].x + b[nj][s].y, t3[mi][nj]);
                    }
        }
    };
    // (complex64 only: the FP64 kernel measured slower with it)
    const bool all_live = sizeof(T) == 4 && live[0][0] && live[0][1] && live[1][0] && live[1][1];
    auto mma = [&](int buf) {
        if (all_live)
            mma_t(buf, std::true_type{});
        else
            mma_t(buf, std::false_type{});
    };
    if (kbeg < kend) {
        gload(kbeg);
        lstore(0, kbeg);
        __syncthreads();
        int buf = 0;
        for (int64_t kb = kbeg; kb < kend; kb += KB) {
            const bool more = kb + KB < kend;
            gload(kb + KB);   // past the chunk end: clamped, never stored
            mma(buf);
            if (more) lstore(buf ^ 1, kb + KB);
            __syncthreads();
            buf ^= 1;
        }
    }
    cpx<T> *P = part + (size_t)split * (herm ? (size_t)ntile * kTile * kTile : (size_t)p * q);
    const int i0 = tm * kTile + ia, j0 = tn * kTile + jb;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * mi + M::row(g, r);
                const int j = j0 + 16 * nj + li;
                const size_t at = herm ? ((size_t)tile * kTile + (j - tn * kTile)) * kTile + (i - tm * kTile)
                                       : (size_t)j * p + i;
                if (i < p && j < q)
                    P[at] = cpx<T>{t1[mi][nj][r] + t2[mi][nj][r], t3[mi][nj][r] - t1[mi][nj][r] + t2[mi][nj][r]};
            }
}

// Sum of the split-K partials: 64 outputs per workgroup of NW waves, wave w
// adding splits w, w + NW, ..., the NW wave sums combined in wave order (fixed
// order: deterministic).  NW = 4, or 16 when fewer than 256 groups of 64
// outputs exist (the 64 x 64 and 128 x 64 Grams: shorter chains per thread;
// 64 x 64 Gram at K = 34181 44 -> 33 us FP64).
template <class T, int NW>
__global__ void __launch_bounds__(64 * NW)
    k_reduce_parts(const cpx<T> *__restrict__ part, int nsplit, int p, int q, cd *C, int64_t ldc,
                   const double *__restrict__ scale_row, double beta, int ntile_herm) {
    __shared__ cd red[NW][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // herm (ntile_herm > 0): partials packed per upper tile; element e of tile
    // t is (ii, jj) = (e % 64, e / 64) of the tile's (tm, tn), and the sum is
    // also stored, conjugated, at the mirrored position below the diagonal
    const bool herm = ntile_herm > 0;
    const int64_t n = herm ? (int64_t)ntile_herm * kTile * kTile : (int64_t)p * q;
    const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
    int i = 0, j = 0;
    bool ok = idx < n;
    if (ok && herm) {
        int t = (int)(idx / (kTile * kTile)), tn = 0;
        const int e = (int)(idx % (kTile * kTile));
        while (t > tn) t -= ++tn;
        i = t * kTile + e % kTile;
        j = tn * kTile + e / kTile;
        ok = i < p && j < q;
    } else if (ok) {
        i = (int)(idx % p);
        j = (int)(idx / p);
    }
    double sr = 0.0, si = 0.0;
    if (ok)
        for (int s = wave; s < nsplit; s += NW) {
            const cpx<T> v = part[(size_t)s * n + idx];
            sr += (double)v.x;
            si += (double)v.y;
        }
    red[wave][lane] = cd{sr, si};
    __syncthreads();
    if (wave != 0 || !ok) return;
    sr = red[0][lane].x;
    si = red[0][lane].y;
#pragma unroll
    for (int w = 1; w < NW; ++w) {   // wave order (deterministic)
        sr += red[w][lane].x;
        si += red[w][lane].y;
    }
    if (scale_row) {
        sr *= scale_row[i];
        si *= scale_row[i];
    }
    cd *c = C + (int64_t)j * ldc + i;
    if (beta != 0.0) {
        sr += beta * c->x;
        si += beta * c->y;
    }
    *c = cd{sr, si};
    if (herm && i / kTile < j / kTile) C[(int64_t)i * ldc + j] = cd{sr, -si};
}

// NN: the k-blocks are staged through LDS: per 16-wide k-block the workgroup
// reads 16 columns x 64 rows of A (one wave instruction = one 1 KB column
// segment) and 16 x 64 of C, both once, into padded LDS tiles; the next
// block's global loads are in flight during the current block's MFMAs.  BF
// as for TN.
template <class T, bool BF>
__global__ void __launch_bounds__(kThreads)
    k_gemm_nn_lds(const cpx<T> *__restrict__ A, int64_t lda, const cd *__restrict__ Cm, int64_t ldc,
                  int64_t K, int p, int q, double alpha, double beta, cpx<T> *Y, int64_t ldy,
                  int tiles_m) {
    using M = Mfma<T>;
    using v4 = typename M::v4;
    constexpr int KB = 16, LDA = kTile + 1, LDCC = KB + 1;
    __shared__ cpx<T> sA[2][KB * LDA], sC[2][kTile * LDCC];
    const int lid = xcd_logical(blockIdx.x, gridDim.x);
    const int tm = lid % tiles_m, tn = lid / tiles_m;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, g = lane >> 4;
    const int64_t rbase = (int64_t)tm * kTile;
    const int cbase = tn * kTile;
    const int ia = (wave & 1) * 32, jb = (wave >> 1) * 32;

    // global -> LDS: A instruction u covers column kb + 4 wave + u, rows lane;
    // C instruction u covers columns 16 wave + 4u + g, k rows li
    const bool arow = rbase + lane < K;
    const cpx<T> *Arow = A + (arow ? rbase + lane : 0);
    const cd *Cc[4];
    bool cok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int col = cbase + 16 * wave + 4 * u + g;
        cok[u] = col < q;
        Cc[u] = Cm + (int64_t)(cok[u] ? col : 0) * ldc;
    }
    cpx<T> ra[4];
    cd rc[4];
    auto gload = [&](int kb) {   // clamped addresses
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = kb + 4 * wave + u;
            ra[u] = tile_load(Arow + (int64_t)(kk < p ? kk : 0) * lda, arow && kk < p);
            const int kc = kb + li;
            rc[u] = coef_load<T>(Cc[u] + (kc < p ? kc : 0), cok[u] && kc < p);
        }
    };
    auto lstore = [&](int buf, int kb) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = kb + 4 * wave + u;
            sA[buf][(4 * wave + u) * LDA + lane] = tile_keep(ra[u], arow && kk < p);
            sC[buf][(16 * wave + 4 * u + g) * LDCC + li] = coef_keep<T>(rc[u], cok[u] && kb + li < p);
        }
    };
    // 3-multiplication complex product: with t1 = sum ar cr, t2 = sum ai ci,
    // t3 = sum (ar + ai)(cr + ci), a c = (t1 - t2) + i (t3 - t1 - t2)
    v4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) t1[a][b] = t2[a][b] = t3[a][b] = v4{0, 0, 0, 0};
    bool live[2][2];   // sub-tiles wholly outside K x q are skipped (uniform per wave)
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
            live[mi][nj] = rbase + ia + 16 * mi < K && cbase + jb + 16 * nj < q;
    auto mma = [&](int buf) {
        cpx<T> a[2][4], b[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                a[t][s] = sA[buf][(4 * g + s) * LDA + ia + 16 * t + li];
                b[t][s] = sC[buf][(jb + 16 * t + li) * LDCC + 4 * g + s];
            }
        if constexpr (BF) {
            mma_bf16<+1>(a, b, live, t1, t2, t3);
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int nj = 0; nj < 2; ++nj) {
                        if (!live[mi][nj]) continue;
                        t1[mi][nj] = M::op(a[mi][s].x, b[nj][s].x, t1[mi][nj]);
                        t2[mi][nj] = M::op(a[mi][s].y, b[nj][s].y, t2[mi][nj]);
                        t3[mi][nj] = M::op(a[mi][s].x + a[mi][s].y, b[nj][s].x + b[nj][s].y, t3[mi][nj]);
                    }
        }
    };
    if (p > 0) {
        gload(0);
        lstore(0, 0);
        __syncthreads();
        int buf = 0;
        for (int kb = 0; kb < p; kb += KB) {
            const bool more = kb + KB < p;
            gload(kb + KB);   // past p: clamped, never stored
            mma(buf);
            if (more) lstore(buf ^ 1, kb + KB);
            __syncthreads();
            buf ^= 1;
        }
    }
    // all reads of A (global -> LDS) finished before the final barrier above:
    // the in-place form Y == A is safe when one workgroup spans all q
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = rbase + ia + 16 * mi + M::row(g, r);
                const int j = cbase + jb + 16 * nj + li;
                if (i < K && j < q) {
                    cpx<T> *y = Y + (int64_t)j * ldy + i;
                    T yr = T(alpha) * (t1[mi][nj][r] - t2[mi][nj][r]);
                    T yi = T(alpha) * (t3[mi][nj][r] - t1[mi][nj][r] - t2[mi][nj][r]);
                    if (beta != 0.0) {
                        const cpx<T> o = *y;
                        yr += T(beta) * o.x;
                        yi += T(beta) * o.y;
                    }
                    *y = cpx<T>{yr, yi};
                }
            }
}

// NN with the rows dealt out in 16-row blocks: workgroup (g, tn) takes row
// blocks [g nblk / G, (g + 1) nblk / G) (at most kNnMaxRb of them) and the 64
// columns of tile tn; its four waves each own 16 columns and every row block.
// G is chosen so that the grid fills whole rounds of resident workgroups
// instead of spilling a few 64-row tiles into an extra round (K = 34181 gives
// 535 tiles of 64 rows for 512 resident workgroups).  Same LDS staging and
// double buffering as k_gemm_nn_lds.
constexpr int kNnMaxRb = 5;
template <class T>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 1 : 3)))
    k_gemm_nn_rows(const cpx<T> *__restrict__ A, int64_t lda, const cd *__restrict__ Cm, int64_t ldc,
                   int64_t K, int p, int q, double alpha, double beta, cpx<T> *Y, int64_t ldy,
                   int groups) {
    using M = Mfma<T>;
    using v4 = typename M::v4;
    constexpr int KB = 16, NRW = 16 * kNnMaxRb, LDA = NRW + 1, LDCC = KB + 1;
    __shared__ cpx<T> sA[2][KB * LDA], sC[2][kTile * LDCC];
    const int lid = xcd_logical(blockIdx.x, gridDim.x);
    const int g = lid % groups, tn = lid / groups;
    const int64_t nblk = (K + 15) / 16;
    const int64_t rb0 = nblk * g / groups, rb1 = nblk * (g + 1) / groups;
    const int nrb = (int)(rb1 - rb0);   // 1 .. kNnMaxRb (host guarantees)
    const int64_t rbase = rb0 * 16;
    const int cbase = tn * kTile;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, gq = lane >> 4;

    // global -> LDS: A instruction (u, h) covers column kb + 4 wave + u, rows
    // 64 h + lane; C instruction u covers columns 16 wave + 4u + gq, k rows li
    const int nrows = 16 * nrb;
    const bool arow0 = lane < nrows && rbase + lane < K;
    const bool arow1 = 64 + lane < nrows && rbase + 64 + lane < K;
    const cpx<T> *Arow0 = A + (arow0 ? rbase + lane : 0);
    const cpx<T> *Arow1 = A + (arow1 ? rbase + 64 + lane : 0);
    const cd *Cc[4];
    bool cok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int col = cbase + 16 * wave + 4 * u + gq;
        cok[u] = col < q;
        Cc[u] = Cm + (int64_t)(cok[u] ? col : 0) * ldc;
    }
    cpx<T> ra0[4], ra1[4];
    cd rc[4];
    auto gload = [&](int kb) {   // clamped addresses
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = kb + 4 * wave + u;
            const int64_t ko = (int64_t)(kk < p ? kk : 0) * lda;
            ra0[u] = tile_load(Arow0 + ko, arow0 && kk < p);
            ra1[u] = tile_load(Arow1 + ko, arow1 && kk < p);
            const int kc = kb + li;
            rc[u] = coef_load<T>(Cc[u] + (kc < p ? kc : 0), cok[u] && kc < p);
        }
    };
    auto lstore = [&](int buf, int kb) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = kb + 4 * wave + u;
            sA[buf][(4 * wave + u) * LDA + lane] = tile_keep(ra0[u], arow0 && kk < p);
            if (lane < NRW - 64)
                sA[buf][(4 * wave + u) * LDA + 64 + lane] = tile_keep(ra1[u], arow1 && kk < p);
            sC[buf][(16 * wave + 4 * u + gq) * LDCC + li] = coef_keep<T>(rc[u], cok[u] && kb + li < p);
        }
    };
    const bool colv = cbase + 16 * wave < q;   // this wave's 16 columns (uniform per wave)
    // For complex64 the k loop and the output are instantiated per row-block
    // count NB, so that the MFMA sequence has no branches (the LDS reads are
    // issued ahead of the MFMAs) and each instance holds only its own
    // accumulators; FP64 (NB = 0) keeps one loop over the runtime count, which
    // measured faster there (the FP32 MFMA takes half the cycles and leaves
    // the LDS latency exposed).
    auto run = [&](auto nbc) {
        constexpr int NB = decltype(nbc)::value;
        constexpr int NA = NB ? NB : kNnMaxRb;
        // 3-multiplication complex product (as in k_gemm_nn_lds)
        v4 t1[NA], t2[NA], t3[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i) t1[i] = t2[i] = t3[i] = v4{0, 0, 0, 0};
        auto mma = [&](int buf) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const cpx<T> b = sC[buf][(16 * wave + li) * LDCC + 4 * gq + s];
                const T bs = b.x + b.y;
#pragma unroll
                for (int i = 0; i < NA; ++i) {
                    if (!NB && i >= nrb) break;
                    const cpx<T> a = sA[buf][(4 * gq + s) * LDA + 16 * i + li];
                    t1[i] = M::op(a.x, b.x, t1[i]);
                    t2[i] = M::op(a.y, b.y, t2[i]);
                    t3[i] = M::op(a.x + a.y, bs, t3[i]);
                }
            }
        };
        if (p > 0) {   // every wave stages its share of A, also when its columns are idle
            gload(0);
            lstore(0, 0);
        }
        __syncthreads();
        if (p > 0) {
            int buf = 0;
            for (int kb = 0; kb < p; kb += KB) {
                const bool more = kb + KB < p;
                gload(kb + KB);   // past p: clamped, never stored
                if (colv) mma(buf);
                if (more) lstore(buf ^ 1, kb + KB);
                __syncthreads();
                buf ^= 1;
            }
        }
        // every read of A finished before the last barrier: Y == A is safe when
        // one workgroup spans all q (each workgroup writes only its own rows)
        if (!colv) return;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            if (!NB && i >= nrb) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = rbase + 16 * i + M::row(gq, r);
                const int j = cbase + 16 * wave + li;
                if (row < K && j < q) {
                    cpx<T> *y = Y + (int64_t)j * ldy + row;
                    T yr = T(alpha) * (t1[i][r] - t2[i][r]);
                    T yi = T(alpha) * (t3[i][r] - t1[i][r] - t2[i][r]);
                    if (beta != 0.0) {
                        const cpx<T> o = *y;
                        yr += T(beta) * o.x;
                        yi += T(beta) * o.y;
                    }
                    *y = cpx<T>{yr, yi};
                }
            }
        }
    };
    static_assert(kNnMaxRb == 5, "row-block cases below");
    if constexpr (sizeof(T) == 8) {
        run(std::integral_constant<int, 0>{});
        return;
    }
    switch (nrb) {
    case 5: run(std::integral_constant<int, 5>{}); break;
    case 4: run(std::integral_constant<int, 4>{}); break;
    case 3: run(std::integral_constant<int, 3>{}); break;
    case 2: run(std::integral_constant<int, 2>{}); break;
    default: run(std::integral_constant<int, 1>{}); break;
    }
}

#ifndef PW_SPLIT_WGS
#define PW_SPLIT_WGS 1024   // target workgroup count of a split-K launch
#endif
// compute units of the current device (queried once per process and device)
int device_cu_count() {
    static std::atomic<int> cached[64];
    int dev = 0;
    PW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) dev = 0;
    int n = cached[dev].load(std::memory_order_relaxed);
    if (!n) {
        PW_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
        if (n <= 0) n = 256;
        cached[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// for_size: an upper bound over every device (sizing the partial buffer on any
// context, host-only ones included), without the CU-count cap
int choose_split(int64_t K, int tiles, int target, bool for_size = false) {
    // outputs of one or two 64 x 64 tiles (the CholQR Grams and the overlaps with
    // [X P]) have too little work per k-block for several workgroups per CU: one
    // round of at most one workgroup per CU, chunks of at least 4 k-blocks
    const bool small = tiles <= 2;
    const int64_t cap = (small && !for_size) ? std::min<int64_t>(target, device_cu_count()) : target;
    int64_t ns = (small && !for_size) ? cap / tiles : (cap + tiles - 1) / tiles;
    // chunks of at least 16 k-blocks (4 for small outputs), except for short K
    // (coefficient-space products, K = 3m), which split down to single k-blocks
    // (at most 16)
    const int64_t minkb = small ? 4 : 16;
    const int64_t kmax = std::max<int64_t>((K + 16 * minkb - 1) / (16 * minkb),
                                           std::min<int64_t>((K + 15) / 16, 16));
    if (ns > kmax) ns = kmax;
    if (ns < 1) ns = 1;
    return (int)ns;
}

}  // namespace

size_t gemm_tn_part_elems(int64_t K, int p, int q, int *nsplit_out) {
    const int tiles = ((p + kTile - 1) / kTile) * ((q + kTile - 1) / kTile);
    const int ns = choose_split(K, tiles, std::max(PW_SPLIT_WGS, kTnSplitMax), true);   // any tuned target fits
    if (nsplit_out) *nsplit_out = ns;
    return (size_t)ns * p * q;
}

// herm: A^H B is Hermitian (B = H A for a Hermitian H, p = q); only the
// tiles on and above the diagonal are formed and the rest is mirrored
template <class T, bool BF = false>
void gemm_tn_impl(const cpx<T> *A, int64_t lda, const cpx<T> *B, int64_t ldb, int64_t K, int p, int q,
                  cd *C, int64_t ldc, const double *scale_row, double beta, cd *part, size_t part_elems,
                  hipStream_t st, bool herm = false) {
    if (p <= 0 || q <= 0) return;
    PW_REQUIRE(K > 0, PW_ERR_ARG, "empty contraction (callers form a zero product themselves)");
    const int tiles_m = (p + kTile - 1) / kTile, tiles_n = (q + kTile - 1) / kTile;
    herm = herm && p == q && tiles_m >= 2 && !scale_row && beta == 0.0;
    const int ntile = herm ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
    const size_t per_split = herm ? (size_t)ntile * kTile * kTile : (size_t)p * q;
    const int target = thread_tuning().tn_split_wgs > 0 ? thread_tuning().tn_split_wgs : PW_SPLIT_WGS;
    int ns = choose_split(K, ntile, target);
    if ((size_t)ns * per_split > part_elems) ns = (int)(part_elems / per_split);
    PW_REQUIRE(ns >= 1, PW_ERR_NOMEM, "GEMM partial buffer too small");
    int64_t kchunk = (K + ns - 1) / ns;
    kchunk = (kchunk + 15) / 16 * 16;
    ns = (int)((K + kchunk - 1) / kchunk);
    if (ns < 1) ns = 1;
    const int total = ntile * ns;
    // partials in the block type (the buffer is sized for complex128)
    cpx<T> *pt = reinterpret_cast<cpx<T> *>(part);
    hipLaunchKernelGGL((k_gemm_tn_lds<T, BF>), dim3(total), dim3(kThreads), 0, st, A, lda, B, ldb, K, p, q,
                       kchunk, tiles_m, tiles_n, ns, pt, herm ? 1 : 0);
    const int64_t n = (int64_t)per_split;
    const unsigned rgroups = (unsigned)((n + 63) / 64);
    if (rgroups < 256)
        hipLaunchKernelGGL((k_reduce_parts<T, 16>), dim3(rgroups), dim3(1024), 0, st, pt, ns, p, q, C, ldc,
                           scale_row, beta, herm ? ntile : 0);
    else
        hipLaunchKernelGGL((k_reduce_parts<T, 4>), dim3(rgroups), dim3(256), 0, st, pt, ns, p, q, C, ldc,
                           scale_row, beta, herm ? ntile : 0);
    PW_HIP(hipGetLastError());
}

template <class T, bool BF = false>
void gemm_nn_impl(const cpx<T> *A, int64_t lda, const cd *C, int64_t ldc, int64_t K, int p, int q,
                  double alpha, double beta, cpx<T> *Y, int64_t ldy, hipStream_t st) {
    if (K <= 0 || q <= 0) return;
    const int tiles_m = (int)((K + kTile - 1) / kTile), tiles_n = (q + kTile - 1) / kTile;
    PW_REQUIRE(!((const void *)A == (const void *)Y) || q <= kTile, PW_ERR_ARG,
               "in-place block update needs q <= 64");
    if constexpr (!BF) {
        // row groups of 4-5 blocks of 16 rows, sized to whole rounds of the
        // resident workgroups when that keeps <= 5 blocks per group
        const int64_t nblk = (K + 15) / 16;
        int64_t G = (nblk + 3) / 4;
        static std::atomic<int> per_cu{0};   // resident workgroups per CU of this kernel
        int occ = per_cu.load(std::memory_order_relaxed);
        if (!occ) {
            PW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_gemm_nn_rows<T>, kThreads, 0));
            if (occ <= 0) occ = 1;
            per_cu.store(occ, std::memory_order_relaxed);
        }
        const int64_t slots = (int64_t)occ * device_cu_count();
        const int64_t rounds = (G * tiles_n + slots - 1) / slots;
        if (nblk * tiles_n <= slots) {
            G = nblk;   // short K (coefficient space): one block per workgroup, all resident
        } else if (rounds > 1) {
            const int64_t Gfit = (rounds - 1) * slots / tiles_n;
            if (Gfit >= (nblk + kNnMaxRb - 1) / kNnMaxRb) G = Gfit;
        }
        hipLaunchKernelGGL(k_gemm_nn_rows<T>, dim3((unsigned)(G * tiles_n)), dim3(kThreads), 0, st, A, lda,
                           C, ldc, K, p, q, alpha, beta, Y, ldy, (int)G);
        PW_HIP(hipGetLastError());
        return;
    }
    hipLaunchKernelGGL((k_gemm_nn_lds<T, BF>), dim3(tiles_m * tiles_n), dim3(kThreads), 0, st, A, lda, C, ldc,
                       K, p, q, alpha, beta, Y, ldy, tiles_m);
    PW_HIP(hipGetLastError());
}

void launch_gemm_tn(const cd *A, int64_t lda, const cd *B, int64_t ldb, int64_t K, int p, int q,
                    cd *C, int64_t ldc, const double *scale_row, double beta, cd *part,
                    size_t part_elems, hipStream_t st) {
    gemm_tn_impl(A, lda, B, ldb, K, p, q, C, ldc, scale_row, beta, part, part_elems, st);
}
void launch_gemm_tn(const cf *A, int64_t lda, const cf *B, int64_t ldb, int64_t K, int p, int q,
                    cd *C, int64_t ldc, const double *scale_row, double beta, cd *part,
                    size_t part_elems, hipStream_t st) {
    gemm_tn_impl(A, lda, B, ldb, K, p, q, C, ldc, scale_row, beta, part, part_elems, st);
}
void launch_gemm_nn(const cd *A, int64_t lda, const cd *C, int64_t ldc, int64_t K, int p, int q,
                    double alpha, double beta, cd *Y, int64_t ldy, hipStream_t st) {
    gemm_nn_impl(A, lda, C, ldc, K, p, q, alpha, beta, Y, ldy, st);
}
void launch_gemm_nn(const cf *A, int64_t lda, const cd *C, int64_t ldc, int64_t K, int p, int q,
                    double alpha, double beta, cf *Y, int64_t ldy, hipStream_t st) {
    gemm_nn_impl(A, lda, C, ldc, K, p, q, alpha, beta, Y, ldy, st);
}
void launch_gemm_tn_bf16(const cf *A, int64_t lda, const cf *B, int64_t ldb, int64_t K, int p, int q,
                         cd *C, int64_t ldc, const double *scale_row, double beta, cd *part,
                         size_t part_elems, hipStream_t st, bool herm) {
    gemm_tn_impl<float, true>(A, lda, B, ldb, K, p, q, C, ldc, scale_row, beta, part, part_elems, st, herm);
}
void launch_gemm_herm(const cd *A, int64_t lda, const cd *B, int64_t ldb, int64_t K, int p, cd *C,
                      int64_t ldc, cd *part, size_t part_elems, hipStream_t st) {
    gemm_tn_impl(A, lda, B, ldb, K, p, p, C, ldc, nullptr, 0.0, part, part_elems, st, true);
}
void launch_gemm_herm(const cf *A, int64_t lda, const cf *B, int64_t ldb, int64_t K, int p, cd *C,
                      int64_t ldc, cd *part, size_t part_elems, hipStream_t st) {
    gemm_tn_impl(A, lda, B, ldb, K, p, p, C, ldc, nullptr, 0.0, part, part_elems, st, true);
}
void launch_gemm_nn_bf16(const cf *A, int64_t lda, const cd *C, int64_t ldc, int64_t K, int p, int q,
                         double alpha, double beta, cf *Y, int64_t ldy, hipStream_t st) {
    gemm_nn_impl<float, true>(A, lda, C, ldc, K, p, q, alpha, beta, Y, ldy, st);
}

}  // namespace pw
