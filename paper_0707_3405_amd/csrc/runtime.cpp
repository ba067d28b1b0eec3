// Host runtime behind the C ABI: context, plane-wave sphere setup, potential
// and projector tables, workspace plan, H.X apply and the block LOBPCG driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <type_traits>
#include <map>
#include <mutex>

#include "pw_internal.h"

using pw::cd;
using pw::Error;

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace (or a dry run that only sizes it).
struct Arena {
    char *base = nullptr;
    size_t used = 0;
    template <class T>
    T *take(size_t count) {
        used = align_up(used, 256);
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
};

// Event pairs around phases; elapsed times are collected after a stream sync.
struct PhaseTimer {
    enum Phase { kApply = 0, kGemm, kDense, kVec, kFinal, kCount };
    hipStream_t st = nullptr;
    bool on = true;   // off: no events are recorded (each one is a marker between kernels)
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> open;
    size_t next = 0;
    double ms[kCount] = {0, 0, 0, 0, 0};
    hipEvent_t get() {
        if (next == pool.size()) {
            hipEvent_t e;
            PW_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[next++];
    }
    hipEvent_t begin() {
        if (!on) return nullptr;
        hipEvent_t e = get();
        PW_HIP(hipEventRecord(e, st));
        return e;
    }
    void end(int phase, hipEvent_t b) {
        if (!on) return;
        hipEvent_t e = get();
        PW_HIP(hipEventRecord(e, st));
        open.push_back({phase, {b, e}});
    }
    // call after the stream has been synchronised
    void collect() {
        for (auto &o : open) {
            float t = 0.f;
            PW_HIP(hipEventElapsedTime(&t, o.second.first, o.second.second));
            ms[o.first] += t;
        }
        open.clear();
        next = 0;
    }
    ~PhaseTimer() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace

namespace pw {
void ensure_smem_limit(const void *kernel, size_t bytes) {
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> done;
    int dev = 0;
    PW_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    size_t &cur = done[{kernel, dev}];
    if (bytes <= cur) return;
    PW_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    cur = bytes;
}
namespace {
const Tuning kDefaultTuning{};
thread_local const Tuning *t_tuning = nullptr;
}  // namespace
const Tuning &thread_tuning() { return t_tuning ? *t_tuning : kDefaultTuning; }
const Tuning *set_thread_tuning(const Tuning *t) {
    const Tuning *prev = t_tuning;
    t_tuning = t;
    return prev;
}
}  // namespace pw

struct pw_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // basis
    bool has_basis = false;
    double cell[9] = {0}, kfrac[3] = {0}, ecut = 0;
    int n = 0;
    int64_t npw = 0, ldp = 0;   // ldp: padded leading dimension of internal blocks
    std::vector<int32_t> miller;   // [npw][3]
    std::vector<double> kin;       // [npw]
    std::vector<double> qvec;      // [npw][3]
    pw::SphereDev sp;
    std::vector<void *> dev_allocs;   // context-owned device memory
    double *d_qvec = nullptr;

    // potential (V / N^3 in [z][y][x]); float copy for the mixed form
    bool has_v = false;
    double *d_v = nullptr;
    int v_r2 = 0;   // radix split (second factor) whose x-order d_v is stored in
    float *d_v32 = nullptr;

    // projectors
    int natom = 0, nlm = 0;
    cd *d_B = nullptr;
    pw::cf *d_B32 = nullptr;   // complex64 copy for the mixed form
    bool proj_bf16 = false;    // complex64 projector products on split-bf16 MFMA
    bool gram_bf16 = false;    // complex64 Rayleigh-Ritz Gram on split-bf16 MFMA
    bool rr_fp32 = false;      // complex64 stage: Rayleigh-Ritz tridiagonal reduction in FP32
    bool phase_timing = false; // per-phase HIP events in the solves (pw_set_phase_timing)
    pw::Tuning tune;           // launch parameters (pw_autotune / pw_set_tuning)
    double *d_D = nullptr;
    double *d_Q = nullptr;     // overlap coefficients (generalized form); null: O = I

    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int plan_nbands = 0, plan_block = 0;
    pw_precision plan_prec = PW_PREC_FP64;

    int *d_status = nullptr;
    int nst_host = 0, ncx_host = 0;
    hipError_t static_scratch_status = hipSuccess;   // pw::static_scratch_setup at pw_create

    // pinned host staging of the per-iteration round trip (residual norms and
    // status down, active columns up), allocated with the context: copies to
    // and from it are asynchronous, and a solve allocates no host memory
    static constexpr size_t kPinnedBytes = 4096;   // >= 3 * 64 doubles + (1 + 3 * 64) ints
    void *h_pinned = nullptr;
    char *pinned(size_t bytes) {
        PW_REQUIRE(h_pinned && bytes <= kPinnedBytes, PW_ERR_STATE, "pinned staging too small");
        return static_cast<char *>(h_pinned);
    }

    // last solve
    std::vector<double> res;
    pw_stats stats{};

    template <class T>
    T *dev_alloc(size_t count) {
        void *p = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) throw Error{PW_ERR_NOMEM, "device allocation failed"};
        dev_allocs.push_back(p);
        return static_cast<T *>(p);
    }
    void dev_free(void *p) {
        if (!p) return;
        auto it = std::find(dev_allocs.begin(), dev_allocs.end(), p);
        if (it != dev_allocs.end()) {
            (void)hipFree(p);
            dev_allocs.erase(it);
        }
    }
    int nproj() const { return natom * nlm; }
};

namespace {

// Mixed form: the complex64 LOBPCG runs each block to this residual (or its
// iteration cap, or its precision floor: no halving of the largest residual
// in kMixedFloorIters iterations), then the FP64 iteration refines from its
// vectors.
constexpr double kMixedTol = 1e-5;
constexpr int kMixedMaxIter = 200;
constexpr int kMixedFloorIters = 10;
// complex64 stage: H X (and O X) formed from X itself every this many
// iterations instead of carried by the block updates, so the FP32 rounding of
// the updates does not accumulate into the Rayleigh quotients and residuals
constexpr int kMixedRefresh = 10;

// ---- workspace plan ----------------------------------------------------------
// S is the block storage type: cd (complex128) or cf (complex64).  Small
// matrices (Grams, coefficients, overlaps) are complex128 in both forms.
template <class S>
struct Plan {
    S *Sb = nullptr;              // stick buffer [block][n][ldst]
    S *Z[2] = {nullptr, nullptr};     // [ldp x 3m] basis blocks [X | P | W]
    S *HZ[2] = {nullptr, nullptr};    // [ldp x 3m]
    S *HXall = nullptr;           // [ldp x M]
    S *OZ[2] = {nullptr, nullptr};    // [ldp x 3m] O Z (generalized form only)
    S *OXall = nullptr;           // [ldp x M] O X (generalized form only)
    S *T = nullptr;               // [ldp x M] rotation temp
    S *Xs = nullptr;              // [ldp x M] internal copy of X (complex64 form only)
    cd *Pj = nullptr;             // projector overlaps [nproj x block]
    cd *part = nullptr;           // GEMM split-K partials
    size_t part_elems = 0;
    cd *Agram = nullptr;          // [max(3m, M)]^2
    cd *Cc = nullptr;             // [3m x 2m] coefficients [C | c_p]
    cd *U = nullptr;              // [M x M] final eigenvectors (also [3m x m])
    cd *Ov = nullptr;             // [M x m] overlaps
    cd *Gs = nullptr;             // [m x m]
    cd *Rinv = nullptr;           // [m x m]
    cd *T1 = nullptr;             // [m x m]
    double *theta = nullptr;      // [M]
    double *ekin = nullptr;       // [2M]
    double *res = nullptr;        // [M]
    double *w = nullptr;          // [max(3m, M)]
    double *rpart = nullptr;      // residual partials
    int *act = nullptr;           // [m] active column map
    void *heev_scratch = nullptr;
    size_t bytes = 0;
};

template <class S>
Plan<S> make_plan(const pw_ctx_s &c, int M, int m, char *base) {
    Plan<S> p;
    Arena a;
    a.base = base;
    const int64_t ld = c.ldp;
    const int nproj = c.nproj();
    const int n3 = std::max(3 * m, M);
    p.Sb = a.take<S>((size_t)m * c.n * c.sp.ldst);
    for (int i = 0; i < 2; ++i) {
        p.Z[i] = a.take<S>((size_t)ld * 3 * m);
        p.HZ[i] = a.take<S>((size_t)ld * 3 * m);
    }
    p.HXall = a.take<S>((size_t)ld * M);
    if (c.d_Q) {
        for (int i = 0; i < 2; ++i) p.OZ[i] = a.take<S>((size_t)ld * 3 * m);
        p.OXall = a.take<S>((size_t)ld * M);
    }
    p.T = a.take<S>((size_t)ld * M);
    if (!std::is_same<S, cd>::value) p.Xs = a.take<S>((size_t)ld * M);
    p.Pj = a.take<cd>((size_t)std::max(nproj, 1) * m);
    size_t pe = 0;
    auto upd = [&](int64_t K, int pp, int qq) {
        pe = std::max(pe, pw::gemm_tn_part_elems(K, pp, qq, nullptr));
    };
    upd(c.npw, 3 * m, 3 * m);
    upd(c.npw, 2 * m, m);
    upd(c.npw, M, m);
    upd(c.npw, m, m);
    upd(c.npw, M, M);
    if (nproj) upd(c.npw, nproj, m);
    upd(3 * m, m, m);
    p.part_elems = pe;
    p.part = a.take<cd>(pe);
    p.Agram = a.take<cd>((size_t)n3 * n3);
    p.Cc = a.take<cd>((size_t)3 * m * 2 * m);
    p.U = a.take<cd>((size_t)n3 * n3);
    p.Ov = a.take<cd>((size_t)std::max(M, 3 * m) * m);
    p.Gs = a.take<cd>((size_t)m * m);
    p.Rinv = a.take<cd>((size_t)m * m);
    p.T1 = a.take<cd>((size_t)m * m);
    p.theta = a.take<double>(n3);
    p.ekin = a.take<double>(2 * (size_t)n3);
    p.res = a.take<double>(n3);
    p.w = a.take<double>(n3);
    p.rpart = a.take<double>(pw::resid_part_elems(c.npw, n3));
    p.act = a.take<int>(m);
    p.heev_scratch = a.take<char>(pw::heev_scratch_bytes(n3, n3));
    p.bytes = align_up(a.used, 256);
    return p;
}

// scratch of pw_density for nb bands in chunks of `chunk` (laid out as it takes it)
size_t density_bytes(const pw_ctx_s &c, int chunk, int nb) {
    Arena a;
    const int64_t n3 = (int64_t)c.n * c.n * c.n;
    a.take<cd>((size_t)chunk * c.n * c.sp.ldst);
    a.take<double>((size_t)n3);
    a.take<double>((size_t)nb);
    return align_up(a.used, 256);
}

// the solver's plan, and enough for pw_density of up to M bands with the same block
size_t plan_bytes(const pw_ctx_s &c, int M, int m, pw_precision prec) {
    size_t b = make_plan<cd>(c, M, m, nullptr).bytes;
    if (prec != PW_PREC_FP64) b = std::max(b, make_plan<pw::cf>(c, M, m, nullptr).bytes);
    return std::max(b, density_bytes(c, m, M));
}

void require_precision(pw_precision prec) {
    PW_REQUIRE(prec == PW_PREC_FP64 || prec == PW_PREC_MIXED || prec == PW_PREC_MIXED_BF16 ||
                   prec == PW_PREC_MIXED_BF16_GRAM || prec == PW_PREC_MIXED_FP32_RR,
               PW_ERR_ARG, "unknown precision");
}

void require_basis(const pw_ctx_s *c) {
    PW_REQUIRE(c->has_basis, PW_ERR_STATE, "pw_init_basis has not been called");
}
void require_device(const pw_ctx_s *c) {
    PW_REQUIRE(c->device >= 0, PW_ERR_STATE, "host-only context (device < 0) cannot run kernels");
}

template <class S>
Plan<S> ready_plan(pw_ctx_s *c, int M, int m) {
    require_basis(c);
    require_device(c);
    PW_REQUIRE(c->has_v, PW_ERR_STATE, "pw_set_local_potential has not been called");
    PW_REQUIRE(c->ws != nullptr, PW_ERR_STATE, "pw_set_workspace has not been called");
    Plan<S> dry = make_plan<S>(*c, M, m, nullptr);
    PW_REQUIRE(dry.bytes <= c->ws_bytes, PW_ERR_NOMEM,
               "workspace too small for this (nbands, block, precision); query pw_workspace_size");
    return make_plan<S>(*c, M, m, c->ws);
}

// complex64 copies of the potential and projector table, made on first use
void ensure_mixed_tables(pw_ctx_s *c) {
    const size_t n3 = (size_t)c->n * c->n * c->n;
    if (!c->d_v32) {
        c->d_v32 = c->dev_alloc<float>(n3);
        pw::launch_convert_f64_f32(c->d_v, c->d_v32, (int64_t)n3, c->stream);
    }
    const int np = c->nproj();
    if (np > 0 && !c->d_B32) {
        c->d_B32 = c->dev_alloc<pw::cf>((size_t)c->ldp * np);
        pw::launch_copy_cols(c->d_B, c->ldp, c->d_B32, c->ldp, c->ldp, np, c->stream);
    }
}

// R2 of the radix split the context's tuning selects for its grid
int tuned_r2(const pw_ctx_s *c) { return c->tune.fft_r2 > 0 ? c->tune.fft_r2 : pw::fft_default_r2(c->n); }
bool split_available(int n, int r2) {
    const std::vector<int> v = pw::fft_radix_splits(n);
    return std::find(v.begin(), v.end(), r2) != v.end();
}
// keep the stored potential in the x-order of the tuned radix split
void relayout_potential(pw_ctx_s *c) {
    if (!c->has_v) return;
    const int want = tuned_r2(c);
    if (want == c->v_r2) return;
    const size_t n3 = (size_t)c->n * c->n * c->n;
    double *nv = c->dev_alloc<double>(n3);
    pw::launch_repermute_potential(c->d_v, c->n, c->v_r2, want, nv, c->stream);
    PW_HIP(hipStreamSynchronize(c->stream));
    c->dev_free(c->d_v);
    c->d_v = nv;
    c->v_r2 = want;
    c->dev_free(c->d_v32);   // the float copy is rebuilt on the next mixed-form call
    c->d_v32 = nullptr;
}

const double *potential_of(const pw_ctx_s *c, const cd *) { return c->d_v; }
const float *potential_of(const pw_ctx_s *c, const pw::cf *) { return c->d_v32; }
const cd *projectors_of(const pw_ctx_s *c, const cd *) { return c->d_B; }
const pw::cf *projectors_of(const pw_ctx_s *c, const pw::cf *) { return c->d_B32; }

// ---- H.X and O.X -----------------------------------------------------------------
// Y += B diag(s) B^H X over nc <= block columns (projector table B [npw x nproj])
template <class S>
void proj_add(pw_ctx_s *c, const Plan<S> &p, const double *s, const S *X, int64_t ldx, S *Y,
              int64_t ldy, int nc) {
    const S *B = projectors_of(c, X);
    const int np = c->nproj();
    if constexpr (std::is_same<S, pw::cf>::value) {
        if (c->proj_bf16) {
            pw::launch_gemm_tn_bf16(B, c->ldp, X, ldx, c->npw, np, nc, p.Pj, np, s, 0.0, p.part,
                                    p.part_elems, c->stream);
            pw::launch_gemm_nn_bf16(B, c->ldp, p.Pj, np, c->npw, np, nc, 1.0, 1.0, Y, ldy, c->stream);
            return;
        }
    }
    pw::launch_gemm_tn(B, c->ldp, X, ldx, c->npw, np, nc, p.Pj, np, s, 0.0, p.part, p.part_elems,
                       c->stream);
    pw::launch_gemm_nn(B, c->ldp, p.Pj, np, c->npw, np, nc, 1.0, 1.0, Y, ldy, c->stream);
}

// Rayleigh-Ritz Gram A = Z^H (HZ) [nz x nz] (the Rayleigh-Ritz of sec. 3.2, Algorithm 1); in the
// complex64 stage of PW_PREC_MIXED_BF16_GRAM on split-bf16 MFMA
template <class S>
void rr_gram(pw_ctx_s *c, const Plan<S> &p, const S *Z, const S *HZ, int64_t ld, int nz) {
    if constexpr (std::is_same<S, pw::cf>::value) {
        if (c->gram_bf16) {
            pw::launch_gemm_tn_bf16(Z, ld, HZ, ld, c->npw, nz, nz, p.Agram, nz, nullptr, 0.0, p.part,
                                    p.part_elems, c->stream, true);
            return;
        }
    }
    // Z^H H Z is Hermitian: the tiles below the diagonal are mirrored
    pw::launch_gemm_herm(Z, ld, HZ, ld, c->npw, nz, p.Agram, nz, p.part, p.part_elems, c->stream);
}

template <class S>
void apply_H(pw_ctx_s *c, const Plan<S> &p, int chunk, const S *X, int64_t ldx, S *Y, int64_t ldy,
             int nb) {
    for (int b0 = 0; b0 < nb; b0 += chunk) {
        const int nc = std::min(chunk, nb - b0);
        const S *Xc = X + (int64_t)b0 * ldx;
        S *Yc = Y + (int64_t)b0 * ldy;
        pw::launch_fft_apply(c->sp, potential_of(c, X), Xc, ldx, Yc, ldy, nc, p.Sb, c->stream);
        if (c->nproj() > 0) proj_add(c, p, c->d_D, Xc, ldx, Yc, ldy, nc);   // + B diag(D) B^H X
    }
}

// Y = O X = X + B diag(q) B^H X (generalized form; the overlap is set)
template <class S>
void apply_O(pw_ctx_s *c, const Plan<S> &p, int chunk, const S *X, int64_t ldx, S *Y, int64_t ldy,
             int nb) {
    pw::launch_copy_cols(X, ldx, Y, ldy, c->npw, nb, c->stream);
    for (int b0 = 0; b0 < nb; b0 += chunk) {
        const int nc = std::min(chunk, nb - b0);
        proj_add(c, p, c->d_Q, X + (int64_t)b0 * ldx, ldx, Y + (int64_t)b0 * ldy, ldy, nc);
    }
}

int read_status(pw_ctx_s *c) {
    int s = 0;
    PW_HIP(hipMemcpyAsync(&s, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    PW_HIP(hipStreamSynchronize(c->stream));
    return s;
}

// CholQR of V [npw x nb] in place: G = V^H V, V <- V R^-1.  In the
// generalized form (OV given, OV = O V) the factor is of G = V^H O V and OV
// is carried along: OV <- OV R^-1.
template <class S>
void cholqr(pw_ctx_s *c, const Plan<S> &p, PhaseTimer &tm, S *V, int64_t ldv, int nb, S *OV = nullptr) {
    auto e0 = tm.begin();
    pw::launch_gemm_tn(V, ldv, OV ? OV : V, ldv, c->npw, nb, nb, p.Gs, nb, nullptr, 0.0, p.part,
                       p.part_elems, c->stream);
    tm.end(PhaseTimer::kGemm, e0);
    auto e1 = tm.begin();
    pw::launch_chol_inv_f64(p.Gs, nb, nb, p.Rinv, nb, c->d_status, c->stream);
    tm.end(PhaseTimer::kDense, e1);
    auto e2 = tm.begin();
    pw::launch_gemm_nn(V, ldv, p.Rinv, nb, c->npw, nb, nb, 1.0, 0.0, V, ldv, c->stream);
    if (OV) pw::launch_gemm_nn(OV, ldv, p.Rinv, nb, c->npw, nb, nb, 1.0, 0.0, OV, ldv, c->stream);
    tm.end(PhaseTimer::kGemm, e2);
}

// V <- V - Q (Q^H V), Q [npw x nq].  Generalized form: OQ = O Q given, the
// coefficients are (OQ)^H V (O-orthogonal complement), and OV <- OV - OQ (..)
// when OV is given.
template <class S>
void project_out(pw_ctx_s *c, const Plan<S> &p, PhaseTimer &tm, const S *Q, int64_t ldq, int nq,
                 S *V, int64_t ldv, int nb, const S *OQ = nullptr, int64_t ldoq = 0, S *OV = nullptr) {
    if (nq <= 0) return;
    auto e0 = tm.begin();
    if (OQ)
        pw::launch_gemm_tn(OQ, ldoq, V, ldv, c->npw, nq, nb, p.Ov, nq, nullptr, 0.0, p.part,
                           p.part_elems, c->stream);
    else
        pw::launch_gemm_tn(Q, ldq, V, ldv, c->npw, nq, nb, p.Ov, nq, nullptr, 0.0, p.part,
                           p.part_elems, c->stream);
    pw::launch_gemm_nn(Q, ldq, p.Ov, nq, c->npw, nq, nb, -1.0, 1.0, V, ldv, c->stream);
    if (OQ && OV) pw::launch_gemm_nn(OQ, ldoq, p.Ov, nq, c->npw, nq, nb, -1.0, 1.0, OV, ldv, c->stream);
    tm.end(PhaseTimer::kGemm, e0);
}

// Block LOBPCG over M bands in blocks of m.  X (storage S) receives the
// converged vectors; with final_rr the Rayleigh-Ritz over all M bands and the
// residual check follow.  Timing and counters accumulate into stats.
template <class S>
pw_status lobpcg(pw_ctx_s *c, const Plan<S> &p, int M, int m, double tol, int max_iter, S *X,
                 int64_t ldx, int use_guess, double *eig, bool final_rr, pw_stats &stats,
                 int floor_iters = 0, bool *final_res_above_tol = nullptr) {
    hipStream_t st = c->stream;
    const int64_t ld = c->ldp, npw = c->npw;
    // PW_PREC_MIXED_FP32_RR: the complex64 stage, whose blocks carry FP32
    // rounding, reduces its Rayleigh-Ritz problems to tridiagonal form in FP32
    // as well (its FP64 stage, and every other form, reduce in FP64)
    const bool lowp_reduction = std::is_same<S, pw::cf>::value && c->rr_fp32;
    PhaseTimer tm;
    tm.st = st;
    tm.on = c->phase_timing;
    hipEvent_t t_begin, t_end;
    PW_HIP(hipEventCreate(&t_begin));
    PW_HIP(hipEventCreate(&t_end));
    PW_HIP(hipEventRecord(t_begin, st));
    PW_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), st));
    bool all_converged = true;
    // pinned: residual norms [3m] | status | active columns [3m]
    char *hp = c->pinned(sizeof(double) * 3 * m + sizeof(int) * (1 + 3 * m));
    double *hres = reinterpret_cast<double *>(hp);
    int *hstat = reinterpret_cast<int *>(hp + sizeof(double) * 3 * m);
    int *hact = hstat + 1;
    // residual norms below this are rounding noise (Ha; the spectrum scale is ~ecut)
    const double res_floor = 1e-10 * std::max(1.0, c->ecut);

    // Each block iterates mb = min(m, keep + guard) columns; the lowest `keep`
    // must converge and are stored, the top `guard` columns only shield them
    // from a near-degenerate neighbour just above the block.
    const int guard = m / 5;   // measured best of m/8 .. m/3 with the warm start below
    // the guard Ritz vectors of the previous block (bands just above it) seed
    // the next block when the caller gives no guess
    S *prevZ = nullptr;
    int prev_keep = 0, prev_mb = 0;
    for (int b0 = 0; b0 < M;) {
        const int keep = std::min(m - guard, M - b0);
        const int mb = (int)std::min<int64_t>(std::min(m, keep + guard), npw - b0);
        ++stats.blocks;
        int cur = 0;
        S *Z = p.Z[cur], *HZ = p.HZ[cur];
        // generalized form: O Z is carried beside Z and H Z, and every
        // orthogonality is in the O inner product
        const bool gen = c->d_Q != nullptr;
        S *OZ = gen ? p.OZ[cur] : nullptr;
        S *OXprev = gen ? p.OXall : nullptr;
        // start block: X in slot 0 (caller guess for the stored columns)
        const int nguess = use_guess ? std::min(mb, M - b0) : 0;
        if (nguess > 0) pw::launch_copy_cols(X + (int64_t)b0 * ldx, ldx, Z, ld, npw, nguess, st);
        int nwarm = 0;
        if (nguess == 0 && prevZ && prev_mb > prev_keep) {
            // source columns [prev_keep, prev_mb) never overlap [0, nwarm) (prev_keep >= guard)
            nwarm = std::min(prev_mb - prev_keep, mb);
            pw::launch_copy_cols(prevZ + (int64_t)prev_keep * ld, ld, Z, ld, npw, nwarm, st);
        }
        const int nfill = std::max(nguess, nwarm);
        if (nfill < mb)
            pw::launch_random_block(Z + (int64_t)nfill * ld, ld, npw, mb - nfill,
                                    0x5EED0000ull + (uint64_t)b0, c->sp.kin, st);
        // orthogonal to previous blocks, orthonormal (twice)
        auto orthonormalise_start = [&]() {
            if (gen) {
                auto e = tm.begin();
                apply_O(c, p, m, Z, ld, OZ, ld, mb);
                tm.end(PhaseTimer::kApply, e);
            }
            for (int pass = 0; pass < 2; ++pass) {
                project_out(c, p, tm, (const S *)X, ldx, b0, Z, ld, mb, OXprev, ld, OZ);
                cholqr(c, p, tm, Z, ld, mb, OZ);
            }
        };
        orthonormalise_start();
        if (nguess > 0) {
            // columns of the caller's guess with nothing independent left (zero,
            // repeated, or spanned by the earlier blocks) leave the
            // orthonormalisation as null columns, which would pass as converged:
            // they are replaced by random columns from a seed range of their own
            // (distinct per block, round and column) until every column is unit
            std::vector<cd> g((size_t)mb * mb);
            for (int round = 0; round < 3; ++round) {
                pw::launch_gemm_tn(Z, ld, gen ? OZ : Z, ld, npw, mb, mb, p.Gs, mb, nullptr, 0.0, p.part,
                                   p.part_elems, st);
                PW_HIP(hipMemcpyAsync(g.data(), p.Gs, sizeof(cd) * g.size(), hipMemcpyDeviceToHost, st));
                PW_HIP(hipStreamSynchronize(st));
                PW_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), st));   // breakdowns of the guess
                bool redo = false;
                for (int j = 0; j < mb; ++j) {
                    if (!(std::fabs(g[(size_t)j * mb + j].x - 1.0) <= 1e-6)) {
                        const uint64_t seed = 0x5EED0000ull + ((uint64_t)(b0 + 1) << 16) +
                                              ((uint64_t)round << 12) + (uint64_t)j;
                        pw::launch_random_block(Z + (int64_t)j * ld, ld, npw, 1, seed, c->sp.kin, st);
                        redo = true;
                    }
                }
                if (!redo) break;
                orthonormalise_start();
            }
        }
        {
            auto e = tm.begin();
            apply_H(c, p, m, Z, ld, HZ, ld, mb);
            tm.end(PhaseTimer::kApply, e);
            stats.h_applies += mb;
        }
        // initial Rayleigh-Ritz on span(X)
        {
            auto e0 = tm.begin();
            rr_gram(c, p, Z, HZ, ld, mb);
            tm.end(PhaseTimer::kGemm, e0);
            auto e1 = tm.begin();
            pw::launch_heev_f64(p.Agram, mb, mb, mb, p.w, p.Cc, 3 * m, p.heev_scratch, c->d_status, st,
                                lowp_reduction);
            tm.end(PhaseTimer::kDense, e1);
            auto e2 = tm.begin();
            pw::launch_gemm_nn(Z, ld, p.Cc, 3 * m, npw, mb, mb, 1.0, 0.0, p.Z[1 - cur], ld, st);
            pw::launch_gemm_nn(HZ, ld, p.Cc, 3 * m, npw, mb, mb, 1.0, 0.0, p.HZ[1 - cur], ld, st);
            if (gen) pw::launch_gemm_nn(OZ, ld, p.Cc, 3 * m, npw, mb, mb, 1.0, 0.0, p.OZ[1 - cur], ld, st);
            tm.end(PhaseTimer::kGemm, e2);
            cur = 1 - cur;
            Z = p.Z[cur];
            HZ = p.HZ[cur];
            if (gen) OZ = p.OZ[cur];
        }
        // Active set: only columns whose residual is still above tol receive a
        // new direction W and a conjugate direction P, so H.W, the
        // projections and the Rayleigh-Ritz size shrink as the block converges.
        // Basis layout in Z / HZ: [X (mb) | P (np) | W (na)].
        int np = 0, converged_it = -1;
        std::vector<int> act;
        // floor detection (floor_iters > 0): the block ends early once its
        // largest residual has not halved for floor_iters iterations
        double best = HUGE_VAL;
        int since_best = 0;
        int it = 0;
        for (it = 0; it < max_iter; ++it) {
            if (std::is_same<S, pw::cf>::value && it > 0 && it % kMixedRefresh == 0) {
                auto e = tm.begin();
                apply_H(c, p, m, Z, ld, HZ, ld, mb);
                if (gen) apply_O(c, p, m, Z, ld, OZ, ld, mb);
                tm.end(PhaseTimer::kApply, e);
                stats.h_applies += mb;
            }
            {
                auto e = tm.begin();
                // R = HZ - theta OZ (OZ = Z when O = I)
                pw::launch_band_dots(Z, ld, HZ, ld, c->sp.kin, npw, mb, p.rpart, p.theta, p.ekin, st, OZ,
                                     ld);
                pw::launch_resid_precond(gen ? OZ : Z, ld, HZ, ld, c->sp.kin, npw, mb, p.theta, p.ekin,
                                         (S *)nullptr, 0, p.rpart, p.res, st, c->d_status);
                tm.end(PhaseTimer::kVec, e);
            }
            // the norms and, in res[mb], the status word: one copy per iteration
            PW_HIP(hipMemcpyAsync(hres, p.res, sizeof(double) * (mb + 1), hipMemcpyDeviceToHost, st));
            PW_HIP(hipStreamSynchronize(st));
            const int status = (int)hres[mb];
            tm.collect();
            if (status & 4) throw Error{PW_ERR_NUMERIC, "non-finite value in the iteration"};
            if (status & 1) {
                // a CholQR broke down (P or W): restart without P
                PW_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), st));
                if (np > 0) ++stats.p_restarts;
                np = 0;
            }
            for (int j = 0; j < mb; ++j)
                if (!std::isfinite(hres[j])) throw Error{PW_ERR_NUMERIC, "non-finite residual"};
            bool done = true;
            for (int j = 0; j < keep; ++j)
                if (!(hres[j] <= tol)) done = false;
            if (done) {
                converged_it = it;
                break;
            }
            if (floor_iters > 0) {
                double rmax = 0.0;
                for (int j = 0; j < keep; ++j) rmax = std::max(rmax, hres[j]);
                if (rmax < 0.5 * best) {
                    best = rmax;
                    since_best = 0;
                } else if (++since_best >= floor_iters) {
                    break;
                }
            }
            // soft locking: a column at the rounding floor of its residual gets no new
            // direction either (in the fixed-sweep mode, tol = 0, such a direction
            // would be rounding noise that CholQR blows up to unit norm)
            act.clear();
            for (int j = 0; j < mb; ++j)
                if (hres[j] > std::max(tol, res_floor)) act.push_back(j);
            const int na = (int)act.size();
            if (na == 0) {   // every column at the floor: the block is stationary
                if (tol == 0.0) it = max_iter;   // the remaining fixed sweeps are no-ops
                break;
            }
            // hact is rewritten only after the next synchronisation, when this copy has run
            std::copy(act.begin(), act.end(), hact);
            PW_HIP(hipMemcpyAsync(p.act, hact, sizeof(int) * na, hipMemcpyHostToDevice, st));
            const int wcol = mb + np;
            S *W = Z + (int64_t)wcol * ld;
            {
                auto e = tm.begin();
                pw::launch_precond_map(gen ? OZ : Z, ld, HZ, ld, c->sp.kin, npw, p.theta, p.ekin, p.act,
                                       na, W, ld, st);
                tm.end(PhaseTimer::kVec, e);
            }
            // constraint to previous blocks, then orthogonal to [X P] (twice) and orthonormal;
            // generalized form: O W is formed after the first projection and then carried
            S *OW = gen ? OZ + (int64_t)wcol * ld : nullptr;
            project_out(c, p, tm, (const S *)X, ldx, b0, W, ld, na, OXprev, ld, (S *)nullptr);
            for (int pass = 0; pass < 2; ++pass) {
                project_out(c, p, tm, (const S *)Z, ld, wcol, W, ld, na, (const S *)OZ, ld,
                            pass ? OW : nullptr);
                if (gen && pass == 0) {
                    auto e = tm.begin();
                    apply_O(c, p, m, W, ld, OW, ld, na);
                    tm.end(PhaseTimer::kApply, e);
                }
                cholqr(c, p, tm, W, ld, na, OW);
            }
            {
                auto e = tm.begin();
                apply_H(c, p, m, W, ld, HZ + (int64_t)wcol * ld, ld, na);
                tm.end(PhaseTimer::kApply, e);
                stats.h_applies += na;
            }
            const int nz = wcol + na;
            // Rayleigh-Ritz on span{X, P, W} (orthonormal basis)
            {
                auto e0 = tm.begin();
                rr_gram(c, p, Z, HZ, ld, nz);
                tm.end(PhaseTimer::kGemm, e0);
                auto e1 = tm.begin();
                pw::launch_heev_f64(p.Agram, nz, nz, mb, p.w, p.Cc, 3 * m, p.heev_scratch, c->d_status,
                                    st, lowp_reduction);
                tm.end(PhaseTimer::kDense, e1);
            }
            // P coefficients for the active columns: C with the X rows removed,
            // made orthogonal to C and orthonormal (in coefficient space, the
            // basis being orthonormal)
            cd *Cp = p.Cc + (int64_t)mb * 3 * m;
            {
                auto e0 = tm.begin();
                pw::launch_pcoef_map_f64(p.Cc, 3 * m, nz, mb, p.act, na, Cp, 3 * m, st);
                for (int pass = 0; pass < 2; ++pass) {
                    pw::launch_gemm_tn(p.Cc, 3 * m, Cp, 3 * m, nz, mb, na, p.T1, mb, nullptr, 0.0,
                                       p.part, p.part_elems, st);
                    pw::launch_gemm_nn(p.Cc, 3 * m, p.T1, mb, nz, mb, na, -1.0, 1.0, Cp, 3 * m, st);
                    pw::launch_gemm_tn(Cp, 3 * m, Cp, 3 * m, nz, na, na, p.Gs, na, nullptr, 0.0,
                                       p.part, p.part_elems, st);
                    pw::launch_chol_inv_f64(p.Gs, na, na, p.Rinv, na, c->d_status, st);
                    pw::launch_gemm_nn(Cp, 3 * m, p.Rinv, na, nz, na, na, 1.0, 0.0, Cp, 3 * m, st);
                }
                tm.end(PhaseTimer::kDense, e0);
            }
            // [X P]_new = Z [C c_p], same for HZ
            {
                auto e = tm.begin();
                pw::launch_gemm_nn(Z, ld, p.Cc, 3 * m, npw, nz, mb + na, 1.0, 0.0, p.Z[1 - cur], ld, st);
                pw::launch_gemm_nn(HZ, ld, p.Cc, 3 * m, npw, nz, mb + na, 1.0, 0.0, p.HZ[1 - cur], ld,
                                   st);
                if (gen)
                    pw::launch_gemm_nn(OZ, ld, p.Cc, 3 * m, npw, nz, mb + na, 1.0, 0.0, p.OZ[1 - cur], ld,
                                       st);
                tm.end(PhaseTimer::kGemm, e);
            }
            cur = 1 - cur;
            Z = p.Z[cur];
            HZ = p.HZ[cur];
            if (gen) OZ = p.OZ[cur];
            np = na;
        }
        const bool converged = converged_it >= 0;
        stats.iterations += it;
        if (!converged) all_converged = false;
        // store the converged columns of the block
        pw::launch_copy_cols(Z, ld, X + (int64_t)b0 * ldx, ldx, npw, keep, st);
        pw::launch_copy_cols(HZ, ld, p.HXall + (int64_t)b0 * ld, ld, npw, keep, st);
        if (gen) pw::launch_copy_cols(OZ, ld, p.OXall + (int64_t)b0 * ld, ld, npw, keep, st);
        prevZ = Z;
        prev_keep = keep;
        prev_mb = mb;
        b0 += keep;
    }

    if (final_rr) {   // Rayleigh-Ritz over all M bands
        auto ef = tm.begin();
        pw::launch_gemm_herm(X, ldx, p.HXall, ld, npw, M, p.Agram, M, p.part, p.part_elems, st);
        pw::launch_heev_f64(p.Agram, M, M, M, p.w, p.U, M, p.heev_scratch, c->d_status, st);
        pw::launch_gemm_nn(X, ldx, p.U, M, npw, M, M, 1.0, 0.0, p.T, ld, st);
        pw::launch_copy_cols(p.T, ld, X, ldx, npw, M, st);
        pw::launch_gemm_nn(p.HXall, ld, p.U, M, npw, M, M, 1.0, 0.0, p.T, ld, st);
        pw::launch_copy_cols(p.T, ld, p.HXall, ld, npw, M, st);
        if (p.OXall && c->d_Q) {
            pw::launch_gemm_nn(p.OXall, ld, p.U, M, npw, M, M, 1.0, 0.0, p.T, ld, st);
            pw::launch_copy_cols(p.T, ld, p.OXall, ld, npw, M, st);
            pw::launch_band_dots(X, ldx, p.HXall, ld, c->sp.kin, npw, M, p.rpart, p.theta, p.ekin, st,
                                 p.OXall, ld);
            pw::launch_resid_precond(p.OXall, ld, p.HXall, ld, c->sp.kin, npw, M, p.theta, p.ekin,
                                     (S *)nullptr, 0, p.rpart, p.res, st);
        } else {
            pw::launch_band_dots(X, ldx, p.HXall, ld, c->sp.kin, npw, M, p.rpart, p.theta, p.ekin, st);
            pw::launch_resid_precond(X, ldx, p.HXall, ld, c->sp.kin, npw, M, p.theta, p.ekin, (S *)nullptr,
                                     0, p.rpart, p.res, st);
        }
        tm.end(PhaseTimer::kFinal, ef);
    }
    PW_HIP(hipEventRecord(t_end, st));
    if (final_rr) {
        c->res.assign(M, 0.0);
        PW_HIP(hipMemcpyAsync(eig, p.theta, sizeof(double) * M, hipMemcpyDeviceToHost, st));
        PW_HIP(hipMemcpyAsync(c->res.data(), p.res, sizeof(double) * M, hipMemcpyDeviceToHost, st));
    }
    const int status = read_status(c);
    tm.collect();
    float total = 0.f;
    PW_HIP(hipEventElapsedTime(&total, t_begin, t_end));
    (void)hipEventDestroy(t_begin);
    (void)hipEventDestroy(t_end);
    stats.ms_total += total;
    stats.ms_apply += tm.ms[PhaseTimer::kApply];
    stats.ms_gemm += tm.ms[PhaseTimer::kGemm];
    stats.ms_dense += tm.ms[PhaseTimer::kDense];
    stats.ms_vec += tm.ms[PhaseTimer::kVec];
    stats.ms_final_rr += tm.ms[PhaseTimer::kFinal];
    if (status & 4) throw Error{PW_ERR_NUMERIC, "non-finite value in the final Rayleigh-Ritz"};
    if (!final_rr) return all_converged ? PW_OK : PW_ERR_NOT_CONVERGED;
    for (int j = 0; j < M; ++j) {
        if (!std::isfinite(eig[j])) throw Error{PW_ERR_NUMERIC, "non-finite eigenvalue"};
    }
    if (tol == 0.0) return PW_OK;   // fixed-sweep mode: max_iter iterations per block, no test
    bool res_ok = true;
    for (int j = 0; j < M; ++j)
        if (!(c->res[j] <= tol)) res_ok = false;
    if (!all_converged || !res_ok) {
        if (all_converged && final_res_above_tol) *final_res_above_tol = true;
        c->err = all_converged ? "a final residual exceeds tol after the final Rayleigh-Ritz"
                               : "max_iter reached before every block converged";
        return PW_ERR_NOT_CONVERGED;
    }
    return PW_OK;
}

// The FP64 iteration with its final Rayleigh-Ritz; if every block converged
// but the rotation over all bands left a residual above tol, one more sweep
// from the rotated vectors (each block then starts at or near convergence).
template <class S>
pw_status lobpcg_final(pw_ctx_s *c, const Plan<S> &p, int M, int m, double tol, int max_iter, S *X,
                       int64_t ldx, int use_guess, double *eig, pw_stats &stats) {
    bool resweep = false;
    pw_status rc = lobpcg(c, p, M, m, tol, max_iter, X, ldx, use_guess, eig, true, stats, 0, &resweep);
    if (rc == PW_ERR_NOT_CONVERGED && resweep)
        rc = lobpcg(c, p, M, m, tol, max_iter, X, ldx, 1, eig, true, stats);
    return rc;
}

// FP64 solve, or the mixed form: complex64 LOBPCG to kMixedTol, then the FP64
// iteration (with its final Rayleigh-Ritz) from those vectors.
pw_status solve(pw_ctx_s *c, int M, int m, double tol, int max_iter, pw_precision prec, cd *X,
                int64_t ldx, int use_guess, double *eig) {
    pw_stats stats{};
    pw_status rc;
    if (prec != PW_PREC_FP64) {
        ensure_mixed_tables(c);
        c->proj_bf16 = prec == PW_PREC_MIXED_BF16 || prec == PW_PREC_MIXED_BF16_GRAM;
        c->gram_bf16 = prec == PW_PREC_MIXED_BF16_GRAM;
        c->rr_fp32 = prec == PW_PREC_MIXED_FP32_RR;
        Plan<pw::cf> p32 = ready_plan<pw::cf>(c, M, m);
        if (use_guess) pw::launch_copy_cols(X, ldx, p32.Xs, c->ldp, c->npw, M, c->stream);
        // an unconverged block here is not an error: the FP64 stage continues from it
        (void)lobpcg(c, p32, M, m, std::max(tol, kMixedTol), std::min(max_iter, kMixedMaxIter), p32.Xs,
                     c->ldp, use_guess, eig, false, stats, kMixedFloorIters);
        pw::launch_copy_cols(p32.Xs, c->ldp, X, ldx, c->npw, M, c->stream);
        stats.mixed_iterations = stats.iterations;
        Plan<cd> p64 = ready_plan<cd>(c, M, m);
        rc = lobpcg_final(c, p64, M, m, tol, max_iter, X, ldx, 1, eig, stats);
    } else {
        Plan<cd> p64 = ready_plan<cd>(c, M, m);
        rc = lobpcg_final(c, p64, M, m, tol, max_iter, X, ldx, use_guess, eig, stats);
    }
    c->stats = stats;
    return rc;
}

// ---- basis setup -------------------------------------------------------------------
void init_basis(pw_ctx_s *c, const double cell[9], const double kfrac[3], double ecut,
                const int32_t fft_n[3], int64_t *npw_out) {
    PW_REQUIRE(cell && kfrac && fft_n && npw_out, PW_ERR_ARG, "null argument");
    PW_REQUIRE(ecut > 0 && std::isfinite(ecut), PW_ERR_ARG, "ecut must be positive");
    PW_REQUIRE(fft_n[0] == fft_n[1] && fft_n[1] == fft_n[2], PW_ERR_ARG, "FFT grid must be cubic");
    PW_REQUIRE(pw::fft_size_supported(fft_n[0]), PW_ERR_ARG, "unsupported FFT size");
    // reset everything that depends on the basis (a tuned radix split the new
    // grid cannot use falls back to the default)
    if (c->tune.fft_r2 > 0 && !split_available(fft_n[0], c->tune.fft_r2)) c->tune.fft_r2 = 0;
    if (c->device >= 0)
        for (void *p : c->dev_allocs) (void)hipFree(p);
    c->dev_allocs.clear();
    c->has_basis = c->has_v = false;
    c->natom = c->nlm = 0;
    c->d_B = nullptr;
    c->d_B32 = nullptr;
    c->d_D = nullptr;
    c->d_Q = nullptr;
    c->d_v = nullptr;
    c->d_v32 = nullptr;
    c->d_qvec = nullptr;
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->plan_nbands = c->plan_block = 0;
    c->d_status = nullptr;

    std::memcpy(c->cell, cell, sizeof(c->cell));
    std::memcpy(c->kfrac, kfrac, sizeof(c->kfrac));
    c->ecut = ecut;
    const int N = fft_n[0];
    c->n = N;
    // reciprocal rows b_i = 2 pi (cell^-1)^T rows
    const double *a = cell;
    const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                       a[2] * (a[3] * a[7] - a[4] * a[6]);
    PW_REQUIRE(std::fabs(det) > 1e-12, PW_ERR_ARG, "singular cell");
    double inv[9];
    inv[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    inv[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    inv[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    inv[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    inv[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    inv[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    inv[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    inv[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    inv[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    double B[9];   // B[i][j] = 2 pi inv[j][i]
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[3 * i + j] = 2.0 * M_PI * inv[3 * j + i];
    const double qmax = std::sqrt(2.0 * ecut);
    int lim[3];
    for (int i = 0; i < 3; ++i) {
        const double an = std::sqrt(a[3 * i] * a[3 * i] + a[3 * i + 1] * a[3 * i + 1] +
                                    a[3 * i + 2] * a[3 * i + 2]);
        lim[i] = (int)std::ceil(an * qmax / (2.0 * M_PI) + std::fabs(kfrac[i])) + 1;
    }
    c->miller.clear();
    c->kin.clear();
    c->qvec.clear();
    for (int nx = -lim[0]; nx <= lim[0]; ++nx)
        for (int ny = -lim[1]; ny <= lim[1]; ++ny)
            for (int nz = -lim[2]; nz <= lim[2]; ++nz) {
                const double f[3] = {nx + kfrac[0], ny + kfrac[1], nz + kfrac[2]};
                double q[3];
                for (int j = 0; j < 3; ++j) q[j] = f[0] * B[j] + f[1] * B[3 + j] + f[2] * B[6 + j];
                const double t = 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
                if (t <= ecut) {
                    c->miller.insert(c->miller.end(), {nx, ny, nz});
                    c->kin.push_back(t);
                    c->qvec.insert(c->qvec.end(), {q[0], q[1], q[2]});
                }
            }
    const int64_t npw = (int64_t)c->kin.size();
    PW_REQUIRE(npw > 0, PW_ERR_ARG, "empty plane-wave sphere");
    int mx[3] = {0, 0, 0};
    int xmin = 1 << 30, xmax = -(1 << 30);
    for (int64_t g = 0; g < npw; ++g) {
        for (int j = 0; j < 3; ++j) mx[j] = std::max(mx[j], std::abs(c->miller[3 * g + j]));
        xmin = std::min(xmin, c->miller[3 * g]);
        xmax = std::max(xmax, c->miller[3 * g]);
    }
    for (int j = 0; j < 3; ++j)
        PW_REQUIRE(N >= 2 * mx[j] + 1, PW_ERR_ARG, "FFT grid too small for the sphere (need n >= 2 nmax + 1)");
    // sticks: runs of equal (n_x, n_y)
    std::vector<int32_t> st_start, st_len, st_z0, st_y, st_xc, g_map(npw);
    for (int64_t g = 0; g < npw; ++g) {
        const int nx = c->miller[3 * g], ny = c->miller[3 * g + 1], nz = c->miller[3 * g + 2];
        if (g == 0 || nx != c->miller[3 * (g - 1)] || ny != c->miller[3 * (g - 1) + 1]) {
            st_start.push_back((int32_t)g);
            st_len.push_back(0);
            st_z0.push_back(nz);
            st_y.push_back(((ny % N) + N) % N);
            st_xc.push_back(nx - xmin);
        }
        const int s = (int)st_start.size() - 1;
        ++st_len[s];
        g_map[g] = s * N + ((nz % N) + N) % N;
    }
    const int nst = (int)st_start.size();
    c->npw = npw;
    c->nst_host = nst;
    c->ncx_host = xmax - xmin + 1;
    // sizes (also on a host-only context, so pw_workspace_size can plan there)
    c->ldp = (int64_t)align_up((size_t)npw, 32);
    pw::SphereDev &sp = c->sp;
    sp = pw::SphereDev{};
    sp.npw = npw;
    sp.n = N;
    sp.nst = nst;
    sp.ldst = (int32_t)align_up((size_t)nst, 16);
    sp.ncx = xmax - xmin + 1;
    sp.xmin = xmin;
    if (c->device < 0) {   // host-only context: tables stay on the host
        c->has_basis = true;
        *npw_out = npw;
        return;
    }
    c->d_status = c->dev_alloc<int>(1);
    PW_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
    auto up_i = [&](const std::vector<int32_t> &v) {
        int32_t *d = c->dev_alloc<int32_t>(v.size());
        PW_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        return d;
    };
    sp.st_start = up_i(st_start);
    sp.st_len = up_i(st_len);
    sp.st_z0 = up_i(st_z0);
    sp.st_y = up_i(st_y);
    sp.st_xc = up_i(st_xc);
    sp.g_map = up_i(g_map);
    sp.kin = c->dev_alloc<double>(npw);
    PW_HIP(hipMemcpy(sp.kin, c->kin.data(), npw * sizeof(double), hipMemcpyHostToDevice));
    std::vector<double> tw(2 * N);
    for (int j = 0; j < N; ++j) {
        const long double ang = 2.0L * 3.141592653589793238462643383279502884L * j / N;
        tw[2 * j] = (double)std::cos(ang);
        tw[2 * j + 1] = (double)std::sin(ang);
    }
    sp.twid = c->dev_alloc<double>(2 * N);
    PW_HIP(hipMemcpy(sp.twid, tw.data(), 2 * N * sizeof(double), hipMemcpyHostToDevice));
    c->d_qvec = c->dev_alloc<double>(3 * npw);
    PW_HIP(hipMemcpy(c->d_qvec, c->qvec.data(), 3 * npw * sizeof(double), hipMemcpyHostToDevice));
    c->has_basis = true;
    *npw_out = npw;
}

void set_potential(pw_ctx_s *c, const double *v, int on_device) {
    require_basis(c);
    require_device(c);
    PW_REQUIRE(v != nullptr, PW_ERR_ARG, "null potential");
    const int N = c->n;
    const size_t tot = (size_t)N * N * N;
    double *src = nullptr;
    double *tmp = c->dev_alloc<double>(tot);
    if (on_device) {
        src = const_cast<double *>(v);
    } else {
        PW_HIP(hipMemcpyAsync(tmp, v, tot * sizeof(double), hipMemcpyHostToDevice, c->stream));
        src = tmp;
    }
    if (!c->d_v) c->d_v = c->dev_alloc<double>(tot);
    c->dev_free(c->d_v32);   // the float copy is rebuilt on the next mixed-form call
    c->d_v32 = nullptr;
    PW_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
    const int r2 = tuned_r2(c);
    PW_REQUIRE(split_available(N, r2), PW_ERR_ARG, "the tuned radix split does not divide this FFT size");
    pw::launch_permute_potential(src, N, 1.0 / (double(N) * N * N), c->d_v, c->d_status, r2, c->stream);
    c->v_r2 = r2;
    const int s = read_status(c);
    c->dev_free(tmp);
    PW_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
    PW_REQUIRE(!(s & 1), PW_ERR_NUMERIC, "potential contains NaN or Inf");
    c->has_v = true;
}

void set_projectors(pw_ctx_s *c, int natom, const double *pos, int nlm, const int32_t *lm,
                    const double *D) {
    require_basis(c);
    require_device(c);
    PW_REQUIRE(natom >= 0 && nlm >= 0, PW_ERR_ARG, "negative projector count");
    c->dev_free(c->d_B);
    c->dev_free(c->d_B32);
    c->dev_free(c->d_D);
    c->dev_free(c->d_Q);
    c->d_B = nullptr;
    c->d_B32 = nullptr;
    c->d_D = nullptr;
    c->d_Q = nullptr;   // the overlap is defined on the projectors: cleared with them
    c->natom = c->nlm = 0;
    if (natom == 0 || nlm == 0) return;
    PW_REQUIRE(pos && lm && D, PW_ERR_ARG, "null projector argument");
    for (int p = 0; p < nlm; ++p) {
        const int l = lm[2 * p], m = lm[2 * p + 1];
        PW_REQUIRE((l == 0 && m == 0) || (l == 1 && m >= -1 && m <= 1), PW_ERR_ARG,
                   "projectors support l = 0, 1 only");
    }
    for (int i = 0; i < natom * nlm; ++i) PW_REQUIRE(std::isfinite(D[i]), PW_ERR_NUMERIC, "non-finite D");
    const int np = natom * nlm;
    double *d_pos = c->dev_alloc<double>(3 * natom);
    int *d_lm = c->dev_alloc<int>(2 * nlm);
    PW_HIP(hipMemcpy(d_pos, pos, 3 * natom * sizeof(double), hipMemcpyHostToDevice));
    PW_HIP(hipMemcpy(d_lm, lm, 2 * nlm * sizeof(int), hipMemcpyHostToDevice));
    c->d_B = c->dev_alloc<cd>((size_t)c->ldp * np);
    c->d_D = c->dev_alloc<double>(np);
    PW_HIP(hipMemcpy(c->d_D, D, np * sizeof(double), hipMemcpyHostToDevice));
    const double *a = c->cell;
    const double omega = std::fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                                   a[2] * (a[3] * a[7] - a[4] * a[6]));
    const double pref = std::sqrt(32.0 * std::pow(M_PI, 2.5)) / std::sqrt(omega);
    pw::launch_zero(c->d_B, c->ldp, c->ldp, np, c->stream);
    pw::launch_build_projectors_f64(c->d_qvec, c->npw, natom, d_pos, nlm, lm ? d_lm : nullptr, pref,
                                    c->d_B, c->ldp, c->stream);
    PW_HIP(hipStreamSynchronize(c->stream));
    c->dev_free(d_pos);
    c->dev_free(d_lm);
    c->natom = natom;
    c->nlm = nlm;
}

void set_overlap(pw_ctx_s *c, const double *q) {
    require_basis(c);
    require_device(c);
    c->dev_free(c->d_Q);
    c->d_Q = nullptr;
    if (!q) return;
    const int np = c->nproj();
    PW_REQUIRE(np > 0, PW_ERR_STATE, "the overlap needs projectors (pw_set_projectors)");
    for (int i = 0; i < np; ++i)
        PW_REQUIRE(std::isfinite(q[i]) && q[i] >= 0.0, PW_ERR_ARG, "overlap coefficients must be finite and >= 0");
    c->d_Q = c->dev_alloc<double>(np);
    PW_HIP(hipMemcpy(c->d_Q, q, np * sizeof(double), hipMemcpyHostToDevice));
}

// the context's launch parameters for the duration of one API call on this thread
struct TuningScope {
    const pw::Tuning *prev;
    explicit TuningScope(const pw::Tuning *t) : prev(pw::set_thread_tuning(t)) {}
    ~TuningScope() { pw::set_thread_tuning(prev); }
};

template <class F>
pw_status guard(pw_ctx c, F &&f) {
    if (!c) return PW_ERR_ARG;
    TuningScope scope(&c->tune);
    try {
        c->err.clear();
        return f();
    } catch (const Error &e) {
        c->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        c->err = "host allocation failed";
        return PW_ERR_NOMEM;
    } catch (...) {
        c->err = "unexpected exception";
        return PW_ERR_DEVICE;
    }
}

}  // namespace

namespace {
template <class S>
pw_status gram_impl(pw_ctx c, const void *A, int64_t lda, const void *B, int64_t ldb, int64_t K,
                    int32_t p, int32_t q, void *C, int64_t ldc) {
    return guard(c, [&] {
        require_device(c);
        PW_REQUIRE(A && B && C, PW_ERR_ARG, "null argument");
        PW_REQUIRE(K >= 0 && p >= 0 && q >= 0 && lda >= K && ldb >= K && ldc >= p, PW_ERR_ARG,
                   "bad GEMM shape");
        PW_REQUIRE(c->ws != nullptr, PW_ERR_STATE, "pw_set_workspace has not been called");
        if (p == 0 || q == 0) return PW_OK;
        // one K chunk needs p q partials; a smaller workspace than the full split
        // only lowers the number of chunks (the launcher clamps it)
        const size_t need = (size_t)p * q * sizeof(cd);
        PW_REQUIRE(need <= c->ws_bytes, PW_ERR_NOMEM, "workspace too small for this Gram");
        if (K == 0) {
            pw::launch_zero(static_cast<cd *>(C), ldc, p, q, c->stream);
            return PW_OK;
        }
        pw::launch_gemm_tn(static_cast<const S *>(A), lda, static_cast<const S *>(B), ldb, K, p, q,
                           static_cast<cd *>(C), ldc, nullptr, 0.0, reinterpret_cast<cd *>(c->ws),
                           c->ws_bytes / sizeof(cd), c->stream);
        return PW_OK;
    });
}

template <class S>
pw_status block_update_impl(pw_ctx c, const void *A, int64_t lda, const void *C, int64_t ldc,
                            int64_t K, int32_t p, int32_t q, double alpha, double beta, void *Y,
                            int64_t ldy) {
    return guard(c, [&] {
        require_device(c);
        PW_REQUIRE(A && C && Y, PW_ERR_ARG, "null argument");
        PW_REQUIRE(K >= 0 && p >= 0 && q >= 0 && lda >= K && ldy >= K && ldc >= p, PW_ERR_ARG,
                   "bad GEMM shape");
        pw::launch_gemm_nn(static_cast<const S *>(A), lda, static_cast<const cd *>(C), ldc, K, p, q,
                           alpha, beta, static_cast<S *>(Y), ldy, c->stream);
        return PW_OK;
    });
}

}  // namespace

namespace {
// the local part of every context in one launch per FFT pass, then each
// context's projector products, chunk by chunk (the stream is the contexts' one)
template <class S>
void apply_batch_impl(pw_ctx const *ctxs, int nk, const void *const *X, const int64_t *ldx,
                      void *const *Y, const int64_t *ldy, int nb, int chunk, pw_precision prec) {
    using T = decltype(S{}.x);
    pw_ctx c0 = ctxs[0];
    std::vector<Plan<S>> plans;
    plans.reserve(nk);
    for (int k = 0; k < nk; ++k) {
        pw_ctx c = ctxs[k];
        plans.push_back(ready_plan<S>(c, std::max(c->plan_nbands, 1), chunk));
        if constexpr (std::is_same<S, pw::cf>::value) {
            ensure_mixed_tables(c);
            c->proj_bf16 = prec == PW_PREC_MIXED_BF16 || prec == PW_PREC_MIXED_BF16_GRAM;
        }
    }
    std::vector<pw::FftApplyItem<T>> items(nk);
    for (int b0 = 0; b0 < nb; b0 += chunk) {
        const int nc = std::min(chunk, nb - b0);
        for (int k = 0; k < nk; ++k)
            items[k] = pw::FftApplyItem<T>{ctxs[k]->sp, static_cast<const S *>(X[k]) + (int64_t)b0 * ldx[k], ldx[k],
                                           static_cast<S *>(Y[k]) + (int64_t)b0 * ldy[k], ldy[k], plans[k].Sb};
        pw::launch_fft_apply_batch(items.data(), nk, potential_of(c0, (const S *)nullptr), nc, c0->stream);
        for (int k = 0; k < nk; ++k)
            if (ctxs[k]->nproj() > 0)
                proj_add(ctxs[k], plans[k], ctxs[k]->d_D, static_cast<const S *>(X[k]) + (int64_t)b0 * ldx[k], ldx[k],
                         static_cast<S *>(Y[k]) + (int64_t)b0 * ldy[k], ldy[k], nc);
    }
}
}  // namespace

extern "C" {

pw_status pw_create(int device, void *hip_stream, pw_ctx *out) {
    if (!out) return PW_ERR_ARG;
    *out = nullptr;
    if (device >= 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return PW_ERR_DEVICE;
        if (hipSetDevice(device) != hipSuccess) return PW_ERR_DEVICE;
    }
    pw_ctx c = new (std::nothrow) pw_ctx_s;
    if (!c) return PW_ERR_NOMEM;
    // device address of the library's static scratch on this device (once per
    // device; pw_small_eigh_noalloc reports a failure here when it is called)
    if (device >= 0) c->static_scratch_status = pw::static_scratch_setup(device);
    if (device >= 0 && hipHostMalloc(&c->h_pinned, pw_ctx_s::kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return PW_ERR_NOMEM;
    }
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    *out = c;
    return PW_OK;
}

void pw_destroy(pw_ctx c) {
    if (!c) return;
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        for (void *p : c->dev_allocs) (void)hipFree(p);
        if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    }
    delete c;
}

const char *pw_last_error(pw_ctx c) { return c ? c->err.c_str() : "null context"; }

pw_status pw_fft_sizes(int32_t *sizes, int32_t cap, int32_t *count) {
    if (!count) return PW_ERR_ARG;
    const std::vector<int> v = pw::fft_supported_sizes();
    *count = (int32_t)v.size();
    for (int i = 0; i < (int)v.size() && i < cap && sizes; ++i) sizes[i] = v[i];
    return PW_OK;
}

pw_status pw_init_basis(pw_ctx c, const double cell[9], const double kfrac[3], double ecut,
                        const int32_t fft_n[3], int64_t *npw) {
    return guard(c, [&] {
        if (c->device >= 0) PW_HIP(hipSetDevice(c->device));
        init_basis(c, cell, kfrac, ecut, fft_n, npw);
        return PW_OK;
    });
}

pw_status pw_get_miller(pw_ctx c, int32_t *miller) {
    return guard(c, [&] {
        require_basis(c);
        PW_REQUIRE(miller, PW_ERR_ARG, "null output");
        std::memcpy(miller, c->miller.data(), c->miller.size() * sizeof(int32_t));
        return PW_OK;
    });
}

pw_status pw_get_kinetic(pw_ctx c, double *kin) {
    return guard(c, [&] {
        require_basis(c);
        PW_REQUIRE(kin, PW_ERR_ARG, "null output");
        std::memcpy(kin, c->kin.data(), c->kin.size() * sizeof(double));
        return PW_OK;
    });
}

pw_status pw_set_local_potential(pw_ctx c, const double *v, int on_device) {
    return guard(c, [&] {
        if (c->device >= 0) PW_HIP(hipSetDevice(c->device));
        set_potential(c, v, on_device);
        return PW_OK;
    });
}

pw_status pw_set_projectors(pw_ctx c, int32_t natom, const double *pos, int32_t nproj_per_atom,
                            const int32_t *lm, const double *D) {
    return guard(c, [&] {
        if (c->device >= 0) PW_HIP(hipSetDevice(c->device));
        set_projectors(c, natom, pos, nproj_per_atom, lm, D);
        return PW_OK;
    });
}

pw_status pw_set_overlap(pw_ctx c, const double *q) {
    return guard(c, [&] {
        if (c->device >= 0) PW_HIP(hipSetDevice(c->device));
        set_overlap(c, q);
        return PW_OK;
    });
}

pw_status pw_workspace_size(pw_ctx c, int32_t nbands, int32_t block, pw_precision prec, size_t *bytes) {
    return guard(c, [&] {
        require_basis(c);
        PW_REQUIRE(bytes, PW_ERR_ARG, "null output");
        require_precision(prec);
        PW_REQUIRE(nbands >= 1 && block >= 1 && block <= 64, PW_ERR_ARG, "need nbands >= 1 and 1 <= block <= 64");
        PW_REQUIRE(nbands <= 1024 && (int64_t)nbands + 3 * std::min(block, nbands) <= c->npw, PW_ERR_ARG,
                   "need nbands <= 1024 and nbands + 3 * block <= npw");
        const int m = std::min(block, nbands);
        c->plan_nbands = nbands;
        c->plan_block = m;
        c->plan_prec = prec;
        *bytes = plan_bytes(*c, nbands, m, prec);
        return PW_OK;
    });
}

pw_status pw_set_workspace(pw_ctx c, void *dptr, size_t bytes) {
    return guard(c, [&] {
        require_basis(c);
        PW_REQUIRE(dptr, PW_ERR_ARG, "null workspace");
        PW_REQUIRE(((uintptr_t)dptr & 255) == 0, PW_ERR_ARG, "workspace must be 256-byte aligned");
        if (c->plan_nbands > 0) {
            const size_t need = plan_bytes(*c, c->plan_nbands, c->plan_block, c->plan_prec);
            PW_REQUIRE(bytes >= need, PW_ERR_NOMEM, "workspace smaller than pw_workspace_size");
        }
        c->ws = static_cast<char *>(dptr);
        c->ws_bytes = bytes;
        return PW_OK;
    });
}

// shared body of pw_apply_H and pw_apply_O
static pw_status apply_entry(pw_ctx c, const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t nb,
                             pw_precision prec, bool overlap) {
    return guard(c, [&] {
        require_precision(prec);
        require_basis(c);
        PW_REQUIRE(X && Y, PW_ERR_ARG, "null block");
        PW_REQUIRE(nb >= 0, PW_ERR_ARG, "negative column count");
        PW_REQUIRE(ldx >= c->npw && ldy >= c->npw, PW_ERR_ARG, "leading dimension < npw");
        PW_REQUIRE(!overlap || c->d_Q, PW_ERR_STATE, "pw_set_overlap has not been called");
        if (nb == 0) return PW_OK;
        const int chunk = c->plan_block > 0 ? c->plan_block : 1;
        if (prec != PW_PREC_FP64) {
            Plan<pw::cf> p = ready_plan<pw::cf>(c, std::max(c->plan_nbands, 1), chunk);
            ensure_mixed_tables(c);
            c->proj_bf16 = prec == PW_PREC_MIXED_BF16 || prec == PW_PREC_MIXED_BF16_GRAM;
            auto Xc = static_cast<const pw::cf *>(X);
            auto Yc = static_cast<pw::cf *>(Y);
            if (overlap) apply_O(c, p, chunk, Xc, ldx, Yc, ldy, nb);
            else apply_H(c, p, chunk, Xc, ldx, Yc, ldy, nb);
        } else {
            Plan<cd> p = ready_plan<cd>(c, std::max(c->plan_nbands, 1), chunk);
            auto Xc = static_cast<const cd *>(X);
            auto Yc = static_cast<cd *>(Y);
            if (overlap) apply_O(c, p, chunk, Xc, ldx, Yc, ldy, nb);
            else apply_H(c, p, chunk, Xc, ldx, Yc, ldy, nb);
        }
        return PW_OK;
    });
}

pw_status pw_apply_H(pw_ctx c, const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t nb,
                     pw_precision prec) {
    return apply_entry(c, X, ldx, Y, ldy, nb, prec, false);
}

pw_status pw_apply_O(pw_ctx c, const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t nb,
                     pw_precision prec) {
    return apply_entry(c, X, ldx, Y, ldy, nb, prec, true);
}


pw_status pw_apply_H_batch(pw_ctx const *ctxs, int32_t nk, const void *const *X, const int64_t *ldx,
                           void *const *Y, const int64_t *ldy, int32_t nb, pw_precision prec) {
    if (!ctxs || nk < 1 || !ctxs[0]) return PW_ERR_ARG;
    pw_ctx c0 = ctxs[0];
    return guard(c0, [&] {
        require_precision(prec);
        PW_REQUIRE(nk <= pw::kMaxApplyBatch, PW_ERR_ARG, "at most 16 contexts per batched apply");
        PW_REQUIRE(X && Y && ldx && ldy, PW_ERR_ARG, "null argument");
        PW_REQUIRE(nb >= 0, PW_ERR_ARG, "negative column count");
        require_basis(c0);
        require_device(c0);
        PW_REQUIRE(c0->has_v, PW_ERR_STATE, "pw_set_local_potential has not been called");
        int chunk = 1 << 30;
        for (int k = 0; k < nk; ++k) {
            pw_ctx c = ctxs[k];
            PW_REQUIRE(c != nullptr, PW_ERR_ARG, "null context");
            require_basis(c);
            PW_REQUIRE(c->device == c0->device && c->stream == c0->stream, PW_ERR_ARG,
                       "the contexts of a batched apply share one device and one stream");
            PW_REQUIRE(c->n == c0->n, PW_ERR_ARG, "the contexts of a batched apply share one FFT grid");
            PW_REQUIRE(X[k] && Y[k], PW_ERR_ARG, "null block");
            PW_REQUIRE(ldx[k] >= c->npw && ldy[k] >= c->npw, PW_ERR_ARG, "leading dimension < npw");
            for (int q = 0; q < k; ++q) PW_REQUIRE(ctxs[q] != c, PW_ERR_ARG, "a context appears twice");
            chunk = std::min(chunk, c->plan_block > 0 ? c->plan_block : 1);
        }
        if (nb == 0) return PW_OK;
        if (prec != PW_PREC_FP64) apply_batch_impl<pw::cf>(ctxs, nk, X, ldx, Y, ldy, nb, chunk, prec);
        else apply_batch_impl<cd>(ctxs, nk, X, ldx, Y, ldy, nb, chunk, prec);
        return PW_OK;
    });
}

pw_status pw_lobpcg_solve(pw_ctx c, int32_t nbands, int32_t block, double tol, int32_t max_iter,
                          pw_precision prec, void *X, int64_t ldx, int32_t use_guess, double *eig) {
    return guard(c, [&] {
        require_precision(prec);
        require_basis(c);
        PW_REQUIRE(X && eig, PW_ERR_ARG, "null argument");
        PW_REQUIRE(nbands >= 1 && block >= 1 && block <= 64, PW_ERR_ARG, "need nbands >= 1, 1 <= block <= 64");
        // every block needs room for its whole basis [X P W] beside the earlier bands
        PW_REQUIRE(nbands <= 1024 && (int64_t)nbands + 3 * std::min(block, nbands) <= c->npw, PW_ERR_ARG,
                   "need nbands <= 1024 and nbands + 3 * block <= npw");
        PW_REQUIRE(ldx >= c->npw, PW_ERR_ARG, "ldx < npw");
        PW_REQUIRE(tol >= 0 && max_iter >= 1, PW_ERR_ARG, "need tol >= 0 and max_iter >= 1");
        PW_REQUIRE(tol > 0 || prec == PW_PREC_FP64, PW_ERR_ARG, "the fixed-sweep mode (tol = 0) is FP64 only");
        const int m = std::min(block, nbands);
        PW_REQUIRE(c->plan_nbands >= nbands && c->plan_block == m, PW_ERR_STATE,
                   "call pw_workspace_size with this (nbands, block) before the solve");
        require_device(c);
        PW_HIP(hipSetDevice(c->device));
        return solve(c, nbands, m, tol, max_iter, prec, static_cast<cd *>(X), ldx, use_guess, eig);
    });
}

pw_status pw_lobpcg_solve_batch(pw_ctx *ctxs, int32_t n, int32_t nbands, int32_t block, double tol,
                                int32_t max_iter, pw_precision prec, void *const *X,
                                const int64_t *ldx, int32_t use_guess, double *const *eig,
                                pw_status *status) {
    if (!ctxs || !X || !ldx || !eig || !status || n < 1) return PW_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return PW_ERR_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return PW_ERR_ARG;   // one solve per context at a time
    }
    // one host thread per context; each context runs on its own stream
    std::vector<std::thread> th;
    th.reserve(n);
    for (int i = 0; i < n; ++i)
        th.emplace_back([=] {
            status[i] = pw_lobpcg_solve(ctxs[i], nbands, block, tol, max_iter, prec, X[i], ldx[i],
                                        use_guess, eig[i]);
        });
    for (auto &t : th) t.join();
    pw_status worst = PW_OK;
    for (int i = 0; i < n; ++i)
        if (status[i] != PW_OK && (worst == PW_OK || worst == PW_ERR_NOT_CONVERGED)) worst = status[i];
    return worst;
}

pw_status pw_set_tuning(pw_ctx c, const pw_tuning *t) {
    return guard(c, [&] {
        if (!t) {
            c->tune = pw::Tuning{};
            relayout_potential(c);
            return PW_OK;
        }
        PW_REQUIRE(t->fft_sticks_per_block >= 0 && t->fft_sticks_per_block <= 64, PW_ERR_ARG,
                   "fft_sticks_per_block must be in [0, 64]");
        PW_REQUIRE(t->fft_plane_rows >= 0 && t->fft_plane_rows <= 128, PW_ERR_ARG,
                   "fft_plane_rows must be in [0, 128]");
        PW_REQUIRE(t->gemm_split_workgroups >= 0 && t->gemm_split_workgroups <= pw::kTnSplitMax, PW_ERR_ARG,
                   "gemm_split_workgroups must be in [0, 1024]");
        PW_REQUIRE(t->fft_radix2 == 0 || (c->n > 0 ? split_available(c->n, t->fft_radix2)
                                                      : (t->fft_radix2 >= 2 && t->fft_radix2 <= 16)),
                   PW_ERR_ARG, "fft_radix2 must be 0 or the second factor of an available radix split");
        c->tune.fft_spb = t->fft_sticks_per_block;
        c->tune.fft_rb = t->fft_plane_rows;
        c->tune.tn_split_wgs = t->gemm_split_workgroups;
        c->tune.fft_r2 = t->fft_radix2;
        relayout_potential(c);
        return PW_OK;
    });
}

pw_status pw_autotune(pw_ctx c, int32_t nb, pw_tuning *out) {
    return guard(c, [&] {
        require_basis(c);
        require_device(c);
        PW_REQUIRE(out, PW_ERR_ARG, "null output");
        PW_REQUIRE(c->plan_block > 0, PW_ERR_STATE, "call pw_workspace_size before pw_autotune");
        PW_REQUIRE(nb >= 1 && nb <= c->plan_block, PW_ERR_ARG, "need 1 <= nb <= block of the workspace");
        PW_HIP(hipSetDevice(c->device));
        const int m = c->plan_block;
        Plan<cd> p = ready_plan<cd>(c, std::max(c->plan_nbands, 1), m);
        hipStream_t st = c->stream;
        const int64_t ld = c->ldp, npw = c->npw;
        const int np = c->nproj(), nz = (int)std::min<int64_t>(3 * m, npw);
        pw::launch_random_block(p.Z[0], ld, npw, nz, 0xA070ull, c->sp.kin, st);
        pw::launch_random_block(p.HZ[0], ld, npw, nz, 0xA071ull, c->sp.kin, st);
        hipEvent_t e0, e1;
        PW_HIP(hipEventCreate(&e0));
        PW_HIP(hipEventCreate(&e1));
        auto timed = [&](auto &&fn) {   // mean of 5 after one warm-up, ms
            fn();
            PW_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < 5; ++r) fn();
            PW_HIP(hipEventRecord(e1, st));
            PW_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            PW_HIP(hipEventElapsedTime(&ms, e0, e1));
            return (double)ms / 5.0;
        };
        const double *vapply = c->d_v;   // the potential in the layout of the split being timed
        auto apply = [&] { pw::launch_fft_apply(c->sp, vapply, p.Z[0], ld, p.HZ[0] + 0, ld, nb, p.Sb, st); };
        auto gemm = [&] {
            pw::launch_gemm_herm(p.Z[0], ld, p.HZ[0], ld, npw, nz, p.Agram, nz, p.part, p.part_elems, st);
            if (np > 0)
                pw::launch_gemm_tn(c->d_B, c->ldp, p.Z[0], ld, npw, np, m, p.Pj, np, c->d_D, 0.0, p.part,
                                   p.part_elems, st);
        };
        c->tune = pw::Tuning{};
        relayout_potential(c);   // default split
        const double apply_def = timed(apply), gemm_def = timed(gemm);
        pw::Tuning best{};
        double apply_best = apply_def, gemm_best = gemm_def;
        const int spb_c[] = {16, 32, 64}, rb_c[] = {16, 32, 48, 96};
        const std::vector<int> r2_c = pw::fft_radix_splits(c->n);
        const int r2_def = pw::fft_default_r2(c->n);
        double *vtmp = c->dev_alloc<double>((size_t)c->n * c->n * c->n);
        for (int r2 : r2_c) {
            vapply = c->d_v;
            if (r2 != r2_def) {   // the potential in this split's x-order
                pw::launch_repermute_potential(c->d_v, c->n, r2_def, r2, vtmp, st);
                vapply = vtmp;
            }
            for (int spb : spb_c)
                for (int rb : rb_c) {
                    c->tune = pw::Tuning{};
                    c->tune.fft_spb = spb;
                    c->tune.fft_rb = rb;
                    c->tune.fft_r2 = r2 == r2_def ? 0 : r2;
                    const double t = timed(apply);
                    if (t < apply_best) {
                        apply_best = t;
                        best.fft_spb = spb;
                        best.fft_rb = rb;
                        best.fft_r2 = c->tune.fft_r2;
                    }
                }
        }
        PW_HIP(hipStreamSynchronize(st));
        c->dev_free(vtmp);
        vapply = c->d_v;
        const int split_c[] = {384, 512, 768, 1024};
        for (int sw : split_c) {
            c->tune = pw::Tuning{};
            c->tune.tn_split_wgs = sw;
            const double t = timed(gemm);
            if (t < gemm_best) {
                gemm_best = t;
                best.tn_split_wgs = sw;
            }
        }
        c->tune = best;
        relayout_potential(c);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        out->fft_sticks_per_block = best.fft_spb;
        out->fft_plane_rows = best.fft_rb;
        out->gemm_split_workgroups = best.tn_split_wgs;
        out->fft_radix2 = best.fft_r2;
        out->apply_ms_default = apply_def;
        out->apply_ms_tuned = apply_best;
        out->gemm_ms_default = gemm_def;
        out->gemm_ms_tuned = gemm_best;
        return PW_OK;
    });
}

pw_status pw_density(pw_ctx c, const void *X, int64_t ldx, int32_t nb, const double *occ,
                     void *rho) {
    return guard(c, [&] {
        require_device(c);
        require_basis(c);
        PW_REQUIRE(X && occ && rho, PW_ERR_ARG, "null argument");
        PW_REQUIRE(nb >= 1 && ldx >= c->npw, PW_ERR_ARG, "need nb >= 1 and ldx >= npw");
        PW_REQUIRE(c->ws != nullptr, PW_ERR_STATE, "pw_set_workspace has not been called");
        for (int i = 0; i < nb; ++i) PW_REQUIRE(std::isfinite(occ[i]), PW_ERR_ARG, "non-finite occupation");
        const int chunk = c->plan_block > 0 ? c->plan_block : 1;
        const int64_t n3 = (int64_t)c->n * c->n * c->n;
        PW_REQUIRE(density_bytes(*c, chunk, nb) <= c->ws_bytes, PW_ERR_NOMEM, "workspace too small for the density");
        Arena a;
        a.base = c->ws;
        cd *S = a.take<cd>((size_t)chunk * c->n * c->sp.ldst);
        double *rz = a.take<double>((size_t)n3);
        double *docc = a.take<double>((size_t)nb);
        hipStream_t st = c->stream;
        pw::launch_zero(reinterpret_cast<cd *>(rz), n3 / 2, n3 / 2, 1, st);   // N is even
        PW_HIP(hipMemcpyAsync(docc, occ, sizeof(double) * nb, hipMemcpyHostToDevice, st));
        const cd *Xc = static_cast<const cd *>(X);
        for (int b0 = 0; b0 < nb; b0 += chunk) {
            const int nc = std::min(chunk, nb - b0);
            pw::launch_density_accumulate(c->sp, Xc + (int64_t)b0 * ldx, ldx, nc, docc + b0, rz, S, st);
        }
        const double *m = c->cell;
        const double omega = std::fabs(m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                                       m[2] * (m[3] * m[7] - m[4] * m[6]));
        pw::launch_density_finish(rz, c->n, 1.0 / omega, static_cast<double *>(rho), st);
        PW_HIP(hipStreamSynchronize(st));   // occ is read from host memory above
        return PW_OK;
    });
}

pw_status pw_get_residuals(pw_ctx c, double *res) {
    return guard(c, [&] {
        PW_REQUIRE(res, PW_ERR_ARG, "null output");
        PW_REQUIRE(!c->res.empty(), PW_ERR_STATE, "no solve has run");
        std::memcpy(res, c->res.data(), c->res.size() * sizeof(double));
        return PW_OK;
    });
}

pw_status pw_get_stats(pw_ctx c, pw_stats *stats) {
    return guard(c, [&] {
        PW_REQUIRE(stats, PW_ERR_ARG, "null output");
        *stats = c->stats;
        return PW_OK;
    });
}

pw_status pw_set_phase_timing(pw_ctx c, int32_t on) {
    return guard(c, [&] {
        c->phase_timing = on != 0;
        return PW_OK;
    });
}

pw_status pw_gram(pw_ctx c, const void *A, int64_t lda, const void *B, int64_t ldb, int64_t K,
                  int32_t p, int32_t q, void *C, int64_t ldc) {
    return gram_impl<cd>(c, A, lda, B, ldb, K, p, q, C, ldc);
}
pw_status pw_gram_mixed(pw_ctx c, const void *A, int64_t lda, const void *B, int64_t ldb, int64_t K,
                        int32_t p, int32_t q, void *C, int64_t ldc) {
    return gram_impl<pw::cf>(c, A, lda, B, ldb, K, p, q, C, ldc);
}
pw_status pw_block_update(pw_ctx c, const void *A, int64_t lda, const void *C, int64_t ldc,
                          int64_t K, int32_t p, int32_t q, double alpha, double beta, void *Y,
                          int64_t ldy) {
    return block_update_impl<cd>(c, A, lda, C, ldc, K, p, q, alpha, beta, Y, ldy);
}
pw_status pw_block_update_mixed(pw_ctx c, const void *A, int64_t lda, const void *C, int64_t ldc,
                                int64_t K, int32_t p, int32_t q, double alpha, double beta, void *Y,
                                int64_t ldy) {
    return block_update_impl<pw::cf>(c, A, lda, C, ldc, K, p, q, alpha, beta, Y, ldy);
}

pw_status pw_small_eigh(pw_ctx c, void *A, int64_t lda, int32_t n, int32_t k, void *w, void *V,
                        int64_t ldv) {
    return guard(c, [&] {
        require_device(c);
        PW_REQUIRE(A && w && V, PW_ERR_ARG, "null argument");
        PW_REQUIRE(n >= 1 && n <= 1024 && k >= 1 && k <= n && lda >= n && ldv >= n, PW_ERR_ARG,
                   "need 1 <= k <= n <= 1024");
        PW_REQUIRE(c->ws != nullptr, PW_ERR_STATE, "pw_set_workspace has not been called");
        PW_REQUIRE(c->d_status, PW_ERR_STATE, "pw_init_basis has not been called");
        PW_REQUIRE(pw::heev_scratch_bytes(n, k) <= c->ws_bytes, PW_ERR_NOMEM, "workspace too small");
        PW_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
        pw::launch_heev_f64(static_cast<cd *>(A), lda, n, k, static_cast<double *>(w),
                            static_cast<cd *>(V), ldv, c->ws, c->d_status, c->stream);
        const int s = read_status(c);
        PW_REQUIRE(!(s & 4), PW_ERR_NUMERIC, "non-finite eigenvalue");
        return PW_OK;
    });
}

pw_status pw_small_eigh_noalloc(pw_ctx c, void *A, int64_t lda, int32_t n, int32_t k, void *w,
                                void *V, int64_t ldv) {
    return guard(c, [&] {
        require_device(c);
        PW_REQUIRE(A && w && V, PW_ERR_ARG, "null argument");
        PW_REQUIRE(n >= 1 && n <= 1024 && k >= 1 && k <= n && lda >= n && ldv >= n, PW_ERR_ARG,
                   "need 1 <= k <= n <= 1024");
        const size_t need = 256 + pw::heev_scratch_bytes(n, k);
        if (need > pw::static_scratch_bytes())
            throw Error{PW_ERR_ARG, "n = " + std::to_string(n) + ", k = " + std::to_string(k) + " needs " +
                                        std::to_string(need) + " bytes of scratch, more than the " +
                                        std::to_string(pw::static_scratch_bytes()) +
                                        " of the library's static array; use pw_small_eigh"};
        if (c->static_scratch_status != hipSuccess)
            throw Error{PW_ERR_DEVICE, std::string("hipGetSymbolAddress of the static scratch failed: ") +
                                           hipGetErrorString(c->static_scratch_status)};
        char *base = static_cast<char *>(pw::static_scratch(c->device));
        PW_REQUIRE(base, PW_ERR_STATE, "static scratch not resolved on this device");
        // [0, 256): status word; [256, need): the eigensolver's scratch
        int *status = reinterpret_cast<int *>(base);
        pw::launch_clear_ints(status, 1, c->stream);
        pw::launch_heev_f64(static_cast<cd *>(A), lda, n, k, static_cast<double *>(w),
                            static_cast<cd *>(V), ldv, base + 256, status, c->stream);
        int *h = reinterpret_cast<int *>(c->pinned(sizeof(int)));
        PW_HIP(hipMemcpyAsync(h, status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        PW_HIP(hipStreamSynchronize(c->stream));
        PW_REQUIRE(!(*h & 4), PW_ERR_NUMERIC, "non-finite eigenvalue");
        return PW_OK;
    });
}

pw_status pw_chol_inv(pw_ctx c, const void *G, int64_t ldg, int32_t n, void *Rinv, int64_t ldr) {
    return guard(c, [&] {
        require_device(c);
        PW_REQUIRE(G && Rinv, PW_ERR_ARG, "null argument");
        PW_REQUIRE(n >= 1 && n <= 64 && ldg >= n && ldr >= n, PW_ERR_ARG, "need 1 <= n <= 64");
        PW_REQUIRE(c->d_status, PW_ERR_STATE, "pw_init_basis has not been called");
        PW_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
        pw::launch_chol_inv_f64(static_cast<const cd *>(G), ldg, n, static_cast<cd *>(Rinv), ldr,
                                c->d_status, c->stream);
        const int s = read_status(c);
        PW_REQUIRE(!(s & 1), PW_ERR_NUMERIC, "Cholesky breakdown (not positive definite)");
        return PW_OK;
    });
}

pw_status pw_residuals(pw_ctx c, const void *X, int64_t ldx, const void *HX, int64_t ldhx,
                       int32_t nb, void *theta, void *res, void *W, int64_t ldw) {
    return guard(c, [&] {
        require_device(c);
        require_basis(c);
        PW_REQUIRE(X && HX && theta && res, PW_ERR_ARG, "null argument");
        PW_REQUIRE(nb >= 1 && ldx >= c->npw && ldhx >= c->npw && (!W || ldw >= c->npw), PW_ERR_ARG,
                   "bad shape");
        PW_REQUIRE(c->ws != nullptr, PW_ERR_STATE, "pw_set_workspace has not been called");
        const size_t need = (pw::resid_part_elems(c->npw, nb) + 2 * (size_t)nb) * sizeof(double) + 512;
        PW_REQUIRE(need <= c->ws_bytes, PW_ERR_NOMEM, "workspace too small");
        double *part = reinterpret_cast<double *>(c->ws);
        double *ekin = part + align_up(pw::resid_part_elems(c->npw, nb), 32);
        pw::launch_band_dots(static_cast<const cd *>(X), ldx, static_cast<const cd *>(HX), ldhx,
                                 c->sp.kin, c->npw, nb, part, static_cast<double *>(theta), ekin,
                                 c->stream);
        pw::launch_resid_precond(static_cast<const cd *>(X), ldx, static_cast<const cd *>(HX), ldhx,
                                     c->sp.kin, c->npw, nb, static_cast<const double *>(theta), ekin,
                                     static_cast<cd *>(W), ldw, part, static_cast<double *>(res),
                                     c->stream);
        return PW_OK;
    });
}

}  // extern "C"
