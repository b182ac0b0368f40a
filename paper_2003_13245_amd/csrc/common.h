// Internal declarations shared by the ftdmrg host driver and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <atomic>
#include <complex>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ftdmrg.h"

namespace ftd {

inline double wall_seconds() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}


using cplx = std::complex<double>;

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);

struct Error {
    ftd_status code;
    std::string msg;
};

#define FTD_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::ftd::Error{FTD_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define FTD_CHECK(cond, code, msg)                                                      \
    do {                                                                                \
        if (!(cond)) throw ::ftd::Error{code, msg};                                     \
    } while (0)

// --------------------------------------------------------------- constants
constexpr int kMaxTerms = 32;   // summed GEMM products across all problems
constexpr int kMaxProbs = 16;   // independent GEMM outputs per launch
constexpr int kMaxMixJobs = 16;
constexpr int kMaxMixEnts = 40;
constexpr int kMaxKrylov = 64;  // one wavefront holds the tridiagonal problem

// ------------------------------------------------------------------ buffers
struct Ctx;

// Device allocation through the context allocator.
void* dev_alloc(Ctx* ctx, size_t bytes);
void dev_free(Ctx* ctx, void* p);

// A growable device buffer.  Growth synchronises the context stream before the
// old block is released, so kernels still queued on it never see freed memory.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void ensure(Ctx* ctx, size_t need);
    void release(Ctx* ctx);
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- GEMM API
// C_p = sum over terms t of problem p of opA(A + offA_t) * opB(B + offB_t)
// Complex operands in split planes: the imaginary plane of operand X starts
// `planeX` elements after its real plane.  Element (m,k) of A sits at
// m*sAm + k*sAk; (k,n) of B at k*sBk + n*sBn; (m,n) of C at m*sCm + n*sCn.
struct GemmTerm {
    int64_t offA, offB;
};
struct GemmProb {
    int64_t offC;
    int t0, t1;  // term range
};
struct GemmParams {
    int M, N, K;
    int64_t sAm, sAk, sBk, sBn, sCm, sCn;
    int64_t planeA, planeB, planeC;
    int conjA, conjB, accumulate;
    int nprob, ksplit;
    int a_kcontig, b_kcontig;
    const int* stop;   // launch is a no-op when *stop != 0 (Krylov halt), may be null
    // timing slot {first block start, last block end} in wall-clock ticks
    // (atomic min / max), or null
    unsigned long long* tstamp;
    GemmProb prob[kMaxProbs];
    GemmTerm term[kMaxTerms];
};

enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2 };

// kind tags used for timing attribution
enum KernelTag { TAG_NONE = 0, TAG_HEFF = 1, TAG_KEFF = 2 };

// Launch a complex GEMM.  Tin/Tout: double/double, float/float, float/double.
void gemm(Ctx* ctx, Prec prec, bool out_f64, const void* A, const void* B, void* C,
          GemmParams p, int tag);
// The same kernels with caller-provided split-K partial storage (partial_cap
// bytes; fewer splits are used when the chosen count does not fit), no
// allocation and no timing.
void gemm_in(Ctx* ctx, Prec prec, bool out_f64, const void* A, const void* B, void* C,
             GemmParams p, void* partial, size_t partial_cap);
// Device address of this library's static scratch array on `device`, looked
// up once per device (the device must be current).
void scratch_init(int device);

// ---------------------------------------------------------- channel mixing
// out_j[a][p'][q][b] (+)= sum_e op_e[p'][p] in_e[a][p][q][b]
struct MixJob {
    int64_t offOut;
    int e0, e1;
};
struct MixEnt {
    int64_t offIn;
    int op;
};
struct MixParams {
    int Da, d, Db;
    int64_t ldIn, ldOut;   // row strides of the b index (0 = Db)
    int64_t planeIn, planeOut;
    int64_t opStride;   // elements per op (re plane then im plane, d*d each)
    int accumulate;
    int njobs;
    const int* stop;   // launch is a no-op when *stop != 0, may be null
    MixJob job[kMaxMixJobs];
    MixEnt ent[kMaxMixEnts];
};
void chanmix(Ctx* ctx, Prec prec, bool out_f64, const void* in, const void* ops, void* out,
             const MixParams& p);

// ----------------------------------------------------------- vector kernels
void k_copy_f64(Ctx* ctx, const double* src, double* dst, int64_t n);
void k_convert_f64_f32(Ctx* ctx, const double* src, float* dst, int64_t n);
void k_scale_cplx(Ctx* ctx, double* x, int64_t n, int64_t plane, double re, double im);
void k_scale_by_dev(Ctx* ctx, double* x, int64_t n, int64_t plane, const double* s, int inv);
void k_zero(Ctx* ctx, void* p, size_t bytes);
// out[0] = |x|^2 (device)
void k_nrm2(Ctx* ctx, const double* x, int64_t n, int64_t plane, double* out);
// h[j] = <V_j, w>, j < k; V_j at V + j*vstride
void k_multidot(Ctx* ctx, const double* V, int64_t vstride, int k, const double* w, int64_t n,
                int64_t plane, double* h, double* alpha = nullptr);
// w -= sum_j V_j h[j] in one pass, with |w|^2 left as block partials in ctx->ws_red;
// returns their count.  With `skip` (two device doubles: |w|^2 after and before
// the first Gram-Schmidt pass) the kernel does nothing when skip[0] > thr2 *
// skip[1], the test the tridiagonal kernel repeats to pick its norm
int k_multiaxpy_nrm2_part(Ctx* ctx, const double* V, int64_t vstride, int k, const double* h,
                          double* w, int64_t n, int64_t plane, const double* skip = nullptr,
                          double thr2 = 0.0);
// w -= sum_j V_j h[j], then h[j] = <V_j, w> of the updated w, in one pass over
// V and w; also h[k] = (|w|^2 after, |w|^2 before the update).  False (nothing
// done) when k or n is outside its range (k <= 16, long vectors), so that the
// caller falls back to k_multiaxpy + k_multidot
bool k_multiaxpy_dot(Ctx* ctx, const double* V, int64_t vstride, int k, double* h, double* w,
                     int64_t n, int64_t plane);
// w -= sum_j V_j h[j]
void k_multiaxpy(Ctx* ctx, const double* V, int64_t vstride, int k, const double* h, double* w,
                 int64_t n, int64_t plane);
// y = scale * sum_j V_j u[j]
void k_lincomb(Ctx* ctx, const double* V, int64_t vstride, int k, const double* u,
               const double* scale_dev, double* y, int64_t n, int64_t plane);
// embed src[Da][dd][Db] into dst[DA][dd][DB] at (a0, b0), times (re, im)
void k_embed(Ctx* ctx, const double* src, int Da, int dd, int Db, double* dst, int DA, int DB,
             int a0, int b0, double re, double im, int accumulate = 0);
// exact MPO x MPS site product
struct ApplyEnt {
    int cl, cr, op;
};
void k_mpo_apply(Ctx* ctx, const double* A, int Da, int d, int Db, const double* ops,
                 int64_t opStride, int wl, int wr, const ApplyEnt* ents_dev, int nents,
                 double* B);
// B[a][b] planar -> A: dst = src row-major (rows x cols) transposed, with conj
void k_transpose(Ctx* ctx, const double* src, int64_t rows, int64_t cols, int64_t splane,
                 double* dst, int64_t dplane, int conj);

// ------------------------------------------------------------- Krylov tail
// Device state of one Lanczos run.
struct KrylovDev {
    double* alpha;   // [kMaxKrylov]
    double* beta;    // [kMaxKrylov]
    double* h;       // complex [2*(kMaxKrylov+1)]
    double* u;       // complex [2*kMaxKrylov]
    double* nrm;     // [4]
    int* flag;       // [4]: converged, k, failed, halt (converged or failed)
};
// the squared norm of the new residual is given as `nb` block partials, or,
// when skip[0] > thr2 * skip[1] (the second Gram-Schmidt pass was skipped), as
// skip[0]
void k_tridiag_expm(Ctx* ctx, KrylovDev kd, int k, double zr, double zi, double tol,
                    int exhausted, const double* nrm_part, int nb, const double* skip = nullptr,
                    double thr2 = 0.0);
void k_lanczos_post(Ctx* ctx, KrylovDev kd, int k, double* w, int64_t n, int64_t plane,
                    float* out32 = nullptr);
void k_krylov_reset(Ctx* ctx, KrylovDev kd);

// ----------------------------------------------------------------- QR / SVD
// Shifted CholeskyQR (three passes) of a full-column-rank M (m x n, row-major,
// split planes).  Q overwrites M; R (n x n upper, row-major, planar) returned.
void qr_chol(Ctx* ctx, double* M, int64_t m, int64_t n, double* R, bool check = true);
// LQ of a full-row-rank M (n x m row-major): M = L Q, Q overwrites M, L n x n.
void lq_chol(Ctx* ctx, double* M, int64_t n, int64_t m, double* L, bool check = true);
// reads and clears the sticky CholeskyQR breakdown flag; throws if it was set
void chol_flag_check(Ctx* ctx);
// clears that flag (after a failed sweep, whose gauge moves may have set it)
void chol_flag_clear(Ctx* ctx);
// Householder QR for any rank of an m x n matrix A: Q (m x r, row-major, not
// formed when Q is null) and R (r x n, row-major), r = min(m, n), diag(R)
// real >= 0.  A = M (row-major m x n), or A = M^H for a row-major n x m M
// when adjoint is set.
void qr_householder(Ctx* ctx, const double* M, int64_t m, int64_t n, double* Q, double* R,
                    bool adjoint = false);
// Thin SVD of X (m x n, row-major, m >= n) by one-sided Jacobi:
// X = U S V^H, U m x n (columns scaled), S[n] sorted descending, V n x n.
void svd_jacobi(Ctx* ctx, const double* X, int64_t m, int64_t n, double* U, double* S,
                double* V, bool adjoint_input = false);

// ----------------------------------------------------------------- objects
struct MpoEntry {
    int cl, cr;
    bool identity;
    std::vector<cplx> op;  // d x d, row-major [out][in], coefficient folded in
};
struct MpoSite {
    int d = 0, wl = 0, wr = 0;
    int idxI_l = -1, idxF_l = -1, idxI_r = -1, idxF_r = -1;
    std::vector<MpoEntry> ents;
    double* ops64 = nullptr;    // [nents][2][d][d]
    float* ops32 = nullptr;
    ApplyEnt* apply_ents = nullptr;  // device copy of (cl, cr, op)
};
struct Mpo {
    Ctx* ctx = nullptr;
    int L = 0;
    std::vector<MpoSite> s;
    std::vector<int> electronic;   // 1 where the site is a molecule's carrier site
    int wmax = 0, dmax = 0;
};

struct Mps {
    Ctx* ctx = nullptr;
    int L = 0;
    std::vector<int> Dl, Dr, d;
    std::vector<double*> A;   // planar complex, n = Dl*d*d*Dr per plane
    double log_norm = 0.0;
    Prec prec = Prec::F64;
    int64_t size(int i) const { return (int64_t)Dl[i] * d[i] * d[i] * Dr[i]; }
};

struct EventPair {
    hipEvent_t a, b;
    hipEvent_t m;   // after the main kernel (before a split-K reduction), or null
    double flops, bytes;
    int tag;
    int kind;   // kernel identity for dominant-kernel attribution
    int slot;   // device timestamp slot of the main kernel, or -1
};

struct Ctx {
    // Lifetime across the ABI: every ftd_mps / ftd_mpo handle made on this
    // context holds a reference, and so does the ftd_ctx handle until
    // ftd_ctx_destroy; the context is released when the last one goes, so
    // handles may be destroyed before or after their context.
    std::atomic<int> refs{1};
    void* owner = nullptr;   // the ftd_ctx this context belongs to
    int device = 0;
    hipStream_t stream = nullptr;
    bool has_alloc = false;
    ftd_allocator alloc{};
    // timing
    bool timing = false;
    int verbose = 0;
    std::vector<EventPair> events;
    std::vector<hipEvent_t> event_pool;
    size_t event_next = 0;
    // device timestamps of timed GEMM launches: 2 x u64 per slot
    unsigned long long* tslots = nullptr;
    int tslot_next = 0;
    static constexpr int kTimingSlots = 65536;
    ftd_stats stats{};
    // scratch
    DBuf ws_gemm_partial, ws_red;
    DBuf ws_T, ws_U, ws_X32, ws_Y32, ws_Krylov, ws_tmp1, ws_tmp2, ws_tmp3, ws_qr;
    DBuf ws_svd1, ws_svd2, ws_svd3, ws_site, ws_perm, ws_expY, ws_expC;
    // environments of the current sweep: envL[i] left of site i, envR[i]
    // right of site i-1 (i.e. contraction of sites i..L-1)
    std::vector<DBuf> envL, envR;
    std::vector<int> envL_w, envR_w, envL_D, envR_D;
    DBuf ws_A32;
    double* scal = nullptr;       // device scalars (Krylov state etc.)
    int* iscal = nullptr;
    // Float copies of Krylov vectors: every workspace reallocation bumps
    // ws_gen; load_slot records where it put the compute-precision copy of
    // its input (last32_*), and a Lanczos normalisation that already wrote
    // the next vector's copy there marks it (pre32_*) so the next load of
    // that vector is skipped.
    uint64_t ws_gen = 0;
    const double* last32_x = nullptr;
    void* last32_dst = nullptr;
    int64_t last32_n = 0;
    uint64_t last32_gen = 0;
    const double* pre32_x = nullptr;
    const void* pre32_dst = nullptr;
    uint64_t pre32_gen = 0;
    int* h_pinned_i = nullptr;    // host pinned readback
    double* h_pinned_d = nullptr;
    KrylovDev kd{};
    // While a Krylov exponential is being enqueued: its halt flag.  The
    // kernels of one Lanczos iteration return at once when it is set, so
    // iterations can be queued ahead of the convergence test.
    const int* kstop = nullptr;
    // vector counts of the previous exponential at each site / bond
    std::vector<int> khint_site, khint_bond;
};

// Progress line on stderr when the context's verbose level is >= level.
inline void vlog(const Ctx* ctx, int level, const char* fmt, ...) {
    if (ctx->verbose < level) return;
    va_list ap;
    va_start(ap, fmt);
    std::fputs("[ftdmrg] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    std::fflush(stderr);
    va_end(ap);
}

// context set-up / release (device scalars, pinned readback, workspaces)
void ctx_init(Ctx& c, int device, hipStream_t stream, const ftd_allocator* alloc);
void ctx_release(Ctx& c);
// one TDVP step of a (on ca) and of b (on cb) at the same time, from two host
// threads; cb's stream is ordered after ca's prior work and ca's stream after
// both steps
void tdvp_pair(Ctx* ca, Ctx* cb, hipEvent_t fork, hipEvent_t join, const Mpo* H, Mps* a, Mps* b,
               cplx z, double tol, int mmax);

hipEvent_t timing_event(Ctx* ctx);
void record_kernel(Ctx* ctx, hipEvent_t a, hipEvent_t b, double flops, double bytes, int tag,
                   int kind, hipEvent_t mid = nullptr, int slot = -1);
// next device timestamp slot (allocated and cleared on first use), or null
// when all are taken; timing_slots_reset clears them all
unsigned long long* timing_slot(Ctx* ctx, int* index);
void timing_slots_reset(Ctx* ctx);

// ---------------------------------------------------------- high level ops
Mpo* build_mpo(Ctx* ctx, const ftd_model& m, bool current);
void upload_mpo(Ctx* ctx, Mpo* mpo);
Mpo* build_product_mpo(Ctx* ctx, const ftd_model& md, std::vector<int>& carrier);
void reduced_density(Ctx* ctx, const ftd_model& md, const Mps* psi, double* sigma);
void destroy_mpo(Mpo* mpo);

Mps* mps_alloc(Ctx* ctx, const std::vector<int>& Dl, const std::vector<int>& d,
               const std::vector<int>& Dr, Prec prec);
void mps_free(Mps* m);
Mps* mps_clone(const Mps* m);
Mps* identity_mps(Ctx* ctx, const Mpo* H);

// One second-order one-site TDVP step; expand_D > 0 turns on the bond
// expansion up to expand_D with threshold expand_tol (relative to |H_eff A|).
void tdvp_step(Ctx* ctx, const Mpo* H, Mps* psi, cplx z, double tol, int mmax, int expand_D = 0,
               double expand_tol = 0.0);
Mps* apply_compress(Ctx* ctx, const Mpo* O, const Mps* psi, int D, double cutoff);
Mps* compress(Ctx* ctx, Mps* X, int D, double cutoff, bool consume);
void truncate_canonical(Ctx* ctx, Mps* psi, int D, double cutoff);
struct TruncOut {
    int k;
    double* Lq;
    double* Rq;
};
// abs_floor >= 0 switches to the expansion rule: keep the singular values
// above abs_floor, at most D, possibly none (k = 0, no buffers returned).
TruncOut svd_trunc(Ctx* ctx, const double* T, int64_t m, int64_t n, int D, double cutoff,
                   bool s_left, double abs_floor = -1.0);
Mps* taylor_growth(Ctx* ctx, const Mpo* H, const Mps* psi, double dtau, int D, double cutoff);
Mps* pc_stage(Ctx* ctx, const Mps* psi, const Mpo* O, const Mps* phi, cplx c, int D, double cutoff);
Mps* mps_add(Ctx* ctx, const Mps* a, const Mps* b, cplx c);
Mps* mpo_apply(Ctx* ctx, const Mpo* O, const Mps* psi);
double mps_normalize(Ctx* ctx, Mps* psi);
cplx overlap(Ctx* ctx, const Mps* bra, const Mpo* O, const Mps* ket);
void heff_apply_host(Ctx* ctx, const Mpo* H, const Mps* psi, int site, const double* x,
                     double* y, int nrep);
int heff_expm_host(Ctx* ctx, const Mpo* H, const Mps* psi, int site, const double* x, double* y,
                   cplx z, double tol, int mmax, int nrep);

}  // namespace ftd

struct ftd_ctx {
    ftd::Ctx c;
    // second context on its own stream, created on first use: the two states
    // of the correlation loop are propagated concurrently
    ftd::Ctx* aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};
struct ftd_mpo {
    ftd::Mpo* m;
};
struct ftd_mps {
    ftd::Mps* m;
};
