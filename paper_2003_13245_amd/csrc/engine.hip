// Host driver of the hot path: environments, effective Hamiltonians, the
// Krylov exponential, one-site projector-splitting sweeps, compression,
// imaginary-time preparation and the current correlation.
//
// Every floating-point step runs in HIP kernels; the host only orders
// launches, reads back Krylov stop flags and truncation spectra, and keeps
// shapes.  Site tensors A[a][p][q][b] are float64 complex in split planes
// (real plane, then imaginary plane).  Environments hold one D x D block per
// MPO channel, each block [re plane][im plane].
#include <algorithm>
#include <cfloat>
#include <exception>
#include <functional>
#include <numeric>
#include <thread>

#include "common.h"

namespace ftd {

// ================================================================ buffers
void* dev_alloc(Ctx* ctx, size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = nullptr;
    if (ctx->has_alloc) {
        p = ctx->alloc.alloc(bytes, ctx->alloc.user);
        FTD_CHECK(p != nullptr, FTD_ENOMEM, "allocator callback failed");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        FTD_CHECK(e == hipSuccess, FTD_ENOMEM, "hipMalloc failed");
    }
    return p;
}
void dev_free(Ctx* ctx, void* p) {
    if (!p) return;
    if (ctx->has_alloc)
        ctx->alloc.free(p, ctx->alloc.user);
    else
        (void)hipFree(p);
}
void DBuf::ensure(Ctx* ctx, size_t need) {
    if (need <= bytes) return;
    if (p) {
        FTD_HIP(hipStreamSynchronize(ctx->stream));
        dev_free(ctx, p);
        p = nullptr;
        bytes = 0;
    }
    size_t want = need + need / 4 + 256;
    p = dev_alloc(ctx, want);
    bytes = want;
    ctx->ws_gen++;
}
void DBuf::release(Ctx* ctx) {
    dev_free(ctx, p);
    p = nullptr;
    bytes = 0;
}

void ctx_init(Ctx& c, int device, hipStream_t stream, const ftd_allocator* alloc) {
    c.device = device;
    c.stream = stream;
    scratch_init(device);
    if (alloc && alloc->alloc && alloc->free) {
        c.has_alloc = true;
        c.alloc = *alloc;
    }
    c.scal = static_cast<double*>(dev_alloc(&c, sizeof(double) * 4096));
    c.iscal = static_cast<int*>(dev_alloc(&c, sizeof(int) * 64));
    FTD_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_pinned_i), sizeof(int) * 64,
                          hipHostMallocDefault));
    FTD_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_pinned_d), sizeof(double) * 64,
                          hipHostMallocDefault));
    FTD_HIP(hipMemsetAsync(c.scal, 0, sizeof(double) * 4096, c.stream));
    FTD_HIP(hipMemsetAsync(c.iscal, 0, sizeof(int) * 64, c.stream));
    double* s = c.scal + 256;
    c.kd.alpha = s;
    c.kd.beta = s + kMaxKrylov;
    c.kd.h = s + 2 * kMaxKrylov;
    c.kd.u = s + 4 * kMaxKrylov + 2;
    c.kd.nrm = s + 6 * kMaxKrylov + 4;
    c.kd.flag = c.iscal + 32;
    FTD_HIP(hipStreamSynchronize(c.stream));
}

void ctx_release(Ctx& c) {
    (void)hipStreamSynchronize(c.stream);
    for (auto* b : {&c.ws_gemm_partial, &c.ws_red, &c.ws_T, &c.ws_U, &c.ws_X32, &c.ws_Y32,
                    &c.ws_Krylov, &c.ws_tmp1, &c.ws_tmp2, &c.ws_tmp3, &c.ws_qr, &c.ws_svd1,
                    &c.ws_svd2, &c.ws_svd3, &c.ws_site, &c.ws_perm, &c.ws_A32, &c.ws_expY,
                    &c.ws_expC})
        b->release(&c);
    for (auto& b : c.envL) b.release(&c);
    for (auto& b : c.envR) b.release(&c);
    dev_free(&c, c.scal);
    dev_free(&c, c.iscal);
    dev_free(&c, c.tslots);
    c.tslots = nullptr;
    c.scal = nullptr;
    c.iscal = nullptr;
    if (c.h_pinned_i) (void)hipHostFree(c.h_pinned_i);
    if (c.h_pinned_d) (void)hipHostFree(c.h_pinned_d);
    c.h_pinned_i = nullptr;
    c.h_pinned_d = nullptr;
    for (auto e : c.event_pool) (void)hipEventDestroy(e);
    c.event_pool.clear();
}

hipEvent_t timing_event(Ctx* ctx) {
    if (ctx->event_next >= ctx->event_pool.size()) {
        hipEvent_t e;
        FTD_HIP(hipEventCreate(&e));
        ctx->event_pool.push_back(e);
    }
    return ctx->event_pool[ctx->event_next++];
}
void record_kernel(Ctx* ctx, hipEvent_t a, hipEvent_t b, double flops, double bytes, int tag,
                   int kind, hipEvent_t mid, int slot) {
    ctx->events.push_back({a, b, mid, flops, bytes, tag, kind, slot});
}

__global__ void tslot_clear_kernel(unsigned long long* s, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        s[2 * i] = ~0ull;
        s[2 * i + 1] = 0ull;
    }
}
void timing_slots_reset(Ctx* ctx) {
    ctx->tslot_next = 0;
    if (!ctx->tslots) return;
    tslot_clear_kernel<<<64, 256, 0, ctx->stream>>>(ctx->tslots, Ctx::kTimingSlots);
    FTD_HIP(hipGetLastError());
}
unsigned long long* timing_slot(Ctx* ctx, int* index) {
    if (!ctx->tslots) {
        ctx->tslots = static_cast<unsigned long long*>(
            dev_alloc(ctx, sizeof(unsigned long long) * 2 * Ctx::kTimingSlots));
        timing_slots_reset(ctx);
    }
    if (ctx->tslot_next >= Ctx::kTimingSlots) {
        *index = -1;
        return nullptr;
    }
    *index = ctx->tslot_next++;
    return ctx->tslots + 2 * (size_t)*index;
}

// ============================================================ small kernels
__global__ void eye_f64_kernel(double* X, int n, int64_t plane) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        X[e] = (e / n == e % n) ? 1.0 : 0.0;
        X[e + plane] = 0.0;
    }
}
__global__ void eye_f32_kernel(float* X, int n, int64_t plane) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        X[e] = (e / n == e % n) ? 1.0f : 0.0f;
        X[e + plane] = 0.0f;
    }
}
// dst[:, j] = s_j * op(src[:, perm[j]])  (column-major, m rows)
__global__ void gather_cols_kernel(const double* __restrict__ src, int64_t m, int64_t splane,
                                   const int* __restrict__ perm, const double* __restrict__ sc,
                                   int k, int conj, double* __restrict__ dst, int64_t dplane) {
    const int64_t tot = m * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / m);
        const int64_t i = e % m;
        const double s = sc ? sc[j] : 1.0;
        const int64_t o = (int64_t)perm[j] * m + i;
        dst[e] = s * src[o];
        dst[e + dplane] = (conj ? -s : s) * src[o + splane];
    }
}

static dim3 gr(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65535 * 4) b = 65535 * 4;
    return dim3((unsigned)b);
}
static void eye(Ctx* ctx, void* X, int n, int64_t plane, bool f32) {
    if (f32)
        eye_f32_kernel<<<gr((int64_t)n * n), 256, 0, ctx->stream>>>(static_cast<float*>(X), n, plane);
    else
        eye_f64_kernel<<<gr((int64_t)n * n), 256, 0, ctx->stream>>>(static_cast<double*>(X), n, plane);
    FTD_HIP(hipGetLastError());
}

// ===================================================================== MPS
Mps* mps_alloc(Ctx* ctx, const std::vector<int>& Dl, const std::vector<int>& d,
               const std::vector<int>& Dr, Prec prec) {
    Mps* m = new Mps();
    m->ctx = ctx;
    m->L = (int)d.size();
    m->Dl = Dl;
    m->Dr = Dr;
    m->d = d;
    m->prec = prec;
    m->A.assign(m->L, nullptr);
    try {
        for (int i = 0; i < m->L; ++i)
            m->A[i] = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m->size(i)));
    } catch (...) {
        mps_free(m);
        throw;
    }
    return m;
}
void mps_free(Mps* m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->ctx->stream);
    for (auto p : m->A) dev_free(m->ctx, p);
    delete m;
}
Mps* mps_clone(const Mps* s) {
    Mps* m = mps_alloc(s->ctx, s->Dl, s->d, s->Dr, s->prec);
    for (int i = 0; i < s->L; ++i) k_copy_f64(s->ctx, s->A[i], m->A[i], 2 * s->size(i));
    m->log_norm = s->log_norm;
    return m;
}
static void set_site(Ctx* ctx, Mps* m, int i, int Dl, int Dr, double* buf) {
    FTD_HIP(hipStreamSynchronize(ctx->stream));
    dev_free(ctx, m->A[i]);
    m->A[i] = buf;
    m->Dl[i] = Dl;
    m->Dr[i] = Dr;
}

// The purified identity of the one-carrier space, |I> = sum_i |i>_P |i>_Q.
// Bond states: "carrier not yet placed" and "placed"; electronic sites move
// between them with p = q = 1, phonon sites carry the identity on (p, q).
Mps* identity_mps(Ctx* ctx, const Mpo* H) {
    const int L = H->L;
    std::vector<int> d(L), kind(L);
    std::vector<int> epos;
    for (int i = 0; i < L; ++i) {
        d[i] = H->s[i].d;
        kind[i] = H->electronic[i];
        if (kind[i]) epos.push_back(i);
    }
    FTD_CHECK(!epos.empty(), FTD_EINVAL, "MPO has no carrier sites");
    const int fe = epos.front(), le = epos.back();
    std::vector<int> Dl(L), Dr(L);
    for (int i = 0; i < L; ++i) {
        Dl[i] = (i <= fe || i > le) ? 1 : 2;
        Dr[i] = (i < fe || i >= le) ? 1 : 2;
    }
    Mps* m = mps_alloc(ctx, Dl, d, Dr, Prec::F64);
    double dim = (double)epos.size();
    for (int i = 0; i < L; ++i)
        if (!kind[i]) dim *= d[i];
    for (int i = 0; i < L; ++i) {
        const int64_t n = m->size(i);
        std::vector<double> h(2 * n, 0.0);
        const int dd = d[i];
        auto at = [&](int a, int p, int q, int b) -> double& {
            return h[(((int64_t)a * dd + p) * dd + q) * Dr[i] + b];
        };
        // bond labels: 0 none, 1 placed
        auto lab_l = [&](int a) { return (i <= fe) ? 0 : (i > le ? 1 : a); };
        auto lab_r = [&](int b) { return (i < fe) ? 0 : (i >= le ? 1 : b); };
        for (int a = 0; a < Dl[i]; ++a)
            for (int b = 0; b < Dr[i]; ++b) {
                const int la = lab_l(a), lb = lab_r(b);
                if (kind[i]) {
                    if (la == 0 && lb == 0) at(a, 0, 0, b) = 1.0;
                    if (la == 0 && lb == 1) at(a, 1, 1, b) = 1.0;
                    if (la == 1 && lb == 1) at(a, 0, 0, b) = 1.0;
                } else if (la == lb) {
                    for (int v = 0; v < dd; ++v) at(a, v, v, b) = 1.0;
                }
            }
        if (i == 0)
            for (auto& x : h) x /= std::sqrt(dim);
        FTD_HIP(hipMemcpyAsync(m->A[i], h.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice,
                               ctx->stream));
        FTD_HIP(hipStreamSynchronize(ctx->stream));
    }
    m->log_norm = 0.5 * std::log(dim);
    return m;
}

static double read_scalar(Ctx* ctx, const double* dev) {
    FTD_HIP(hipMemcpyAsync(ctx->h_pinned_d, dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    FTD_HIP(hipStreamSynchronize(ctx->stream));
    return ctx->h_pinned_d[0];
}

double mps_normalize(Ctx* ctx, Mps* psi) {
    const int64_t n = psi->size(0);
    k_nrm2(ctx, psi->A[0], n, n, ctx->scal + 4);
    const double nn = read_scalar(ctx, ctx->scal + 4);
    FTD_CHECK(std::isfinite(nn) && nn > 0.0, FTD_ENOCONV, "state norm is zero or not finite");
    const double nrm = std::sqrt(nn);
    k_scale_cplx(ctx, psi->A[0], n, n, 1.0 / nrm, 0.0);
    psi->log_norm += std::log(nrm);
    return nrm;
}

// ============================================================ environments
struct EnvView {
    void* p;      // channel c block at p + c*2*D1*D2 (element type by precision)
    int w, D1, D2;
};

static size_t esz(Prec prec) { return prec == Prec::F64 ? sizeof(double) : sizeof(float); }

static EnvView env_get(Ctx* ctx, std::vector<DBuf>& bufs, std::vector<int>& ws,
                       std::vector<int>& Ds, int i, int w, int D, Prec prec) {
    if ((int)bufs.size() <= i) {
        bufs.resize(i + 1);
        ws.resize(i + 1, 0);
        Ds.resize(i + 1, 0);
    }
    bufs[i].ensure(ctx, esz(prec) * 2 * (size_t)w * D * D);
    ws[i] = w;
    Ds[i] = D;
    return {bufs[i].p, w, D, D};
}

static void boundary_env(Ctx* ctx, EnvView e, Prec prec) {
    eye(ctx, e.p, 1, 1, prec != Prec::F64);
}

// compute-precision copy of a site tensor into slot `slot` of ws_T
static void load_slot(Ctx* ctx, Prec prec, const double* x, int64_t n, void* Tbase, int slot) {
    if (prec == Prec::F64) {
        k_copy_f64(ctx, x, static_cast<double*>(Tbase) + (int64_t)slot * 2 * n, 2 * n);
        ctx->last32_x = nullptr;
        return;
    }
    float* dst = static_cast<float*>(Tbase) + (int64_t)slot * 2 * n;
    const bool ready = x == ctx->pre32_x && dst == ctx->pre32_dst && ctx->pre32_gen == ctx->ws_gen;
    ctx->pre32_x = nullptr;
    if (!ready) k_convert_f64_f32(ctx, x, dst, 2 * n);
    ctx->last32_x = x;
    ctx->last32_dst = dst;
    ctx->last32_n = n;
    ctx->last32_gen = ctx->ws_gen;
}

static const void* ops_of(const MpoSite& W, Prec prec) {
    return prec == Prec::F64 ? (const void*)W.ops64 : (const void*)W.ops32;
}

// Stage 1: T[c] = E[c] * X for the listed channels (batched GEMM).
// X lives in slot xs of Tbase; T[c] in slot c.  Shapes: E[c] Da1 x Da2,
// X Da2 x (dd * Db), T Da1 x (dd * Db).
static void stage_left(Ctx* ctx, Prec prec, const EnvView& E, const std::vector<int>& chans,
                       void* Tbase, int xs, int Da1, int Da2, int dd, int Db, int64_t nslot,
                       int tag) {
    if (chans.empty()) return;
    const int64_t nX = (int64_t)Da2 * dd * Db;
    for (size_t c0 = 0; c0 < chans.size(); c0 += kMaxProbs) {
        GemmParams p{};
        p.M = Da1;
        p.N = dd * Db;
        p.K = Da2;
        p.sAm = Da2; p.sAk = 1; p.planeA = (int64_t)Da1 * Da2; p.a_kcontig = 1;
        p.sBk = (int64_t)dd * Db; p.sBn = 1; p.planeB = nX; p.b_kcontig = 0;
        p.sCm = (int64_t)dd * Db; p.sCn = 1; p.planeC = nslot;
        const size_t c1 = std::min(chans.size(), c0 + kMaxProbs);
        p.nprob = (int)(c1 - c0);
        for (size_t k = c0; k < c1; ++k) {
            const int c = chans[k];
            const int j = (int)(k - c0);
            p.prob[j].offC = (int64_t)c * 2 * nslot;
            p.prob[j].t0 = j;
            p.prob[j].t1 = j + 1;
            p.term[j].offA = (int64_t)c * 2 * Da1 * Da2;
            p.term[j].offB = (int64_t)xs * 2 * nslot;
        }
        gemm(ctx, prec, prec == Prec::F64, E.p, Tbase, Tbase, p, tag);
    }
}

// Stage 2 plan: for each output channel, entries (input slot, op).  Returns
// for every output channel the slot that holds its mixed tensor (alias when
// the column is a single identity entry).
struct MixPlan {
    std::vector<int> out_slot;       // per output channel, -1 if column empty
};

// by_col: entries grouped by output channel; each entry (input channel, op)
static MixPlan stage_mix(Ctx* ctx, Prec prec, const MpoSite& W, bool left_to_right,
                         const std::vector<int>& in_slot, int n_out, int out_base,
                         const std::vector<int>& skip_out, void* Tbase, int Da, int d, int Db,
                         int64_t nslot, int direct_out, void* direct_ptr, bool direct_f64,
                         bool direct_acc) {
    MixPlan plan;
    plan.out_slot.assign(n_out, -1);
    std::vector<std::vector<std::pair<int, int>>> col(n_out);
    for (size_t e = 0; e < W.ents.size(); ++e) {
        const int o = left_to_right ? W.ents[e].cr : W.ents[e].cl;
        const int i = left_to_right ? W.ents[e].cl : W.ents[e].cr;
        col[o].push_back({i, (int)e});
    }
    MixParams mp{};
    mp.Da = Da;
    mp.d = d;
    mp.Db = Db;
    mp.planeIn = nslot;
    mp.planeOut = nslot;
    mp.opStride = 2 * (int64_t)d * d;
    MixParams md = mp;
    int ne = 0, ned = 0;
    for (int o = 0; o < n_out; ++o) {
        if (col[o].empty()) continue;
        if (std::find(skip_out.begin(), skip_out.end(), o) != skip_out.end()) continue;
        if (o == direct_out) {
            md.job[md.njobs] = {0, ned, ned + (int)col[o].size()};
            for (auto& pr : col[o]) md.ent[ned++] = {(int64_t)in_slot[pr.first] * 2 * nslot, pr.second};
            md.njobs++;
            continue;
        }
        if (col[o].size() == 1 && W.ents[col[o][0].second].identity) {
            plan.out_slot[o] = in_slot[col[o][0].first];
            continue;
        }
        const int slot = out_base + o;
        FTD_CHECK(mp.njobs < kMaxMixJobs && ne + (int)col[o].size() <= kMaxMixEnts, FTD_EINVAL,
                  "MPO site too wide for the channel mixer");
        mp.job[mp.njobs] = {(int64_t)slot * 2 * nslot, ne, ne + (int)col[o].size()};
        for (auto& pr : col[o]) mp.ent[ne++] = {(int64_t)in_slot[pr.first] * 2 * nslot, pr.second};
        mp.njobs++;
        plan.out_slot[o] = slot;
    }
    if (mp.njobs) chanmix(ctx, prec, false, Tbase, ops_of(W, prec), Tbase, mp);
    if (md.njobs) {
        md.planeOut = nslot;
        md.accumulate = direct_acc ? 1 : 0;
        chanmix(ctx, prec, direct_f64, Tbase, ops_of(W, prec), direct_ptr, md);
    }
    return plan;
}

// y = H_eff x at a site with left env L (channels W.wl, Da x Da) and right
// env R (channels W.wr, Db x Db).  Canonical gauge: L[I] = 1, R[F] = 1.
static void heff(Ctx* ctx, Prec prec, const MpoSite& W, int Da, int Db, const EnvView& L,
                 const EnvView& R, const double* x, double* y) {
    const int d = W.d;
    const int64_t n = (int64_t)Da * d * d * Db;
    const int wl = W.wl, wr = W.wr;
    ctx->ws_T.ensure(ctx, esz(prec) * 2 * (size_t)n * (wl + wr));
    void* T = ctx->ws_T.p;
    const int xs = W.idxI_l >= 0 ? W.idxI_l : 0;
    load_slot(ctx, prec, x, n, T, xs);
    std::vector<int> used(wl, 0);
    for (auto& e : W.ents) used[e.cl] = 1;
    std::vector<int> chans;
    for (int c = 0; c < wl; ++c)
        if (used[c] && c != W.idxI_l) chans.push_back(c);
    FTD_CHECK(W.idxI_l >= 0 || chans.empty() || true, FTD_EINVAL, "");
    stage_left(ctx, prec, L, chans, T, xs, Da, Da, d * d, Db, n, TAG_HEFF);
    std::vector<int> in_slot(wl);
    for (int c = 0; c < wl; ++c) in_slot[c] = c;
    // columns: F goes straight into y
    bool have_direct = false;
    for (auto& e : W.ents)
        if (e.cr == W.idxF_r) have_direct = true;
    MixPlan plan = stage_mix(ctx, prec, W, true, in_slot, wr, wl, {}, T, Da, d, Db, n,
                             W.idxF_r, y, true, false);
    // stage 3: y += sum_{cr != F} U[cr] R[cr]^T
    GemmParams p{};
    p.M = Da * d * d;
    p.N = Db;
    p.K = Db;
    p.sAm = Db; p.sAk = 1; p.planeA = n; p.a_kcontig = 1;
    p.sBk = 1; p.sBn = Db; p.planeB = (int64_t)Db * Db; p.b_kcontig = 1;
    p.sCm = Db; p.sCn = 1; p.planeC = n;
    p.nprob = 1;
    p.prob[0].offC = 0;
    p.prob[0].t0 = 0;
    int nt = 0;
    for (int c = 0; c < wr; ++c) {
        if (c == W.idxF_r || plan.out_slot[c] < 0) continue;
        FTD_CHECK(nt < kMaxTerms, FTD_EINVAL, "too many channels");
        p.term[nt].offA = (int64_t)plan.out_slot[c] * 2 * n;
        p.term[nt].offB = (int64_t)c * 2 * Db * Db;
        ++nt;
    }
    p.prob[0].t1 = nt;
    p.accumulate = have_direct ? 1 : 0;
    if (nt > 0)
        gemm(ctx, prec, true, T, R.p, y, p, TAG_HEFF);
    else if (!have_direct)
        k_zero(ctx, y, sizeof(double) * 2 * n);
    ctx->stats.matvecs++;
}

// y = K_eff C at the bond between two sites.  C is D1 x D2: the left index
// in the basis of the left environment L (channels of that bond, D1 x D1
// blocks), the right index in that of R (D2 x D2 blocks); they differ only
// right after a bond expansion.  L[I] and R[F] are materialised identities.
static void keff(Ctx* ctx, Prec prec, int w, int idxI, int D1, int D2, const EnvView& L,
                 const EnvView& R, const double* x, double* y) {
    const int64_t n = (int64_t)D1 * D2;
    ctx->ws_T.ensure(ctx, esz(prec) * 2 * (size_t)n * w);
    void* T = ctx->ws_T.p;
    const int xs = idxI >= 0 ? idxI : 0;
    load_slot(ctx, prec, x, n, T, xs);
    std::vector<int> chans;
    for (int c = 0; c < w; ++c)
        if (c != idxI) chans.push_back(c);
    stage_left(ctx, prec, L, chans, T, xs, D1, D1, 1, D2, n, TAG_KEFF);
    GemmParams p{};
    p.M = D1;
    p.N = D2;
    p.K = D2;
    p.sAm = D2; p.sAk = 1; p.planeA = n; p.a_kcontig = 1;
    p.sBk = 1; p.sBn = D2; p.planeB = (int64_t)D2 * D2; p.b_kcontig = 1;
    p.sCm = D2; p.sCn = 1; p.planeC = n;
    p.nprob = 1;
    p.prob[0].offC = 0;
    p.prob[0].t0 = 0;
    p.prob[0].t1 = w;
    for (int c = 0; c < w; ++c) {
        p.term[c].offA = (int64_t)c * 2 * n;
        p.term[c].offB = (int64_t)c * 2 * D2 * D2;
    }
    gemm(ctx, prec, true, T, R.p, y, p, TAG_KEFF);
    ctx->stats.matvecs++;
}

// Left environment of site i+1 from that of site i and the left-orthonormal
// A_i (bra = ket).  Output channels W.wr, Db x Db; channel I set to 1.
static void env_left_update(Ctx* ctx, Prec prec, const MpoSite& W, int Da, int Db,
                            const EnvView& L, const double* A, const EnvView& Lout) {
    const int d = W.d;
    const int64_t n = (int64_t)Da * d * d * Db;
    const int wl = W.wl, wr = W.wr;
    ctx->ws_T.ensure(ctx, esz(prec) * 2 * (size_t)n * (wl + wr));
    void* T = ctx->ws_T.p;
    const int xs = W.idxI_l >= 0 ? W.idxI_l : 0;
    load_slot(ctx, prec, A, n, T, xs);
    std::vector<int> used(wl, 0);
    for (auto& e : W.ents)
        if (e.cr != W.idxI_r) used[e.cl] = 1;
    std::vector<int> chans;
    for (int c = 0; c < wl; ++c)
        if (used[c] && c != W.idxI_l) chans.push_back(c);
    stage_left(ctx, prec, L, chans, T, xs, Da, Da, d * d, Db, n, TAG_NONE);
    std::vector<int> in_slot(wl);
    for (int c = 0; c < wl; ++c) in_slot[c] = c;
    std::vector<int> skip;
    if (W.idxI_r >= 0) skip.push_back(W.idxI_r);
    MixPlan plan = stage_mix(ctx, prec, W, true, in_slot, wr, wl, skip, T, Da, d, Db, n, -1,
                             nullptr, false, false);
    // Lout[cr] = A^H U[cr]
    const bool f32 = prec != Prec::F64;
    const int64_t bb = (int64_t)Db * Db;
    std::vector<int> outs;
    for (int c = 0; c < wr; ++c)
        if (c != W.idxI_r) outs.push_back(c);
    for (size_t o0 = 0; o0 < outs.size(); o0 += kMaxProbs) {
        GemmParams p{};
        p.M = Db;
        p.N = Db;
        p.K = Da * d * d;
        p.sAm = 1; p.sAk = Db; p.planeA = n; p.conjA = 1; p.a_kcontig = 0;
        p.sBk = Db; p.sBn = 1; p.planeB = n; p.b_kcontig = 0;
        p.sCm = Db; p.sCn = 1; p.planeC = bb;
        const size_t o1 = std::min(outs.size(), o0 + kMaxProbs);
        int np = 0;
        std::vector<int> zero_out;
        for (size_t k = o0; k < o1; ++k) {
            const int c = outs[k];
            if (plan.out_slot[c] < 0) {
                zero_out.push_back(c);
                continue;
            }
            p.prob[np].offC = (int64_t)c * 2 * bb;
            p.prob[np].t0 = np;
            p.prob[np].t1 = np + 1;
            p.term[np].offA = (int64_t)xs * 2 * n;
            p.term[np].offB = (int64_t)plan.out_slot[c] * 2 * n;
            ++np;
        }
        p.nprob = np;
        if (np) gemm(ctx, prec, !f32, T, T, Lout.p, p, TAG_NONE);
        for (int c : zero_out)
            k_zero(ctx, static_cast<char*>(Lout.p) + (size_t)c * 2 * bb * esz(prec), esz(prec) * 2 * bb);
    }
    if (W.idxI_r >= 0)
        eye(ctx, static_cast<char*>(Lout.p) + (size_t)W.idxI_r * 2 * bb * esz(prec), Db, bb, f32);
}

// Right environment of site i (contraction of sites i..) from that of site
// i+1 and the right-orthonormal A_i.  Output channels W.wl, Da x Da; F = 1.
static void env_right_update(Ctx* ctx, Prec prec, const MpoSite& W, int Da, int Db,
                             const EnvView& R, const double* A, const EnvView& Rout) {
    const int d = W.d;
    const int64_t n = (int64_t)Da * d * d * Db;
    const int wl = W.wl, wr = W.wr;
    ctx->ws_T.ensure(ctx, esz(prec) * 2 * (size_t)n * (wl + wr));
    void* T = ctx->ws_T.p;
    const int as = W.idxF_r >= 0 ? W.idxF_r : 0;
    load_slot(ctx, prec, A, n, T, as);
    // T'[cr] = A R[cr]^T, cr != F
    std::vector<int> used(wr, 0);
    for (auto& e : W.ents)
        if (e.cl != W.idxF_l) used[e.cr] = 1;
    std::vector<int> chans;
    for (int c = 0; c < wr; ++c)
        if (used[c] && c != W.idxF_r) chans.push_back(c);
    for (size_t c0 = 0; c0 < chans.size(); c0 += kMaxProbs) {
        GemmParams p{};
        p.M = Da * d * d;
        p.N = Db;
        p.K = Db;
        p.sAm = Db; p.sAk = 1; p.planeA = n; p.a_kcontig = 1;
        p.sBk = 1; p.sBn = Db; p.planeB = (int64_t)Db * Db; p.b_kcontig = 1;
        p.sCm = Db; p.sCn = 1; p.planeC = n;
        const size_t c1 = std::min(chans.size(), c0 + kMaxProbs);
        p.nprob = (int)(c1 - c0);
        for (size_t k = c0; k < c1; ++k) {
            const int c = chans[k];
            const int j = (int)(k - c0);
            p.prob[j].offC = (int64_t)c * 2 * n;
            p.prob[j].t0 = j;
            p.prob[j].t1 = j + 1;
            p.term[j].offA = (int64_t)as * 2 * n;
            p.term[j].offB = (int64_t)c * 2 * Db * Db;
        }
        gemm(ctx, prec, prec == Prec::F64, T, R.p, T, p, TAG_NONE);
    }
    std::vector<int> in_slot(wr);
    for (int c = 0; c < wr; ++c) in_slot[c] = c;
    std::vector<int> skip;
    if (W.idxF_l >= 0) skip.push_back(W.idxF_l);
    MixPlan plan = stage_mix(ctx, prec, W, false, in_slot, wl, wr, skip, T, Da, d, Db, n, -1,
                             nullptr, false, false);
    const bool f32 = prec != Prec::F64;
    const int64_t aa = (int64_t)Da * Da;
    const int64_t K = (int64_t)d * d * Db;
    std::vector<int> outs;
    for (int c = 0; c < wl; ++c)
        if (c != W.idxF_l) outs.push_back(c);
    for (size_t o0 = 0; o0 < outs.size(); o0 += kMaxProbs) {
        GemmParams p{};
        p.M = Da;
        p.N = Da;
        p.K = (int)K;
        p.sAm = K; p.sAk = 1; p.planeA = n; p.conjA = 1; p.a_kcontig = 1;
        p.sBk = 1; p.sBn = K; p.planeB = n; p.b_kcontig = 1;
        p.sCm = Da; p.sCn = 1; p.planeC = aa;
        const size_t o1 = std::min(outs.size(), o0 + kMaxProbs);
        int np = 0;
        std::vector<int> zero_out;
        for (size_t k = o0; k < o1; ++k) {
            const int c = outs[k];
            if (plan.out_slot[c] < 0) {
                zero_out.push_back(c);
                continue;
            }
            p.prob[np].offC = (int64_t)c * 2 * aa;
            p.prob[np].t0 = np;
            p.prob[np].t1 = np + 1;
            p.term[np].offA = (int64_t)as * 2 * n;
            p.term[np].offB = (int64_t)plan.out_slot[c] * 2 * n;
            ++np;
        }
        p.nprob = np;
        if (np) gemm(ctx, prec, !f32, T, T, Rout.p, p, TAG_NONE);
        for (int c : zero_out)
            k_zero(ctx, static_cast<char*>(Rout.p) + (size_t)c * 2 * aa * esz(prec), esz(prec) * 2 * aa);
    }
    if (W.idxF_l >= 0)
        eye(ctx, static_cast<char*>(Rout.p) + (size_t)W.idxF_l * 2 * aa * esz(prec), Da, aa, f32);
}

// ================================================================ Krylov
// x <- exp(z H) x for the Hermitian operator `op`, by Lanczos with full
// reorthogonalisation in float64 (classical Gram-Schmidt applied twice) and
// the device tridiagonal exponential.  Iterations are enqueued without
// waiting; every kernel of an iteration returns at once after the device has
// raised the halt flag, so the host reads the flags only from the expected
// vector count on (hint: the count of the previous call at the same site or
// bond); the vector count itself does not depend on the hint.  Timing
// events and matvec counts of iterations that ran as no-ops are discarded.
// In the reduced precisions the normalisation of each new vector also writes
// the float copy the next matvec reads.
static int expm_krylov(Ctx* ctx, const std::function<void(const double*, double*)>& op, double* x,
                       int64_t n, cplx z, double tol, int mmax, int& last) {
    FTD_CHECK(mmax >= 1 && mmax < kMaxKrylov, FTD_EINVAL, "Krylov mmax out of range");
    const int64_t vs = 2 * n;
    ctx->ws_Krylov.ensure(ctx, sizeof(double) * (size_t)vs * (mmax + 1));
    double* V = ctx->ws_Krylov.as<double>();
    KrylovDev kd = ctx->kd;
    k_krylov_reset(ctx, kd);
    k_nrm2(ctx, x, n, n, kd.nrm + 1);
    k_copy_f64(ctx, x, V, vs);
    k_scale_by_dev(ctx, V, n, n, kd.nrm + 1, 0);
    const int kmax = (int)std::min<int64_t>(mmax, n);
    const int hint = std::max(1, last - 1);
    std::vector<size_t> ev_mark(kmax + 1);
    std::vector<int64_t> mv_mark(kmax + 1);
    std::vector<double> fl_mark(kmax + 1);
    ctx->kstop = kd.flag + 3;
    // 100 u / tol (u = 2^-53): a tolerance of about 1e-14 or tighter keeps
    // both Gram-Schmidt passes always
    const double cgs_thr = tol > 0.0 ? 100.0 * 0.5 * DBL_EPSILON / tol : 1.0;
    int done = 0;
    try {
        for (int k = 0; k < kmax; ++k) {
            ev_mark[k] = ctx->events.size();
            mv_mark[k] = ctx->stats.matvecs;
            fl_mark[k] = ctx->stats.all_flops;
            double* vk = V + (int64_t)k * vs;
            double* w = V + (int64_t)(k + 1) * vs;
            ctx->last32_x = nullptr;
            op(vk, w);
            // classical Gram-Schmidt twice; alpha_k = <v_k, w> of the first pass.
            // The second correction is skipped on the device when the first
            // pass kept more than thr of |w| (then its orthogonality error,
            // about u |w| / |w'|, is below tol / 100).
            k_multidot(ctx, V, vs, k + 1, w, n, n, kd.h, kd.alpha + k);
            const double* skip = nullptr;
            if (k_multiaxpy_dot(ctx, V, vs, k + 1, kd.h, w, n, n)) {
                if (cgs_thr < 0.5) skip = kd.h + 2 * (k + 1);
            } else {
                k_multiaxpy(ctx, V, vs, k + 1, kd.h, w, n, n);
                k_multidot(ctx, V, vs, k + 1, w, n, n, kd.h);
            }
            const double thr2 = cgs_thr * cgs_thr;
            const int nb = k_multiaxpy_nrm2_part(ctx, V, vs, k + 1, kd.h, w, n, n, skip, thr2);
            const int exhausted = (k + 1 == n) ? 1 : 0;
            k_tridiag_expm(ctx, kd, k + 1, z.real(), z.imag(), tol, exhausted,
                           ctx->ws_red.as<double>(), nb, skip, thr2);
            // the normalised w is the next matvec's input: when the matvec just
            // loaded its input as a float copy, the normalisation writes the
            // next one in the same place
            float* w32 = nullptr;
            if (ctx->last32_x == vk && ctx->last32_n == n && ctx->last32_gen == ctx->ws_gen &&
                k + 1 < kmax)
                w32 = static_cast<float*>(ctx->last32_dst);
            k_lanczos_post(ctx, kd, k + 1, w, n, n, w32);
            if (w32) {
                ctx->pre32_x = w;
                ctx->pre32_dst = w32;
                ctx->pre32_gen = ctx->ws_gen;
            }
            if (k + 1 < hint && k + 1 < kmax) continue;
            FTD_HIP(hipMemcpyAsync(ctx->h_pinned_i, kd.flag, 4 * sizeof(int),
                                   hipMemcpyDeviceToHost, ctx->stream));
            FTD_HIP(hipStreamSynchronize(ctx->stream));
            if (ctx->h_pinned_i[3]) {
                done = k + 1;
                break;
            }
        }
    } catch (...) {
        ctx->kstop = nullptr;
        ctx->pre32_x = ctx->last32_x = nullptr;
        throw;
    }
    ctx->kstop = nullptr;
    ctx->pre32_x = ctx->last32_x = nullptr;
    if (!done) throw Error{FTD_ENOCONV, "Krylov exponential did not converge within mmax vectors"};
    const int conv = ctx->h_pinned_i[0], failed = ctx->h_pinned_i[2], m = ctx->h_pinned_i[1];
    FTD_CHECK(!failed || conv, FTD_ENOCONV,
              m >= kmax ? "Krylov exponential did not converge within mmax vectors"
                        : "Krylov exponential: non-finite values");
    FTD_CHECK(m >= 1 && m <= done, FTD_EDEVICE, "Krylov exponential: inconsistent vector count");
    // iterations m .. done-1 were enqueued after the halt and did nothing
    if (m < done) {
        ctx->events.resize(ev_mark[m]);
        ctx->stats.matvecs = mv_mark[m];
        ctx->stats.all_flops = fl_mark[m];
    }
    k_lincomb(ctx, V, vs, m, kd.u, kd.nrm + 1, x, n, n);
    last = m;
    ctx->stats.krylov_vectors += m;
    ctx->stats.expm_calls += 1;
    ctx->stats.krylov_max = std::max<int64_t>(ctx->stats.krylov_max, m);
    return m;
}

// ============================================================= gauge moves
static void ensure_env_arrays(Ctx* ctx, int L) {
    if ((int)ctx->envL.size() < L + 1) {
        ctx->envL.resize(L + 1);
        ctx->envL_w.resize(L + 1);
        ctx->envL_D.resize(L + 1);
    }
    if ((int)ctx->envR.size() < L + 1) {
        ctx->envR.resize(L + 1);
        ctx->envR_w.resize(L + 1);
        ctx->envR_D.resize(L + 1);
    }
}
static EnvView envL_view(Ctx* ctx, int i, Prec prec) {
    return {ctx->envL[i].p, ctx->envL_w[i], ctx->envL_D[i], ctx->envL_D[i]};
}
static EnvView envR_view(Ctx* ctx, int i, Prec prec) {
    return {ctx->envR[i].p, ctx->envR_w[i], ctx->envR_D[i], ctx->envR_D[i]};
}

static void build_right_envs(Ctx* ctx, const Mpo* H, const Mps* psi, int from) {
    const int L = psi->L;
    const Prec prec = psi->prec;
    ensure_env_arrays(ctx, L);
    EnvView b = env_get(ctx, ctx->envR, ctx->envR_w, ctx->envR_D, L, 1, 1, prec);
    boundary_env(ctx, b, prec);
    for (int i = L - 1; i >= from; --i) {
        const MpoSite& W = H->s[i];
        EnvView R = envR_view(ctx, i + 1, prec);
        EnvView out = env_get(ctx, ctx->envR, ctx->envR_w, ctx->envR_D, i, W.wl, psi->Dl[i], prec);
        env_right_update(ctx, prec, W, psi->Dl[i], psi->Dr[i], R, psi->A[i], out);
    }
}
static void build_left_envs(Ctx* ctx, const Mpo* H, const Mps* psi, int upto) {
    const int L = psi->L;
    const Prec prec = psi->prec;
    ensure_env_arrays(ctx, L);
    EnvView b = env_get(ctx, ctx->envL, ctx->envL_w, ctx->envL_D, 0, 1, 1, prec);
    boundary_env(ctx, b, prec);
    for (int i = 0; i < upto; ++i) {
        const MpoSite& W = H->s[i];
        EnvView Lv = envL_view(ctx, i, prec);
        EnvView out = env_get(ctx, ctx->envL, ctx->envL_w, ctx->envL_D, i + 1, W.wr, psi->Dr[i], prec);
        env_left_update(ctx, prec, W, psi->Dl[i], psi->Dr[i], Lv, psi->A[i], out);
    }
}

// new A_{i+1} = C A_{i+1}, C: D1 x D2 with D2 the old left bond of A_{i+1};
// the new left bond is D1 (wider after an expansion of bond i).
static void absorb_right(Ctx* ctx, Mps* psi, int i, const double* C, int D1) {
    const int D2 = psi->Dl[i + 1];
    const int64_t nn = psi->size(i + 1);
    const int64_t cols = nn / D2;
    const int64_t nout = (int64_t)D1 * cols;
    double* out;
    if (D1 == D2) {
        ctx->ws_site.ensure(ctx, sizeof(double) * 2 * nn);
        out = ctx->ws_site.as<double>();
    } else {
        out = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * nout));
    }
    GemmParams p{};
    p.M = D1; p.N = (int)cols; p.K = D2;
    p.sAm = D2; p.sAk = 1; p.planeA = (int64_t)D1 * D2; p.a_kcontig = 1;
    p.sBk = cols; p.sBn = 1; p.planeB = nn; p.b_kcontig = 0;
    p.sCm = cols; p.sCn = 1; p.planeC = nout;
    p.nprob = 1; p.prob[0].t1 = 1;
    gemm(ctx, Prec::F64, true, C, psi->A[i + 1], out, p, TAG_NONE);
    if (D1 == D2)
        k_copy_f64(ctx, out, psi->A[i + 1], 2 * nn);
    else
        set_site(ctx, psi, i + 1, D1, psi->Dr[i + 1], out);
}
// new A_{i-1} = A_{i-1} C, C: D1 x D2 with D1 the old right bond of A_{i-1};
// the new right bond is D2 (wider after an expansion of bond i-1).
static void absorb_left(Ctx* ctx, Mps* psi, int i, const double* C, int D2) {
    const int D1 = psi->Dr[i - 1];
    const int64_t nn = psi->size(i - 1);
    const int64_t rows = nn / D1;
    const int64_t nout = rows * D2;
    double* out;
    if (D1 == D2) {
        ctx->ws_site.ensure(ctx, sizeof(double) * 2 * nn);
        out = ctx->ws_site.as<double>();
    } else {
        out = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * nout));
    }
    GemmParams p{};
    p.M = (int)rows; p.N = D2; p.K = D1;
    p.sAm = D1; p.sAk = 1; p.planeA = nn; p.a_kcontig = 1;
    p.sBk = D2; p.sBn = 1; p.planeB = (int64_t)D1 * D2; p.b_kcontig = 0;
    p.sCm = D2; p.sCn = 1; p.planeC = nout;
    p.nprob = 1; p.prob[0].t1 = 1;
    gemm(ctx, Prec::F64, true, psi->A[i - 1], C, out, p, TAG_NONE);
    if (D1 == D2)
        k_copy_f64(ctx, out, psi->A[i - 1], 2 * nn);
    else
        set_site(ctx, psi, i - 1, psi->Dl[i - 1], D2, out);
}

// ---------------------------------------------------------- bond expansion
// Y minus its projection on the orthonormal columns (left) or rows (right)
// of Q, applied twice; Y is m x r (left) or r x m (right), Q likewise.
static void project_out(Ctx* ctx, double* Y, const double* Q, int64_t m, int r, bool rows) {
    const int64_t ny = m * r;
    ctx->ws_expC.ensure(ctx, sizeof(double) * 2 * (size_t)r * r);
    double* G = ctx->ws_expC.as<double>();
    for (int pass = 0; pass < 2; ++pass) {
        GemmParams p{};
        p.nprob = 1; p.prob[0].t1 = 1;
        if (!rows) {   // G = Q^H Y (r x r)
            p.M = r; p.N = r; p.K = (int)m;
            p.sAm = 1; p.sAk = r; p.planeA = ny; p.conjA = 1; p.a_kcontig = 0;
            p.sBk = r; p.sBn = 1; p.planeB = ny; p.b_kcontig = 0;
            p.sCm = r; p.sCn = 1; p.planeC = (int64_t)r * r;
            gemm(ctx, Prec::F64, true, Q, Y, G, p, TAG_NONE);
        } else {       // G = Y Q^H (r x r)
            p.M = r; p.N = r; p.K = (int)m;
            p.sAm = m; p.sAk = 1; p.planeA = ny; p.a_kcontig = 1;
            p.sBk = 1; p.sBn = m; p.planeB = ny; p.conjB = 1; p.b_kcontig = 1;
            p.sCm = r; p.sCn = 1; p.planeC = (int64_t)r * r;
            gemm(ctx, Prec::F64, true, Y, Q, G, p, TAG_NONE);
        }
        k_scale_cplx(ctx, G, (int64_t)r * r, (int64_t)r * r, -1.0, 0.0);
        GemmParams q{};
        q.nprob = 1; q.prob[0].t1 = 1;
        q.accumulate = 1;
        if (!rows) {   // Y -= Q G
            q.M = (int)m; q.N = r; q.K = r;
            q.sAm = r; q.sAk = 1; q.planeA = ny; q.a_kcontig = 1;
            q.sBk = r; q.sBn = 1; q.planeB = (int64_t)r * r; q.b_kcontig = 0;
            q.sCm = r; q.sCn = 1; q.planeC = ny;
            gemm(ctx, Prec::F64, true, Q, G, Y, q, TAG_NONE);
        } else {       // Y -= G Q
            q.M = r; q.N = (int)m; q.K = r;
            q.sAm = r; q.sAk = 1; q.planeA = (int64_t)r * r; q.a_kcontig = 1;
            q.sBk = m; q.sBn = 1; q.planeB = ny; q.b_kcontig = 0;
            q.sCm = m; q.sCn = 1; q.planeC = ny;
            gemm(ctx, Prec::F64, true, G, Q, Y, q, TAG_NONE);
        }
    }
}

// Bond expansion, first half: Y = H_eff A of the evolved centre A (into
// ws_expY, float64) and |Y|_F, before the gauge factorisation overwrites A.
static double expansion_residual(Ctx* ctx, Prec prec, const MpoSite& W, int Da, int Db,
                                 const EnvView& L, const EnvView& R, const double* A) {
    const int64_t n = (int64_t)Da * W.d * W.d * Db;
    ctx->ws_expY.ensure(ctx, sizeof(double) * 2 * (size_t)n);
    double* Y = ctx->ws_expY.as<double>();
    heff(ctx, prec, W, Da, Db, L, R, A, Y);
    ctx->stats.matvecs--;   // not a Krylov matvec
    k_nrm2(ctx, Y, n, n, ctx->scal + 8);
    return std::sqrt(read_scalar(ctx, ctx->scal + 8));
}

// Second half: the leading directions of Y outside the span of the
// orthonormal factor Q (columns of the m x r factor for a left-to-right step,
// rows of the r x m factor for right-to-left), at most cap, singular values of
// the projected Y above tol |Y|_F.  Returns their count and sets *dirs to a
// new buffer (m x k orthonormal columns, or k x m orthonormal rows), or
// nullptr when there are none.
static int expansion_dirs(Ctx* ctx, double ynorm, const double* Q, int64_t m, int r, bool rows,
                          int cap, double tol, double** dirs) {
    *dirs = nullptr;
    if (!(ynorm > 0.0) || !std::isfinite(ynorm)) return 0;
    double* Y = ctx->ws_expY.as<double>();
    project_out(ctx, Y, Q, m, r, rows);
    TruncOut t = rows ? svd_trunc(ctx, Y, r, m, cap, 0.0, true, tol * ynorm)
                      : svd_trunc(ctx, Y, m, r, cap, 0.0, false, tol * ynorm);
    if (t.k == 0) return 0;
    if (rows) {
        dev_free(ctx, t.Lq);
        *dirs = t.Rq;
    } else {
        dev_free(ctx, t.Rq);
        *dirs = t.Lq;
    }
    return t.k;
}

// ============================================================ TDVP sweep
static void tdvp_sweeps(Ctx* ctx, const Mpo* H, Mps* psi, cplx z, double tol, int mmax, int xD,
                        double xtol);

void tdvp_step(Ctx* ctx, const Mpo* H, Mps* psi, cplx z, double tol, int mmax, int expand_D,
               double expand_tol) {
    try {
        tdvp_sweeps(ctx, H, psi, z, tol, mmax, expand_D, expand_tol);
    } catch (...) {
        // a failed sweep may leave the sticky breakdown flag set by gauge
        // moves it had already queued: clear it for the next call
        try {
            chol_flag_clear(ctx);
        } catch (...) {
        }
        throw;
    }
}

// The sweep pair of one step.  With xD > 0 every gauge move is followed by
// a bond expansion while the bond it opens is below min(xD, what the two
// neighbouring sites can carry): the orthonormal factor gets the leading
// directions of H_eff A outside its span (threshold xtol |H_eff A|), the bond
// matrix zero rows (left to right) or columns (right to left) for them, so
// the state is unchanged; the bond's backward step and the next site's step
// then run in the enlarged basis.
static void tdvp_sweeps(Ctx* ctx, const Mpo* H, Mps* psi, cplx z, double tol, int mmax, int xD,
                        double xtol) {
    const int L = psi->L;
    FTD_CHECK(H->L == L, FTD_EINVAL, "MPO and MPS lengths differ");
    const Prec prec = psi->prec;
    build_right_envs(ctx, H, psi, 1);
    EnvView b = env_get(ctx, ctx->envL, ctx->envL_w, ctx->envL_D, 0, 1, 1, prec);
    boundary_env(ctx, b, prec);
    const cplx h = 0.5 * z;
    ctx->ws_tmp1.ensure(ctx, sizeof(double) * 2 * 1024 * 1024);
    if ((int)ctx->khint_site.size() != L) ctx->khint_site.assign(L, 4);
    if ((int)ctx->khint_bond.size() != L) ctx->khint_bond.assign(L, 4);
    auto site_evolve = [&](int i) {
        const MpoSite& W = H->s[i];
        EnvView Lv = envL_view(ctx, i, prec), Rv = envR_view(ctx, i + 1, prec);
        const int Da = psi->Dl[i], Db = psi->Dr[i];
        auto op = [&](const double* x, double* y) { heff(ctx, prec, W, Da, Db, Lv, Rv, x, y); };
        expm_krylov(ctx, op, psi->A[i], psi->size(i), h, tol, mmax, ctx->khint_site[i]);
    };
    // bond between sites i and i+1 (envL[i+1], envR[i+1]); C is D1 x D2
    auto bond_evolve = [&](int i, double* C, int D1, int D2) {
        const MpoSite& W = H->s[i];
        EnvView Lv = envL_view(ctx, i + 1, prec), Rv = envR_view(ctx, i + 1, prec);
        auto op = [&](const double* x, double* y) {
            keff(ctx, prec, W.wr, W.idxI_r, D1, D2, Lv, Rv, x, y);
        };
        expm_krylov(ctx, op, C, (int64_t)D1 * D2, -h, tol, mmax, ctx->khint_bond[i]);
    };
    double* Cx = nullptr;   // the widened bond matrix of an expansion
    try {
        for (int i = 0; i < L - 1; ++i) {
            site_evolve(i);
            const int Da = psi->Dl[i], Db = psi->Dr[i], d = psi->d[i];
            const int64_t m = (int64_t)Da * d * d;
            int cap = 0;
            double ynorm = 0.0;
            if (xD > 0) {
                const int64_t right = (int64_t)psi->d[i + 1] * psi->d[i + 1] * psi->Dr[i + 1];
                cap = (int)std::min<int64_t>(std::min<int64_t>(xD, m), right) - Db;
                if (cap > 0)
                    ynorm = expansion_residual(ctx, prec, H->s[i], Da, Db, envL_view(ctx, i, prec),
                                               envR_view(ctx, i + 1, prec), psi->A[i]);
            }
            ctx->ws_tmp1.ensure(ctx, sizeof(double) * 2 * (size_t)Db * Db);
            double* C = ctx->ws_tmp1.as<double>();
            qr_chol(ctx, psi->A[i], m, Db, C, false);
            double* dirs = nullptr;
            const int k = cap > 0 ? expansion_dirs(ctx, ynorm, psi->A[i], m, Db, false, cap, xtol,
                                                   &dirs)
                                  : 0;
            int Dn = Db;
            if (k > 0) {
                Dn = Db + k;
                double* An = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * Dn));
                k_embed(ctx, psi->A[i], Da, d * d, Db, An, Da, Dn, 0, 0, 1.0, 0.0);
                k_embed(ctx, dirs, Da, d * d, k, An, Da, Dn, 0, Db, 1.0, 0.0);
                Cx = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * (size_t)Dn * Db));
                k_zero(ctx, Cx, sizeof(double) * 2 * (size_t)Dn * Db);
                k_embed(ctx, C, Db, 1, Db, Cx, Dn, Db, 0, 0, 1.0, 0.0);
                set_site(ctx, psi, i, Da, Dn, An);
                dev_free(ctx, dirs);
                C = Cx;
            }
            EnvView Lv = envL_view(ctx, i, prec);
            EnvView out = env_get(ctx, ctx->envL, ctx->envL_w, ctx->envL_D, i + 1, H->s[i].wr, Dn,
                                  prec);
            env_left_update(ctx, prec, H->s[i], Da, Dn, Lv, psi->A[i], out);
            bond_evolve(i, C, Dn, Db);
            absorb_right(ctx, psi, i, C, Dn);
            if (Cx) {
                FTD_HIP(hipStreamSynchronize(ctx->stream));
                dev_free(ctx, Cx);
                Cx = nullptr;
            }
        }
        site_evolve(L - 1);
        site_evolve(L - 1);
        for (int i = L - 1; i >= 1; --i) {
            const int Da = psi->Dl[i], Db = psi->Dr[i], d = psi->d[i];
            const int64_t m = (int64_t)d * d * Db;
            int cap = 0;
            double ynorm = 0.0;
            if (xD > 0) {
                const int64_t left = (int64_t)psi->Dl[i - 1] * psi->d[i - 1] * psi->d[i - 1];
                cap = (int)std::min<int64_t>(std::min<int64_t>(xD, m), left) - Da;
                if (cap > 0)
                    ynorm = expansion_residual(ctx, prec, H->s[i], Da, Db, envL_view(ctx, i, prec),
                                               envR_view(ctx, i + 1, prec), psi->A[i]);
            }
            ctx->ws_tmp1.ensure(ctx, sizeof(double) * 2 * (size_t)Da * Da);
            double* C = ctx->ws_tmp1.as<double>();
            lq_chol(ctx, psi->A[i], Da, m, C, false);
            double* dirs = nullptr;
            const int k = cap > 0 ? expansion_dirs(ctx, ynorm, psi->A[i], m, Da, true, cap, xtol,
                                                   &dirs)
                                  : 0;
            int Dn = Da;
            if (k > 0) {
                Dn = Da + k;
                double* An = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * Dn));
                k_embed(ctx, psi->A[i], Da, d * d, Db, An, Dn, Db, 0, 0, 1.0, 0.0);
                k_embed(ctx, dirs, k, d * d, Db, An, Dn, Db, Da, 0, 1.0, 0.0);
                Cx = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * (size_t)Da * Dn));
                k_zero(ctx, Cx, sizeof(double) * 2 * (size_t)Da * Dn);
                k_embed(ctx, C, Da, 1, Da, Cx, Da, Dn, 0, 0, 1.0, 0.0);
                set_site(ctx, psi, i, Dn, Db, An);
                dev_free(ctx, dirs);
                C = Cx;
            }
            EnvView Rv = envR_view(ctx, i + 1, prec);
            EnvView out = env_get(ctx, ctx->envR, ctx->envR_w, ctx->envR_D, i, H->s[i].wl, Dn, prec);
            env_right_update(ctx, prec, H->s[i], Dn, Db, Rv, psi->A[i], out);
            bond_evolve(i - 1, C, Da, Dn);
            absorb_left(ctx, psi, i, C, Dn);
            if (Cx) {
                FTD_HIP(hipStreamSynchronize(ctx->stream));
                dev_free(ctx, Cx);
                Cx = nullptr;
            }
            site_evolve(i - 1);
        }
    } catch (...) {
        (void)hipStreamSynchronize(ctx->stream);
        dev_free(ctx, Cx);
        throw;
    }
    // gauge moves were enqueued without waiting: report a breakdown now
    chol_flag_check(ctx);
}

void tdvp_pair(Ctx* ca, Ctx* cb, hipEvent_t fork, hipEvent_t join, const Mpo* H, Mps* a, Mps* b,
               cplx z, double tol, int mmax) {
    FTD_HIP(hipEventRecord(fork, ca->stream));
    FTD_HIP(hipStreamWaitEvent(cb->stream, fork, 0));
    std::exception_ptr err_b;
    std::thread worker([&] {
        try {
            FTD_HIP(hipSetDevice(cb->device));
            tdvp_step(cb, H, b, z, tol, mmax);
        } catch (...) {
            err_b = std::current_exception();
        }
    });
    std::exception_ptr err_a;
    try {
        tdvp_step(ca, H, a, z, tol, mmax);
    } catch (...) {
        err_a = std::current_exception();
    }
    worker.join();
    FTD_HIP(hipEventRecord(join, cb->stream));
    FTD_HIP(hipStreamWaitEvent(ca->stream, join, 0));
    if (err_a) std::rethrow_exception(err_a);
    if (err_b) std::rethrow_exception(err_b);
}

// ============================================================ MPS algebra
Mps* mpo_apply(Ctx* ctx, const Mpo* O, const Mps* psi) {
    const int L = psi->L;
    std::vector<int> Dl(L), Dr(L);
    for (int i = 0; i < L; ++i) {
        Dl[i] = psi->Dl[i] * O->s[i].wl;
        Dr[i] = psi->Dr[i] * O->s[i].wr;
    }
    Mps* out = mps_alloc(ctx, Dl, psi->d, Dr, psi->prec);
    for (int i = 0; i < L; ++i) {
        const MpoSite& W = O->s[i];
        k_mpo_apply(ctx, psi->A[i], psi->Dl[i], W.d, psi->Dr[i], W.ops64, 2 * (int64_t)W.d * W.d,
                    W.wl, W.wr, W.apply_ents, (int)W.ents.size(), out->A[i]);
    }
    out->log_norm = psi->log_norm;
    return out;
}

Mps* mps_add(Ctx* ctx, const Mps* a, const Mps* b, cplx c) {
    const int L = a->L;
    FTD_CHECK(b->L == L, FTD_EINVAL, "mps_add: lengths differ");
    std::vector<int> Dl(L), Dr(L);
    for (int i = 0; i < L; ++i) {
        Dl[i] = (i == 0) ? 1 : a->Dl[i] + b->Dl[i];
        Dr[i] = (i == L - 1) ? 1 : a->Dr[i] + b->Dr[i];
    }
    Mps* out = mps_alloc(ctx, Dl, a->d, Dr, a->prec);
    for (int i = 0; i < L; ++i) {
        const int dd = a->d[i] * a->d[i];
        k_zero(ctx, out->A[i], sizeof(double) * 2 * out->size(i));
        k_embed(ctx, a->A[i], a->Dl[i], dd, a->Dr[i], out->A[i], Dl[i], Dr[i], 0, 0, 1.0, 0.0);
        const int a0 = (i == 0) ? 0 : a->Dl[i];
        const int b0 = (i == L - 1) ? 0 : a->Dr[i];
        const cplx s = (i == 0) ? c : cplx(1.0, 0.0);
        k_embed(ctx, b->A[i], b->Dl[i], dd, b->Dr[i], out->A[i], Dl[i], Dr[i], a0, b0, s.real(), s.imag());
    }
    out->log_norm = a->log_norm;
    return out;
}

static int truncation_rank(const std::vector<double>& s, int D, double cutoff) {
    if (s.empty() || s[0] == 0.0) return 1;
    int k = 0;
    for (double x : s)
        if (x > cutoff * s[0]) ++k;
    k = std::max(1, std::min(k, D));
    while (k > 1 && k < (int)s.size() && (s[k - 1] - s[k]) <= 1e-8 * s[k - 1]) --k;
    return k;
}

// Truncated SVD of T (m x n, row-major, split planes m*n):
//   T ~ Lq diag(S) Rq,  Lq m x k (orthonormal columns), Rq k x n (orthonormal
//   rows), k from truncation_rank.  S is multiplied into Lq (s_left) or Rq.
// Tall blocks (m >= 2n) are reduced by Householder QR first and one-sided
// Jacobi runs on the adjoint of the triangular factor; otherwise on T (m >= n)
// or T^H (m < n).  Returns newly allocated buffers.
// Expansion rule: the singular values above `floor` (sorted descending), at
// most cap of them, possibly none, multiplets kept whole.
static int expansion_rank(const std::vector<double>& s, int cap, double floor) {
    if (cap <= 0 || s.empty()) return 0;
    int k = 0;
    for (double x : s)
        if (x > floor) ++k;
    k = std::min(k, cap);
    while (k > 0 && k < (int)s.size() && (s[k - 1] - s[k]) <= 1e-8 * s[k - 1]) --k;
    return k;
}

TruncOut svd_trunc(Ctx* ctx, const double* T, int64_t m, int64_t n, int D, double cutoff,
                   bool s_left, double abs_floor) {
    const int64_t ns = std::min(m, n);
    const int64_t big = std::max(m, n);
    ctx->ws_svd1.ensure(ctx, sizeof(double) * 2 * (size_t)(big * ns + ns * ns + ns));
    double* Ub = ctx->ws_svd1.as<double>();
    double* Vb = Ub + 2 * big * ns;
    double* Sd = Vb + 2 * ns * ns;
    std::vector<double> S(ns);
    std::vector<int> perm(ns);
    int k = 0;
    auto finish = [&]() {
        FTD_HIP(hipMemcpyAsync(S.data(), Sd, sizeof(double) * ns, hipMemcpyDeviceToHost, ctx->stream));
        FTD_HIP(hipStreamSynchronize(ctx->stream));
        std::iota(perm.begin(), perm.end(), 0);
        std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return S[x] > S[y]; });
        std::vector<double> ss(ns);
        for (int j = 0; j < ns; ++j) ss[j] = S[perm[j]];
        k = abs_floor >= 0.0 ? expansion_rank(ss, D, abs_floor) : truncation_rank(ss, D, cutoff);
    };
    ctx->ws_perm.ensure(ctx, 64 + (sizeof(int) + 3 * sizeof(double)) * (size_t)ns);
    int* dperm = ctx->ws_perm.as<int>();
    double* dS = reinterpret_cast<double*>(static_cast<char*>(ctx->ws_perm.p) +
                                           ((sizeof(int) * ns + 63) / 64) * 64);
    double* dInv = dS + ns;
    auto upload = [&]() {
        std::vector<double> sv(k), iv(k);
        for (int j = 0; j < k; ++j) {
            sv[j] = S[perm[j]];
            iv[j] = sv[j] > 0.0 ? 1.0 / sv[j] : 0.0;
        }
        FTD_HIP(hipMemcpyAsync(dperm, perm.data(), sizeof(int) * k, hipMemcpyHostToDevice, ctx->stream));
        FTD_HIP(hipMemcpyAsync(dS, sv.data(), sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
        FTD_HIP(hipMemcpyAsync(dInv, iv.data(), sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
        FTD_HIP(hipStreamSynchronize(ctx->stream));
    };
    auto gather = [&](const double* src, int64_t rows, int64_t splane, const double* sc, int conj,
                      double* dst) {
        gather_cols_kernel<<<gr(rows * k), 256, 0, ctx->stream>>>(src, rows, splane, dperm, sc, k, conj,
                                                                  dst, rows * k);
        FTD_HIP(hipGetLastError());
    };
    TruncOut o{0, nullptr, nullptr};
    if (m >= n) {
        if (m >= 2 * n && n > 1) {
            double* Q = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * n));
            double* R = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n * n));
            qr_householder(ctx, T, m, n, Q, R);
            // Jacobi on R^H (faster convergence after QR): R^H V' = U' S, so
            // R = V' S U'^H: left vectors V', right vectors U' = Ub / S
            svd_jacobi(ctx, R, n, n, Ub, Sd, Vb, true);
            finish();
            if (k == 0) {
                FTD_HIP(hipStreamSynchronize(ctx->stream));
                dev_free(ctx, Q);
                dev_free(ctx, R);
                return o;
            }
            upload();
            double* G = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n * k));
            gather(Vb, n, n * n, s_left ? dS : nullptr, 0, G);
            o.Lq = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * k));
            GemmParams p{};
            p.M = (int)m; p.N = k; p.K = (int)n;
            p.sAm = n; p.sAk = 1; p.planeA = m * n; p.a_kcontig = 1;
            p.sBk = 1; p.sBn = n; p.planeB = n * k; p.b_kcontig = 1;
            p.sCm = k; p.sCn = 1; p.planeC = m * k;
            p.nprob = 1; p.prob[0].t1 = 1;
            gemm(ctx, Prec::F64, true, Q, G, o.Lq, p, TAG_NONE);
            o.Rq = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n * k));
            gather(Ub, n, n * n, s_left ? dInv : nullptr, 1, o.Rq);
            FTD_HIP(hipStreamSynchronize(ctx->stream));
            dev_free(ctx, Q);
            dev_free(ctx, R);
            dev_free(ctx, G);
        } else {
            svd_jacobi(ctx, T, m, n, Ub, Sd, Vb);       // T V = U S, Ub = U S (m x n)
            finish();
            if (k == 0) return o;
            upload();
            double* G = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * k));
            gather(Ub, m, m * n, s_left ? nullptr : dInv, 0, G);
            o.Lq = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * k));
            k_transpose(ctx, G, k, m, m * k, o.Lq, m * k, 0);
            o.Rq = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n * k));
            gather(Vb, n, n * n, s_left ? nullptr : dS, 1, o.Rq);
            FTD_HIP(hipStreamSynchronize(ctx->stream));
            dev_free(ctx, G);
        }
    } else {
        ctx->ws_tmp3.ensure(ctx, sizeof(double) * 2 * (size_t)m * n);
        double* TH = ctx->ws_tmp3.as<double>();
        k_transpose(ctx, T, m, n, m * n, TH, m * n, 1);   // n x m
        svd_jacobi(ctx, TH, n, m, Ub, Sd, Vb);           // T^H = U S V^H, Ub = U S (n x m)
        finish();
        if (k == 0) return o;
        upload();
        double* G = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * k));
        gather(Vb, m, m * m, s_left ? dS : nullptr, 0, G);
        o.Lq = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * k));
        k_transpose(ctx, G, k, m, m * k, o.Lq, m * k, 0);
        o.Rq = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n * k));
        gather(Ub, n, n * m, s_left ? dInv : nullptr, 1, o.Rq);
        FTD_HIP(hipStreamSynchronize(ctx->stream));
        dev_free(ctx, G);
    }
    o.k = k;
    return o;
}

// SVD compression of sum_t c_t O_t |psi_t> (O_t an MPO or the identity)
// without storing the exact sum X, whose bonds are as wide as the MPO bond
// times the state bond:
//   1. right to left, the exact remainder of X beyond each bond is factored
//      as R_b Q_{>b} with Q right-orthonormal; only the small factor R_b
//      (bond width x rank) is kept: R_b is the L factor of X_{b+1} R_{b+1};
//   2. left to right, the partial product T_i = C X_i is multiplied by R_i,
//      which makes it the true centre matrix across bond i, and truncated by
//      SVD (at most D singular values with s/s_max > cutoff, whole
//      multiplets); the kept left vectors become the site tensor and
//      C = U^H T_i is carried on;
//   3. an LQ sweep returns the state to right-canonical form.
// The result depends only on the state X, not on the MPO's channel basis.
struct ZipTerm {
    cplx c;
    const Mpo* O;   // nullptr: identity
    const Mps* psi;
};

namespace {
// bond b = right of site b; b = L-1 is the boundary where the terms add up
struct BondLayout {
    int64_t width;
    std::vector<int64_t> off;   // per term
};
BondLayout bond_layout(const std::vector<ZipTerm>& terms, int b, int L) {
    BondLayout bl;
    bl.width = 0;
    for (auto& t : terms) {
        bl.off.push_back(bl.width);
        if (b >= L - 1)
            bl.width += 1;
        else
            bl.width += (t.O ? (int64_t)t.O->s[b].wr : 1) * t.psi->Dr[b];
    }
    return bl;
}
}  // namespace

// M = X_s R_in as a (width of bond s-1) x (d^2 r) row-major matrix.
static void form_M(Ctx* ctx, const std::vector<ZipTerm>& terms, int s, const double* Rin,
                   int64_t rin_rows, int r, const BondLayout& left, const BondLayout& right,
                   double* M) {
    const int d = terms[0].psi->d[s];
    const int64_t rowlen = (int64_t)d * d * r;
    const int64_t nM = left.width * rowlen;
    k_zero(ctx, M, sizeof(double) * 2 * nM);
    const int64_t rplane = rin_rows * r;
    for (size_t t = 0; t < terms.size(); ++t) {
        const Mps* ps = terms[t].psi;
        const int Dl = ps->Dl[s], Dr = ps->Dr[s];
        const int64_t npsi = ps->size(s);
        GemmParams p{};
        p.M = Dl * d * d; p.N = r; p.K = Dr;
        p.sAm = Dr; p.sAk = 1; p.planeA = npsi; p.a_kcontig = 1;
        p.sBk = r; p.sBn = 1; p.planeB = rplane; p.b_kcontig = 0;
        if (!terms[t].O) {
            p.sCm = r; p.sCn = 1; p.planeC = nM;
            p.nprob = 1; p.prob[0].t1 = 1;
            p.prob[0].offC = left.off[t] * rowlen;
            p.term[0].offB = right.off[t] * r;
            gemm(ctx, Prec::F64, true, ps->A[s], Rin, M, p, TAG_NONE);
            continue;
        }
        const MpoSite& W = terms[t].O->s[s];
        const int wl = W.wl, wr = W.wr;
        const int64_t nY = (int64_t)Dl * d * d * r;
        ctx->ws_U.ensure(ctx, sizeof(double) * 2 * nY * wr);
        double* Y = ctx->ws_U.as<double>();
        p.sCm = r; p.sCn = 1; p.planeC = nY;
        for (int c0 = 0; c0 < wr; c0 += kMaxProbs) {
            const int c1 = std::min(wr, c0 + kMaxProbs);
            p.nprob = c1 - c0;
            for (int c = c0; c < c1; ++c) {
                const int j = c - c0;
                p.prob[j].offC = (int64_t)c * 2 * nY;
                p.prob[j].t0 = j;
                p.prob[j].t1 = j + 1;
                p.term[j].offA = 0;
                p.term[j].offB = (right.off[t] + (int64_t)c * Dr) * r;
            }
            gemm(ctx, Prec::F64, true, ps->A[s], Rin, Y, p, TAG_NONE);
        }
        // M[(cl, a), p', q, j] = sum_cr sum_p W[cl, cr][p', p] Y_cr[a, p, q, j]
        std::vector<std::vector<std::pair<int, int>>> col(wl);
        for (size_t e = 0; e < W.ents.size(); ++e) col[W.ents[e].cl].push_back({W.ents[e].cr, (int)e});
        MixParams mp{};
        mp.Da = Dl; mp.d = d; mp.Db = r;
        mp.planeIn = nY; mp.planeOut = nM;
        mp.opStride = 2 * (int64_t)d * d;
        int ne = 0;
        for (int cl = 0; cl < wl; ++cl) {
            if (col[cl].empty()) continue;
            if (mp.njobs == kMaxMixJobs || ne + (int)col[cl].size() > kMaxMixEnts) {
                chanmix(ctx, Prec::F64, true, Y, W.ops64, M, mp);
                mp.njobs = 0;
                ne = 0;
            }
            mp.job[mp.njobs] = {(left.off[t] + (int64_t)cl * Dl) * rowlen, ne, ne + (int)col[cl].size()};
            for (auto& pr : col[cl]) mp.ent[ne++] = {(int64_t)pr.first * 2 * nY, pr.second};
            mp.njobs++;
        }
        if (mp.njobs) chanmix(ctx, Prec::F64, true, Y, W.ops64, M, mp);
    }
}

// T = C X_i: (Dp d^2) x (width of bond i), or at the last site the sum over
// terms as a single column.
static double* form_T(Ctx* ctx, const std::vector<ZipTerm>& terms, int i, const double* C,
                      int64_t ldC, int Dp, const BondLayout& left, const BondLayout& right,
                      bool last, int64_t& ncols) {
    const int d = terms[0].psi->d[i];
    ncols = last ? 1 : right.width;
    const int64_t m = (int64_t)Dp * d * d;
    const int64_t Tn = m * ncols;
    double* T = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * Tn));
    k_zero(ctx, T, sizeof(double) * 2 * Tn);
    for (size_t t = 0; t < terms.size(); ++t) {
        const Mps* ps = terms[t].psi;
        const int Dlt = ps->Dl[i], Drt = ps->Dr[i];
        const int64_t nX = (int64_t)Dp * d * d * Drt;
        const int64_t npsi = ps->size(i);
        const int64_t toff = last ? 0 : right.off[t];
        if (!terms[t].O) {
            ctx->ws_U.ensure(ctx, sizeof(double) * 2 * nX);
            double* X = ctx->ws_U.as<double>();
            GemmParams p{};
            p.M = Dp; p.N = d * d * Drt; p.K = Dlt;
            p.sAm = ldC; p.sAk = 1; p.planeA = (int64_t)Dp * ldC; p.a_kcontig = 1;
            p.sBk = (int64_t)d * d * Drt; p.sBn = 1; p.planeB = npsi; p.b_kcontig = 0;
            p.sCm = (int64_t)d * d * Drt; p.sCn = 1; p.planeC = nX;
            p.nprob = 1; p.prob[0].t1 = 1;
            p.term[0].offA = left.off[t];
            gemm(ctx, Prec::F64, true, C, ps->A[i], X, p, TAG_NONE);
            k_embed(ctx, X, Dp, d * d, Drt, T, Dp, (int)ncols, 0, (int)toff, 1.0, 0.0, 1);
            continue;
        }
        const MpoSite& W = terms[t].O->s[i];
        const int wl = W.wl, wr = W.wr;
        ctx->ws_U.ensure(ctx, sizeof(double) * 2 * nX * wl);
        double* X = ctx->ws_U.as<double>();
        for (int c0 = 0; c0 < wl; c0 += kMaxProbs) {
            const int c1 = std::min(wl, c0 + kMaxProbs);
            GemmParams p{};
            p.M = Dp; p.N = d * d * Drt; p.K = Dlt;
            p.sAm = ldC; p.sAk = 1; p.planeA = (int64_t)Dp * ldC; p.a_kcontig = 1;
            p.sBk = (int64_t)d * d * Drt; p.sBn = 1; p.planeB = npsi; p.b_kcontig = 0;
            p.sCm = (int64_t)d * d * Drt; p.sCn = 1; p.planeC = nX;
            p.nprob = c1 - c0;
            for (int c = c0; c < c1; ++c) {
                const int j = c - c0;
                p.prob[j].offC = (int64_t)c * 2 * nX;
                p.prob[j].t0 = j;
                p.prob[j].t1 = j + 1;
                p.term[j].offA = left.off[t] + (int64_t)c * Dlt;
                p.term[j].offB = 0;
            }
            gemm(ctx, Prec::F64, true, C, ps->A[i], X, p, TAG_NONE);
        }
        std::vector<std::vector<std::pair<int, int>>> col(wr);
        for (size_t e = 0; e < W.ents.size(); ++e) col[W.ents[e].cr].push_back({W.ents[e].cl, (int)e});
        MixParams mp{};
        mp.Da = Dp; mp.d = d; mp.Db = Drt;
        mp.ldIn = Drt; mp.ldOut = ncols;
        mp.planeIn = nX; mp.planeOut = Tn;
        mp.opStride = 2 * (int64_t)d * d;
        mp.accumulate = 1;
        int ne = 0;
        for (int cr = 0; cr < wr; ++cr) {
            if (col[cr].empty()) continue;
            if (mp.njobs == kMaxMixJobs || ne + (int)col[cr].size() > kMaxMixEnts) {
                chanmix(ctx, Prec::F64, true, X, W.ops64, T, mp);
                mp.njobs = 0;
                ne = 0;
            }
            mp.job[mp.njobs] = {toff + (int64_t)cr * Drt, ne, ne + (int)col[cr].size()};
            for (auto& pr : col[cr]) mp.ent[ne++] = {(int64_t)pr.first * 2 * nX, pr.second};
            mp.njobs++;
        }
        if (mp.njobs) chanmix(ctx, Prec::F64, true, X, W.ops64, T, mp);
    }
    return T;
}

// LQ sweep from the right (no truncation): right-canonical, norm on site 0.
static void lq_sweep(Ctx* ctx, Mps* Y) {
    for (int i = Y->L - 1; i >= 1; --i) {
        const int Da = Y->Dl[i], d = Y->d[i], Db = Y->Dr[i];
        ctx->ws_tmp1.ensure(ctx, sizeof(double) * 2 * (size_t)Da * Da);
        double* Lm = ctx->ws_tmp1.as<double>();
        lq_chol(ctx, Y->A[i], Da, (int64_t)d * d * Db, Lm);
        absorb_left(ctx, Y, i, Lm, Y->Dl[i]);
    }
}

static Mps* compress_terms(Ctx* ctx, const std::vector<ZipTerm>& terms, int D, double cutoff) {
    FTD_CHECK(!terms.empty(), FTD_EINVAL, "compress: no terms");
    const int L = terms[0].psi->L;
    for (auto& t : terms) {
        FTD_CHECK(t.psi->L == L && (!t.O || t.O->L == L), FTD_EINVAL, "compress: lengths differ");
        FTD_CHECK(std::abs(t.psi->log_norm - terms[0].psi->log_norm) <=
                      1e-15 * std::max(1.0, std::abs(terms[0].psi->log_norm)),
                  FTD_EINVAL, "compress: terms carry different norms");
    }
    const int nt = (int)terms.size();
    std::vector<BondLayout> bonds(L);
    for (int b = 0; b < L; ++b) bonds[b] = bond_layout(terms, b, L);
    BondLayout left0;
    left0.width = nt;
    for (int t = 0; t < nt; ++t) left0.off.push_back(t);
    // 1. metric factors R_b (bond width x rank), right to left
    std::vector<double*> Rf(L, nullptr);
    std::vector<int> rk(L, 0);
    Mps* Y = nullptr;
    double* C = nullptr;
    const double t0 = wall_seconds();
    double t1 = t0, t_svd = 0.0;
    int wmax = 0;
    for (auto& b : bonds) wmax = std::max<int>(wmax, (int)b.width);
    try {
        {
            std::vector<double> ones(2 * nt, 0.0);
            for (int t = 0; t < nt; ++t) ones[t] = 1.0;
            Rf[L - 1] = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * nt));
            FTD_HIP(hipMemcpyAsync(Rf[L - 1], ones.data(), sizeof(double) * 2 * nt, hipMemcpyHostToDevice, ctx->stream));
            FTD_HIP(hipStreamSynchronize(ctx->stream));
            rk[L - 1] = 1;
        }
        for (int s = L - 1; s >= 1; --s) {
            const BondLayout& lb = bonds[s - 1];
            const BondLayout& rb = bonds[s];
            const int d = terms[0].psi->d[s];
            const int r = rk[s];
            const int64_t cols = (int64_t)d * d * r;
            ctx->ws_tmp2.ensure(ctx, sizeof(double) * 2 * (size_t)(lb.width * cols));
            double* M = ctx->ws_tmp2.as<double>();
            form_M(ctx, terms, s, Rf[s], rb.width, r, lb, rb, M);
            // M = L Q: QR of M^H (cols x width), L = R^H
            const int64_t rr = std::min<int64_t>(cols, lb.width);
            double* Rp = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * rr * lb.width));
            qr_householder(ctx, M, cols, lb.width, nullptr, Rp, true);
            Rf[s - 1] = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * lb.width * rr));
            k_transpose(ctx, Rp, rr, lb.width, rr * lb.width, Rf[s - 1], rr * lb.width, 1);
            FTD_HIP(hipStreamSynchronize(ctx->stream));
            dev_free(ctx, Rp);
            rk[s - 1] = (int)rr;
        }
        t1 = wall_seconds();
        // 2. left-to-right truncation of the true centre matrices
        Y = new Mps();
        Y->ctx = ctx;
        Y->L = L;
        Y->d = terms[0].psi->d;
        Y->Dl.assign(L, 1);
        Y->Dr.assign(L, 1);
        Y->A.assign(L, nullptr);
        Y->prec = terms[0].psi->prec;
        Y->log_norm = terms[0].psi->log_norm;
        {
            std::vector<double> h(2 * nt);
            for (int t = 0; t < nt; ++t) {
                h[t] = terms[t].c.real();
                h[nt + t] = terms[t].c.imag();
            }
            C = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * nt));
            FTD_HIP(hipMemcpyAsync(C, h.data(), sizeof(double) * 2 * nt, hipMemcpyHostToDevice, ctx->stream));
            FTD_HIP(hipStreamSynchronize(ctx->stream));
        }
        int64_t ldC = nt;
        int Dp = 1;
        for (int i = 0; i < L; ++i) {
            const bool last = (i == L - 1);
            const BondLayout& lb = (i == 0) ? left0 : bonds[i - 1];
            int64_t ncols = 0;
            double* T = form_T(ctx, terms, i, C, ldC, Dp, lb, bonds[i], last, ncols);
            const int d = Y->d[i];
            const int64_t m = (int64_t)Dp * d * d;
            if (last) {
                FTD_HIP(hipStreamSynchronize(ctx->stream));
                dev_free(ctx, C);
                C = nullptr;
                Y->A[i] = T;
                Y->Dl[i] = Dp;
                break;
            }
            const int r = rk[i];
            double* P = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * m * r));
            {
                GemmParams p{};
                p.M = (int)m; p.N = r; p.K = (int)ncols;
                p.sAm = ncols; p.sAk = 1; p.planeA = m * ncols; p.a_kcontig = 1;
                p.sBk = r; p.sBn = 1; p.planeB = ncols * r; p.b_kcontig = 0;
                p.sCm = r; p.sCn = 1; p.planeC = m * r;
                p.nprob = 1; p.prob[0].t1 = 1;
                gemm(ctx, Prec::F64, true, T, Rf[i], P, p, TAG_NONE);
            }
            const double ts = ctx->verbose >= 2 ? wall_seconds() : 0.0;
            TruncOut tr = svd_trunc(ctx, P, m, r, D, cutoff, false);
            if (ctx->verbose >= 2) t_svd += wall_seconds() - ts;
            const int k = tr.k;
            double* Cn = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * (int64_t)k * ncols));
            {
                GemmParams p{};
                p.M = k; p.N = (int)ncols; p.K = (int)m;
                p.sAm = 1; p.sAk = k; p.planeA = m * k; p.conjA = 1; p.a_kcontig = 0;
                p.sBk = ncols; p.sBn = 1; p.planeB = m * ncols; p.b_kcontig = 0;
                p.sCm = ncols; p.sCn = 1; p.planeC = (int64_t)k * ncols;
                p.nprob = 1; p.prob[0].t1 = 1;
                gemm(ctx, Prec::F64, true, tr.Lq, T, Cn, p, TAG_NONE);
            }
            FTD_HIP(hipStreamSynchronize(ctx->stream));
            dev_free(ctx, T);
            dev_free(ctx, P);
            dev_free(ctx, tr.Rq);
            dev_free(ctx, C);
            C = Cn;
            ldC = ncols;
            Y->A[i] = tr.Lq;
            Y->Dl[i] = Dp;
            Y->Dr[i] = k;
            Dp = k;
        }
    } catch (...) {
        for (auto p : Rf) dev_free(ctx, p);
        dev_free(ctx, C);
        mps_free(Y);
        throw;
    }
    for (auto p : Rf) dev_free(ctx, p);
    const double t2 = wall_seconds();
    // 3. back to right-canonical form
    lq_sweep(ctx, Y);
    FTD_HIP(hipStreamSynchronize(ctx->stream));
    vlog(ctx, 2, "compress %d terms, widest bond %d: metric %.3f s, truncation %.3f s "
         "(svd %.3f s), lq sweep %.3f s", nt, wmax, t1 - t0, t2 - t1, t_svd, wall_seconds() - t2);
    return Y;
}

// SVD truncation of a right-canonical state in place: left to right, each
// centre A_i (Dl d^2 x Dr) keeps at most D singular values with
// s/s_max > cutoff (whole multiplets), its left vectors become the site and
// S V^H moves into the next site; then an LQ sweep restores right-canonical
// form.  For a right-canonical input this is the SVD compression of the
// state (the right-canonical sweep compress() starts with is the identity).
void truncate_canonical(Ctx* ctx, Mps* psi, int D, double cutoff) {
    const int L = psi->L;
    for (int i = 0; i < L - 1; ++i) {
        const int Da = psi->Dl[i], Db = psi->Dr[i], d = psi->d[i];
        const int64_t m = (int64_t)Da * d * d;
        TruncOut t = svd_trunc(ctx, psi->A[i], m, Db, D, cutoff, false);
        try {
            set_site(ctx, psi, i, Da, t.k, t.Lq);
            t.Lq = nullptr;
            absorb_right(ctx, psi, i, t.Rq, t.k);
        } catch (...) {
            FTD_HIP(hipStreamSynchronize(ctx->stream));
            dev_free(ctx, t.Lq);
            dev_free(ctx, t.Rq);
            throw;
        }
        FTD_HIP(hipStreamSynchronize(ctx->stream));
        dev_free(ctx, t.Rq);
    }
    lq_sweep(ctx, psi);
    FTD_HIP(hipStreamSynchronize(ctx->stream));
}

Mps* compress(Ctx* ctx, Mps* X, int D, double cutoff, bool consume) {
    Mps* Y = compress_terms(ctx, {ZipTerm{cplx(1.0, 0.0), nullptr, X}}, D, cutoff);
    if (consume) mps_free(X);
    return Y;
}

Mps* apply_compress(Ctx* ctx, const Mpo* O, const Mps* psi, int D, double cutoff) {
    return compress_terms(ctx, {ZipTerm{cplx(1.0, 0.0), O, psi}}, D, cutoff);
}

Mps* pc_stage(Ctx* ctx, const Mps* psi, const Mpo* O, const Mps* phi, cplx c, int D, double cutoff) {
    return compress_terms(ctx, {ZipTerm{cplx(1.0, 0.0), nullptr, psi}, ZipTerm{c, O, phi}}, D, cutoff);
}

Mps* taylor_growth(Ctx* ctx, const Mpo* H, const Mps* psi, double dtau, int D, double cutoff) {
    Mps* phi = nullptr;
    try {
        for (int k = 4; k >= 1; --k) {
            const Mps* src = phi ? phi : psi;
            Mps* nxt = compress_terms(ctx, {ZipTerm{cplx(1.0, 0.0), nullptr, psi},
                                            ZipTerm{cplx(-dtau / k, 0.0), H, src}},
                                      D, cutoff);
            mps_free(phi);
            phi = nxt;
        }
    } catch (...) {
        mps_free(phi);
        throw;
    }
    return phi;
}

// ============================================================== overlap
// <bra| O |ket> by a left-to-right transfer contraction in float64.
// sigma_ij = <psi| c+_j c_i |psi> / <psi|psi>: one bond-1 MPO whose two
// carrier-site op tables are rewritten per pair (sigma- on e_i, sigma+ on e_j;
// n on e_i when i == j), each pair one overlap.  sigma: 2*N*N doubles,
// interleaved complex, row i column j.
void reduced_density(Ctx* ctx, const ftd_model& md, const Mps* psi, double* sigma) {
    std::vector<int> epos;
    Mpo* O = build_product_mpo(ctx, md, epos);
    try {
        FTD_CHECK(O->L == psi->L, FTD_EINVAL, "state and model have different chains");
        for (int s = 0; s < O->L; ++s)
            FTD_CHECK(O->s[s].d == psi->d[s], FTD_EINVAL, "state and model have different sites");
        upload_mpo(ctx, O);
        // electron basis |0> empty, |1> occupied; op tables [re plane][im plane], [out][in]
        const double eye[8] = {1, 0, 0, 1, 0, 0, 0, 0};
        const double sm[8] = {0, 1, 0, 0, 0, 0, 0, 0};   // |0><1|
        const double sp[8] = {0, 0, 1, 0, 0, 0, 0, 0};   // |1><0|
        const double nn[8] = {0, 0, 0, 1, 0, 0, 0, 0};
        auto put = [&](int site, const double* op) {
            FTD_HIP(hipMemcpyAsync(O->s[site].ops64, op, sizeof(double) * 8, hipMemcpyHostToDevice,
                                   ctx->stream));
        };
        const double z = overlap(ctx, psi, O, psi).real();
        FTD_CHECK(z > 0.0 && std::isfinite(z), FTD_EINVAL, "state has zero norm");
        const int N = md.n_mol;
        for (int i = 0; i < N; ++i) {
            for (int j = 0; j < N; ++j) {
                if (i == j) {
                    put(epos[i], nn);
                } else {
                    put(epos[i], sm);
                    put(epos[j], sp);
                }
                const cplx v = overlap(ctx, psi, O, psi) / z;
                sigma[2 * (i * N + j)] = v.real();
                sigma[2 * (i * N + j) + 1] = v.imag();
                put(epos[i], eye);
                put(epos[j], eye);
            }
        }
        FTD_HIP(hipStreamSynchronize(ctx->stream));
    } catch (...) {
        destroy_mpo(O);
        throw;
    }
    destroy_mpo(O);
}

cplx overlap(Ctx* ctx, const Mps* bra, const Mpo* O, const Mps* ket) {
    const int L = bra->L;
    FTD_CHECK(ket->L == L && O->L == L, FTD_EINVAL, "overlap: lengths differ");
    DBuf Ea, Eb;
    std::vector<double> one = {1.0, 0.0};
    Ea.ensure(ctx, sizeof(double) * 2);
    FTD_HIP(hipMemcpyAsync(Ea.p, one.data(), sizeof(double) * 2, hipMemcpyHostToDevice, ctx->stream));
    FTD_HIP(hipStreamSynchronize(ctx->stream));
    int w = 1;
    for (int i = 0; i < L; ++i) {
        const MpoSite& W = O->s[i];
        const int d = W.d;
        const int Da1 = bra->Dl[i], Db1 = bra->Dr[i];
        const int Da2 = ket->Dl[i], Db2 = ket->Dr[i];
        FTD_CHECK(w == W.wl, FTD_EINVAL, "overlap: channel mismatch");
        const int64_t n = (int64_t)Da1 * d * d * Db2;   // T shape (a', p, q, b)
        const int64_t nk = ket->size(i);
        const int wl = W.wl, wr = W.wr;
        ctx->ws_T.ensure(ctx, sizeof(double) * 2 * (size_t)n * (wl + wr + 1) + sizeof(double) * 2 * nk);
        double* T = ctx->ws_T.as<double>();
        // ket tensor into the extra slot wl + wr
        const int ks = wl + wr;
        // stage_left expects X laid out with slot stride 2n; use a direct GEMM here
        k_copy_f64(ctx, ket->A[i], T + (int64_t)ks * 2 * n, 2 * nk);
        {
            GemmParams p{};
            p.M = Da1; p.N = d * d * Db2; p.K = Da2;
            p.sAm = Da2; p.sAk = 1; p.planeA = (int64_t)Da1 * Da2; p.a_kcontig = 1;
            p.sBk = (int64_t)d * d * Db2; p.sBn = 1; p.planeB = nk; p.b_kcontig = 0;
            p.sCm = (int64_t)d * d * Db2; p.sCn = 1; p.planeC = n;
            p.nprob = wl;
            for (int c = 0; c < wl; ++c) {
                p.prob[c].offC = (int64_t)c * 2 * n;
                p.prob[c].t0 = c;
                p.prob[c].t1 = c + 1;
                p.term[c].offA = (int64_t)c * 2 * Da1 * Da2;
                p.term[c].offB = (int64_t)ks * 2 * n;
            }
            gemm(ctx, Prec::F64, true, Ea.p, T, T, p, TAG_NONE);
        }
        std::vector<int> in_slot(wl);
        for (int c = 0; c < wl; ++c) in_slot[c] = c;
        MixPlan plan = stage_mix(ctx, Prec::F64, W, true, in_slot, wr, wl, {}, T, Da1, d, Db2, n,
                                 -1, nullptr, true, false);
        const int64_t bb = (int64_t)Db1 * Db2;
        Eb.ensure(ctx, sizeof(double) * 2 * (size_t)wr * bb);
        for (int c = 0; c < wr; ++c)
            if (plan.out_slot[c] < 0) k_zero(ctx, Eb.as<double>() + (int64_t)c * 2 * bb, sizeof(double) * 2 * bb);
        GemmParams p{};
        p.M = Db1; p.N = Db2; p.K = Da1 * d * d;
        p.sAm = 1; p.sAk = Db1; p.planeA = bra->size(i); p.conjA = 1; p.a_kcontig = 0;
        p.sBk = Db2; p.sBn = 1; p.planeB = n; p.b_kcontig = 0;
        p.sCm = Db2; p.sCn = 1; p.planeC = bb;
        int np = 0;
        for (int c = 0; c < wr; ++c) {
            if (plan.out_slot[c] < 0) continue;
            p.prob[np].offC = (int64_t)c * 2 * bb;
            p.prob[np].t0 = np;
            p.prob[np].t1 = np + 1;
            p.term[np].offA = 0;
            p.term[np].offB = (int64_t)plan.out_slot[c] * 2 * n;
            ++np;
        }
        p.nprob = np;
        // bra operand and T are different buffers: run per problem with A = bra
        if (np) gemm(ctx, Prec::F64, true, bra->A[i], T, Eb.p, p, TAG_NONE);
        std::swap(Ea, Eb);
        w = wr;
    }
    std::vector<double> out(2);
    FTD_HIP(hipMemcpyAsync(out.data(), Ea.p, sizeof(double) * 2, hipMemcpyDeviceToHost, ctx->stream));
    FTD_HIP(hipStreamSynchronize(ctx->stream));
    Ea.release(ctx);
    Eb.release(ctx);
    return cplx(out[0], out[1]);
}

// ========================================================= kernel access
void heff_apply_host(Ctx* ctx, const Mpo* H, const Mps* psi, int site, const double* x,
                     double* y, int nrep) {
    const int L = psi->L;
    FTD_CHECK(site >= 0 && site < L, FTD_EINVAL, "site out of range");
    const Prec prec = psi->prec;
    build_left_envs(ctx, H, psi, site);
    build_right_envs(ctx, H, psi, site + 1);
    const int64_t n = psi->size(site);
    double* dx = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n));
    double* dy = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n));
    std::vector<double> hx(2 * n);
    for (int64_t k = 0; k < n; ++k) {
        hx[k] = x[2 * k];
        hx[k + n] = x[2 * k + 1];
    }
    FTD_HIP(hipMemcpyAsync(dx, hx.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice, ctx->stream));
    EnvView Lv = envL_view(ctx, site, prec), Rv = envR_view(ctx, site + 1, prec);
    for (int r = 0; r < std::max(1, nrep); ++r)
        heff(ctx, prec, H->s[site], psi->Dl[site], psi->Dr[site], Lv, Rv, dx, dy);
    FTD_HIP(hipMemcpyAsync(hx.data(), dy, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, ctx->stream));
    FTD_HIP(hipStreamSynchronize(ctx->stream));
    for (int64_t k = 0; k < n; ++k) {
        y[2 * k] = hx[k];
        y[2 * k + 1] = hx[k + n];
    }
    dev_free(ctx, dx);
    dev_free(ctx, dy);
}

// y = exp(z H_eff) x at one site, by the Krylov exponential of the TDVP
// sweep (same environments and operator as heff_apply_host); repeated nrep
// times from the same x (timing).  Returns the Krylov vector count.
int heff_expm_host(Ctx* ctx, const Mpo* H, const Mps* psi, int site, const double* x, double* y,
                   cplx z, double tol, int mmax, int nrep) {
    const int L = psi->L;
    FTD_CHECK(site >= 0 && site < L, FTD_EINVAL, "site out of range");
    FTD_CHECK(H->L == L, FTD_EINVAL, "MPO and MPS lengths differ");
    const Prec prec = psi->prec;
    build_left_envs(ctx, H, psi, site);
    build_right_envs(ctx, H, psi, site + 1);
    const int64_t n = psi->size(site);
    double* dx0 = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n));
    double* dx = nullptr;
    int m = 0;
    try {
        dx = static_cast<double*>(dev_alloc(ctx, sizeof(double) * 2 * n));
        std::vector<double> hx(2 * n);
        for (int64_t k = 0; k < n; ++k) {
            hx[k] = x[2 * k];
            hx[k + n] = x[2 * k + 1];
        }
        FTD_HIP(hipMemcpyAsync(dx0, hx.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice,
                               ctx->stream));
        EnvView Lv = envL_view(ctx, site, prec), Rv = envR_view(ctx, site + 1, prec);
        const MpoSite& W = H->s[site];
        const int Da = psi->Dl[site], Db = psi->Dr[site];
        auto op = [&](const double* a, double* b) { heff(ctx, prec, W, Da, Db, Lv, Rv, a, b); };
        int hint = 4;
        for (int r = 0; r < std::max(1, nrep); ++r) {
            k_copy_f64(ctx, dx0, dx, 2 * n);
            m = expm_krylov(ctx, op, dx, n, z, tol, mmax, hint);
        }
        FTD_HIP(hipMemcpyAsync(hx.data(), dx, sizeof(double) * 2 * n, hipMemcpyDeviceToHost,
                               ctx->stream));
        FTD_HIP(hipStreamSynchronize(ctx->stream));
        for (int64_t k = 0; k < n; ++k) {
            y[2 * k] = hx[k];
            y[2 * k + 1] = hx[k + n];
        }
    } catch (...) {
        dev_free(ctx, dx0);
        if (dx) dev_free(ctx, dx);
        throw;
    }
    dev_free(ctx, dx0);
    dev_free(ctx, dx);
    return m;
}

}  // namespace ftd
