// C ABI of the library (see include/ftdmrg.h): argument checks, handle
// ownership, status codes, and the drivers of the imaginary-time preparation
// and the current correlation.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace ftd {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

template <typename F>
static ftd_status guarded(F&& f) {
    try {
        f();
        return FTD_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return FTD_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return FTD_EDEVICE;
    } catch (...) {
        set_error("unknown error");
        return FTD_EDEVICE;
    }
}

static void check_krylov(const ftd_krylov_opts* ko, double& tol, int& mmax) {
    tol = ko ? ko->tol : 1e-14;
    mmax = ko ? ko->mmax : 40;
    FTD_CHECK(std::isfinite(tol) && tol > 0.0, FTD_EINVAL, "Krylov tolerance must be > 0");
    FTD_CHECK(mmax >= 1 && mmax < kMaxKrylov, FTD_EINVAL, "Krylov mmax must be in [1, 63]");
}

static Prec to_prec(int32_t p) {
    FTD_CHECK(p == FTD_C128 || p == FTD_C64 || p == FTD_BF16X3, FTD_EINVAL, "unknown precision");
    return static_cast<Prec>(p);
}

// largest possible rank of every bond: min(prod_left d^2, prod_right d^2)
static std::vector<double> max_bond(const Mps* psi) {
    const int L = psi->L;
    std::vector<double> out(std::max(0, L - 1));
    std::vector<double> lp(L), rp(L);
    double acc = 1.0;
    for (int i = 0; i < L; ++i) {
        acc = std::min(acc * psi->d[i] * psi->d[i], 1e18);
        lp[i] = acc;
    }
    acc = 1.0;
    for (int i = L - 1; i >= 0; --i) {
        acc = std::min(acc * psi->d[i] * psi->d[i], 1e18);
        rp[i] = acc;
    }
    for (int i = 0; i < L - 1; ++i) out[i] = std::min(lp[i], rp[i + 1]);
    return out;
}

}  // namespace ftd

using namespace ftd;

// The auxiliary context of a handle: own non-blocking stream (no implicit
// ordering against the caller's stream, which may be the null stream), plain
// hipMalloc workspaces.
static Ctx* aux_ctx(ftd_ctx* ctx) {
    if (ctx->aux) return ctx->aux;
    hipStream_t s = nullptr;
    FTD_HIP(hipSetDevice(ctx->c.device));
    FTD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    Ctx* a = new Ctx();
    try {
        ctx_init(*a, ctx->c.device, s, nullptr);
        if (!ctx->ev_fork) FTD_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
        if (!ctx->ev_join) FTD_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    } catch (...) {
        ctx_release(*a);
        (void)hipStreamDestroy(s);
        delete a;
        throw;
    }
    a->timing = ctx->c.timing;
    a->verbose = ctx->c.verbose;
    ctx->aux = a;
    return a;
}

static void ctx_free(ftd_ctx* ctx) {
    if (ctx->aux) {
        ctx_release(*ctx->aux);
        (void)hipStreamDestroy(ctx->aux->stream);
        delete ctx->aux;
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    ctx_release(ctx->c);
    delete ctx;
}

// drop one reference to the context a handle was made on
static void ctx_unref(Ctx* c) {
    if (c->refs.fetch_sub(1) == 1) ctx_free(static_cast<ftd_ctx*>(c->owner));
}

static ftd_mps* mps_handle(Mps* m) {
    m->ctx->refs.fetch_add(1);
    return new ftd_mps{m};
}

static ftd_mpo* mpo_handle(Mpo* m) {
    m->ctx->refs.fetch_add(1);
    return new ftd_mpo{m};
}

extern "C" {

const char* ftd_last_error(void) { return g_last_error.c_str(); }

ftd_status ftd_ctx_create(int32_t device, void* hip_stream, const ftd_allocator* alloc,
                          ftd_ctx** out) {
    return guarded([&] {
        FTD_CHECK(out != nullptr, FTD_EINVAL, "null output pointer");
        int n = 0;
        FTD_HIP(hipGetDeviceCount(&n));
        FTD_CHECK(device >= 0 && device < n, FTD_EINVAL, "device index out of range");
        FTD_HIP(hipSetDevice(device));
        ftd_ctx* h = new ftd_ctx();
        h->c.owner = h;
        try {
            ctx_init(h->c, device, static_cast<hipStream_t>(hip_stream), alloc);
        } catch (...) {
            ctx_release(h->c);
            delete h;
            throw;
        }
        *out = h;
    });
}

void ftd_ctx_destroy(ftd_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->c.stream);
    ctx_unref(&ctx->c);
}

ftd_status ftd_ctx_set_timing(ftd_ctx* ctx, int32_t enable) {
    return guarded([&] {
        FTD_CHECK(ctx, FTD_EINVAL, "null context");
        ctx->c.timing = enable != 0;
        if (ctx->aux) ctx->aux->timing = enable != 0;
    });
}

ftd_status ftd_ctx_set_verbose(ftd_ctx* ctx, int32_t level) {
    return guarded([&] {
        FTD_CHECK(ctx, FTD_EINVAL, "null context");
        ctx->c.verbose = level;
        if (ctx->aux) ctx->aux->verbose = level;
    });
}

ftd_status ftd_ctx_stats_reset(ftd_ctx* ctx) {
    return guarded([&] {
        FTD_CHECK(ctx, FTD_EINVAL, "null context");
        for (Ctx* c : {&ctx->c, ctx->aux}) {
            if (!c) continue;
            FTD_HIP(hipStreamSynchronize(c->stream));
            c->events.clear();
            c->event_next = 0;
            c->stats = ftd_stats{};
            timing_slots_reset(c);
            FTD_HIP(hipStreamSynchronize(c->stream));
        }
    });
}

ftd_status ftd_ctx_stats(ftd_ctx* ctx, ftd_stats* out) {
    return guarded([&] {
        FTD_CHECK(ctx && out, FTD_EINVAL, "null argument");
        Ctx& c = ctx->c;
        FTD_HIP(hipStreamSynchronize(c.stream));
        if (ctx->aux) FTD_HIP(hipStreamSynchronize(ctx->aux->stream));
        ftd_stats s = c.stats;
        if (ctx->aux) {
            const ftd_stats& a = ctx->aux->stats;
            s.matvecs += a.matvecs;
            s.krylov_vectors += a.krylov_vectors;
            s.expm_calls += a.expm_calls;
            s.krylov_max = std::max(s.krylov_max, a.krylov_max);
            s.all_flops += a.all_flops;
        }
        s.heff_launches = 0;
        s.heff_ms = 0;
        s.heff_flops = 0;
        // per kernel identity totals, over both streams
        std::vector<double> kms(32, 0.0), kfl(32, 0.0), kby(32, 0.0);
        std::vector<int64_t> kn(32, 0);
        // device timestamps of the timed GEMM launches, per context
        int rate_khz = 0;
        FTD_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c.device));
        std::vector<std::vector<unsigned long long>> slots;
        std::vector<EventPair> all;
        std::vector<int> owner;
        for (Ctx* x : {&c, ctx->aux}) {
            if (!x) continue;
            std::vector<unsigned long long> h;
            if (x->tslots && x->tslot_next > 0) {
                h.resize(2 * (size_t)x->tslot_next);
                FTD_HIP(hipMemcpy(h.data(), x->tslots, sizeof(unsigned long long) * h.size(),
                                  hipMemcpyDeviceToHost));
            }
            slots.push_back(std::move(h));
            for (auto& e : x->events) {
                all.push_back(e);
                owner.push_back((int)slots.size() - 1);
            }
        }
        for (size_t ie = 0; ie < all.size(); ++ie) {
            const EventPair& e = all[ie];
            float ms = 0.f;
            FTD_HIP(hipEventElapsedTime(&ms, e.a, e.b));
            if (e.tag == TAG_HEFF || e.tag == TAG_KEFF) {
                s.heff_launches++;
                s.heff_ms += ms;
                s.heff_flops += e.flops;
            }
            if (e.tag == TAG_HEFF || e.tag == TAG_KEFF) {
                // every launch of a kernel instance (H_eff and K_eff matvecs share
                // instances); the kernel alone: its device timestamps (first block start to
                // last block end), else the events around the main launch
                float kms_one = ms;
                const auto& sl = slots[owner[ie]];
                if (e.slot >= 0 && 2 * (size_t)e.slot + 1 < sl.size() &&
                    sl[2 * e.slot + 1] >= sl[2 * e.slot] && rate_khz > 0) {
                    kms_one = (float)((double)(sl[2 * e.slot + 1] - sl[2 * e.slot]) / rate_khz);
                } else if (e.m) {
                    FTD_HIP(hipEventElapsedTime(&kms_one, e.a, e.m));
                }
                const int k = e.kind & 31;
                kms[k] += kms_one;
                kfl[k] += e.flops;
                kby[k] += e.bytes;
                kn[k]++;
            }
        }
        int best = 0;
        for (int k = 1; k < 32; ++k)
            if (kms[k] > kms[best]) best = k;
        for (int k = 0; k < 32; ++k) {
            s.kind_launches[k] = kn[k];
            s.kind_ms[k] = kms[k];
            s.kind_flops[k] = kfl[k];
            s.kind_bytes[k] = kby[k];
        }
        s.dom_launches = kn[best];
        s.dom_ms = kms[best];
        s.dom_flops = kfl[best];
        s.dom_bytes = kby[best];
        s.dom_kind = best;
        *out = s;
    });
}

ftd_status ftd_ctx_synchronize(ftd_ctx* ctx) {
    return guarded([&] {
        FTD_CHECK(ctx, FTD_EINVAL, "null context");
        FTD_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

static void check_model(const ftd_model* m) {
        FTD_CHECK(m->n_mol >= (m->periodic ? 3 : 2), FTD_EINVAL,
                  "need n_mol >= 3 on a ring (>= 2 open)");
        FTD_CHECK(m->n_loc >= 0 && m->n_nl >= 0, FTD_EINVAL, "negative mode count");
        FTD_CHECK(m->n_loc == 0 || m->levels_loc >= 1, FTD_EINVAL, "levels_loc < 1");
        FTD_CHECK(m->n_nl == 0 || m->levels_nl >= 1, FTD_EINVAL, "levels_nl < 1");
        FTD_CHECK(m->levels_loc <= 32 && m->levels_nl <= 32, FTD_EINVAL, "levels above 32");
        FTD_CHECK(m->n_loc == 0 || (m->omega_loc && m->g_loc), FTD_EINVAL, "null local-mode arrays");
        FTD_CHECK(m->n_nl == 0 || (m->omega_nl && m->g_nl), FTD_EINVAL, "null bond-mode arrays");
        auto fin = [](double x) { return std::isfinite(x); };
        FTD_CHECK(fin(m->V) && fin(m->R) && fin(m->e0), FTD_EINVAL, "non-finite V, R or e0");
        for (int i = 0; i < m->n_loc; ++i)
            FTD_CHECK(fin(m->omega_loc[i]) && fin(m->g_loc[i]), FTD_EINVAL, "non-finite local mode");
        for (int i = 0; i < m->n_nl; ++i)
            FTD_CHECK(fin(m->omega_nl[i]) && fin(m->g_nl[i]), FTD_EINVAL, "non-finite bond mode");
}

ftd_status ftd_mpo_build(ftd_ctx* ctx, const ftd_model* m, ftd_mpo** H, ftd_mpo** J) {
    return guarded([&] {
        FTD_CHECK(ctx && m && H && J, FTD_EINVAL, "null argument");
        check_model(m);
        Ctx* c = &ctx->c;
        Mpo* h = build_mpo(c, *m, false);
        Mpo* j = nullptr;
        try {
            upload_mpo(c, h);
            j = build_mpo(c, *m, true);
            upload_mpo(c, j);
        } catch (...) {
            destroy_mpo(h);
            destroy_mpo(j);
            throw;
        }
        *H = mpo_handle(h);
        *J = mpo_handle(j);
    });
}

void ftd_mpo_destroy(ftd_mpo* mpo) {
    if (!mpo) return;
    Ctx* c = mpo->m->ctx;
    (void)hipStreamSynchronize(c->stream);
    destroy_mpo(mpo->m);
    delete mpo;
    ctx_unref(c);
}

ftd_status ftd_mpo_info(const ftd_mpo* mpo, int32_t* n_sites, int32_t* dims, int32_t* bond_w) {
    return guarded([&] {
        FTD_CHECK(mpo && n_sites, FTD_EINVAL, "null argument");
        *n_sites = mpo->m->L;
        for (int i = 0; i < mpo->m->L; ++i) {
            if (dims) dims[i] = mpo->m->s[i].d;
            if (bond_w && i < mpo->m->L - 1) bond_w[i] = mpo->m->s[i].wr;
        }
    });
}

void ftd_mps_destroy(ftd_mps* psi) {
    if (!psi) return;
    Ctx* c = psi->m->ctx;
    (void)hipStreamSynchronize(c->stream);
    mps_free(psi->m);
    delete psi;
    ctx_unref(c);
}

ftd_status ftd_mps_copy(ftd_ctx* ctx, const ftd_mps* src, ftd_mps** out) {
    return guarded([&] {
        FTD_CHECK(ctx && src && out, FTD_EINVAL, "null argument");
        *out = mps_handle(mps_clone(src->m));
    });
}

ftd_status ftd_mps_info(const ftd_mps* psi, int32_t* n_sites, int32_t* bond_dims,
                        double* log_norm, int32_t* precision) {
    return guarded([&] {
        FTD_CHECK(psi, FTD_EINVAL, "null argument");
        if (n_sites) *n_sites = psi->m->L;
        if (bond_dims)
            for (int i = 0; i < psi->m->L - 1; ++i) bond_dims[i] = psi->m->Dr[i];
        if (log_norm) *log_norm = psi->m->log_norm;
        if (precision) *precision = (int32_t)psi->m->prec;
    });
}

ftd_status ftd_mps_get_site(ftd_ctx* ctx, const ftd_mps* psi, int32_t site, double* host,
                            int64_t count) {
    return guarded([&] {
        FTD_CHECK(ctx && psi && host, FTD_EINVAL, "null argument");
        const Mps* m = psi->m;
        FTD_CHECK(site >= 0 && site < m->L, FTD_EINVAL, "site out of range");
        const int64_t n = m->size(site);
        FTD_CHECK(count >= n, FTD_EINVAL, "host buffer too small");
        std::vector<double> tmp(2 * n);
        FTD_HIP(hipMemcpyAsync(tmp.data(), m->A[site], sizeof(double) * 2 * n, hipMemcpyDeviceToHost,
                               ctx->c.stream));
        FTD_HIP(hipStreamSynchronize(ctx->c.stream));
        for (int64_t k = 0; k < n; ++k) {
            host[2 * k] = tmp[k];
            host[2 * k + 1] = tmp[k + n];
        }
    });
}

ftd_status ftd_mps_from_host(ftd_ctx* ctx, int32_t n_sites, const int32_t* dims,
                             const double* host, double log_norm, ftd_precision prec,
                             ftd_mps** out) {
    return guarded([&] {
        FTD_CHECK(ctx && dims && host && out && n_sites >= 1, FTD_EINVAL, "bad argument");
        std::vector<int> Dl(n_sites), d(n_sites), Dr(n_sites);
        for (int i = 0; i < n_sites; ++i) {
            Dl[i] = dims[4 * i];
            d[i] = dims[4 * i + 1];
            FTD_CHECK(dims[4 * i + 2] == d[i], FTD_EINVAL, "P and Q legs must match");
            Dr[i] = dims[4 * i + 3];
            FTD_CHECK(Dl[i] >= 1 && d[i] >= 1 && Dr[i] >= 1, FTD_EINVAL, "bad site shape");
            if (i > 0) FTD_CHECK(Dl[i] == Dr[i - 1], FTD_EINVAL, "bond dimensions do not chain");
        }
        FTD_CHECK(Dl[0] == 1 && Dr[n_sites - 1] == 1, FTD_EINVAL, "open boundary bonds must be 1");
        Mps* m = mps_alloc(&ctx->c, Dl, d, Dr, to_prec(prec));
        int64_t off = 0;
        for (int i = 0; i < n_sites; ++i) {
            const int64_t n = m->size(i);
            std::vector<double> tmp(2 * n);
            for (int64_t k = 0; k < n; ++k) {
                tmp[k] = host[2 * (off + k)];
                tmp[k + n] = host[2 * (off + k) + 1];
            }
            FTD_HIP(hipMemcpyAsync(m->A[i], tmp.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice,
                                   ctx->c.stream));
            FTD_HIP(hipStreamSynchronize(ctx->c.stream));
            off += n;
        }
        m->log_norm = log_norm;
        *out = mps_handle(m);
    });
}

ftd_status ftd_mps_set_site(ftd_ctx* ctx, ftd_mps* psi, int32_t site, const double* host,
                            int64_t count) {
    return guarded([&] {
        FTD_CHECK(ctx && psi && host, FTD_EINVAL, "null argument");
        Mps* m = psi->m;
        FTD_CHECK(site >= 0 && site < m->L, FTD_EINVAL, "site out of range");
        const int64_t n = m->size(site);
        FTD_CHECK(count == n, FTD_EINVAL, "element count differs from the site's shape");
        std::vector<double> tmp(2 * n);
        for (int64_t k = 0; k < n; ++k) {
            FTD_CHECK(std::isfinite(host[2 * k]) && std::isfinite(host[2 * k + 1]), FTD_EINVAL,
                      "non-finite tensor element");
            tmp[k] = host[2 * k];
            tmp[k + n] = host[2 * k + 1];
        }
        FTD_HIP(hipMemcpyAsync(m->A[site], tmp.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice,
                               ctx->c.stream));
        FTD_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

static const char kMpsMagic[8] = {'F', 'T', 'D', 'M', 'P', 'S', '0', '1'};

ftd_status ftd_mps_save(ftd_ctx* ctx, const ftd_mps* psi, const char* path) {
    return guarded([&] {
        FTD_CHECK(ctx && psi && path, FTD_EINVAL, "null argument");
        const Mps* m = psi->m;
        FILE* f = std::fopen(path, "wb");
        FTD_CHECK(f != nullptr, FTD_EINVAL, std::string("cannot open for writing: ") + path);
        bool ok = true;
        auto put = [&](const void* p, size_t n) { ok = ok && std::fwrite(p, 1, n, f) == n; };
        try {
            put(kMpsMagic, 8);
            const int32_t L = m->L, prec = (int32_t)m->prec;
            put(&L, 4);
            put(&prec, 4);
            put(&m->log_norm, 8);
            for (int i = 0; i < L; ++i) {
                const int32_t dims[4] = {m->Dl[i], m->d[i], m->d[i], m->Dr[i]};
                put(dims, sizeof(dims));
            }
            std::vector<double> tmp;
            for (int i = 0; i < L && ok; ++i) {
                const int64_t n = m->size(i);
                tmp.resize(2 * n);
                FTD_HIP(hipMemcpyAsync(tmp.data(), m->A[i], sizeof(double) * 2 * n,
                                       hipMemcpyDeviceToHost, ctx->c.stream));
                FTD_HIP(hipStreamSynchronize(ctx->c.stream));
                put(tmp.data(), sizeof(double) * 2 * n);
            }
        } catch (...) {
            std::fclose(f);
            throw;
        }
        ok = (std::fclose(f) == 0) && ok;
        FTD_CHECK(ok, FTD_EDEVICE, std::string("write failed: ") + path);
    });
}

ftd_status ftd_mps_load(ftd_ctx* ctx, const char* path, ftd_mps** out) {
    return guarded([&] {
        FTD_CHECK(ctx && path && out, FTD_EINVAL, "null argument");
        FILE* f = std::fopen(path, "rb");
        FTD_CHECK(f != nullptr, FTD_EINVAL, std::string("cannot open: ") + path);
        Mps* m = nullptr;
        auto get = [&](void* p, size_t n) {
            FTD_CHECK(std::fread(p, 1, n, f) == n, FTD_EINVAL, "state file is short");
        };
        try {
            char magic[8];
            get(magic, 8);
            FTD_CHECK(std::memcmp(magic, kMpsMagic, 8) == 0, FTD_EINVAL, "not a state file");
            int32_t L = 0, prec = 0;
            double log_norm = 0.0;
            get(&L, 4);
            get(&prec, 4);
            get(&log_norm, 8);
            FTD_CHECK(L >= 1 && L <= (1 << 20), FTD_EINVAL, "bad site count in state file");
            FTD_CHECK(prec == FTD_C128 || prec == FTD_C64 || prec == FTD_BF16X3, FTD_EINVAL,
                      "bad precision in state file");
            FTD_CHECK(std::isfinite(log_norm), FTD_EINVAL, "non-finite log norm in state file");
            std::vector<int> Dl(L), d(L), Dr(L);
            for (int i = 0; i < L; ++i) {
                int32_t dims[4];
                get(dims, sizeof(dims));
                FTD_CHECK(dims[0] >= 1 && dims[1] >= 1 && dims[1] == dims[2] && dims[3] >= 1 &&
                              dims[0] <= (1 << 16) && dims[1] <= 64 && dims[3] <= (1 << 16),
                          FTD_EINVAL, "bad site shape in state file");
                Dl[i] = dims[0];
                d[i] = dims[1];
                Dr[i] = dims[3];
                if (i > 0) FTD_CHECK(Dl[i] == Dr[i - 1], FTD_EINVAL, "bonds do not chain");
            }
            FTD_CHECK(Dl[0] == 1 && Dr[L - 1] == 1, FTD_EINVAL, "open boundary bonds must be 1");
            m = mps_alloc(&ctx->c, Dl, d, Dr, static_cast<Prec>(prec));
            std::vector<double> tmp;
            for (int i = 0; i < L; ++i) {
                const int64_t n = m->size(i);
                tmp.resize(2 * n);
                get(tmp.data(), sizeof(double) * 2 * n);
                FTD_HIP(hipMemcpyAsync(m->A[i], tmp.data(), sizeof(double) * 2 * n,
                                       hipMemcpyHostToDevice, ctx->c.stream));
                FTD_HIP(hipStreamSynchronize(ctx->c.stream));
            }
            char extra;
            FTD_CHECK(std::fread(&extra, 1, 1, f) == 0, FTD_EINVAL, "trailing bytes in state file");
            m->log_norm = log_norm;
        } catch (...) {
            std::fclose(f);
            mps_free(m);
            throw;
        }
        std::fclose(f);
        *out = mps_handle(m);
    });
}

ftd_status ftd_mps_set_precision(ftd_mps* psi, ftd_precision prec) {
    return guarded([&] {
        FTD_CHECK(psi, FTD_EINVAL, "null argument");
        psi->m->prec = to_prec(prec);
    });
}

ftd_status ftd_mps_norm(ftd_ctx* ctx, const ftd_mps* psi, double* out) {
    return guarded([&] {
        FTD_CHECK(ctx && psi && out, FTD_EINVAL, "null argument");
        // <psi|psi> via the identity transfer: build a trivial MPO-free overlap
        // by contracting bra and ket through the Q and P legs site by site.
        const Mps* m = psi->m;
        Ctx* c = &ctx->c;
        DBuf E, F;
        std::vector<double> one = {1.0, 0.0};
        E.ensure(c, sizeof(double) * 2);
        FTD_HIP(hipMemcpyAsync(E.p, one.data(), sizeof(double) * 2, hipMemcpyHostToDevice, c->stream));
        for (int i = 0; i < m->L; ++i) {
            const int Da = m->Dl[i], Db = m->Dr[i], dd = m->d[i] * m->d[i];
            const int64_t n = m->size(i);
            c->ws_site.ensure(c, sizeof(double) * 2 * n);
            double* T = c->ws_site.as<double>();
            GemmParams p{};
            p.M = Da; p.N = dd * Db; p.K = Da;
            p.sAm = Da; p.sAk = 1; p.planeA = (int64_t)Da * Da; p.a_kcontig = 1;
            p.sBk = (int64_t)dd * Db; p.sBn = 1; p.planeB = n; p.b_kcontig = 0;
            p.sCm = (int64_t)dd * Db; p.sCn = 1; p.planeC = n;
            p.nprob = 1; p.prob[0].t1 = 1;
            gemm(c, Prec::F64, true, E.p, m->A[i], T, p, TAG_NONE);
            F.ensure(c, sizeof(double) * 2 * (size_t)Db * Db);
            GemmParams q{};
            q.M = Db; q.N = Db; q.K = Da * dd;
            q.sAm = 1; q.sAk = Db; q.planeA = n; q.conjA = 1; q.a_kcontig = 0;
            q.sBk = Db; q.sBn = 1; q.planeB = n; q.b_kcontig = 0;
            q.sCm = Db; q.sCn = 1; q.planeC = (int64_t)Db * Db;
            q.nprob = 1; q.prob[0].t1 = 1;
            gemm(c, Prec::F64, true, m->A[i], T, F.p, q, TAG_NONE);
            std::swap(E, F);
        }
        std::vector<double> h(2);
        FTD_HIP(hipMemcpyAsync(h.data(), E.p, sizeof(double) * 2, hipMemcpyDeviceToHost, c->stream));
        FTD_HIP(hipStreamSynchronize(c->stream));
        E.release(c);
        F.release(c);
        *out = h[0];
    });
}

ftd_status ftd_thermal_prep(ftd_ctx* ctx, const ftd_mpo* H, double beta, int32_t n_imag,
                            int32_t n_grow, int32_t D, double cutoff, double expand_tol,
                            ftd_precision prec, const ftd_krylov_opts* ko, ftd_mps** psi_beta,
                            double* log_Z) {
    return guarded([&] {
        FTD_CHECK(ctx && H && psi_beta && log_Z, FTD_EINVAL, "null argument");
        FTD_CHECK(std::isfinite(beta) && beta >= 0.0, FTD_EINVAL, "beta must be >= 0");
        FTD_CHECK(n_imag >= 1, FTD_EINVAL, "n_imag must be >= 1");
        FTD_CHECK(D >= 1, FTD_EINVAL, "D must be >= 1");
        FTD_CHECK(std::isfinite(cutoff) && cutoff >= 0.0 && cutoff < 1.0, FTD_EINVAL, "bad cutoff");
        FTD_CHECK(n_grow <= n_imag, FTD_EINVAL, "n_grow > n_imag");
        FTD_CHECK(std::isfinite(expand_tol) && expand_tol >= 0.0 && expand_tol < 1.0, FTD_EINVAL,
                  "expand_tol must lie in [0, 1)");
        double tol;
        int mmax;
        check_krylov(ko, tol, mmax);
        const Prec pr = to_prec(prec);
        Ctx* c = &ctx->c;
        const Mpo* h = H->m;
        const double t_start = wall_seconds();
        auto maxb = [](const Mps* m) {
            int b = 1;
            for (int i = 0; i + 1 < m->L; ++i) b = std::max(b, m->Dr[i]);
            return b;
        };
        Mps* psi = identity_mps(c, h);
        try {
            Mps* t = compress(c, psi, D, cutoff, true);
            psi = t;
            mps_normalize(c, psi);
            const double dtau = beta / (2.0 * n_imag);
            int steps = 0;
            const bool adaptive = n_grow < 0;
            const int ng = adaptive ? n_imag : n_grow;
            const std::vector<double> mb = max_bond(psi);
            for (int s = 0; s < ng; ++s) {
                std::vector<int> before(psi->Dr.begin(), psi->Dr.end() - 1);
                Mps* nxt = taylor_growth(c, h, psi, dtau, D, cutoff);
                mps_free(psi);
                psi = nxt;
                mps_normalize(c, psi);
                ++steps;
                vlog(c, 1, "prep growth step %d/%d: max bond %d, %.2f s", steps, n_imag, maxb(psi),
                     wall_seconds() - t_start);
                if (adaptive) {
                    // stop after a step that raised no bond, or raised the summed
                    // bond dimension by less than 2 %, or left every bond full
                    bool all_full = true, grew = false;
                    double sum_before = 0.0, sum_after = 0.0;
                    for (int i = 0; i < psi->L - 1; ++i) {
                        if (psi->Dr[i] < std::min<double>(D, mb[i])) all_full = false;
                        if (psi->Dr[i] > before[i]) grew = true;
                        sum_before += before[i];
                        sum_after += psi->Dr[i];
                    }
                    if (all_full || !grew || sum_after < 1.02 * sum_before) break;
                }
            }
            psi->prec = pr;
            const int xD = expand_tol > 0.0 ? D : 0;
            for (int s = steps; s < n_imag; ++s) {
                tdvp_step(c, h, psi, cplx(-dtau, 0.0), tol, mmax, xD, expand_tol);
                // imaginary time damps some added directions towards zero
                // weight: drop Schmidt values below the cutoff, so no gauge
                // move meets a numerically null direction
                if (xD > 0) truncate_canonical(c, psi, D, cutoff);
                mps_normalize(c, psi);
                vlog(c, 1, "prep tdvp step %d/%d: max bond %d, %.2f s", s + 1, n_imag, maxb(psi),
                     wall_seconds() - t_start);
            }
        } catch (...) {
            mps_free(psi);
            throw;
        }
        *log_Z = 2.0 * psi->log_norm;
        *psi_beta = mps_handle(psi);
    });
}

ftd_status ftd_tdvp_step(ftd_ctx* ctx, const ftd_mpo* H, ftd_mps* psi, double dt_real,
                         double dt_imag, const ftd_krylov_opts* ko) {
    return guarded([&] {
        FTD_CHECK(ctx && H && psi, FTD_EINVAL, "null argument");
        FTD_CHECK(std::isfinite(dt_real) && std::isfinite(dt_imag), FTD_EINVAL, "non-finite step");
        double tol;
        int mmax;
        check_krylov(ko, tol, mmax);
        FTD_CHECK(H->m->L == psi->m->L, FTD_EINVAL, "MPO and MPS lengths differ");
        tdvp_step(&ctx->c, H->m, psi->m, cplx(-dt_imag, -dt_real), tol, mmax);
    });
}

ftd_status ftd_tdvp_step_expand(ftd_ctx* ctx, const ftd_mpo* H, ftd_mps* psi, double dt_real,
                                double dt_imag, int32_t D, double expand_tol,
                                const ftd_krylov_opts* ko) {
    return guarded([&] {
        FTD_CHECK(ctx && H && psi, FTD_EINVAL, "null argument");
        FTD_CHECK(std::isfinite(dt_real) && std::isfinite(dt_imag), FTD_EINVAL, "non-finite step");
        FTD_CHECK(D >= 1, FTD_EINVAL, "D must be >= 1");
        FTD_CHECK(std::isfinite(expand_tol) && expand_tol > 0.0 && expand_tol < 1.0, FTD_EINVAL,
                  "expand_tol must lie in (0, 1)");
        double tol;
        int mmax;
        check_krylov(ko, tol, mmax);
        FTD_CHECK(H->m->L == psi->m->L, FTD_EINVAL, "MPO and MPS lengths differ");
        tdvp_step(&ctx->c, H->m, psi->m, cplx(-dt_imag, -dt_real), tol, mmax, D, expand_tol);
    });
}

ftd_status ftd_tdvp_pair(ftd_ctx* ctx, const ftd_mpo* H, ftd_mps* psi, ftd_mps* phi,
                         double dt_real, double dt_imag, const ftd_krylov_opts* ko) {
    return guarded([&] {
        FTD_CHECK(ctx && H && psi && phi, FTD_EINVAL, "null argument");
        FTD_CHECK(psi != phi && psi->m != phi->m, FTD_EINVAL, "the two states must differ");
        FTD_CHECK(std::isfinite(dt_real) && std::isfinite(dt_imag), FTD_EINVAL, "non-finite step");
        double tol;
        int mmax;
        check_krylov(ko, tol, mmax);
        FTD_CHECK(H->m->L == psi->m->L && H->m->L == phi->m->L, FTD_EINVAL,
                  "MPO and MPS lengths differ");
        Ctx* a = aux_ctx(ctx);
        tdvp_pair(&ctx->c, a, ctx->ev_fork, ctx->ev_join, H->m, psi->m, phi->m,
                  cplx(-dt_imag, -dt_real), tol, mmax);
    });
}

ftd_status ftd_apply_compress(ftd_ctx* ctx, const ftd_mpo* O, const ftd_mps* psi, int32_t D,
                              double cutoff, ftd_mps** out) {
    return guarded([&] {
        FTD_CHECK(ctx && O && psi && out, FTD_EINVAL, "null argument");
        FTD_CHECK(D >= 1, FTD_EINVAL, "D must be >= 1");
        FTD_CHECK(O->m->L == psi->m->L, FTD_EINVAL, "MPO and MPS lengths differ");
        Mps* r = apply_compress(&ctx->c, O->m, psi->m, D, cutoff);
        r->prec = psi->m->prec;
        *out = mps_handle(r);
    });
}

ftd_status ftd_pc_stage(ftd_ctx* ctx, const ftd_mps* psi, const ftd_mpo* O, const ftd_mps* phi,
                        const double* c, int32_t D, double cutoff, ftd_mps** out) {
    return guarded([&] {
        FTD_CHECK(ctx && psi && O && phi && c && out, FTD_EINVAL, "null argument");
        FTD_CHECK(D >= 1, FTD_EINVAL, "D must be >= 1");
        Mps* r = pc_stage(&ctx->c, psi->m, O->m, phi->m, cplx(c[0], c[1]), D, cutoff);
        *out = mps_handle(r);
    });
}

ftd_status ftd_overlap(ftd_ctx* ctx, const ftd_mps* bra, const ftd_mpo* O, const ftd_mps* ket,
                       double* out) {
    return guarded([&] {
        FTD_CHECK(ctx && bra && O && ket && out, FTD_EINVAL, "null argument");
        cplx v = overlap(&ctx->c, bra->m, O->m, ket->m);
        out[0] = v.real();
        out[1] = v.imag();
    });
}

ftd_status ftd_corr_current(ftd_ctx* ctx, const ftd_mpo* H, const ftd_mpo* J,
                            const ftd_mps* psi_beta, int32_t D, double cutoff, double dt,
                            int32_t n_steps, const ftd_krylov_opts* ko, double* C_out) {
    return guarded([&] {
        FTD_CHECK(ctx && H && J && psi_beta && C_out, FTD_EINVAL, "null argument");
        FTD_CHECK(n_steps >= 0 && D >= 1 && std::isfinite(dt), FTD_EINVAL, "bad run arguments");
        double tol;
        int mmax;
        check_krylov(ko, tol, mmax);
        Ctx* c = &ctx->c;
        Mps* psi = mps_clone(psi_beta->m);
        Mps* phi = nullptr;
        try {
            const double t_start = wall_seconds();
            psi->log_norm = 0.0;
            phi = apply_compress(c, J->m, psi, D, cutoff);
            vlog(c, 1, "corr: j|psi> compressed, %.2f s", wall_seconds() - t_start);
            phi->prec = psi->prec;
            phi->log_norm = 0.0;
            cplx c0 = overlap(c, psi, J->m, phi);
            C_out[0] = c0.real();
            C_out[1] = c0.imag();
            Ctx* a = n_steps > 0 ? aux_ctx(ctx) : nullptr;
            for (int k = 1; k <= n_steps; ++k) {
                tdvp_pair(c, a, ctx->ev_fork, ctx->ev_join, H->m, psi, phi, cplx(0.0, -dt), tol,
                          mmax);
                cplx ck = overlap(c, psi, J->m, phi);
                C_out[2 * k] = ck.real();
                C_out[2 * k + 1] = ck.imag();
                vlog(c, 1, "corr step %d/%d: %.2f s", k, n_steps, wall_seconds() - t_start);
            }
        } catch (...) {
            mps_free(psi);
            mps_free(phi);
            throw;
        }
        mps_free(psi);
        mps_free(phi);
    });
}

ftd_status ftd_mobility(const double* C, int32_t n, double dt, double beta, double e0,
                        double* mu_au, double* mu_cm2Vs) {
    return guarded([&] {
        FTD_CHECK(C && mu_au && mu_cm2Vs, FTD_EINVAL, "null argument");
        FTD_CHECK(n >= 2, FTD_EINVAL, "need at least two samples");
        FTD_CHECK(dt > 0.0 && beta >= 0.0 && e0 != 0.0, FTD_EINVAL, "bad dt, beta or e0");
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
            const double w = (k == 0 || k == n - 1) ? 0.5 : 1.0;
            s += w * C[2 * k];
        }
        const double mu = beta / e0 * dt * s;
        // e a0^2 / hbar in cm^2/(V s), CODATA 2018
        const double e = 1.602176634e-19, a0 = 5.29177210903e-11, hbar = 1.054571817e-34;
        *mu_au = mu;
        *mu_cm2Vs = mu * e * a0 * a0 / hbar * 1e4;
    });
}

// the entry points below report through the same thread-local message
static void call(ftd_status st) {
    if (st != FTD_OK) throw Error{st, g_last_error};
}

// One mobility run of model m at beta: MPOs, Psi_beta, C(t), mu (a.u.).
static double run_mobility(ftd_ctx* ctx, const ftd_model& m, double beta, int32_t n_imag,
                           int32_t n_grow, int32_t D, double cutoff, double dt, int32_t n_steps,
                           ftd_precision prec, const ftd_krylov_opts* ko, double* log_Z) {
    ftd_mpo* H = nullptr;
    ftd_mpo* J = nullptr;
    ftd_mps* psi = nullptr;
    std::vector<double> C(2 * ((size_t)n_steps + 1));
    auto release = [&] {
        if (psi) ftd_mps_destroy(psi);
        if (J) ftd_mpo_destroy(J);
        if (H) ftd_mpo_destroy(H);
    };
    double mu = 0.0, mu_cm = 0.0, lz = 0.0;
    try {
        call(ftd_mpo_build(ctx, &m, &H, &J));
        call(ftd_thermal_prep(ctx, H, beta, n_imag, n_grow, D, cutoff, 0.0, prec, ko, &psi, &lz));
        call(ftd_corr_current(ctx, H, J, psi, D, cutoff, dt, n_steps, ko, C.data()));
        call(ftd_mobility(C.data(), n_steps + 1, dt, beta, m.e0, &mu, &mu_cm));
    } catch (...) {
        release();
        throw;
    }
    release();
    if (log_Z) *log_Z = lz;
    return mu;
}

ftd_status ftd_mobility_sweep(ftd_ctx* ctx, const ftd_model* base, const ftd_sweep_point* pts,
                              int32_t n_pts, int32_t n_imag, int32_t n_grow, int32_t D,
                              double cutoff, double dt, int32_t n_steps, ftd_precision prec,
                              const ftd_krylov_opts* ko, double* mu_au, double* log_Z) {
    return guarded([&] {
        FTD_CHECK(ctx && base && pts && mu_au && log_Z, FTD_EINVAL, "null argument");
        FTD_CHECK(n_pts >= 1 && n_steps >= 1, FTD_EINVAL, "need n_pts >= 1 and n_steps >= 1");
        check_model(base);
        for (int p = 0; p < n_pts; ++p) {
            const ftd_sweep_point& q = pts[p];
            FTD_CHECK(std::isfinite(q.beta) && q.beta > 0.0 && std::isfinite(q.V) &&
                          std::isfinite(q.omega_scale) && q.omega_scale > 0.0,
                      FTD_EINVAL, "sweep point needs beta > 0, finite V and omega_scale > 0");
        }
        for (int p = 0; p < n_pts; ++p) {
            const ftd_sweep_point& q = pts[p];
            const double s = q.omega_scale, r = 1.0 / std::sqrt(s);
            std::vector<double> wl(base->n_loc), gl(base->n_loc), wn(base->n_nl), gn(base->n_nl);
            for (int i = 0; i < base->n_loc; ++i) {
                wl[i] = s * base->omega_loc[i];
                gl[i] = r * base->g_loc[i];
            }
            for (int i = 0; i < base->n_nl; ++i) {
                wn[i] = s * base->omega_nl[i];
                gn[i] = r * base->g_nl[i];
            }
            ftd_model m = *base;
            m.omega_loc = wl.data();
            m.g_loc = gl.data();
            m.omega_nl = wn.data();
            m.g_nl = gn.data();
            m.V = q.V;
            mu_au[p] = run_mobility(ctx, m, q.beta, n_imag, n_grow, D, cutoff, dt, n_steps, prec,
                                    ko, &log_Z[p]);
            vlog(&ctx->c, 1, "sweep point %d/%d: beta %.6g, V %.6g, s %.6g: mu %.9g a.u.", p + 1,
                 n_pts, q.beta, q.V, s, mu_au[p]);
        }
    });
}

ftd_status ftd_mobility_grad(ftd_ctx* ctx, const ftd_model* model, double beta, int32_t n_imag,
                             int32_t n_grow, int32_t D, double cutoff, double dt,
                             int32_t n_steps, ftd_precision prec, const ftd_krylov_opts* ko,
                             double rel_step, double* mu, double* dmu_domega_loc,
                             double* dmu_dg_loc, double* dmu_domega_nl, double* dmu_dg_nl) {
    return guarded([&] {
        FTD_CHECK(ctx && model && mu, FTD_EINVAL, "null argument");
        FTD_CHECK(std::isfinite(beta) && beta > 0.0 && n_steps >= 1, FTD_EINVAL,
                  "need beta > 0 and n_steps >= 1");
        FTD_CHECK(std::isfinite(rel_step) && rel_step > 0.0 && rel_step < 0.1, FTD_EINVAL,
                  "rel_step must lie in (0, 0.1)");
        check_model(model);
        FTD_CHECK((model->n_loc == 0 || (dmu_domega_loc && dmu_dg_loc)) &&
                      (model->n_nl == 0 || (dmu_domega_nl && dmu_dg_nl)),
                  FTD_EINVAL, "null gradient array");
        std::vector<double> wl(model->omega_loc, model->omega_loc + model->n_loc);
        std::vector<double> gl(model->g_loc, model->g_loc + model->n_loc);
        std::vector<double> wn(model->omega_nl, model->omega_nl + model->n_nl);
        std::vector<double> gn(model->g_nl, model->g_nl + model->n_nl);
        ftd_model m = *model;
        m.omega_loc = wl.data();
        m.g_loc = gl.data();
        m.omega_nl = wn.data();
        m.g_nl = gn.data();
        auto run = [&] {
            return run_mobility(ctx, m, beta, n_imag, n_grow, D, cutoff, dt, n_steps, prec, ko,
                                nullptr);
        };
        *mu = run();
        // central difference in one parameter; step rel_step |x|, or rel_step
        // itself for a parameter that is zero
        auto central = [&](double& x) {
            const double x0 = x, h = rel_step * (x0 != 0.0 ? std::fabs(x0) : 1.0);
            x = x0 + h;
            const double up = run();
            x = x0 - h;
            const double dn = run();
            x = x0;
            return (up - dn) / (2.0 * h);
        };
        for (int i = 0; i < model->n_loc; ++i) {
            dmu_domega_loc[i] = central(wl[i]);
            dmu_dg_loc[i] = central(gl[i]);
        }
        for (int i = 0; i < model->n_nl; ++i) {
            dmu_domega_nl[i] = central(wn[i]);
            dmu_dg_nl[i] = central(gn[i]);
        }
    });
}

ftd_status ftd_reduced_density(ftd_ctx* ctx, const ftd_model* m, const ftd_mps* psi,
                               double* sigma) {
    return guarded([&] {
        FTD_CHECK(ctx && m && psi && sigma, FTD_EINVAL, "null argument");
        check_model(m);
        reduced_density(&ctx->c, *m, psi->m, sigma);
    });
}

ftd_status ftd_coherent_length(const double* sigma, int32_t n, double* L) {
    return guarded([&] {
        FTD_CHECK(sigma && L, FTD_EINVAL, "null argument");
        FTD_CHECK(n >= 1, FTD_EINVAL, "n must be >= 1");
        double s1 = 0.0, s2 = 0.0;
        for (int64_t k = 0; k < (int64_t)n * n; ++k) {
            const double a = std::hypot(sigma[2 * k], sigma[2 * k + 1]);
            FTD_CHECK(std::isfinite(a), FTD_EINVAL, "non-finite sigma");
            s1 += a;
            s2 += a * a;
        }
        FTD_CHECK(s2 > 0.0, FTD_EINVAL, "sigma is zero");
        *L = s1 * s1 / ((double)n * s2);
    });
}

ftd_status ftd_mean_free_path(const double* C, int32_t n, double dt, double e0, double* l_mfp,
                              double* v, double* tau) {
    return guarded([&] {
        FTD_CHECK(C && l_mfp && v && tau, FTD_EINVAL, "null argument");
        FTD_CHECK(n >= 2, FTD_EINVAL, "need at least two samples");
        FTD_CHECK(dt > 0.0 && e0 != 0.0 && std::isfinite(dt), FTD_EINVAL, "bad dt or e0");
        const double c0 = C[0];
        FTD_CHECK(c0 > 0.0 && std::isfinite(c0), FTD_EINVAL, "Re C(0) must be positive");
        // tau = (1/2) int_{-inf}^{inf} |Re C / Re C(0)| dt = int_0^tmax (Re C even)
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
            const double w = (k == 0 || k == n - 1) ? 0.5 : 1.0;
            s += w * std::fabs(C[2 * k] / c0);
        }
        *tau = dt * s;
        *v = std::sqrt(c0) / std::fabs(e0);
        *l_mfp = *v * *tau;
    });
}

ftd_status ftd_fgr_corr(const double* t, int32_t nt, const double* omega, const double* g,
                        int32_t n_modes, double V, double beta, double e0, double R,
                        double* C_out) {
    return guarded([&] {
        FTD_CHECK(t && C_out && (n_modes == 0 || (omega && g)), FTD_EINVAL, "null argument");
        FTD_CHECK(nt >= 0 && n_modes >= 0, FTD_EINVAL, "bad sizes");
        // finite temperature only: the occupations diverge at beta = 0
        FTD_CHECK(beta > 0.0 && std::isfinite(beta), FTD_EINVAL, "beta must be positive");
        std::vector<double> nb(n_modes);
        for (int m = 0; m < n_modes; ++m) {
            FTD_CHECK(omega[m] > 0.0 && std::isfinite(omega[m]) && std::isfinite(g[m]), FTD_EINVAL,
                      "mode frequencies must be positive and finite");
            const double x = beta * omega[m];
            nb[m] = x < 700.0 ? 1.0 / std::expm1(x) : 0.0;   // Bose occupation
        }
        const double pre = 2.0 * (e0 * R * V) * (e0 * R * V);
        for (int k = 0; k < nt; ++k) {
            // exponent sum_m 2 g^2 [(2n+1) - (n+1) e^{-i w t} - n e^{i w t}]
            double er = 0.0, ei = 0.0;
            for (int m = 0; m < n_modes; ++m) {
                const double wt = omega[m] * t[k], c = std::cos(wt), sn = std::sin(wt);
                const double g2 = 2.0 * g[m] * g[m];
                er += g2 * ((2.0 * nb[m] + 1.0) - (2.0 * nb[m] + 1.0) * c);
                ei += g2 * ((nb[m] + 1.0) * sn - nb[m] * sn);
            }
            const double mag = pre * std::exp(-er);
            C_out[2 * k] = mag * std::cos(-ei);
            C_out[2 * k + 1] = mag * std::sin(-ei);
        }
    });
}

ftd_status ftd_heff_apply(ftd_ctx* ctx, const ftd_mpo* H, const ftd_mps* psi, int32_t site,
                          const double* x, double* y, int32_t n_repeat) {
    return guarded([&] {
        FTD_CHECK(ctx && H && psi && x && y, FTD_EINVAL, "null argument");
        heff_apply_host(&ctx->c, H->m, psi->m, site, x, y, n_repeat);
    });
}

ftd_status ftd_heff_expm(ftd_ctx* ctx, const ftd_mpo* H, const ftd_mps* psi, int32_t site,
                         const double* x, double* y, double zr, double zi,
                         const ftd_krylov_opts* ko, int32_t n_repeat, int32_t* m_out) {
    return guarded([&] {
        FTD_CHECK(ctx && H && psi && x && y, FTD_EINVAL, "null argument");
        FTD_CHECK(std::isfinite(zr) && std::isfinite(zi), FTD_EINVAL, "non-finite z");
        double tol;
        int mmax;
        check_krylov(ko, tol, mmax);
        const int m = heff_expm_host(&ctx->c, H->m, psi->m, site, x, y, cplx(zr, zi), tol, mmax,
                                     n_repeat);
        if (m_out) *m_out = m;
    });
}

ftd_status ftd_svd_trunc(ftd_ctx* ctx, int32_t M, int32_t N, const double* T, int32_t D,
                         double cutoff, int32_t s_left, double* L, double* R, int32_t* kout) {
    return guarded([&] {
        FTD_CHECK(ctx && T && L && R && kout, FTD_EINVAL, "null argument");
        FTD_CHECK(M >= 1 && N >= 1 && D >= 1, FTD_EINVAL, "bad sizes");
        Ctx* c = &ctx->c;
        const int64_t n = (int64_t)M * N;
        double* dT = static_cast<double*>(dev_alloc(c, sizeof(double) * 2 * n));
        std::vector<double> t(2 * n);
        for (int64_t i = 0; i < n; ++i) {
            t[i] = T[2 * i];
            t[i + n] = T[2 * i + 1];
        }
        FTD_HIP(hipMemcpy(dT, t.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice));
        TruncOut o = svd_trunc(c, dT, M, N, D, cutoff, s_left != 0);
        const int k = o.k;
        auto down = [&](const double* d, int64_t cnt, double* h) {
            std::vector<double> b(2 * cnt);
            FTD_HIP(hipMemcpy(b.data(), d, sizeof(double) * 2 * cnt, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < cnt; ++i) {
                h[2 * i] = b[i];
                h[2 * i + 1] = b[i + cnt];
            }
        };
        down(o.Lq, (int64_t)M * k, L);
        down(o.Rq, (int64_t)k * N, R);
        dev_free(c, dT);
        dev_free(c, o.Lq);
        dev_free(c, o.Rq);
        *kout = k;
    });
}

ftd_status ftd_qr(ftd_ctx* ctx, int32_t rows, int32_t cols, const double* M, int32_t lq,
                  double* Q, double* F) {
    return guarded([&] {
        FTD_CHECK(ctx && M && Q && F, FTD_EINVAL, "null argument");
        FTD_CHECK(rows >= 1 && cols >= 1, FTD_EINVAL, "bad sizes");
        FTD_CHECK(lq ? rows <= cols : rows >= cols, FTD_EINVAL,
                  lq ? "ftd_qr: LQ needs rows <= cols" : "ftd_qr: QR needs rows >= cols");
        Ctx* c = &ctx->c;
        const int64_t n = (int64_t)rows * cols;
        const int64_t k = lq ? rows : cols;
        double* dM = static_cast<double*>(dev_alloc(c, sizeof(double) * 2 * n));
        double* dF = static_cast<double*>(dev_alloc(c, sizeof(double) * 2 * k * k));
        try {
            std::vector<double> t(2 * n);
            for (int64_t i = 0; i < n; ++i) {
                t[i] = M[2 * i];
                t[i + n] = M[2 * i + 1];
            }
            FTD_HIP(hipMemcpy(dM, t.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice));
            if (lq)
                lq_chol(c, dM, rows, cols, dF, true);
            else
                qr_chol(c, dM, rows, cols, dF, true);
            auto down = [&](const double* d, int64_t cnt, double* h) {
                std::vector<double> b(2 * cnt);
                FTD_HIP(hipMemcpy(b.data(), d, sizeof(double) * 2 * cnt, hipMemcpyDeviceToHost));
                for (int64_t i = 0; i < cnt; ++i) {
                    h[2 * i] = b[i];
                    h[2 * i + 1] = b[i + cnt];
                }
            };
            down(dM, n, Q);
            down(dF, k * k, F);
        } catch (...) {
            dev_free(c, dM);
            dev_free(c, dF);
            throw;
        }
        dev_free(c, dM);
        dev_free(c, dF);
    });
}

ftd_status ftd_gemm(ftd_ctx* ctx, int32_t precision, int32_t M, int32_t N, int32_t K,
                    int32_t transA, int32_t transB, const double* A, const double* B, double* C) {
    return guarded([&] {
        FTD_CHECK(ctx && A && B && C, FTD_EINVAL, "null argument");
        FTD_CHECK(M >= 1 && N >= 1 && K >= 1, FTD_EINVAL, "empty GEMM");
        FTD_CHECK(transA >= 0 && transA <= 2 && transB >= 0 && transB <= 2, FTD_EINVAL, "bad trans");
        const Prec pr = to_prec(precision);
        Ctx* c = &ctx->c;
        const int64_t na = (int64_t)M * K, nb = (int64_t)K * N, nc = (int64_t)M * N;
        const size_t es = pr == Prec::F64 ? 8 : 4;
        void* dA = dev_alloc(c, es * 2 * na);
        void* dB = dev_alloc(c, es * 2 * nb);
        double* dC = static_cast<double*>(dev_alloc(c, 8 * 2 * nc));
        auto up = [&](const double* h, void* d, int64_t n) {
            if (pr == Prec::F64) {
                std::vector<double> t(2 * n);
                for (int64_t k = 0; k < n; ++k) {
                    t[k] = h[2 * k];
                    t[k + n] = h[2 * k + 1];
                }
                FTD_HIP(hipMemcpy(d, t.data(), 8 * 2 * n, hipMemcpyHostToDevice));
            } else {
                std::vector<float> t(2 * n);
                for (int64_t k = 0; k < n; ++k) {
                    t[k] = (float)h[2 * k];
                    t[k + n] = (float)h[2 * k + 1];
                }
                FTD_HIP(hipMemcpy(d, t.data(), 4 * 2 * n, hipMemcpyHostToDevice));
            }
        };
        up(A, dA, na);
        up(B, dB, nb);
        GemmParams p{};
        p.M = M; p.N = N; p.K = K;
        if (transA == 0) { p.sAm = K; p.sAk = 1; p.a_kcontig = 1; }
        else { p.sAm = 1; p.sAk = M; p.a_kcontig = 0; p.conjA = transA == 2; }
        if (transB == 0) { p.sBk = N; p.sBn = 1; p.b_kcontig = 0; }
        else { p.sBk = 1; p.sBn = K; p.b_kcontig = 1; p.conjB = transB == 2; }
        p.planeA = na; p.planeB = nb;
        p.sCm = N; p.sCn = 1; p.planeC = nc;
        p.nprob = 1; p.prob[0].t1 = 1;
        gemm(c, pr, true, dA, dB, dC, p, TAG_NONE);
        std::vector<double> t(2 * nc);
        FTD_HIP(hipMemcpyAsync(t.data(), dC, 8 * 2 * nc, hipMemcpyDeviceToHost, c->stream));
        FTD_HIP(hipStreamSynchronize(c->stream));
        for (int64_t k = 0; k < nc; ++k) {
            C[2 * k] = t[k];
            C[2 * k + 1] = t[k + nc];
        }
        dev_free(c, dA);
        dev_free(c, dB);
        dev_free(c, dC);
    });
}

}  // extern "C"
