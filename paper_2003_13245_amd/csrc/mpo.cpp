// Matrix-product operators of the Hamiltonian and of the current.
//
// Channel automaton (finite-state construction).  A channel is the state of an
// operator string as it is read from left to right along the chain:
//   I    nothing placed yet
//   F    a complete term has been placed
//   P    c+_n c_n placed on e_n, waiting for the displacement x of one of
//        molecule n's local modes (Holstein term of Eq. (1))
//   A    c_n placed on e_n, waiting for c+_{n+1}   (hop n -> n+1)
//   C    c+_n placed on e_n, waiting for c_{n+1}   (hop n+1 -> n)
//   A2,C2  the same after a Peierls displacement x of a bond mode of
//        (n, n+1) was placed (Holstein-Peierls coupling)
//   WA,WC  the periodic hop across the wrap bond, opened on e_0
//   W2   the wrap hop closed on e_{N-1}, waiting for a wrap-bond mode's x
// The transfer factor V + sum_m g2_m w_m x_m is a sum, so the V path closes
// directly (A -> F with V) while each bond mode moves A to A2.  With one
// carrier the Jordan-Wigner strings are +1, so c+ c pairs map onto hard-core
// sigma+ sigma- (also across the wrap bond).
//
// For j the same automaton without the on-site and Holstein terms, with hop
// coefficients -i e0 R (carrier moves n -> n+1) and +i e0 R (n+1 -> n).
#include <algorithm>
#include <map>

#include "common.h"

namespace ftd {

enum Chan { CH_I = 0, CH_P, CH_A, CH_C, CH_A2, CH_C2, CH_WA, CH_WC, CH_W2, CH_F, CH_N };

namespace {

struct SiteDesc {
    int kind;   // 0 electron, 1 local mode, 2 bond mode
    int mol, mode;
};

std::vector<cplx> op_identity(int d) {
    std::vector<cplx> o(d * d, 0.0);
    for (int i = 0; i < d; ++i) o[i * d + i] = 1.0;
    return o;
}
std::vector<cplx> op_number(int d) {   // b+ b
    std::vector<cplx> o(d * d, 0.0);
    for (int i = 0; i < d; ++i) o[i * d + i] = (double)i;
    return o;
}
std::vector<cplx> op_disp(int d) {     // b + b+
    std::vector<cplx> o(d * d, 0.0);
    for (int v = 1; v < d; ++v) {
        o[(v - 1) * d + v] = std::sqrt((double)v);
        o[v * d + (v - 1)] = std::sqrt((double)v);
    }
    return o;
}
// electron basis |0> empty, |1> occupied; [out][in]
std::vector<cplx> op_sp() { return {0.0, 0.0, 1.0, 0.0}; }   // |1><0|
std::vector<cplx> op_sm() { return {0.0, 1.0, 0.0, 0.0}; }   // |0><1|
std::vector<cplx> op_n() { return {0.0, 0.0, 0.0, 1.0}; }

std::vector<cplx> scaled(std::vector<cplx> o, cplx c) {
    for (auto& x : o) x *= c;
    return o;
}

}  // namespace

Mpo* build_mpo(Ctx* ctx, const ftd_model& md, bool current) {
    const int N = md.n_mol, ML = md.n_loc, MN = md.n_nl;
    const bool per = md.periodic != 0;
    // chain layout
    std::vector<SiteDesc> sites;
    std::vector<int> epos(N);
    for (int n = 0; n < N; ++n) {
        epos[n] = (int)sites.size();
        sites.push_back({0, n, -1});
        for (int m = 0; m < ML; ++m) sites.push_back({1, n, m});
        if (per || n < N - 1)
            for (int m = 0; m < MN; ++m) sites.push_back({2, n, m});
    }
    const int L = (int)sites.size();
    const cplx fwd = current ? cplx(0.0, -md.e0 * md.R) : cplx(1.0, 0.0);
    const cplx bwd = current ? cplx(0.0, md.e0 * md.R) : cplx(1.0, 0.0);
    const bool hterms = !current;

    // activity of channels on the bond to the right of site s
    auto active = [&](int s, int ch) -> bool {
        if (s >= L - 1) return ch == CH_F;
        const SiteDesc& sd = sites[s];
        const int n = sd.mol;
        switch (ch) {
            case CH_I: return true;
            case CH_F: return true;
            case CH_P:
                if (!hterms || ML == 0) return false;
                if (sd.kind == 0) return true;
                return sd.kind == 1 && sd.mode < ML - 1;
            case CH_A:
            case CH_C:
                // open from e_n up to the site before e_{n+1}, n < N-1
                return n < N - 1;
            case CH_A2:
            case CH_C2:
                return n < N - 1 && sd.kind == 2;
            case CH_WA:
            case CH_WC:
                // from e_0 up to the site before e_{N-1}
                return per && s < epos[N - 1];
            case CH_W2:
                if (!per || MN == 0 || n != N - 1) return false;
                if (sd.kind == 0 || sd.kind == 1) return true;
                return sd.mode < MN - 1;
        }
        return false;
    };

    Mpo* mpo = new Mpo();
    mpo->ctx = ctx;
    mpo->L = L;
    mpo->s.resize(L);
    mpo->electronic.resize(L);
    for (int i = 0; i < L; ++i) mpo->electronic[i] = sites[i].kind == 0 ? 1 : 0;
    // channel lists per bond (bond b = right of site b; bond -1 = left edge)
    auto chans = [&](int b) {
        std::vector<int> out;
        if (b < 0) {
            out.push_back(CH_I);
            return out;
        }
        const int order[CH_N] = {CH_I, CH_P, CH_A, CH_C, CH_A2, CH_C2, CH_WA, CH_WC, CH_W2, CH_F};
        for (int c : order)
            if (active(b, c)) out.push_back(c);
        return out;
    };

    for (int s = 0; s < L; ++s) {
        const SiteDesc& sd = sites[s];
        const int d = sd.kind == 0 ? 2 : (sd.kind == 1 ? md.levels_loc : md.levels_nl);
        const std::vector<int> cl = chans(s - 1), cr = chans(s);
        std::map<int, int> il, ir;
        for (size_t i = 0; i < cl.size(); ++i) il[cl[i]] = (int)i;
        for (size_t i = 0; i < cr.size(); ++i) ir[cr[i]] = (int)i;
        MpoSite& S = mpo->s[s];
        S.d = d;
        S.wl = (int)cl.size();
        S.wr = (int)cr.size();
        S.idxI_l = il.count(CH_I) ? il[CH_I] : -1;
        S.idxF_l = il.count(CH_F) ? il[CH_F] : -1;
        S.idxI_r = ir.count(CH_I) ? ir[CH_I] : -1;
        S.idxF_r = ir.count(CH_F) ? ir[CH_F] : -1;
        auto add = [&](int a, int b, std::vector<cplx> op, bool ident) {
            if (!il.count(a) || !ir.count(b)) return;
            MpoEntry e;
            e.cl = il[a];
            e.cr = ir[b];
            e.identity = ident;
            e.op = std::move(op);
            S.ents.push_back(std::move(e));
        };
        const std::vector<cplx> id = op_identity(d);
        add(CH_I, CH_I, id, true);
        add(CH_F, CH_F, id, true);
        const int n = sd.mol;
        if (sd.kind == 0) {
            // close the hop of bond (n-1, n)
            if (n >= 1) {
                add(CH_A, CH_F, scaled(op_sp(), md.V), false);
                add(CH_A2, CH_F, op_sp(), false);
                add(CH_C, CH_F, scaled(op_sm(), md.V), false);
                add(CH_C2, CH_F, op_sm(), false);
            }
            // open the hop of bond (n, n+1)
            if (n < N - 1) {
                add(CH_I, CH_A, scaled(op_sm(), fwd), false);
                add(CH_I, CH_C, scaled(op_sp(), bwd), false);
            }
            if (hterms && ML > 0) add(CH_I, CH_P, op_n(), false);
            if (per) {
                if (n == 0) {
                    // c+_0 c_{N-1} (carrier N-1 -> 0, forward) and c+_{N-1} c_0
                    add(CH_I, CH_WA, scaled(op_sp(), fwd), false);
                    add(CH_I, CH_WC, scaled(op_sm(), bwd), false);
                } else if (n == N - 1) {
                    add(CH_WA, CH_F, scaled(op_sm(), md.V), false);
                    add(CH_WC, CH_F, scaled(op_sp(), md.V), false);
                    if (MN > 0) {
                        add(CH_WA, CH_W2, op_sm(), false);
                        add(CH_WC, CH_W2, op_sp(), false);
                    }
                } else {
                    add(CH_WA, CH_WA, id, true);
                    add(CH_WC, CH_WC, id, true);
                }
            }
        } else {
            const double w = sd.kind == 1 ? md.omega_loc[sd.mode] : md.omega_nl[sd.mode];
            if (hterms) add(CH_I, CH_F, scaled(op_number(d), w), false);
            add(CH_WA, CH_WA, id, true);
            add(CH_WC, CH_WC, id, true);
            add(CH_W2, CH_W2, id, true);
            if (sd.kind == 1) {
                if (hterms) {
                    add(CH_P, CH_F, scaled(op_disp(d), md.g_loc[sd.mode] * w), false);
                    add(CH_P, CH_P, id, true);
                }
                add(CH_A, CH_A, id, true);
                add(CH_C, CH_C, id, true);
            } else {
                const double gw = md.g_nl[sd.mode] * w;
                if (n < N - 1) {
                    add(CH_A, CH_A, id, true);
                    add(CH_C, CH_C, id, true);
                    add(CH_A, CH_A2, scaled(op_disp(d), gw), false);
                    add(CH_C, CH_C2, scaled(op_disp(d), gw), false);
                    add(CH_A2, CH_A2, id, true);
                    add(CH_C2, CH_C2, id, true);
                } else {
                    add(CH_W2, CH_F, scaled(op_disp(d), gw), false);
                }
            }
        }
        mpo->wmax = std::max(mpo->wmax, std::max(S.wl, S.wr));
        mpo->dmax = std::max(mpo->dmax, d);
    }
    return mpo;
}

// Bond-dimension-1 MPO of a product of local operators, all identities as
// built: the chain layout of build_mpo, one channel per bond.  Entries on
// carrier sites are flagged non-identity so that their device op tables,
// which the caller overwrites (e.g. with sigma- and sigma+ for c+_j c_i), are
// always applied.  carrier[n] receives the chain position of e_n.
Mpo* build_product_mpo(Ctx* ctx, const ftd_model& md, std::vector<int>& carrier) {
    const int N = md.n_mol, ML = md.n_loc, MN = md.n_nl;
    const bool per = md.periodic != 0;
    std::vector<int> dims;
    carrier.assign(N, -1);
    for (int n = 0; n < N; ++n) {
        carrier[n] = (int)dims.size();
        dims.push_back(2);
        for (int m = 0; m < ML; ++m) dims.push_back(md.levels_loc);
        if (per || n < N - 1)
            for (int m = 0; m < MN; ++m) dims.push_back(md.levels_nl);
    }
    Mpo* mpo = new Mpo();
    mpo->ctx = ctx;
    mpo->L = (int)dims.size();
    mpo->s.resize(mpo->L);
    mpo->electronic.assign(mpo->L, 0);
    for (int n = 0; n < N; ++n) mpo->electronic[carrier[n]] = 1;
    for (int s = 0; s < mpo->L; ++s) {
        MpoSite& S = mpo->s[s];
        S.d = dims[s];
        S.wl = S.wr = 1;
        // no I/F channel semantics: never used to build environments
        S.idxI_l = S.idxF_l = S.idxI_r = S.idxF_r = -1;
        MpoEntry e;
        e.cl = e.cr = 0;
        e.identity = !mpo->electronic[s];
        e.op = op_identity(S.d);
        S.ents.push_back(std::move(e));
        mpo->wmax = std::max(mpo->wmax, 1);
        mpo->dmax = std::max(mpo->dmax, S.d);
    }
    return mpo;
}

void upload_mpo(Ctx* ctx, Mpo* mpo) {
    for (auto& S : mpo->s) {
        const int d = S.d;
        const size_t ne = S.ents.size();
        std::vector<double> h64(2 * d * d * ne);
        std::vector<float> h32(2 * d * d * ne);
        std::vector<ApplyEnt> ae(ne);
        for (size_t e = 0; e < ne; ++e) {
            for (int k = 0; k < d * d; ++k) {
                h64[e * 2 * d * d + k] = S.ents[e].op[k].real();
                h64[e * 2 * d * d + d * d + k] = S.ents[e].op[k].imag();
            }
            ae[e] = {S.ents[e].cl, S.ents[e].cr, (int)e};
        }
        for (size_t k = 0; k < h64.size(); ++k) h32[k] = (float)h64[k];
        S.ops64 = static_cast<double*>(dev_alloc(ctx, sizeof(double) * std::max<size_t>(1, h64.size())));
        S.ops32 = static_cast<float*>(dev_alloc(ctx, sizeof(float) * std::max<size_t>(1, h32.size())));
        S.apply_ents = static_cast<ApplyEnt*>(dev_alloc(ctx, sizeof(ApplyEnt) * std::max<size_t>(1, ne)));
        if (ne) {
            FTD_HIP(hipMemcpy(S.ops64, h64.data(), sizeof(double) * h64.size(), hipMemcpyHostToDevice));
            FTD_HIP(hipMemcpy(S.ops32, h32.data(), sizeof(float) * h32.size(), hipMemcpyHostToDevice));
            FTD_HIP(hipMemcpy(S.apply_ents, ae.data(), sizeof(ApplyEnt) * ne, hipMemcpyHostToDevice));
        }
    }
}

void destroy_mpo(Mpo* mpo) {
    if (!mpo) return;
    for (auto& S : mpo->s) {
        dev_free(mpo->ctx, S.ops64);
        dev_free(mpo->ctx, S.ops32);
        dev_free(mpo->ctx, S.apply_ents);
    }
    delete mpo;
}

}  // namespace ftd
