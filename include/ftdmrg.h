/*
 * ftdmrg — finite-temperature TD-DMRG for carrier mobility on AMD MI355X (gfx950).
 *
 * C ABI of the hot path of the method of "Finite Temperature TD-DMRG for the
 * Carrier Mobility of Organic Semiconductors" (J. Phys. Chem. Lett. 2020):
 * a purified thermal state |Psi_beta> = exp(-beta H / 2)|I> is prepared by
 * imaginary-time evolution, |Psi_beta> and j|Psi_beta> are propagated in real
 * time with the one-site projector-splitting time-dependent variational
 * principle, and the current-current correlation
 *     C(t) = <Psi_beta| exp(iHt) j exp(-iHt) j |Psi_beta> / Z
 * is integrated by the Kubo formula into the mobility mu.
 *
 * Conventions (all calls):
 *   - Atomic units (hbar = e0 = k_B = 1 unless e0 is given).  Conversions from
 *     cm^-1, meV, K or fs happen in the caller.
 *   - Every call returns an ftd_status.  Outputs are unspecified when the
 *     status is not FTD_OK.  ftd_last_error() returns a thread-local message.
 *   - No exceptions cross the ABI.  Handles are not thread-safe: use one
 *     context per host thread.
 *   - Device work is enqueued on the context's HIP stream.  Calls that return
 *     host values (log Z, C(t), norms, statistics) synchronise that stream.
 *   - Complex numbers in host buffers are interleaved (re, im) doubles.
 */
#ifndef FTDMRG_H
#define FTDMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ftd_status;
#define FTD_OK 0
#define FTD_EINVAL 1     /* invalid argument (shape, range, non-finite value)  */
#define FTD_ENOMEM 2     /* device allocation failed                           */
#define FTD_EDEVICE 3    /* HIP runtime error                                  */
#define FTD_ENOCONV 4    /* Krylov exponential not converged / non-finite data */
#define FTD_ESTATE 5     /* handle in the wrong state (e.g. precision mismatch)*/

typedef enum {
    FTD_C128 = 0,        /* every contraction in complex float64               */
    FTD_C64 = 1,         /* contractions in complex float32 on MFMA, Krylov,
                            QR, norms and log Z in float64                     */
    FTD_BF16X3 = 2       /* contractions on bf16 matrix cores: every float32
                            operand split as hi + lo (two bf16), each real
                            product as hi*hi + hi*lo + lo*hi, float32
                            accumulation (relative error ~2^-17 per product);
                            Krylov, QR, norms and log Z in float64          */
} ftd_precision;

typedef struct ftd_ctx ftd_ctx;
typedef struct ftd_mpo ftd_mpo;
typedef struct ftd_mps ftd_mps;

/* Optional device allocator (e.g. a framework's caching allocator).
 * alloc returns NULL on failure. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} ftd_allocator;

/* The (Holstein-)Peierls chain: Eq. (1) of the paper, and the Holstein-Peierls
 * coupling of its closing section.  N molecules on a ring (periodic = 1) or an
 * open chain; each molecule carries n_loc local modes (frequency omega_loc[m],
 * dimensionless Holstein coupling g_loc[m]); each bond (n, n+1) carries n_nl
 * non-local modes (omega_nl[m], Peierls coupling g_nl[m]).  Each mode keeps
 * `levels` harmonic-oscillator number states.  One carrier.  V is the transfer
 * integral, R the inter-molecular distance and e0 the carrier charge, both of
 * which scale the current operator j = (e0 R / i) sum_n (V + sum_m g_nl[m]
 * omega_nl[m] x_{n,m}) (c+_{n+1} c_n - c+_n c_{n+1}).
 * Arrays are borrowed and copied during ftd_mpo_build. */
typedef struct {
    int32_t n_mol;
    int32_t n_loc;
    int32_t n_nl;
    int32_t periodic;
    int32_t levels_loc;
    int32_t levels_nl;
    const double* omega_loc;   /* [n_loc] */
    const double* g_loc;       /* [n_loc] */
    const double* omega_nl;    /* [n_nl]  */
    const double* g_nl;        /* [n_nl]  */
    double V;
    double R;
    double e0;
} ftd_model;

/* Krylov exponential settings: Lanczos with full reorthogonalisation (float64,
 * classical Gram-Schmidt; for tol above about 2e-14 the second pass runs only
 * when the first left at most 100 u / tol of the residual's norm, u = 2^-53,
 * so that one pass's orthogonality error stays below tol / 100), stopped when
 * beta_k |e_k^T exp(zT_k) e_1| <= tol |exp(zT_k) e_1| or when the Krylov
 * space is exhausted; more than mmax vectors -> FTD_ENOCONV. */
typedef struct {
    double tol;
    int32_t mmax;
} ftd_krylov_opts;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  `hip_stream` is a borrowed
 * hipStream_t (NULL = the null stream).  `alloc` may be NULL (hipMalloc).
 * ftd_ctx_destroy synchronises the stream and gives up the caller's
 * reference: every MPO and MPS handle made on the context holds one too, so
 * the context's memory is released when the last of them is destroyed, in
 * whatever order (the context itself may not be used after destroy). */
ftd_status ftd_ctx_create(int32_t device, void* hip_stream, const ftd_allocator* alloc,
                          ftd_ctx** out);
void ftd_ctx_destroy(ftd_ctx* ctx);
const char* ftd_last_error(void);

/* Kernel timing: when enabled, every launch of the effective-Hamiltonian
 * contraction kernels is bracketed by HIP events on the context stream.
 * ftd_ctx_stats synchronises and returns, for the contraction kernels of the
 * H_eff / K_eff matvecs since the last reset: number of launches, summed
 * kernel milliseconds and summed algorithmic flops (8 m n k per complex
 * product), each bracketed by events; the same for the single GEMM kernel
 * instance with the largest time share over all H_eff and K_eff launches
 * (dom_*; those matvecs share kernel instances), whose launches are timed on
 * the device (first block start to last block end, the kernel alone without
 * its split-K reduction); and over the whole context the number of matvecs
 * and Krylov vectors.  Statistics are reset by ftd_ctx_stats_reset. */
typedef struct {
    int64_t heff_launches;
    double heff_ms;
    double heff_flops;
    int64_t dom_launches;      /* the single kernel with the largest share */
    double dom_ms;
    double dom_flops;
    double dom_bytes;          /* algorithmic bytes of that kernel's operands */
    int64_t matvecs;
    int64_t krylov_vectors;
    int64_t expm_calls;
    int64_t krylov_max;
    int32_t dom_kind;          /* identity of that kernel: 8*precision (0 f64,
                                  1 f32, 2 bf16x3) + 4*(f64 output)
                                  + 2*(A k-contiguous) + (B k-contiguous) */
    double all_flops;          /* algorithmic flops (8 m n k per complex
                                  product) of every contraction launched,
                                  timed or not: matvecs, environments,
                                  overlaps, gauge and compression GEMMs */
    /* per kernel identity (index = dom_kind's encoding): the device-timed
     * H_eff / K_eff launches of that instance, as for dom_* */
    int64_t kind_launches[32];
    double kind_ms[32];
    double kind_flops[32];
    double kind_bytes[32];
} ftd_stats;
ftd_status ftd_ctx_set_timing(ftd_ctx* ctx, int32_t enable);
ftd_status ftd_ctx_stats(ftd_ctx* ctx, ftd_stats* out);
ftd_status ftd_ctx_stats_reset(ftd_ctx* ctx);
ftd_status ftd_ctx_synchronize(ftd_ctx* ctx);
/* Progress log on stderr: level 0 silent (default), 1 one line per
 * imaginary-time step of ftd_thermal_prep and per real-time step of
 * ftd_corr_current (wall seconds, largest bond), 2 also one line per
 * compression phase. */
ftd_status ftd_ctx_set_verbose(ftd_ctx* ctx, int32_t level);

/* ------------------------------------------------------------------- MPO */

/* Build the MPOs of H (Eq. (1) plus the Peierls term) and of the current j
 * (the operator written with the Kubo formula, generalised by the Peierls
 * factor).  Site order: e_0, the local modes of molecule 0, the bond modes of
 * bond (0,1), e_1, ...; the wrap-bond modes follow molecule N-1.
 * Errors: FTD_EINVAL for n_mol < 3 on a ring (the two hops of a 2-ring
 * coincide), n_mol < 2 open, levels < 1 where modes exist, non-finite
 * parameters.  H and J belong to the caller (ftd_mpo_destroy). */
ftd_status ftd_mpo_build(ftd_ctx* ctx, const ftd_model* model, ftd_mpo** H, ftd_mpo** J);
void ftd_mpo_destroy(ftd_mpo* mpo);
/* Number of sites, and per-site physical dimension d (host array, n_sites). */
ftd_status ftd_mpo_info(const ftd_mpo* mpo, int32_t* n_sites, int32_t* dims, int32_t* bond_w);

/* ------------------------------------------------------------------- MPS */

/* Purified MPS: site tensors A[a][p][q][b] (left bond, P leg, Q leg, right
 * bond), float64 complex on the device.  A scalar log-norm factor is kept
 * outside the tensors. */
void ftd_mps_destroy(ftd_mps* psi);
ftd_status ftd_mps_copy(ftd_ctx* ctx, const ftd_mps* src, ftd_mps** out);
/* bond_dims receives n_sites - 1 values. */
ftd_status ftd_mps_info(const ftd_mps* psi, int32_t* n_sites, int32_t* bond_dims,
                        double* log_norm, int32_t* precision);
/* Host copies of one site tensor, interleaved complex, row-major [a][p][q][b].
 * `count` is the number of complex elements the host buffer holds. */
ftd_status ftd_mps_get_site(ftd_ctx* ctx, const ftd_mps* psi, int32_t site, double* host,
                            int64_t count);
/* Build an MPS from host tensors: dims[4*i..4*i+3] = (Dl, d, d, Dr) of site i;
 * tensors concatenated in site order, interleaved complex. */
ftd_status ftd_mps_from_host(ftd_ctx* ctx, int32_t n_sites, const int32_t* dims,
                             const double* host, double log_norm, ftd_precision prec,
                             ftd_mps** out);
/* Select the arithmetic of the contractions applied to psi from now on
 * (site tensors stay float64).  Errors: FTD_EINVAL for an unknown precision. */
ftd_status ftd_mps_set_precision(ftd_mps* psi, ftd_precision prec);
/* <psi|psi> of the tensors (log_norm excluded), float64. */
ftd_status ftd_mps_norm(ftd_ctx* ctx, const ftd_mps* psi, double* out);
/* Overwrite site `site` of psi with host data of the same shape (count
 * complex elements, interleaved, row-major [a][p][q][b]); the shape must be
 * psi's (Dl, d, d, Dr) of that site.  For tests that plant a tensor.
 * Errors: FTD_EINVAL (site out of range, count != Dl d d Dr, non-finite). */
ftd_status ftd_mps_set_site(ftd_ctx* ctx, ftd_mps* psi, int32_t site, const double* host,
                            int64_t count);
/* Checkpoint and resume of a state, e.g. between two parts of a long C(t)
 * run.  The file holds the exact float64 tensors, the log-norm factor and the
 * contraction precision, so that continuing from a loaded state gives the
 * same bits as not stopping.  Layout (little-endian): 8 bytes "FTDMPS01",
 * int32 n_sites, int32 precision, double log_norm, int32 (Dl, d, d, Dr) per
 * site, then per site the real plane and the imaginary plane of the tensor,
 * each Dl*d*d*Dr doubles in [a][p][q][b] order.  save synchronises the
 * context stream; load returns a new state owned by the caller.
 * Errors: FTD_EINVAL (null path, file missing, short or malformed, bonds
 * that do not chain), FTD_EDEVICE (write failure), FTD_ENOMEM. */
ftd_status ftd_mps_save(ftd_ctx* ctx, const ftd_mps* psi, const char* path);
ftd_status ftd_mps_load(ftd_ctx* ctx, const char* path, ftd_mps** out);

/* ------------------------------------------------------- the hot path calls */

/* Imaginary-time preparation (purification section of the paper):
 * |Psi_beta> = exp(-beta H / 2)|I> from the purified identity |I> of the
 * one-carrier space, in n_imag steps of dtau = beta / (2 n_imag).  The first
 * n_grow steps are propagation-and-compression steps (fourth-order Taylor in
 * Horner form, each stage an exact MPO x MPS product compressed to at most D
 * singular values with s/s_max > cutoff); the remaining steps are one-site
 * TDVP sweeps, with the bond expansion of ftd_tdvp_step_expand up to D when
 * expand_tol > 0, each such step followed by an SVD truncation of the state
 * at the cutoff (imaginary time damps some added directions to zero weight);
 * expand_tol = 0: plain one-site sweeps, which keep the bonds the growth
 * left.  If n_grow < 0 the growth continues until every bond has reached
 * min(D, its maximal rank) or n_imag steps are used.
 * Output: the normalised state (right-canonical, centre on site 0; caller
 * owns it) and ln Z, Z = <Psi_beta|Psi_beta>.  Errors: FTD_EINVAL (beta < 0,
 * n_imag < 1, D < 1, expand_tol < 0 or >= 1), FTD_ENOCONV, FTD_ENOMEM. */
ftd_status ftd_thermal_prep(ftd_ctx* ctx, const ftd_mpo* H, double beta, int32_t n_imag,
                            int32_t n_grow, int32_t D, double cutoff, double expand_tol,
                            ftd_precision prec, const ftd_krylov_opts* ko, ftd_mps** psi_beta,
                            double* log_Z);

/* One second-order one-site TDVP projector-splitting step, in place:
 * psi <- exp(z H) psi with z = -i dt_real - dt_imag (real time: dt_imag = 0,
 * imaginary time: dt_real = 0).  psi must be right-canonical with its centre
 * on site 0 (as every call here leaves it).  Contractions run in psi's
 * precision.  Errors: FTD_ENOCONV (Krylov or non-finite), FTD_EINVAL. */
ftd_status ftd_tdvp_step(ftd_ctx* ctx, const ftd_mpo* H, ftd_mps* psi, double dt_real,
                         double dt_imag, const ftd_krylov_opts* ko);

/* One TDVP step as ftd_tdvp_step with bond expansion (the adaptive bond
 * dimension the paper needs at low temperature and strong coupling): after
 * each site's forward step and gauge factorisation, while the bond it opens
 * is below min(D, what the two neighbouring sites can carry), the orthonormal
 * factor is widened by the leading directions of H_eff A outside its span
 * (singular values of the projected H_eff A above expand_tol |H_eff A|,
 * whole near-degenerate multiplets), with zero coefficients in the bond
 * matrix, so the state is unchanged and the bond's backward step and the
 * next site's step evolve into the new directions.  Bonds never shrink.
 * Both sweep directions expand.  Errors: as ftd_tdvp_step; FTD_EINVAL
 * (D < 1, expand_tol <= 0 or >= 1). */
ftd_status ftd_tdvp_step_expand(ftd_ctx* ctx, const ftd_mpo* H, ftd_mps* psi, double dt_real,
                                double dt_imag, int32_t D, double expand_tol,
                                const ftd_krylov_opts* ko);

/* One TDVP step (as ftd_tdvp_step) of each of two different states, run
 * concurrently: psi on the context's stream, phi on a second stream of the
 * context (created on first use, released with the context) from a second
 * host thread.  The states are independent; this is the per-time-step work
 * of the current correlation (real time: both states advance by dt).  Work
 * the caller queued before the call is visible to both; the call returns
 * with the caller's stream ordered after both steps.  Statistics and timing
 * cover both streams.  Errors: as ftd_tdvp_step; FTD_EINVAL if psi == phi. */
ftd_status ftd_tdvp_pair(ftd_ctx* ctx, const ftd_mpo* H, ftd_mps* psi, ftd_mps* phi,
                         double dt_real, double dt_imag, const ftd_krylov_opts* ko);

/* Exact MPO x MPS product followed by compression to D (s/s_max > cutoff):
 * out = compress(O psi).  Used for j|Psi_beta>.  out belongs to the caller. */
ftd_status ftd_apply_compress(ftd_ctx* ctx, const ftd_mpo* O, const ftd_mps* psi, int32_t D,
                              double cutoff, ftd_mps** out);

/* One propagation-and-compression stage of the bond growth:
 * out = compress(psi + c O phi, D), the exact SVD compression of the sum
 * (the same as ftd_apply_compress): the exact remainder right of every bond
 * is factored right to left without forming the sum, then a left-to-right
 * sweep keeps at most D singular values with s/s_max > cutoff per bond
 * (whole near-degenerate multiplets), then an LQ sweep returns the state to
 * right-canonical form.  psi and phi must carry the same log_norm; c is
 * complex (c[0] + i c[1]).  out belongs to the caller. */
ftd_status ftd_pc_stage(ftd_ctx* ctx, const ftd_mps* psi, const ftd_mpo* O, const ftd_mps* phi,
                        const double* c, int32_t D, double cutoff, ftd_mps** out);

/* <bra| O |ket> (log_norm factors excluded), complex, host out[2]. */
ftd_status ftd_overlap(ftd_ctx* ctx, const ftd_mps* bra, const ftd_mpo* O, const ftd_mps* ket,
                       double* out);

/* C(t_k), k = 0..n_steps, t_k = k dt, for a normalised psi_beta (not
 * mutated): phi = compress(j psi_beta, D); then per step one TDVP step of psi
 * and of phi and C_k = <psi|j|phi>.  C_out: host, 2*(n_steps+1) doubles. */
ftd_status ftd_corr_current(ftd_ctx* ctx, const ftd_mpo* H, const ftd_mpo* J,
                            const ftd_mps* psi_beta, int32_t D, double cutoff, double dt,
                            int32_t n_steps, const ftd_krylov_opts* ko, double* C_out);

/* Kubo formula: mu = (1/(2 k_B T e0)) int C(t) dt over the whole real line,
 * evaluated as (beta/e0) int_0^{t_max} Re C(t) dt with C(-t) = conj(C(t)),
 * trapezoid rule on the uniform grid of n samples (interleaved complex C).
 * mu_cm2Vs uses 1 a.u. of mobility = e a0^2 / hbar (CODATA 2018).
 * Host-only.  Errors: FTD_EINVAL (n < 2, dt <= 0, beta < 0). */
ftd_status ftd_mobility(const double* C, int32_t n, double dt, double beta, double e0,
                        double* mu_au, double* mu_cm2Vs);

/* Mean free path of the carrier from C(t) (the mean-free-path passage, after
 * the mobility-versus-coupling figure): group velocity v = sqrt(<j(0) j(0)>)
 * / |e0| = sqrt(Re C(0)) / |e0| and relaxation time
 * tau = (1/2) int_{-inf}^{inf} |Re C(t) / Re C(0)| dt, evaluated as the
 * trapezoid of |Re C / Re C(0)| over [0, t_max] (Re C is even); l_mfp = v tau
 * (bohr when C is in atomic units).  C: n interleaved complex samples on the
 * uniform grid of step dt.  Host-only.  Errors: FTD_EINVAL (n < 2, dt <= 0,
 * e0 == 0, Re C(0) <= 0). */
ftd_status ftd_mean_free_path(const double* C, int32_t n, double dt, double e0, double* l_mfp,
                              double* v, double* tau);

/* Hopping-limit (V -> 0) current correlation of the Holstein ring, the
 * Fermi-golden-rule comparator of the hopping-limit equation, in the form
 * derived for this library's C(t) and j (the printed form is its complex
 * conjugate without the two factors 2, which leaves the mobility unchanged):
 *   C(t) = 2 (e0 R V)^2 exp(-sum_m 2 g_m^2 [(2 n_m + 1) - (n_m + 1) e^{-i w_m t}
 *                                           - n_m e^{i w_m t}]),
 * n_m the Bose occupation at beta.  t: nt times; omega, g: n_modes local-mode
 * frequencies and couplings; C_out: 2*nt doubles (interleaved complex).
 * Host-only.  Errors: FTD_EINVAL (non-positive frequency, beta <= 0: the
 * occupations diverge at infinite temperature). */
ftd_status ftd_fgr_corr(const double* t, int32_t nt, const double* omega, const double* g,
                        int32_t n_modes, double V, double beta, double e0, double R,
                        double* C_out);

/* One point of a mobility sweep: inverse temperature beta = 1/(k_B T) (> 0),
 * transfer integral V, and a frequency scale s > 0 applied to every mode
 * (local and bond): omega -> s omega with g -> g / sqrt(s), which keeps each
 * mode's reorganisation energy g^2 omega fixed.  s = sqrt(m/m') is an isotope
 * substitution of mass m by m' (the isotope-effect passage), so the isotope
 * effect mu'/mu - 1 is the ratio of two points that differ only in s. */
typedef struct {
    double beta;
    double V;
    double omega_scale;
} ftd_sweep_point;

/* Batched mobility runs (the temperature, coupling and isotope studies):
 * for every point, the model `base` with V and the frequency scale of the
 * point, its MPOs, Psi_beta (ftd_thermal_prep with n_imag, n_grow, D, cutoff,
 * prec, ko), C(t_k) for k = 0..n_steps (ftd_corr_current with D, cutoff, dt,
 * ko) and the Kubo mobility (ftd_mobility, e0 of the model).  mu_au and
 * log_Z: host, n_pts doubles each.  The points run one after another on the
 * context's streams; every intermediate is released before the next.
 * Errors: those of the calls it makes, and FTD_EINVAL (n_pts < 1,
 * n_steps < 1, beta <= 0, s <= 0, non-finite point). */
ftd_status ftd_mobility_sweep(ftd_ctx* ctx, const ftd_model* base, const ftd_sweep_point* pts,
                              int32_t n_pts, int32_t n_imag, int32_t n_grow, int32_t D,
                              double cutoff, double dt, int32_t n_steps, ftd_precision prec,
                              const ftd_krylov_opts* ko, double* mu_au, double* log_Z);

/* Gradient of the mobility with respect to the shared mode parameters, by
 * central finite differences through the whole GPU path (not the reverse-mode
 * adjoint): mu of `model` at beta (runs as in ftd_mobility_sweep), and
 * d mu / d omega_loc[k], d mu / d g_loc[k], d mu / d omega_nl[k],
 * d mu / d g_nl[k], each (mu(x + h) - mu(x - h)) / 2h with h = rel_step |x|
 * (rel_step itself for a parameter that is zero).  Cost: 1 + 4 (n_loc + n_nl)
 * mobility runs.  The isotope derivative follows as
 * d mu / d ln m = -1/2 sum_k omega_k d mu / d omega_k + 1/4 sum_k g_k d mu / d g_k.
 * Gradient arrays: host, n_loc and n_nl doubles (may be null when the count
 * is zero).  Errors: those of the runs, and FTD_EINVAL (beta <= 0,
 * n_steps < 1, rel_step outside (0, 0.1)). */
ftd_status ftd_mobility_grad(ftd_ctx* ctx, const ftd_model* model, double beta, int32_t n_imag,
                             int32_t n_grow, int32_t D, double cutoff, double dt,
                             int32_t n_steps, ftd_precision prec, const ftd_krylov_opts* ko,
                             double rel_step, double* mu, double* dmu_domega_loc,
                             double* dmu_dg_loc, double* dmu_domega_nl, double* dmu_dg_nl);

/* Electronic reduced density matrix of a (purified) state, the phonon trace
 * of the coherent-length section: sigma = Tr_ph rho with rho = |psi><psi| /
 * <psi|psi> traced over the ancillas, i.e.
 *   sigma_ij = <psi| c+_j c_i |psi> / <psi|psi>,
 * each element one FP64 overlap with a bond-dimension-1 product MPO (sigma-
 * on e_i, sigma+ on e_j; n_i on the diagonal; no string is needed in the
 * one-carrier sector).  For psi_beta, Tr sigma = 1 and sigma is Hermitian.
 * m: the model psi was prepared for (validated as in ftd_mpo_build; its
 * chain must match psi's).  sigma: host, 2*N*N doubles, interleaved complex,
 * row i column j.  Cost: N^2 overlaps.  Errors: FTD_EINVAL (null, model
 * mismatch, zero norm). */
ftd_status ftd_reduced_density(ftd_ctx* ctx, const ftd_model* m, const ftd_mps* psi,
                               double* sigma);

/* Coherent length of the coherent-length equation,
 *   L = (sum_ij |sigma_ij|)^2 / (N sum_ij |sigma_ij|^2),
 * 1 for a fully localised and N for a fully delocalised thermal state.
 * sigma: host, 2*n*n doubles (interleaved complex).  Host-only.  Errors:
 * FTD_EINVAL (n < 1, non-finite or all-zero sigma). */
ftd_status ftd_coherent_length(const double* sigma, int32_t n, double* L);

/* ------------------------------------------------- kernel-level entry points
 * Apply the one-site effective Hamiltonian of `site` to x, with the left
 * environment built from sites < site of psi (assumed left-orthonormal there)
 * and the right environment from sites > site (right-orthonormal), exactly as
 * inside ftd_tdvp_step.  x, y: host interleaved complex of psi's site shape.
 * n_repeat > 1 repeats the product (timing).  Used by the parity tests and the
 * roofline measurement. */
ftd_status ftd_heff_apply(ftd_ctx* ctx, const ftd_mpo* H, const ftd_mps* psi, int32_t site,
                          const double* x, double* y, int32_t n_repeat);

/* The local step of the projector-splitting integrator (the paper's
 * time-dependent variational method: each site tensor is propagated by the
 * exponential of its effective Hamiltonian): y = exp(z H_eff) x at `site`,
 * with the environments of ftd_heff_apply and the Krylov exponential of
 * ftd_tdvp_step (settings `ko`, NULL: tol 1e-14, mmax 40), in psi's
 * precision.  x, y: host interleaved complex of psi's site shape.  n_repeat
 * > 1 repeats the exponential from the same x (timing of the Lanczos
 * kernels).  *m_out (may be NULL) receives the Krylov vector count.  Errors:
 * FTD_EINVAL (site, lengths, non-finite z, Krylov settings), FTD_ENOCONV. */
ftd_status ftd_heff_expm(ftd_ctx* ctx, const ftd_mpo* H, const ftd_mps* psi, int32_t site,
                         const double* x, double* y, double zr, double zi,
                         const ftd_krylov_opts* ko, int32_t n_repeat, int32_t* m_out);

/* Gauge move of the TDVP sweep on the device (shifted CholeskyQR in three
 * passes, the orthonormalisation the projector-splitting integrator needs
 * between a site and the next bond): lq = 0: M (rows x cols, rows >= cols,
 * full column rank) = Q R, Q with orthonormal columns, R upper triangular with
 * a real positive diagonal; lq = 1: M (rows <= cols, full row rank) = L Q, Q
 * with orthonormal rows, L lower triangular with a real positive diagonal.
 * M, Q: host, rows*cols interleaved complex, row-major; F: host, k*k with
 * k = min(rows, cols), receives R or L.  Errors: FTD_EINVAL (shapes),
 * FTD_ENOCONV (Cholesky breakdown: M numerically rank deficient). */
ftd_status ftd_qr(ftd_ctx* ctx, int32_t rows, int32_t cols, const double* M, int32_t lq,
                  double* Q, double* F);

/* Truncated SVD on the device (the compression kernel): T (M x N, host,
 * interleaved complex, row-major) ~ L diag(S) R with L (M x k) orthonormal
 * columns and R (k x N) orthonormal rows, keeping at most D singular values
 * with s/s_max > cutoff and whole near-degenerate multiplets.  S is folded
 * into L (s_left = 1) or R (s_left = 0).  L and R are host buffers of at
 * least M*min(M,N) and min(M,N)*N complex values; *k receives the rank. */
ftd_status ftd_svd_trunc(ftd_ctx* ctx, int32_t M, int32_t N, const double* T, int32_t D,
                         double cutoff, int32_t s_left, double* L, double* R, int32_t* k);

/* Complex GEMM on the device kernels: C = op(A) op(B) with op = identity,
 * transpose or conjugate transpose per operand (trans = 0, 1, 2), M x N
 * result, inner dimension K; host buffers interleaved complex, row-major:
 * A is M x K (trans 0) or K x M (trans 1, 2), B is K x N (0) or N x K (1, 2).
 * precision FTD_C128 (float64), FTD_C64 (float32 operands, float64 out) or
 * FTD_BF16X3 (float32 operands, bf16 split products, float64 out).
 * Used by the kernel parity tests. */
ftd_status ftd_gemm(ftd_ctx* ctx, int32_t precision, int32_t M, int32_t N, int32_t K,
                    int32_t transA, int32_t transB, const double* A, const double* B, double* C);

/* ftd_gemm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product C = op(A) op(B) by the same kernels, on device buffers, with
 * no allocation of any kind.  A, B, C: device memory of the context's GPU in
 * split planes (the whole real plane, then the whole imaginary plane), each
 * plane row-major as in ftd_gemm: A is M x K (trans 0) or K x M (trans 1, 2),
 * B is K x N (0) or N x K (1, 2); element type double for FTD_C128, float for
 * FTD_C64; C is M x N double (both precisions).  Buffers stay owned by the
 * caller.  The split-K partial sums go to a fixed 32 MiB device array that
 * the library holds on every GPU it has run on until the process ends, so M*N
 * is limited to 2^20 output elements (larger requests: FTD_EINVAL, nothing
 * enqueued); when the split count ftd_gemm would use does not fit, fewer
 * splits are used.  Asynchronous on the context stream (no synchronisation).
 * Every call on one GPU shares that array, which keeps the last call's
 * contents: calls that overlap on one GPU (two streams, two contexts, two
 * host threads) race and must be ordered by the caller.  Errors: FTD_EINVAL
 * (null, sizes, trans, precision), FTD_EDEVICE (launch failure). */
ftd_status ftd_gemm_noalloc(ftd_ctx* ctx, int32_t precision, int32_t M, int32_t N, int32_t K,
                            int32_t transA, int32_t transB, const void* A, const void* B,
                            double* C);

#ifdef __cplusplus
}
#endif
#endif
