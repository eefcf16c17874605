/*
 * risp.h - C ABI of the MI355X (gfx950) TDA-risp library (librisp.so).
 *
 * The library computes the lowest excitation energies and vectors of the TDA-risp matrix
 * (Zhou et al., "GPU Accelerated Minimal Auxiliary Basis Approach TDDFT for Large Organic
 * Molecules", eq. TDA and eq. TDA-risp):
 *
 *   A_{ia,jb} = (e_a - e_i) d_ij d_ab + 2 (ia|jb) - (ij|J^|ab)          (exchange only inside the window)
 *
 * with the RI approximation of eq. TDDFT-axs_approx_integral over the minimal auxiliary basis of
 * eq. gr (one primitive s + p per non-hydrogen atom for Coulomb, one s for exchange, hydrogen
 * omitted), the exchange-space energy window of the section on exchange-space truncation and the
 * range-separated operator J^ = (alpha + beta erf(omega r))/r of eq. RSH / eq. K_mia_RSH.
 *
 * Conventions shared by every entry point:
 *  - Units: bohr and Hartree. Cartesian p components are ordered x, y, z.
 *  - Matrices are row-major. Orbital pairs (i, a) are flattened as i * nvir + a.
 *  - Status: RISP_OK (0) or a negative RISP_E_* code; the message of the last failure on the calling
 *    thread is returned by risp_last_error(). On failure no output is written. No C++ exception
 *    crosses the ABI.
 *  - Inputs are borrowed for the duration of the call only. Outputs go to caller buffers.
 *  - "dev" pointers are device (HBM) addresses on the context's device; every other pointer is host.
 *  - Work is ordered on the context stream. Calls that return host results synchronise that stream;
 *    risp_sigma does not synchronise.
 *  - A context is used by one thread at a time.
 */
#ifndef RISP_H
#define RISP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t risp_status;
enum {
  RISP_OK = 0,
  RISP_PENDING = 1,
  RISP_E_ARG = -1,      /* invalid argument (null pointer, bad enum, negative size) */
  RISP_E_SHAPE = -2,    /* inconsistent sizes (nao vs shells, nocc > nmo, ...) */
  RISP_E_NOMEM = -3,    /* device allocation failed */
  RISP_E_HIP = -4,      /* HIP runtime error */
  RISP_E_NOTCONV = -5,  /* Davidson reached max_iter; results are the last Ritz pairs */
  RISP_E_STATE = -6,    /* object used with the wrong context or after free */
  RISP_E_NOTFOUND = -7
};

/* precision of the stored factors and of the sigma contractions */
enum { RISP_FP64 = 0, RISP_FP32 = 1, RISP_BF16 = 2 };

/* Coulomb route (section on on-the-fly Coulomb evaluation). RISP_J_MO stores T_ia and forms
 * 2 T_ia (T_jb^T X) in two streaming passes. RISP_J_AO_DIRECT stores no T_ia: per sigma block it
 * forms the AO transition densities D_m = C_occ X_m C_vir^T, contracts them with (mu nu|Q)
 * regenerated over the screened pairs, applies the inverse metric, contracts back with (mu nu|P)
 * regenerated again and transforms J_m = C_occ^T U_m C_vir, all in FP64; for molecules whose T_ia
 * does not fit in device memory. The integrals are regenerated in a packed layout over the kept
 * pairs (per-atom partner lists), so only the AO densities of a group of trial vectors are dense
 * FP64 [nao][nao]. Served jobs take RISP_J_MO only (the route synchronises inside sigma and cannot
 * run in the serving loop's graphs). */
enum { RISP_J_MO = 0, RISP_J_AO_DIRECT = 1 };
/* reading of the range-separated exchange: one RI in the J^ metric (paper eq. K_mia_RSH) or
 * alpha RI(1/r) + beta RI(erf) stacked along the auxiliary index */
enum { RISP_RSH_COMBINED = 0, RISP_RSH_SPLIT = 1 };
/* window reference: absolute orbital energies (as written in the paper) or distances to the
 * frontier orbitals */
enum { RISP_WIN_ABSOLUTE = 0, RISP_WIN_FRONTIER = 1 };

/* One uncontracted primitive Cartesian Gaussian shell: coef * N * x^lx y^ly z^lz exp(-exponent r^2)
 * centred on `atom`, with N the normalisation of the primitive (l = 0 or 1 only). */
typedef struct {
  int32_t atom;
  int32_t l;
  double exponent;
  double coef;
} risp_shell;

/* The problem as the paper states it: geometry, AO basis, MO coefficients and energies. */
typedef struct {
  int32_t natm;
  const double *coords;     /* [natm][3] bohr */
  const int32_t *Z;         /* [natm] nuclear charges; Z == 1 marks hydrogen */
  const double *aux_radius; /* [natm] semi-empirical radius R_A (bohr) of eq. gr */
  int32_t nshell;
  const risp_shell *shells; /* AO shells; functions are numbered shell by shell */
  int32_t nao, nmo, nocc;
  const double *mo_coeff;   /* [nao][nmo] */
  const double *mo_energy;  /* [nmo], ascending within occupied and within virtual */
} risp_system;

typedef struct {
  double c_x;         /* alpha of J^ (full-range exact-exchange fraction), e.g. 0.22 */
  double beta;        /* beta of J^ (long-range erf part), e.g. 0.78; 0 for a global hybrid */
  double omega;       /* range-separation parameter (bohr^-1), e.g. 0.2 */
  double window_ev;   /* exchange window (eV), e.g. 40 */
  double theta;       /* auxiliary exponent parameter of eq. gr: exponent = theta / R_A^2 */
  double schwarz_tau; /* shell-pair screening threshold on Q_AB * max_P sqrt((P|P)); 0 keeps all */
  int32_t rsh_mode;   /* RISP_RSH_* */
  int32_t window_mode;/* RISP_WIN_* */
  int32_t precision;  /* RISP_FP64 / RISP_FP32 / RISP_BF16 */
  int32_t h_in_aux;   /* 0: hydrogen omitted from both auxiliary bases (paper's production setting) */
  int32_t bf16_scale; /* BF16 only: 1 stores each auxiliary slice scaled by a power of two */
  int32_t build_chunk_kib; /* device memory for one chunk of FP64 transformed integrals during the
                              build, in KiB; the T_ia and T_ab builds run in as many chunks of
                              occupied / window-virtual orbitals as needed; 0 = as large as the
                              free device memory allows (the stored factors are allocated first,
                              the build's temporaries then come from one allocation) */
  int32_t j_mode;     /* RISP_J_*: how the Coulomb term of sigma is formed */
  int32_t full_tddft; /* nonzero: also build the windowed exchange factor over (i, a) pairs that
                         full TDDFT-risp needs (Fig. tensors_shape, T_ia^P'); FP64/FP32 factors,
                         combined exchange reading, stored-factor Coulomb route; 0 = TDA only */
  int32_t dense_transform; /* nonzero: the first MO transform of the build contracts dense (mu nu|P)
                              slabs; 0 = per-atom partner lists of the kept shell pairs (the same
                              sums without the screened-out zeros; results equal up to rounding) */
  int32_t bf16_coulomb_fp32; /* BF16 only: nonzero forms the Coulomb term of every sigma from the FP32
                                copy of T_ia that the correction pass uses (the exchange stays BF16);
                                0 = BF16 T_ia */
} risp_params;

typedef struct {
  int32_t nstates;         /* number of lowest roots */
  int32_t block;           /* trial vectors per sigma block; 0 = min(2 nstates, 30) */
  int32_t max_space;       /* subspace size that triggers a restart; 0 = 8 * block */
  int32_t max_iter;        /* 0 = 200 */
  double tol;              /* residual 2-norm convergence threshold per state */
  int32_t correction_pass; /* BF16 factors: refine the BF16-converged vectors with FP32 products */
  int32_t correction_steps;/* at most this many FP32 Davidson steps after the FP32 Rayleigh-Ritz;
                              0 = 16 */
  double bf16_tol;         /* BF16 stage stops at max(tol, bf16_tol) or when its residual stalls;
                              0 = 1e-3 (on the 1000-atom molecule the correction pass then needs
                              2 more steps but the BF16 stage 5 fewer: 2.5 s less in all) */
  int32_t nx0;             /* optional initial vectors (resume): count, 0 = unit-vector guess */
  int32_t flags;           /* RISP_DAV_* bits, 0 = none */
  const float *x0;         /* [nx0][nocc*nvir] host */
  int32_t ncorr;           /* correction vectors per iteration only for the lowest ncorr Ritz pairs
                              with residual >= tol (at least nstates, at most block); the other
                              Ritz vectors of the block stay in the subspace; 0 = nstates */
  int32_t correction_ncorr;/* the same for the FP32 correction stage; 0 = nstates */
} risp_dav_opts;

/* risp_dav_opts.flags: RISP_DAV_VERBOSE prints one line per iteration (stage, iteration, subspace
 * size, largest residual over the requested states) to stderr. RISP_DAV_SPILL keeps the subspace
 * vectors and their products (2 (max_space + block) nocc nvir elements) in pinned host memory that
 * the kernels read and write over the host link, for subspaces that do not fit next to the factors
 * (same arithmetic, same results; slower subspace steps). RISP_DAV_OLSEN forms each correction as
 * (D - theta)^-1 (r - eps x) with eps chosen so that it is orthogonal to the Ritz vector x (Olsen's
 * correction; D the diagonal of A) instead of (D - theta)^-1 r. The correction pass of BF16
 * factors rounds the basis vectors it multiplies to BF16 values, so its split-BF16 exchange skips
 * the vectors' lo halves, and solves the subspace problem with their overlap;
 * RISP_DAV_FP32_BASIS keeps FP32 basis vectors there instead (three split products per
 * contraction). */
enum { RISP_DAV_VERBOSE = 1, RISP_DAV_SPILL = 2, RISP_DAV_OLSEN = 4, RISP_DAV_FP32_BASIS = 8 };

typedef struct {
  int32_t iters, restarts, sigma_vectors, converged; /* main stage (BF16 stage for BF16 factors) */
  int32_t correction_iters, correction_vectors;       /* FP32 correction stage */
  double t_build;                  /* seconds in risp_build_factors for these factors */
  double t_sigma, t_subspace;      /* main stage: sigma blocks and subspace work (seconds) */
  double t_correct;                /* correction stage, all of it (seconds) */
  double t_sigma_correct;          /* correction stage sigma blocks (seconds) */
  double sigma_flops;              /* algorithmic flops of the main-stage sigma blocks */
  double sigma_flops_correct;      /* algorithmic flops of the correction-stage sigma blocks */
  int64_t hbm_bytes;               /* device bytes held by the factors */
  double resid_hist[256];          /* max residual norm per iteration (main, then correction) */
} risp_dav_info;

typedef struct {
  int32_t nao, nmo, nocc, nvir;
  int32_t naux_j, naux_k; /* Coulomb and exchange auxiliary functions (naux_k counts both RI
                             blocks in RISP_RSH_SPLIT) */
  int32_t nocc_k, nvir_k; /* orbitals inside the exchange window */
  int32_t npair;          /* shell pairs kept by screening */
  int32_t precision;
  int64_t bytes;          /* device bytes held by the factor object */
  const void *t_ia;       /* dev [naux_j][ld_ia], row = (i, a) pairs nocc*nvir then zero padding,
                             in `precision` (BF16: stored / scale) */
  const void *t_ij;       /* dev [nocc_k][naux_k][ld_ij], last index j < nocc_k, rest zero */
  const void *t_ab;       /* dev [naux_k][nvir_k][ld_ab], last index b < nvir_k, rest zero */
  const float *scale_ia;  /* dev [naux_j] power-of-two scales (BF16), else NULL */
  const float *scale_k;   /* dev [naux_k] product of the T_ij and T_ab scales (BF16), else NULL */
  const int32_t *occ_k;   /* dev [nocc_k] window occupied indices, ascending */
  const int32_t *vir_k;   /* dev [nvir_k] window virtual indices (0-based in the virtual space) */
  int64_t ld_ia;          /* row stride of t_ia: nocc*nvir rounded up to a multiple of 8 (t_ia is
                             NULL for factors built with RISP_J_AO_DIRECT) */
  int32_t ld_ij, ld_ab;   /* row strides of t_ij and t_ab: nocc_k, nvir_k rounded up likewise */
  const double *diag_a;   /* dev [nocc][nvir] FP64 diagonal of A from the FP64 factors before
                             storage: e_a - e_i + 2 sum_P B_ia^2 - [window] sum_P Bx_ii Bx_aa (the
                             Coulomb part is left out on the AO route); Davidson guess and
                             preconditioner */
  const void *t_ij_lo;    /* BF16 factors: dev BF16 remainders of t_ij and t_ab in their layouts
                             (same scales; T / scale = hi + lo to about 2^-17), used by the
                             correction pass's split-BF16 exchange; NULL otherwise */
  const void *t_ab_lo;
} risp_factors_desc;

/* Per-phase timing of sigma products (HIP events on the context stream around each launch). */
enum {
  RISP_PHASE_COULOMB_Y = 0, /* Y[P][m] = sum_ia T_ia^P X_mia (split-K product and its reduction) */
  RISP_PHASE_COULOMB_J = 1, /* sigma_mia = 2 sum_P Y[P][m] T_ia^P */
  RISP_PHASE_EXCHANGE_M = 2,/* M^P_mja = sum_b T_ab^P X_mjb, one launch per auxiliary chunk */
  RISP_PHASE_EXCHANGE_K = 3,/* K_mia += sum_(P, j) T_ij^P M^P_mja, one launch per auxiliary chunk */
  RISP_PHASE_OTHER = 4,     /* window gather, conversions, diagonal term and combine */
  RISP_NPHASE = 5,
  /* counters are kept per arithmetic of the sigma call: slot = precision * RISP_NPHASE + phase,
   * precision RISP_FP64 / RISP_FP32 / RISP_BF16 (the FP32 correction pass of BF16 factors counts
   * as RISP_FP32) */
  RISP_NPHASE_SLOTS = 15
};
typedef struct {
  int64_t launches; /* timed launches (or launch groups) */
  double ms;        /* summed event time */
  double flops;     /* algorithmic flops of those launches */
  double bytes;     /* algorithmic HBM bytes (each operand read once, each result written once) */
} risp_phase_stat;

typedef struct risp_ctx risp_ctx;
typedef struct risp_factors risp_factors;

/* Last error message of the calling thread ("" if none). */
const char *risp_last_error(void);

/* Create a context on HIP device `device`. hip_stream: a hipStream_t to order work on, or NULL for
 * a stream owned by the context. */
risp_status risp_ctx_create(int32_t device, void *hip_stream, risp_ctx **out);
/* Stop serving (queued jobs are dropped, running ones finish), synchronise the stream and release
 * the context. Factor objects still alive are detached: their only valid call is then
 * risp_factors_free. */
risp_status risp_ctx_destroy(risp_ctx *ctx);

/* Enable (1) or disable (0) sigma phase timing; reset != 0 clears the counters. If out is not
 * NULL it receives RISP_NPHASE_SLOTS entries (the stream is synchronised first). */
risp_status risp_ctx_profile(risp_ctx *ctx, int32_t enable, int32_t reset, risp_phase_stat *out);

/* ---- stages of the factor build (exposed for validation; risp_build_factors runs them all) ---- */

/* Auxiliary basis of eq. gr (section on exchange-space truncation for the hydrogen rule): for each
 * atom with Z > 1 (or every atom when h_in_aux) one s and one p primitive with exponent
 * theta / R_A^2 for Coulomb, and the s primitive for exchange. Writes up to `cap` shells to each
 * array (host) and the counts. */
risp_status risp_select_aux(const risp_system *sys, const risp_params *prm, int32_t cap,
                            risp_shell *aux_j, int32_t *n_j, risp_shell *aux_k, int32_t *n_k);

/* Exchange window (section on exchange-space truncation): indices of occupied orbitals i with
 * e_i * 27.211386245988 > -window_ev and of virtual orbitals a (0-based in the virtual space) with
 * e_a * 27.211386245988 < window_ev (RISP_WIN_ABSOLUTE; RISP_WIN_FRONTIER keeps i with (e_LUMO - e_i) * 27.211386245988 < window_ev
 * and a with (e_a - e_HOMO) * 27.211386245988 < window_ev), computed on the device, in
 * ascending order. occ_k [nocc] and vir_k [nmo - nocc] are host buffers; counts returned in
 * *nocc_k, *nvir_k. */
risp_status risp_window(risp_ctx *ctx, int32_t nmo, int32_t nocc, const double *mo_energy,
                        double window_ev, int32_t window_mode, int32_t *occ_k, int32_t *nocc_k,
                        int32_t *vir_k, int32_t *nvir_k);

/* Schwarz shell-pair screening on the device: keeps (A >= B) when
 * max_{mu in A, nu in B} sqrt((mu nu|mu nu)) * max_P sqrt((P|P)) >= tau over the given auxiliary
 * shells. pairs: host [cap][2] receives the kept pairs in ascending (A, B) order. */
risp_status risp_screen(risp_ctx *ctx, const risp_system *sys, int32_t naux_shell,
                        const risp_shell *aux, double tau, int32_t cap, int32_t *pairs,
                        int32_t *npair);

/* Two-centre integrals (P|Q) (omega <= 0) or (P|erf(omega r)/r|Q) over the auxiliary shells,
 * FP64 on the device, written to host out [naux][naux]. */
risp_status risp_int2c(risp_ctx *ctx, const risp_system *sys, int32_t naux_shell,
                       const risp_shell *aux, double omega, double *out);

/* Three-centre integrals (mu nu|P) (omega <= 0) or with erf(omega r)/r, FP64 Obara-Saika on the
 * device for the auxiliary shells [aux_begin, aux_end), all AO pairs (tau = 0) or the pairs kept by
 * screening against `aux` at tau. out: host [naux_sel][nao][nao]. */
risp_status risp_int3c(risp_ctx *ctx, const risp_system *sys, int32_t naux_shell,
                       const risp_shell *aux, int32_t aux_begin, int32_t aux_end, double omega,
                       double tau, double *out);

/* ---- the method ---- */

/* Build every factor of the TDA-risp matrix on the device: auxiliary selection, window, screening,
 * metric (P|Q) and (P|J^|Q) with FP64 Cholesky, (mu nu|P) and (mu nu|J^|P) integrals, MO transforms
 * and metric application in FP64, storage in `precision` (section on exchange-space truncation;
 * eq. TDDFT-axs_approx_integral). */
risp_status risp_build_factors(risp_ctx *ctx, const risp_system *sys, const risp_params *prm,
                               risp_factors **out);
/* Sizes and device pointers of a factor object (valid until risp_factors_free). */
risp_status risp_factors_query(const risp_factors *f, risp_factors_desc *out);
/* Release a factor object (waits for its queued work); NULL is accepted. */
risp_status risp_factors_free(risp_factors *f);

/* sigma = A X for m trial vectors (eq. TDA-risp with the factors): diagonal term, Coulomb
 * 2 T_ia (T_jb^T X) and windowed exchange sum_P T_ij^P X T_ab^P. X_dev and sigma_dev are device
 * [m][nocc][nvir] arrays of doubles (dtype RISP_FP64) or floats (RISP_FP32). Stream-ordered, no
 * synchronisation (except for factors built with RISP_J_AO_DIRECT, whose integral passes
 * synchronise the stream). Factors stored in BF16 compute in BF16 with FP32 accumulation and take
 * FP32 X / sigma. */
risp_status risp_sigma(risp_ctx *ctx, const risp_factors *f, int32_t m, const void *X_dev,
                       void *sigma_dev, int32_t dtype);

/* Bytes of the library's fixed device scratch array (one copy per device, held from the moment
 * the library's code object is loaded on that device until the process ends). */
#define RISP_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): risp_sigma with every workspace (padded X copy, Coulomb partial
 * sums, window block, exchange intermediate and accumulator) taken from the fixed scratch array of
 * RISP_SCRATCH_BYTES; it calls no hipMalloc/hipFree. Same arguments, layouts, stream and
 * precision rules as risp_sigma; the caller owns X_dev and sigma_dev. The result equals
 * risp_sigma's up to the summation order of the exchange accumulation (fewer auxiliary functions per
 * chunk). Returns RISP_E_SHAPE, writing nothing, when m vectors of these factors need more scratch
 * than the array holds (e.g. BF16 factors of a 300-atom molecule take up to about 60 vectors per
 * call), and RISP_E_ARG for factors built with RISP_J_AO_DIRECT. Every call on a device shares that
 * device's array and leaves its contents behind: calls that overlap on one device (two streams, two
 * threads, two contexts) race, so serialise them. Stream-ordered, no synchronisation. */
risp_status risp_sigma_noalloc(risp_ctx *ctx, const risp_factors *f, int32_t m, const void *X_dev,
                               void *sigma_dev, int32_t dtype);

/* Products of full TDDFT-risp (eq. hessian, XC kernel dropped) for m vectors V: P = (A + B) V and
 * M = (A - B) V, with A + B = de + 4 (ia|jb) - [window] ((ij|J^|ab) + (ib|J^|ja)) and
 * A - B = de - [window] ((ij|J^|ab) - (ib|J^|ja)) (the Coulomb part of A + B is 4 (ia|jb) so that A
 * is that of eq. TDA-risp; the printed eq. hessian shows 2). V_dev, P_dev, M_dev: device
 * [m][nocc][nvir] in the factor precision (dtype RISP_FP64 or RISP_FP32); factors built with
 * full_tddft. Synchronises the factors' stream (it allocates the exchange intermediate). */
risp_status risp_sigma_full(risp_ctx *ctx, const risp_factors *f, int32_t m, const void *V_dev, void *P_dev,
                            void *M_dev, int32_t dtype);

/* Full TDDFT-risp (eq. tddft with the matrices of eq. hessian, XC kernel dropped, the same RI
 * factors, window and exchange operator as TDA-risp plus the windowed exchange factor over (i, a)
 * pairs): the lowest nstates excitation energies Omega and amplitudes X + Y, X - Y with
 * (X + Y).(X - Y) = 1. Needs factors built with risp_params.full_tddft (FP64 or FP32 storage).
 * Davidson-like solver on one subspace for (A + B) and (A - B) (section on Davidson settings):
 * FP64 projected matrices, A - B = L L^T (Cholesky), the symmetric problem L^T (A + B) L c =
 * Omega^2 c by the same subspace eigensolver, both residuals preconditioned with 1/(Omega - diag A)
 * and added to the subspace; restarts rebuild the subspace from the current X + Y and X - Y.
 * opts: nstates (<= 32), block, max_space, max_iter, tol (both residual norms per state) and
 * RISP_DAV_VERBOSE; nx0 must be 0. energies: host [nstates]; xpy, xmy: host [nstates][nocc*nvir]
 * or NULL. Returns RISP_E_NOTCONV (results written) when max_iter is reached and RISP_E_STATE when
 * the projected A - B is not positive definite (unstable ground state). */
risp_status risp_davidson_full(risp_ctx *ctx, const risp_factors *f, const risp_dav_opts *opts,
                               double *energies, float *xpy, float *xmy, risp_dav_info *info);

/* Transition properties of nstates excited states (eq. oscillator_strength, eq. rotator_strength,
 * eq. transition and eq. transition_magnetic in the dipole-length form with TDA amplitudes, Y = 0):
 *   mu_0n = sqrt(2) sum_ia <i| r - O |a> X_nia,   m_0n = sqrt(2) sum_ia <i| (r - O) x nabla |a> X_nia,
 *   f_0n = 2/3 Omega_n |mu_0n|^2,                 R_0n = 1/2 mu_0n . m_0n,
 * where sqrt(2) makes the closed-shell singlet of unit-normalised amplitudes X (as risp_davidson
 * returns them) and (r - O) x nabla is taken as the real antisymmetric operator over the real MOs.
 * sys: the same system as for the factor build (geometry, AO shells, MO coefficients; the auxiliary
 * fields are not used); origin: host [3] gauge origin in bohr (NULL: 0, 0, 0); energies: host
 * [nstates] Hartree; X_dev: device FP32 [nstates][nocc][nvir]. Outputs (host, caller-allocated):
 * mu [nstates][3] and mdip [nstates][3] (either may be NULL), f [nstates], R [nstates]. AO
 * integrals by Obara-Saika on the device, FP64 MFMA transforms; allocates device memory and
 * synchronises the context stream. */
risp_status risp_properties(risp_ctx *ctx, const risp_system *sys, const double *origin, int32_t nstates,
                            const double *energies, const void *X_dev, double *mu, double *mdip, double *f,
                            double *R);

/* Lorentzian-broadened stick spectrum (the paper's UV-vis and ECD figures; half width at half
 * maximum hwhm, unit-area lines): out[q] = sum_n s_n (hwhm/pi) / ((e0 + q de - E_n)^2 + hwhm^2)
 * for q < npts. energies and strengths: host [nstates] (f for UV-vis, R for ECD, in any consistent
 * energy unit); out: host [npts]. Synchronises the context stream. */
risp_status risp_spectrum(risp_ctx *ctx, int32_t nstates, const double *energies, const double *strengths,
                          double hwhm, double e0, double de, int32_t npts, double *out);

/* Lowest nstates eigenpairs of A by block Davidson (section on large-system Davidson
 * diagonalisation): guess and preconditioner from the diagonal of A, sigma blocks on MFMA, FP64
 * subspace projection, Gram-Schmidt and tridiagonal eigensolver on the device, thick restart when
 * the subspace reaches max_space; BF16 factors add the FP32 correction pass (risp_dav_opts).
 * energies: host [nstates]; vectors: host [nstates][nocc*nvir] or NULL; info may be NULL.
 * Returns RISP_E_NOTCONV (with the last Ritz pairs written) if max_iter is reached. */
risp_status risp_davidson(risp_ctx *ctx, const risp_factors *f, const risp_dav_opts *opts,
                          double *energies, float *vectors, risp_dav_info *info);

/* ---- serving: continuous batching of excitation jobs ---- */

typedef struct {
  int64_t hbm_budget_bytes; /* device bytes the resident jobs may use; 0 = 85 % of the free memory
                               when serving starts */
  int32_t max_active;       /* jobs resident at once; 0 = 8 */
  int32_t use_graphs;       /* 1: each tick's sigma blocks are captured and launched as one hipGraph */
} risp_serve_opts;

typedef struct {
  int32_t status;     /* the job's own status: RISP_OK, RISP_E_NOTCONV or an error code */
  int32_t nstates;    /* energies written */
  double *energies;   /* caller buffer [nstates] or NULL */
  float *vectors;     /* caller buffer [nstates][nocc*nvir] or NULL */
  risp_dav_info info;
  double t_submit, t_admit, t_first_sigma, t_done; /* seconds since serving started */
  char message[256];  /* error text when status < 0 */
} risp_result;

typedef struct {
  int32_t queued, active, done, reserved;
  int64_t budget_bytes, used_bytes;
  int64_t ticks, graph_ticks;
} risp_serve_stats;

/* Configure serving before the first submit (RISP_E_STATE afterwards). */
risp_status risp_serve_config(risp_ctx *ctx, const risp_serve_opts *opts);

/* Estimated device footprint of a job (host-only computation; the admission rule uses it). */
risp_status risp_job_footprint(const risp_system *sys, const risp_params *prm, const risp_dav_opts *opts,
                               int64_t *bytes);

/* Queue a job: the inputs are deep-copied (the caller may free them at once). A job that does not
 * fit the free budget waits in the queue; one larger than the whole budget is rejected with
 * RISP_E_NOMEM. opts->x0 is not supported here. Thread-safe. */
risp_status risp_submit(risp_ctx *ctx, const risp_system *sys, const risp_params *prm,
                        const risp_dav_opts *opts, uint64_t *job_id);

/* RISP_PENDING while the job is queued or running; RISP_OK once finished, with out filled (the
 * job's own outcome in out->status) and the job released; RISP_E_NOTFOUND for an unknown or already
 * polled id. Thread-safe. */
risp_status risp_poll(risp_ctx *ctx, uint64_t job_id, risp_result *out);

risp_status risp_serve_stats_get(risp_ctx *ctx, risp_serve_stats *out);

/* Device memory held by the library's own allocations in this process (factors, workspaces,
 * Davidson buffers, served jobs; not the HIP runtime's internal allocations), and its high-water mark.
 * reset_peak != 0 first sets the mark to the current value. Host outputs. Thread-safe. */
risp_status risp_device_usage(int64_t *live_bytes, int64_t *peak_bytes, int32_t reset_peak);

#ifdef __cplusplus
}
#endif

#endif /* RISP_H */
