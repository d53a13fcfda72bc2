/*
 * apx.h -- C ABI of the MI355X (gfx950) adaptive-precision EAM-ACE force library.
 *
 * The library evaluates, on one GPU, the per-step force routine of the
 * adaptive-precision potential of Immel, Drautz and Sutmann (arXiv:2411.03002):
 * neighbour lists, centro-symmetry detection and switching weights, classical EAM
 * for every atom, the atomic cluster expansion (ACE) only where the precise weight is
 * non-zero, the site-weighted blend, and velocity-Verlet integration.
 *
 * Conventions for every entry point:
 *  - Return value: apx_status, APX_OK (0) on success, a negative code otherwise.
 *    Nothing throws across the ABI and nothing aborts; apx_last_error() returns the
 *    message of the last failure on that context.
 *  - Array arguments are caller-owned DEVICE pointers unless marked "host".  The
 *    library never frees caller memory.  Arrays of vectors use structure-of-arrays
 *    layout [3][n]: x components at [0, n), y at [n, 2n), z at [2n, 3n).
 *  - Work is enqueued on the context's HIP stream and the call returns at once.
 *    Only calls that return a host scalar synchronise; each says "(sync)".
 *  - A context is not thread-safe: use one per host thread.
 *  - Weights: w is the weight of the precise potential (ACE).  The paper's switching
 *    parameter is the weight of the fast potential, lambda = 1 - w.
 *  - Periodic coordinates must lie in [lo, hi); coordinates in a non-periodic
 *    dimension must lie in [lo, hi) as well (APX_EINVAL otherwise, reported by the
 *    neighbour build).
 */
#ifndef APX_H
#define APX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t apx_status;
#define APX_OK 0
#define APX_EINVAL (-1)     /* bad argument: null pointer, size mismatch, unsupported size */
#define APX_ENOMEM (-2)     /* device allocation failed */
#define APX_EDEVICE (-3)    /* a HIP runtime call failed */
#define APX_ECAPACITY (-4)  /* a caller buffer is too small; the needed size is returned */
#define APX_ENONFINITE (-5) /* a non-finite value where a finite one is required */
#define APX_ERADICAND (-6)  /* a thermostat correction had a negative radicand and was skipped */

#define APX_FP64 0
#define APX_FP32 1

typedef struct apx_ctx apx_ctx;
typedef struct apx_ace_model apx_ace_model;
typedef struct apx_md apx_md;

/* ------------------------------------------------------------------ context */
/* Create a context on HIP device `device` enqueuing on `stream` (a hipStream_t; NULL
 * means the null stream).  The context owns its scratch memory. */
apx_status apx_ctx_create(int32_t device, void* stream, apx_ctx** out);
apx_status apx_ctx_set_stream(apx_ctx* ctx, void* stream);
void apx_ctx_destroy(apx_ctx* ctx);
const char* apx_last_error(const apx_ctx* ctx);
apx_status apx_ctx_synchronize(apx_ctx* ctx); /* (sync) */
const char* apx_version(void);

/* Per-kernel timing with HIP events recorded on the context stream around every
 * kernel launch of the library (off by default).  Enabling resets the counters.
 * apx_profile_count (sync) returns the number of kernel names seen; entry k gives the
 * name (owned by the context), the number of launches and their summed duration. */
apx_status apx_profile_enable(apx_ctx* ctx, int32_t on);
int32_t apx_profile_count(apx_ctx* ctx);
apx_status apx_profile_entry(apx_ctx* ctx, int32_t k, const char** name, int64_t* launches,
                             double* total_ms);

/* Diagnostic: the FP64 functions the pair loops use, on x [n] (device): exp (Tang's
 * table-driven method, ACM TOMS 15(2), 1989), 1/x and 1/sqrt(x) (hardware estimates with
 * two Newton steps).  Outputs (device [n], each nullable). */
apx_status apx_fp64_functions(apx_ctx* ctx, int64_t n, const double* x, double* exp_out, double* rcp_out,
                              double* rsq_out);

/* ------------------------------------------------------------------- atoms */
typedef struct {
  int64_t n;             /* number of atoms */
  const double* pos;     /* device [3][n] positions, Angstrom */
  double lo[3], hi[3];   /* box bounds */
  int32_t periodic[3];   /* 1 = periodic along that axis */
  const uint8_t* frozen; /* device [n] or NULL: 1 = never moved, w pinned to 0, no CSP */
} apx_atoms;

/* --------------------------------------------------------- neighbour lists */
/* Full Verlet list in neighbour-major ELL layout: row i holds count[i] neighbours
 * idx[k*n + i], k < count[i], in ascending j; every j != i whose minimum-image
 * squared distance (dx*dx + dy*dy) + dz*dz is below r_list^2.  (The paper's force
 * routine works on such lists, Sec. II D; the definition is the plain one.) */
typedef struct {
  int64_t n;      /* atoms the list was built for */
  int32_t max_nb; /* row capacity, 1..128 */
  int32_t* count; /* device [n] */
  int32_t* idx;   /* device [max_nb][n] */
  double r_list;  /* cutoff the list was built with (force cutoff + skin) */
} apx_nlist;

/* Build `nl` for `atoms` with cutoff `r_list`.  Periodic dimensions need
 * r_list < L/2.  If some row needs more than nl->max_nb entries the call returns
 * APX_ECAPACITY and stores the largest row length in *needed (host, required; (sync)).
 * The rows' contents are then unspecified.  Otherwise *needed receives the largest row
 * length. */
apx_status apx_build_neighbors(apx_ctx* ctx, const apx_atoms* atoms, double r_list,
                               apx_nlist* nl, int32_t* needed);

/* ------------------------------------------------ detection and switching */
/* CSP: Sec. II B eq. csp_1_i with Appendix A (LAMMPS definition with N + N_buffer
 * candidates within r_cut, chosen by (squared distance, index); N/2 smallest pair
 * values |r_a + r_b|^2 summed in ascending order; fewer candidates: +inf).
 * w0: Appendix B eq. lambda_1_i read as the precise weight,
 *     switch_kind 1: w0 = 1 - f_cut((CSP - csp_lo)/(csp_hi - csp_lo)),
 *     switch_kind 0: w0 = clamp((CSP - csp_lo)/(csp_hi - csp_lo), 0, 1).
 * Spreading: Appendix B eq. lambda_2_i, precise-weight form
 *     w_i = max(w0_i, max_{j: r_ij < r_hi} w0_j f_cut((r_ij - r_lo)/(r_hi - r_lo)));
 *     r_hi = 0 disables it (w = w0).
 * f_cut: Appendix B, evaluated as ((1 - 1.875x) + 1.25x^3) - 0.375x^5 with
 * x^3 = (x*x)*x, x^5 = x^3*(x*x), every operation rounded separately. */
typedef struct {
  int32_t n_nn;        /* N, even, 2..16 (12 for FCC) */
  int32_t n_buffer;    /* N_buffer, N + N_buffer <= 16 */
  int32_t switch_kind; /* 0 linear, 1 f_cut */
  int32_t flags;       /* APX_PREC_CSP_GIVEN: csp is an input, the CSP pass is skipped;
                          APX_PREC_EXTRA_LOCAL: w0_extra joins after the spreading */
  double csp_lo, csp_hi; /* Angstrom^2 */
  double r_cut;          /* CSP candidate cutoff, <= nl->r_list */
  double r_lo, r_hi;     /* spreading radii, Angstrom */
} apx_prec_params;

#define APX_PREC_CSP_GIVEN 1
#define APX_PREC_EXTRA_LOCAL 2

/* Outputs (device, length n): csp, w0, w, mask (1 where w > 0); active receives the
 * indices with w > 0 in ascending order and *n_active (host, (sync)) their number.
 * w0_extra (device [n] or NULL) is an additional detection weight (the learned
 * criterion's) combined by max with the CSP-based w0 before spreading, or, with
 * APX_PREC_EXTRA_LOCAL, with the spread weight after it (its detections are then not
 * spread; w0 is the CSP-based weight alone).  Frozen atoms keep 0 either way. */
apx_status apx_compute_precision(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl,
                                 const apx_prec_params* p, const double* w0_extra,
                                 double* csp, double* w0, double* w, uint8_t* mask,
                                 int32_t* active, int64_t* n_active);

/* Time-averaged switching: Appendix B eqs. csp_2_i, lambda_1_i, lambda_2_i, lambda_3_i,
 * lambda_4_i (N_CSP,avg = N_lambda,avg = n_avg; Delta lambda_min = dw_min), in the
 * precise-weight form w = 1 - lambda.  One call takes one sample at the given positions:
 *   csp      the instantaneous CSP (as apx_compute_precision; an input with
 *            APX_PREC_CSP_GIVEN), pushed into csp_ring;
 *   csp_avg  window APX_WINDOW_PAST (eq. csp_2_i as printed, a sum over n = 1..N of
 *            earlier samples): the mean of the min(samples, n_avg) CSP samples taken
 *            before this call (this call's sample alone on the first call);
 *            APX_WINDOW_CURRENT: the mean of the newest min(samples + 1, n_avg) samples,
 *            this call's included;
 *   w0       the switch of csp_avg, combined with w0_extra by max; frozen atoms 0;
 *   w_min    w0 spread as in apx_compute_precision, pushed into w_ring;
 *   w_avg    (nullable) the mean of the newest min(samples + 1, n_avg) w_min samples
 *            (eq. lambda_3_i: the weight for the force evaluations after this sample);
 *   w        in: the filtered weight returned by the previous call (ignored on the
 *            first); out: w_avg where |w_avg - w_prev| >= dw_min or w_avg is 0 or 1,
 *            else w_prev (on the first call w_avg);
 *   mask, active, *n_active (host, (sync)) as in apx_compute_precision, from the new w.
 * A mean adds its samples newest first from 0.0 and divides by their number.  The rings
 * are caller-owned device arrays [n_avg][n] (slot-major) whose contents the calls keep;
 * `samples` counts the samples taken (0 before the first call) and each successful call
 * advances it by one; the ring slot of a call is samples % n_avg.  All arrays are device
 * arrays of length n.  EINVAL: n_avg outside 1..4096, samples < 0, dw_min < 0 or NaN,
 * an unknown window, missing rings, csp_avg or w_min, or any condition of
 * apx_compute_precision. */
#define APX_WINDOW_PAST 0
#define APX_WINDOW_CURRENT 1
typedef struct {
  int32_t n_avg;      /* samples per moving mean */
  int32_t window;     /* APX_WINDOW_PAST or APX_WINDOW_CURRENT */
  int64_t samples;    /* samples taken so far */
  double dw_min;      /* minimum step of the filtered weight */
  double* csp_ring;   /* device [n_avg][n] */
  double* w_ring;     /* device [n_avg][n] */
} apx_avg_state;

apx_status apx_compute_precision_avg(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl,
                                     const apx_prec_params* p, apx_avg_state* st,
                                     const double* w0_extra, double* csp, double* csp_avg,
                                     double* w0, double* w_min, double* w_avg, double* w,
                                     uint8_t* mask, int32_t* active, int64_t* n_active);

/* ------------------------------------------------------------------- EAM */
/* Sec. III B eq. energy_eam: E_i = F(rho_i) + 1/2 sum_j phi(r_ij), rho_i = sum_j rho(r_ij)
 * over r_ij < r_cut, psi(x) = x^4/(1 + x^4) for x < 0 else 0 (the taper of Appendix E).
 * kind APX_EAM_CLOSED: phi(r) = A exp(-alpha(r - r0)) psi((r - r_cut)/h),
 *     rho(r) = exp(-beta(r - r0)) psi((r - r_cut)/h), F(rho) = -sqrt(rho).
 * kind APX_EAM2: the paper's EAM2 copper potential (Appendix E, parameters of Table III;
 *     the refit's offset of Sec. III B added to the embedding), eam2[] holding in order
 *     E1, E2, delta, alpha1, alpha2, r01, r02, S1, S2, S3, rs1, rs2, rs3, a, beta1, beta2,
 *     r03, r04, xi0, xi2, q1, q2, q3, q4, Q1, Q2, f0:
 *     phi(r)  = (E1 M(r, r01, alpha1) + E2 M(r, r02, alpha2) + delta) psi((r - r_cut)/h)
 *               - sum_n [r <= rs_n] S_n (rs_n - r)^4,
 *     M(r, r0, alpha) = exp(-2 alpha (r - r0)) - 2 exp(-alpha (r - r0)),
 *     rho(r)  = (a exp(-beta1 (r - r03)^2) + exp(-beta2 (r - r04))) psi((r - r_cut)/h),
 *     F(x)    = xi0 + xi2 d^2/2 + sum_n q_n d^(n+2) for x <= 1, else
 *               (xi0 + xi2 d^2/2 + q1 d^3 + Q1 d^4)/(1 + Q2 d^3), d = x - 1; plus f0.
 * A, alpha, beta, r0 are unused for APX_EAM2. */
#define APX_EAM_CLOSED 0
#define APX_EAM2 1
typedef struct {
  double A, alpha, beta, r0, r_cut, h;
  int32_t kind;
  int32_t reserved;
  double eam2[27];
} apx_eam_params;

/* Outputs: e_site[n] = E_i^EAM (unweighted), rho[n], f[3][n] (overwritten) =
 * -d/dx sum_k (1 - w_k) E_k^EAM (Appendix C eq. F_i_d, fast part).  w NULL means 0.
 * rho may be NULL. */
apx_status apx_eam_forces(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl,
                          const apx_eam_params* p, const double* w, double* e_site,
                          double* rho, double* f);

/* ------------------------------------------------------------------- ACE */
/* Sec. III A: E_i = phi_i^(1) + sqrt(phi_i^(2)), phi^(p) = sum_v c_v^(p) B_iv, with the
 * synthetic basis: radial g_k(r) = T_k(2r/r_cut - 1) psi((r - r_cut)/h), k < n_max;
 * R_nl = sum_k W[l][n][k] g_k; real orthonormal Y_lm; A_nlm = (1/s_a) sum_j R_nl Y_lm;
 * B1_n = A_n00; B2_(n1<=n2,l) = sum_m A_n1lm A_n2lm; B3 over (n,l) labels
 * p = n(l_max+1) + l, p1 <= p2 <= p3, l1+l2+l3 even, triangle: sum G A A A with the
 * real Gaunt coefficients.  Basis order: B1 (n), B2 (n1, n2, l), B3 (p1, p2, p3).
 * sqrt is replaced by F_eps(x) = sign(x)(sqrt(|x| + eps^2) - eps).  If `anchored`, an
 * EAM site energy with parameters `anchor` (kind APX_EAM_CLOSED; EINVAL otherwise) is added
 * to E_i. */
typedef struct {
  int32_t n_max;    /* 1..12 */
  int32_t l_max;    /* 3 or 4 */
  double r_cut, h, s_a, eps;
  const double* W;  /* host [l_max+1][n_max][n_max] */
  const double* c1; /* host [n_basis] */
  const double* c2; /* host [n_basis] */
  int32_t anchored;
  int32_t reserved;
  apx_eam_params anchor;
} apx_ace_desc;

int64_t apx_ace_num_basis(int32_t n_max, int32_t l_max);
/* Work counts of a model per evaluated atom (host, no device work): out[0] label pairs,
 * out[1] third-block terms (triples), out[2] coupling terms summed over pairs,
 * out[3] sum over triples of (2L+1), out[4] product-basis size, out[5] atomic-base size. */
apx_status apx_ace_model_stats(const apx_ace_model* m, int64_t* out6);
/* Copies the descriptor's arrays to the device and builds the coupling tables. */
apx_status apx_ace_model_create(apx_ctx* ctx, const apx_ace_desc* desc, apx_ace_model** out);
void apx_ace_model_destroy(apx_ace_model* m);
/* Replaces the coefficient vectors c1, c2 (host [n_basis] each) of a model; used to
 * differentiate with respect to the coefficients.  Synchronises the context stream. */
apx_status apx_ace_model_set_coeffs(apx_ctx* ctx, apx_ace_model* m, const double* c1, const double* c2);

/* Evaluate ACE for the atoms listed in `active` (device, n_active entries, distinct).
 * e_site[n] (overwritten): E_i^ACE at active atoms, 0 elsewhere.  f[3][n]
 * (overwritten): -d/dx sum_{i active} w_i E_i^ACE (Appendix C eq. F_i_d, precise part);
 * w NULL means 1.  dE_dc1/dE_dc2 (device [n_basis] or NULL, overwritten):
 * d/dc of sum_i w_i E_i^ACE.  precision: APX_FP64, or APX_FP32 (basis, products and
 * adjoint in float32 with compensated energy sums; forces accumulated in float64). */
apx_status apx_ace_energy_forces(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl,
                                 const apx_ace_model* m, const double* w,
                                 const int32_t* active, int64_t n_active, int32_t precision,
                                 double* e_site, double* f, double* dE_dc1, double* dE_dc2);

/* ------------------------------------------------------------------ blend */
/* Sec. II A eq. energy_hyb (precise-weight form): e_site = (1-w) e_eam + w e_ace (the ACE
 * term only where w > 0); f = f_eam + f_ace; *e_pot (device scalar) = sum_i e_site,
 * deterministic pairwise order. */
apx_status apx_blend(apx_ctx* ctx, int64_t n, const double* w, const double* e_eam,
                     const double* e_ace, const double* f_eam, const double* f_ace,
                     double* e_site, double* f, double* e_pot);

/* *out (device scalar) = sum_i w_i e_i over n atoms (w NULL: all 1), summed in the blend's
 * deterministic pairwise order: the weighted precise energy sum_i w_i E_i^ACE of the
 * site-weighted energy (Sec. II A eq. energy_hyb), used as the autograd forward value. */
apx_status apx_weighted_sum(apx_ctx* ctx, int64_t n, const double* w, const double* e, double* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): apx_blend with the same arguments,
 * results and error behaviour, whose block partial sums live in a static device array
 * of the library (65,536 doubles per GPU, held until the process ends) instead of the
 * context's scratch.  It calls no allocation routine.  Limit: n <= 134,217,728 atoms
 * (65,536 blocks of 2,048); larger n returns APX_EINVAL.  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (different streams or contexts) race. */
apx_status apx_blend_noalloc(apx_ctx* ctx, int64_t n, const double* w, const double* e_eam,
                             const double* e_ace, const double* f_eam, const double* f_ace,
                             double* e_site, double* f, double* e_pot);

/* ---------------------------------------------------------- integration */
#define APX_MODE_ADAPTIVE 0 /* EAM everywhere, ACE where w > 0, w from the criterion */
#define APX_MODE_FULL_ACE 1 /* w = 1 for every atom, no EAM, no detection (frozen atoms keep their
                             site energies, which depend on mobile neighbours) */
#define APX_MODE_EAM 2      /* w = 0, no ACE, no detection */

/* ------------------------------------------------------- local thermostat */
/* Energy correction of a weight update (Sec. II C 2; Appendix C), precise-weight form
 * w = 1 - lambda.  Energy errors, eqs. Delta_V_i, Delta_T_i, Delta_E_i, per atom:
 *   dV_i = (w_d_i - w_c_i)(e_fast_i - e_precise_i)   (0 where w_d_i == w_c_i),
 *   dT_i = sum_a [dt^2/(8m)((F^c_ia)^2 - (F^d_ia)^2) + (F^c_ia - F^d_ia) v_half_ia dt/2],
 *   dE_i = dV_i + dT_i (0 for frozen atoms),
 * with F^d = f_d, F^c = f_d + df (interatomic forces only, eV/A; [3][n]), v_half the
 * velocities after the first half kick (A/ps, [3][n]), m = mass/9648.5332 (mass in amu),
 * dt in ps.  w_c: the constant reference weights (those of the previous force
 * evaluation); w_d: the updated ones.  frozen may be NULL.  Output dE [n] (eV). */
apx_status apx_thermostat_energy_errors(apx_ctx* ctx, int64_t n, const uint8_t* frozen, const double* w_c,
                                        const double* w_d, const double* e_fast, const double* e_precise,
                                        const double* f_d, const double* df, const double* v_half, double dt,
                                        double mass, double* dE);

/* Correction, eqs. p_resc_omega and beta_omega_i: every mobile atom i with dE_i != 0
 * rescales the velocities of its group Omega_i about the group's centre-of-mass velocity
 * v_cm by beta = sqrt(dE_i / K_rel + 1), K_rel = sum_j m |v_j - v_cm|^2 / 2, which keeps
 * the group's momentum and changes its kinetic energy by dE_i.  Omega_i is atom i plus the
 * mobile atoms j != i with minimum-image r_ij^2 < r_omega^2 at the given positions, all of
 * them if there are fewer than omega_max, else the omega_max - 1 with the smallest
 * priority: the first word of Philox4x64-10 (Salmon et al., SC'11) with counter
 * (i, j, step, 0) and key (seed, 0), ties to the smaller j.  Corrections run one after the
 * other in the order (colour, atom index), the colour being the parity pattern of the
 * atom's cell in a grid of floor(L/(2 r_omega)) cells per axis (at least 1; one fewer if
 * odd on a periodic axis), cell floor((x - lo) * (nc / L)) clamped; atoms of one colour in
 * different cells are 2 r_omega apart, so their groups are disjoint.  vel [3][n] (A/ps) is
 * updated in place.  *n_corrected and *n_failed (host, (sync)) count the corrections made
 * and those skipped because the radicand was negative or the group had no relative
 * momentum; any skip returns APX_ERADICAND after the others are applied (the paper
 * enlarges the group then, Appendix D).  APX_ECAPACITY: more than 8192 corrections in one
 * colour cell or more than 4096 candidates within r_omega of one atom (reduce r_omega). */
typedef struct {
  double r_omega;      /* group radius, A */
  int32_t omega_max;   /* |Omega|, the largest group (Appendix F: 800) */
  int32_t group_batch; /* most groups drawn and held at once (0: as many as 1 GiB holds); the
                          corrections and their order do not depend on it */
  uint64_t seed;       /* key of the group draw */
} apx_thermo_params;

apx_status apx_thermostat_correct(apx_ctx* ctx, const apx_atoms* atoms, double* vel, const double* dE,
                                  const apx_thermo_params* p, int64_t step, double mass, int64_t* n_corrected,
                                  int64_t* n_failed);

typedef struct {
  double dt;               /* ps */
  double mass;             /* amu */
  double skin;             /* neighbour skin, Angstrom; rebuild when an atom moved > skin/2 */
  int32_t max_nb;          /* neighbour row capacity (<= 128) */
  int32_t precision_every; /* recompute w every k steps (0: keep w) */
  int32_t ace_precision;   /* APX_FP64 or APX_FP32 */
  int32_t mode;            /* APX_MODE_* */
  int32_t indenter;        /* 1: spherical indenter on */
  int32_t avg_samples;     /* adaptive mode: 0 instantaneous weights; n > 0 time-averaged
                              weights (apx_compute_precision_avg) over n samples, one
                              sample per weight update, the history restarted by apx_md_init */
  double ind_radius, ind_k;  /* R (A), K (eV/A^3): U = K/3 (R - d)^3, force K (R - d)^2 */
  double ind_center[3];      /* centre at step 0 */
  double ind_velocity[3];    /* A/ps */
  double avg_dw_min;         /* minimum step of the time-averaged weight */
  int32_t avg_window;        /* APX_WINDOW_PAST: the sample of an update step is taken after
                                that step's forces (the force routine's order of Appendix G:
                                fast potential, precise potential, CSP, lambda) and its
                                weight serves the following steps; APX_WINDOW_CURRENT: the
                                update precedes the step's forces (eq. vv step 2) */
  int32_t thermostat;        /* 1: local thermostat at every step whose weights differ from
                                the previous force evaluation's (apx_thermostat_*) */
  apx_thermo_params thermo;  /* group radius, size and draw key of the thermostat */
} apx_md_params;

typedef struct {
  int64_t steps;         /* steps taken by the call */
  int64_t rebuilds;      /* neighbour rebuilds */
  int64_t precision_updates;
  int64_t n_active;      /* atoms with w > 0 after the call */
  double e_pot, e_kin;   /* at the end of the call, eV (potential excludes the indenter) */
  double e_indenter;     /* indenter energy at the end, eV */
  int64_t ace_atoms;     /* sum over the call's steps of the atoms ACE was evaluated for */
  int64_t thermo_steps;      /* steps whose weights changed and were corrected */
  int64_t thermo_corrected;  /* corrections applied */
  int64_t thermo_failed;     /* corrections skipped (negative radicand) */
} apx_md_stats;

/* An integrator bound to a box, potentials and criterion.  `atoms` supplies n, box,
 * periodicity and the frozen mask (pos is ignored).  The ACE model and EAM parameters
 * are referenced/copied; the model must outlive the integrator. */
apx_status apx_md_create(apx_ctx* ctx, const apx_atoms* atoms, const apx_md_params* p,
                         const apx_eam_params* eam, const apx_ace_model* ace,
                         const apx_prec_params* prec, apx_md** out);
void apx_md_destroy(apx_md* md);
/* Neighbour list, weights (unless mode fixes them) and forces at the current
 * positions: pos[3][n] (in), f[3][n] (out), w[n] (out). */
apx_status apx_md_init(apx_md* md, const double* pos, double* f, double* w);
/* Sec. II C eq. vv: n_steps velocity-Verlet steps with the weight update as step 2 (or,
 * with time-averaged weights and APX_WINDOW_PAST, after the step's forces).  pos, vel
 * (A/ps), f, w are device arrays updated in place; w holds the weights of the next force
 * evaluation.  With the thermostat on, a step whose weights changed evaluates the forces of
 * both weight sets in one pass (the difference only where weights differ; ACE over the
 * atoms with either weight > 0), then corrects the velocities after the second half kick.
 * A skipped correction ends the call after its step with APX_ERADICAND (stats filled).
 * stats: host, (sync). */
apx_status apx_verlet_step(apx_md* md, double* pos, double* vel, double* f, double* w,
                           int64_t n_steps, apx_md_stats* stats);
/* Switches the integrator's detection to the learned criterion combined with the
 * centro-symmetry one (mlp NULL: back to the centro-symmetry criterion alone).  The
 * network must outlive the integrator.  Adaptive mode only. */
typedef struct apx_mlp apx_mlp;
apx_status apx_md_set_mlp(apx_md* md, apx_mlp* mlp, double tau_lo, double tau_hi);
/* Device timers of the last apx_verlet_step call, milliseconds summed over its steps:
 * out[0] half kick + drift + neighbour rebuilds, [1] weight updates, [2] EAM, [3] ACE,
 * [4] blend + indenter + half kick.  Collected only while profiling is on for the context
 * (apx_profile_enable), which adds one device wait per step; zeros otherwise. */
apx_status apx_md_timings(apx_md* md, double* out5);

/* ------------------------------------------------ learned precision indicator */
/* The detection argument of the switching function may be replaced by another criterion
 * (Appendix B, after eq. lambda_1_i).  Learned criterion: a 4-64-64-64-1 tanh network on
 * per-atom features [rho_EAM, min(CSP, 50), coordination (neighbours closer than 3.08 A),
 * |F_EAM|] (inputs standardised with mu, sd) predicting log(|F_ACE - F_EAM| + 1e-3).
 * Parameters (float32, APX_MLP_PARAMS values): W1 [64][4], b1 [64], W2 [64][64], b2 [64],
 * W3 [64][64], b3 [64], W4 [64], b4 [1]. */
#define APX_MLP_PARAMS 8705
apx_status apx_mlp_create(apx_ctx* ctx, const float* params /*host*/, const float* mu /*host [4]*/,
                          const float* sd /*host [4]*/, apx_mlp** out);
void apx_mlp_destroy(apx_mlp* m);
apx_status apx_mlp_get_params(apx_ctx* ctx, const apx_mlp* m, float* params /*host; (sync)*/);
/* Feature range seen in training (host [4] each); outside it the learned weight is 0. */
apx_status apx_mlp_set_range(apx_mlp* m, const float* fmin, const float* fmax);
/* feat [n][4] float32 from rho [n], csp [n] and the unweighted EAM force f_eam [3][n]. */
apx_status apx_features(apx_ctx* ctx, const apx_atoms* atoms, const apx_nlist* nl, const double* rho,
                        const double* csp, const double* f_eam, float* feat);
/* float32 forward: out [n]. */
apx_status apx_mlp_forward(apx_ctx* ctx, const apx_mlp* m, const float* feat, int64_t n, float* out);
/* Gradient of the mean squared error over the nb samples sel[0..nb) (sel NULL: 0..nb-1)
 * of feat/target: grad [APX_MLP_PARAMS] and *loss (device) overwritten. */
apx_status apx_mlp_gradients(apx_ctx* ctx, apx_mlp* m, const float* feat, const float* target,
                             const int32_t* sel, int64_t nb, float* grad, float* loss);
/* Adam update of the parameters with grad (bias-corrected; the step counter is kept in m);
 * grad is cleared. */
apx_status apx_mlp_adam_step(apx_ctx* ctx, apx_mlp* m, const float* grad, float lr, float beta1,
                             float beta2, float eps);
/* One training step: gradients on the batch then Adam (lr, 0.9, 0.999, 1e-8); loss
 * (device scalar, may be NULL) receives the batch mean squared error. */
apx_status apx_mlp_train_step(apx_ctx* ctx, apx_mlp* m, const float* feat, const float* target,
                              const int32_t* sel, int64_t nb, float lr, float* loss);
/* Inference with bfloat16 weights and activations on the matrix cores, float32 sums. */
apx_status apx_mlp_infer_bf16(apx_ctx* ctx, apx_mlp* m, const float* feat, int64_t n, float* out);
/* Training labels of the learned criterion from the two potentials' forces f_precise,
 * f_fast [3][n] (float64, eV/A): dF [n] (float64, nullable) = |f_precise - f_fast| and
 * label [n] (float32) = log(dF + 1e-3). */
apx_status apx_mlp_labels(apx_ctx* ctx, int64_t n, const double* f_precise, const double* f_fast, double* dF,
                          float* label);
/* Statistics of the features feat [n][4] (float32), n >= 1: stats [16] (device, float64) =
 * per column the mean [0..3], the standard deviation with n - 1 [4..7] (the input
 * standardisation), the minimum [8..11] and the maximum [12..15] (the training range). */
apx_status apx_mlp_feature_stats(apx_ctx* ctx, const float* feat, int64_t n, double* stats);
/* Detection weight of the learned criterion (Appendix B: the argument of eq. lambda_1_i
 * replaced by the predicted force gap) from given predictions pred [n] (float32,
 * log(|dF| + 1e-3)) and features feat [n][4]: w0_extra [n] = 1 - f_cut((exp(pred) - 1e-3 -
 * tau_lo) / (tau_hi - tau_lo)) (exp in float64) for atoms whose features all lie in the
 * training range [fmin, fmax] (inclusive; apx_mlp_set_range), 0 outside (those keep the
 * centro-symmetry weight alone when combined by apx_compute_precision). */
apx_status apx_mlp_weight(apx_ctx* ctx, const apx_mlp* m, const float* pred, const float* feat, int64_t n,
                          double tau_lo, double tau_hi, double* w0_extra);
/* pred [n] = bfloat16 inference, then w0_extra [n] as apx_mlp_weight. */
apx_status apx_mlp_precision(apx_ctx* ctx, apx_mlp* m, const float* feat, int64_t n, double tau_lo,
                             double tau_hi, float* pred, double* w0_extra);

#ifdef __cplusplus
}
#endif
#endif /* APX_H */
