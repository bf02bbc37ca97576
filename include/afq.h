/*
 * afq.h -- C ABI of the MI355X phaseless-AFQMC walker-step library.
 *
 * Method: Sukurma et al., "Towards Large-Scale AFQMC Calculations: Large Time
 * Step Auxiliary-Field Quantum Monte Carlo" (arXiv 2403.02542).  The library
 * runs the batched walker step of Sec. II.A with the Split-2 propagator of
 * Sec. III.B, the Krylov (Sec. IV.C) or Taylor (Sec. IV.A) exponential, the
 * capping rules of Sec. V.A-D and the local energy of Eq. (eloc), entirely
 * in hand-written HIP kernels for gfx950.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Closed shell: N_alpha == N_beta == N.  One complex M x N orbital matrix
 *    per walker carries both spins; <Psi_T|Phi> = det(Psi_T^T Phi)^2.
 *  - Matrices at the boundary are row-major.  Complex arrays are interleaved
 *    (re, im) float64 pairs, i.e. the layout of complex128 / torch.cdouble.
 *  - `ptr_is_device` = 0: pointers are host memory and the call copies
 *    synchronously.  = 1: pointers are device memory on the context's device;
 *    the call enqueues on the context stream and returns (the caller keeps
 *    the buffers alive until the stream has passed the call).
 *  - Inputs are copied: the caller may free host inputs when a call returns.
 *  - The context owns all device state it allocates; nothing is shared
 *    between contexts.  One context per host thread.
 *  - Errors: every call returns an afq_status; no C++ exception crosses the
 *    boundary.  On error the context is unchanged and afq_last_error()
 *    describes the failure.
 */
#ifndef AFQ_H
#define AFQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct afq_ctx afq_ctx;
typedef int32_t afq_status;

enum {
  AFQ_OK = 0,
  AFQ_EINVAL = 1,   /* bad argument: shape, range, asymmetric input, ...       */
  AFQ_ENOMEM = 2,   /* device allocation failed                                 */
  AFQ_EDEVICE = 3,  /* HIP runtime error (text in afq_last_error)               */
  AFQ_ESTATE = 4,   /* call out of order (e.g. propagate before init_trial)     */
  AFQ_ENUMERIC = 5  /* every walker of a system is non-finite                   */
};
/* Exponential of the one-body operator on the orbitals: per-orbital Krylov
 * (Sec. IV.C, Eq. krylov), Taylor (Sec. IV.A, Eq. taylor), or block Krylov
 * (Sec. IV.D, Eq. bkrylov: one kN-dimensional Krylov space per walker for
 * all N orbitals, k N <= M; its small exponential needs one host
 * synchronisation per step, so the graph schedule does not run it). */
enum { AFQ_EXP_KRYLOV = 0, AFQ_EXP_TAYLOR = 1, AFQ_EXP_BLOCK_KRYLOV = 2, AFQ_EXP_CHEBYSHEV = 3 };
/* AFQ_EXP_CHEBYSHEV (Sec. IV.B, Eq. chebpoly): sum_{n=0}^{k} c_n T_n(A) Phi
 * with the three-term recurrence T_n = 2 A T_{n-1} - T_{n-2} applied to A
 * as it stands (no spectral shift or scaling), c_0 = J_0(i) = I_0(1),
 * c_n = 2 i^n J_n(-i) = 2 I_n(1); k operator applications. */
/* Precision of the dense contractions: FP64, or BF16-split operands on the
 * BF16 matrix cores with FP32 accumulation, three pieces per value (six
 * piece products, ~24 significand bits) or two pieces (three products, ~16
 * bits).
 *  MIXED:        local energy / Coulomb vector, operator build, one-body
 *                half-steps (as Phi + (B - I) Phi) and the operator-orbital
 *                products of the exponential, three pieces.
 *  MIXED_FAST:   the same with two pieces.
 *  MIXED_ENERGY: only the local-energy contraction (the exchange blocks
 *                T_g and the one-body energy), three pieces; propagation
 *                in FP64.
 * The Coulomb vector (force bias, Hartree term) is FP64 in every mode, a
 * contraction N times smaller than the exchange one, so that under
 * MIXED_ENERGY the walkers follow the FP64 trajectory.  Overlap, inverse,
 * QR, Arnoldi, weights and energy sums stay FP64. */
enum { AFQ_PREC_FP64 = 0, AFQ_PREC_MIXED = 1, AFQ_PREC_MIXED_FAST = 2, AFQ_PREC_MIXED_ENERGY = 3 };

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on, or NULL for a stream owned by the context (default priority). */
afq_status afq_create(afq_ctx** out, int device, void* hip_stream);
void afq_destroy(afq_ctx* ctx);
/* Text of the last error on this context; valid until the next call. */
const char* afq_last_error(const afq_ctx* ctx);

/* Hamiltonian of Eq. (mbham) in Cholesky form, Sec. II.A:
 *   h      M x M one-body matrix, symmetric (checked to 1e-12 relative),
 *   L      n_chol x M x M Cholesky vectors, each symmetric (checked),
 *          <pq|rs> = sum_g L[g,p,r] L[g,q,s],
 *   e_core constant energy.
 * Returns a system id (0, 1, ...) in *sys_id.  Several systems may live in
 * one context; they are propagated together by afq_propagate_batch. */
afq_status afq_init_hamiltonian(afq_ctx* ctx, int64_t M, int64_t n_chol,
                                const double* h, const double* L, double e_core,
                                int ptr_is_device, int32_t* sys_id);

/* Trial determinant Psi_T (Sec. II.A), row-major, host or device memory
 * (copied), columns orthonormal (checked to 1e-10).
 * Closed shell (n_beta == n_alpha): Psi_T is M x n_alpha; the alpha and
 * beta blocks of every walker are equal, so each trace of Eqs. eloc, hyben
 * and force_shift carries a spin factor 2.
 * Open shell (n_beta != n_alpha, either may be 0): Psi_T is
 * M x (n_alpha + n_beta), the alpha orbitals then the beta orbitals (each
 * set orthonormal; a UHF determinant).  The system is then rewritten in
 * the 2M spin orbitals as for afq_init_trial_spin_orbital (h and L_g become
 * diag(X, X) on the device, 4x their memory; 2M <= 512, n_alpha + n_beta <=
 * 80) and every later call sees M' = 2M and N = n_alpha + n_beta (an
 * AFQ_ENOMEM or AFQ_EDEVICE after the rewrite leaves the system in spin
 * orbitals without a trial: initialise a new system).  A trial with equal
 * counts but separate alpha and beta orbitals goes through
 * afq_init_trial_spin_orbital.  Precomputes the mean-field shift Lbar_g
 * (Eq. force_shift), the one-body matrix H1 = h - 1/2 sum_g L_g L_g +
 * sum_g Lbar_g L_g that accompanies the shifted HS transform, its
 * eigendecomposition for the exact half-step exp(-tau H1/2) of Sec. III.B,
 * the half-rotated Psi_T^T h and Psi_T^T L_g, and the trial energy
 * E_L(Psi_T).  AFQ_ESTATE if the system already has a trial. */
afq_status afq_init_trial(afq_ctx* ctx, int32_t sys_id, int64_t n_alpha,
                          int64_t n_beta, const double* psi_t, int ptr_is_device);

/* Trial of one determinant of spin orbitals (any N_alpha, N_beta, including
 * a UHF or a general determinant): the system's M basis functions are spin
 * orbitals (for a spatial Hamiltonian
 * (h, L) of M/2 orbitals, h and every L_g block-diagonal diag(X, X)) and
 * Psi_T is one M x n_elec determinant of spin orbitals (for (Psi_a, Psi_b)
 * the block-diagonal diag(Psi_a, Psi_b), n_elec = N_alpha + N_beta).  The
 * traces of Eqs. eloc, hyben and force_shift then run over one
 * determinant: spin factor 1.  Everything else, and every other entry point,
 * is as for afq_init_trial: walkers are M x n_elec, log-overlaps are of the
 * whole determinant; the two adjoints return AFQ_EINVAL on such a system.
 * The propagator keeps a walker in the block structure of H1 and L_g, so a
 * block-diagonal start stays block-diagonal. */
afq_status afq_init_trial_spin_orbital(afq_ctx* ctx, int32_t sys_id, int64_t n_elec,
                                       const double* psi_t, int ptr_is_device);

/* Walker store of a system (Eq. wavefun_rep): n_walkers determinants set to
 * phi0 (complex128, n_walkers x M x N) or, if phi0 is NULL, to Psi_T; weights
 * 1; log-overlaps log det(Psi_T^T Phi). */
afq_status afq_init_walkers(afq_ctx* ctx, int32_t sys_id, int64_t n_walkers,
                            const void* phi0, int ptr_is_device);

typedef struct {
  double tau;            /* imaginary time step                                  */
  int32_t exp_method;    /* AFQ_EXP_KRYLOV, AFQ_EXP_TAYLOR or AFQ_EXP_BLOCK_KRYLOV */
  int32_t exp_order;     /* k: Krylov dimension / Taylor order / block-Krylov
                            order (1..16), the number of operator applications */
  int32_t reorth_every;  /* QR after global step t when (t+1) % reorth_every == 0 */
  int32_t precision;     /* AFQ_PREC_*: FP64, MIXED, MIXED_FAST or MIXED_ENERGY  */
  int32_t n_steps;       /* steps to run                                         */
  int32_t energy_every;  /* local energy every this many steps (and at the last);
                            0 is read as 1.  Other steps form only the Coulomb
                            vector the next force bias needs, a ~100x cheaper
                            product than the local-energy contraction          */
  double e0;             /* energy shift E0 of Eq. (imag_prop): a value sets the
                            system's E0 and clears its update history; NaN keeps
                            the system's current E0 (the trial energy E_L(Psi_T)
                            after afq_init_walkers, unless updates moved it)    */
  uint64_t seed;         /* Philox key word 0 (word 1 is the system id)          */
  uint64_t step0;        /* global index of the first step (RNG counter, QR)     */
  const double* fields;  /* optional DEVICE array [n_steps][W][n_chol] of N(0,1)
                            fields (single-system calls only); NULL = Philox     */
  double* energies_out;  /* optional DEVICE array [n_sys][n_steps][2]:
                            (sum_w W E_L capped, sum_w W) per step               */
  int32_t schedule;      /* AFQ_SCHED_*: how the steps of several systems are
                            issued (results are the same for every schedule)     */
  int32_t e0_window;     /* 0: E0 stays fixed.  1..64: after every measured step
                            E0 becomes the mean of the last e0_window per-step
                            estimates sum W E_L / sum W that had sum W > 0 (the
                            "best estimate" reading of Sec. II.A); a step with
                            sum W = 0 leaves E0 unchanged                        */
  int32_t pop_every;     /* 0: no population control (the paper describes none).
                            > 0: after global step t with (t+1) % pop_every == 0,
                            comb resampling by weight: with T = sum_w W_w and
                            running sums C_i, slot j copies walker
                            min{i : C_i > (j + u) T / W}, u in [0, 1) from
                            Philox4x64-10 key (seed, sys_id + 2^32), counter
                            t + 1, word 0, u = (x >> 11) 2^-53; every copy gets
                            weight 1; T = 0 leaves the walkers alone             */
  int32_t propagator;    /* AFQ_PROP_*: the orbital update of a step (Sec. III);
                            all but SPLIT2 need precision FP64 or MIXED_ENERGY  */
  int32_t force_bias_at; /* AFQ_FB_START: f from the Green's function of the
                            walker at the start of the step (default).
                            AFQ_FB_HALF: f from that of exp(-tau H1/2) Phi,
                            after the first Split-2 half-step (SPLIT2 only;
                            one more overlap and Coulomb-vector product per
                            step).  The paper does not place f (Eq.
                            force_shift); any f is a change of variables of
                            the field integral                                  */
} afq_prop_params;
enum { AFQ_FB_START = 0, AFQ_FB_HALF = 1 };

/* Propagators (Sec. III), with A = -tau H_int^w and H1 the effective
 * one-body matrix (h - 1/2 sum_g L_g L_g + sum_g Lbar_g L_g):
 *  SPLIT2: exp(-tau H1 / 2) exp(A) exp(-tau H1 / 2) Phi (Sec. III.B),
 *  SPLIT1: exp(-tau H1) exp(A) Phi (Sec. III.A),
 *  TAYLOR: exp(A - tau H1) Phi, the refactorised exp(-tau H_eff^w) of
 *          Sec. III.C, by the step's exponential method (exp_method),
 *  CN:     (I - A_T / 2)^-1 (I + A_T / 2) Phi with A_T = A - tau H1, the
 *          Crank-Nicolson form of Sec. III.D, by a dense solve per walker
 *          (Gauss-Jordan with partial pivoting; exp_method is not used).
 * exp(-tau H1) and exp(-tau H1 / 2) are exact (eigendecomposition). */
enum { AFQ_PROP_SPLIT2 = 0, AFQ_PROP_SPLIT1 = 1, AFQ_PROP_TAYLOR = 2, AFQ_PROP_CN = 3 };

/* Schedules of afq_propagate_batch.
 *  SERIAL:  system after system, phase after phase, on the context stream.
 *  STREAMS: per step, the per-system work up to the new Green's function runs
 *           on four branch streams (systems assigned longest-first), then one
 *           local-energy launch per kernel instance covers all systems (FP64;
 *           tiles ordered longest-first), then the energies.
 *  GRAPH:   STREAMS captured once as a two-step HIP graph and replayed (the
 *           step index, reorthonormalisation schedule and estimator slot are
 *           read from device memory).  Krylov exponential only.
 *  AUTO:    SERIAL for one system; GRAPH (Krylov) or STREAMS (Taylor) for
 *           several.  STREAMS and GRAPH need library fields (fields == NULL),
 *           energy_every <= 1 and profiling off (EINVAL otherwise); AUTO then
 *           falls back to SERIAL. */
enum { AFQ_SCHED_AUTO = 0, AFQ_SCHED_SERIAL = 1, AFQ_SCHED_STREAMS = 2, AFQ_SCHED_GRAPH = 3 };

/* Run n_steps Split-2 walker steps on every walker of the listed systems.
 * Per step and walker (Sec. II.A, III.B, IV, V): force bias from the current
 * mixed Green's function with the |f| < 1 cap; shifted fields; operator
 * A = i sqrt(tau) sum_g (x_g - f_g) L_g; Phi <- B exp(A) B Phi with
 * B = exp(-tau H1/2); overlap ratio, hybrid energy and phaseless weight with
 * the reweighting cap; QR reorthonormalisation on schedule; local energy with
 * the energy window.  Enqueued on the context stream; no host synchronisation
 * inside the loop.  A walker whose new overlap or Green's function is not
 * finite, or whose reorthonormalisation fails (numerically rank-deficient
 * orbitals), is frozen: its state is held, its weight set to 0 and it is
 * counted (not an error; see afq_get_counters).  Workspace the call needs is
 * allocated by the library on first use and owned by the context: the
 * Krylov basis, the block table of the operator build and, for MIXED and
 * MIXED_FAST, three BF16 pieces of L per system (6 Gp M^2 bytes, Gp = G
 * rounded up to 32, made once) and of the operator per walker set
 * (6 W M Kq bytes, Kq = 2M rounded up to 32); a failed allocation returns
 * AFQ_ENOMEM. */
afq_status afq_propagate_batch(afq_ctx* ctx, const int32_t* sys_ids, int32_t n_sys,
                               const afq_prop_params* params);

/* Tile shapes from measurement.  For each listed system (with walkers), the
 * local-energy contraction is timed with the six tile shapes (Cholesky
 * blocks x walkers per workgroup) its occupancy model ranks best, and the
 * operator-orbital product with 1x, 2x, 4x ... its default number of column
 * blocks; each launch is timed `reps` times (< 1: 3) after a warm-up launch
 * on the context stream, with the system's current walkers and outputs to
 * scratch memory.  The fastest shapes are kept by the system and used by
 * every later call.  Walker state is not changed, and later results do not
 * depend on the choice (every output is the same sum in the same order).
 * Synchronises the context stream. */
afq_status afq_autotune(afq_ctx* ctx, const int32_t* sys_ids, int32_t n_sys, int32_t reps);

/* Local energy of every walker (Eq. eloc) at its current determinant:
 * eloc_out complex128 [W].  The Coulomb vector ell_g = <Lhat_g>_mixed,
 * complex128 [W][n_chol], is written to ell_out if it is not NULL.
 * precision: AFQ_PREC_* of the contraction (FP64 or BF16-split). */
afq_status afq_local_energy_batch(afq_ctx* ctx, int32_t sys_id, int32_t precision,
                                  double* eloc_out, double* ell_out, int ptr_is_device);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the FP64 local energy of every
 * walker exactly as afq_local_energy_batch computes it (same kernels, same
 * sums), with device pointers only -- eloc_out complex128 [W], ell_out
 * complex128 [W][n_chol] or NULL -- and without any device allocation.  The
 * per-(walker, Cholesky block) partial results live in a fixed 32 MiB
 * workspace that the library holds on each GPU it runs on for the life of
 * the process, so n_walkers * (n_chol + 1) must not exceed 1048576
 * (AFQ_EINVAL otherwise).  Unlike afq_local_energy_batch the call leaves the
 * step's own Coulomb vector alone.  Every call on a GPU shares that GPU's
 * workspace: calls that overlap on one GPU (other contexts or streams) race;
 * calls ordered on one stream are safe.  Enqueued on the context stream. */
afq_status afq_local_energy_batch_noalloc(afq_ctx* ctx, int32_t sys_id, double* eloc_out,
                                          double* ell_out);

/* Adjoint of the local energy at fixed walkers and fixed Psi_T:
 * grad_h[M][M]      = sum_w dE_dEL[w] d Re E_L^w / d h,
 * grad_L[g][M][M]   = sum_w dE_dEL[w] d Re E_L^w / d L_g,
 * with respect to unconstrained matrix entries (symmetrise for symmetric
 * parameters).  dE_dEL is real [W]. */
afq_status afq_local_energy_adjoint(afq_ctx* ctx, int32_t sys_id, const double* dE_dEL,
                                    double* grad_h, double* grad_L, int ptr_is_device);

/* Adjoint of the Coulomb vector (force bias without its affine map):
 * grad_L[g][M][M] = sum_w Re(d_ell[w][g]) d Re ell_g^w / d L_g
 *                 + Im(d_ell[w][g]) d Im ell_g^w / d L_g;  d_ell complex128. */
afq_status afq_force_bias_adjoint(afq_ctx* ctx, int32_t sys_id, const double* d_ell,
                                  double* grad_L, int ptr_is_device);

/* Read / write the walker store: phi complex128 [W][M][N], weight [W],
 * log_ovlp complex128 [W] (log det(Psi_T^T Phi) of the one stored
 * determinant: one spin block of a closed-shell walker), alive int32 [W].
 * Any output pointer may be NULL.  afq_set_walkers recomputes the Green's
 * functions and the log-overlaps of the given determinants. */
afq_status afq_get_walkers(afq_ctx* ctx, int32_t sys_id, void* phi, double* weight,
                           double* log_ovlp, int32_t* alive, int ptr_is_device);
afq_status afq_set_walkers(afq_ctx* ctx, int32_t sys_id, const void* phi,
                           const double* weight, int ptr_is_device);

/* Auxiliary fields of one step from the library's Philox4x64-10 generator:
 * out[w][g], n_walkers x n_chol float64 (device pointer). */
afq_status afq_fill_fields(afq_ctx* ctx, uint64_t seed, uint64_t sys_id, uint64_t step,
                           int64_t n_walkers, int64_t n_chol, double* out_dev);

/* Per-system diagnostics of the last afq_propagate_batch call (synchronises),
 * the first n (1..5) of: out[0] walkers not frozen at the last measured
 * step, out[1] capped force-bias components, out[2] Krylov happy
 * breakdowns, out[3] walkers frozen, out[4] walkers with weight W > 0 at
 * the last measured step (0 means the population is extinct: the estimator
 * sum W is 0). */
afq_status afq_get_counters(afq_ctx* ctx, int32_t sys_id, int64_t* out, int32_t n);

/* Current E0 of a system (synchronises): the value the next step uses. */
afq_status afq_get_e0(afq_ctx* ctx, int32_t sys_id, double* e0_out);

/* Per-phase timing with HIP events on the context stream.  While enabled,
 * afq_propagate_batch records an event pair around every phase of every
 * step; afq_profile_read synchronises, returns the accumulated milliseconds
 * and launch counts of the first n phases (AFQ_PH_*) and clears them. */
enum {
  AFQ_PH_FIELDS = 0, AFQ_PH_FORCE_BIAS, AFQ_PH_OPBUILD, AFQ_PH_ONEBODY, AFQ_PH_EXPONENTIAL,
  AFQ_PH_OVERLAP, AFQ_PH_WEIGHT, AFQ_PH_QR, AFQ_PH_EXCHANGE, AFQ_PH_ENERGY, AFQ_PH_COULOMB,
  AFQ_PH_POPCTL, AFQ_PH_COUNT
};
afq_status afq_profile(afq_ctx* ctx, int enable);
afq_status afq_profile_read(afq_ctx* ctx, double* ms_out, int64_t* launches_out, int n);

/* Wait for all work enqueued on the context stream. */
afq_status afq_sync(afq_ctx* ctx);

/* ---- statistics of a run's per-step estimates (host arrays; no context,
 * no device work).  The series are the (sum W Ebar, sum W) pairs of
 * energies_out, split into W_k and E_k by the caller. */

/* Sec. II.A: the time average over the steps k >= n_eq (0-based),
 *   out[0] = E_bar = sum W_k E_k / sum W_k,
 *   out[1] = sigma_E^2 = (sum W_k E_k^2 / sum W_k) - E_bar^2 (the squared
 *            energies take the same weights),
 *   out[2] = the number N of those steps.
 * E_bar and sigma_E^2 are NaN when N = 0 or sum W_k = 0.  EINVAL on null
 * pointers or negative sizes. */
afq_status afq_stats_time_average(const double* w, const double* e, int64_t n, int64_t n_eq,
                                  double* out);

/* The correlation length kappa of Eq. (variance), sigma_Ebar^2 =
 * sigma_E^2 kappa / N, from the unweighted series e[0..n):
 *   out[0] = 1 + 2 sum_{t=1}^{M} rho(t), rho(t) = C(t) / C(0) with
 *            C(t) = sum_i (E_i - m)(E_{i+t} - m) / (n - t), and the window
 *            M the smallest with M >= c kappa(M) (Sokal; c = 5 is usual),
 *   out[1] = M,
 *   out[2] = (se_l / se_0)^2 from the blocking transformation (block means
 *            of 2^l samples) at the smallest level l with
 *            (2^l)^3 > 2 n (se_l / se_0)^4 (Lee, Needs, Drummond, Towler),
 *   out[3] = l.
 * EINVAL for n < 2, c <= 0 or a non-finite entry. */
afq_status afq_stats_kappa(const double* e, int64_t n, double c, double* out);

/* The blocking levels behind out[2] above: for l < min(*n_levels,
 * max_levels), levels[3 l + 0..2] = (n_l, se_l, se_l / sqrt(2 (n_l - 1)))
 * with se_l^2 = sum (x - x_bar)^2 / (n_l (n_l - 1)) over the n_l block
 * means (a trailing odd sample dropped at each halving).  *n_levels gets
 * the number of levels with n_l >= 2. */
afq_status afq_stats_blocking(const double* e, int64_t n, double* levels, int32_t max_levels,
                              int32_t* n_levels);

/* Time-step extrapolation (Sec. V.G): least squares (weights 1 / sigma_i^2,
 * or 1 when sigma is NULL) of E(tau_i) = E0 + alpha tau + beta tau^2
 * (Eq. square_fit; AFQ_FIT_QUADRATIC), E0 + beta tau^2 (Eq.
 * pure_square_fit; AFQ_FIT_PURE_SQUARE) or E0 + alpha tau (AFQ_FIT_LINEAR).
 * coef[3] = (E0, alpha, beta) with the absent term 0; err[0] = the standard
 * error of E0 from (A^T Sigma^-1 A)^-1, err[1] = sigma_x = sqrt(sum
 * sigma_i^2) / n (Eq. staterr; NaN when sigma is NULL).  EINVAL for fewer
 * points than terms or a non-positive sigma, ENUMERIC for a singular
 * system (repeated tau). */
enum { AFQ_FIT_QUADRATIC = 0, AFQ_FIT_PURE_SQUARE = 1, AFQ_FIT_LINEAR = 2 };
afq_status afq_tau_fit(const double* tau, const double* e, const double* sigma, int32_t n,
                       int32_t form, double* coef, double* err);

#ifdef __cplusplus
}
#endif

#endif /* AFQ_H */
