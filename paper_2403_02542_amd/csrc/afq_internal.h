// Internal state of the walker-step library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

// E0 of a system on the device (read by the weight and energy kernels, so
// that captured launches follow updates): the current value and a ring of
// the last per-step estimates for the running-mean update.
constexpr int kE0Max = 64;
constexpr int kCounters = 5;
struct E0Dev {
  double e0;
  int count, head;
  double ring[kE0Max];
};

// Device arrays of one system.  Complex walker data are planar (separate
// real and imaginary arrays); a walker's orbitals are stored orbital-major,
// [w][j][p], so that one orbital is a contiguous M-vector.
struct SysDev {
  int M = 0, N = 0, G = 0, W = 0;
  double e_core = 0.0;
  // spin factor of the traces of one determinant: 2 for a closed-shell
  // determinant of spatial orbitals (both spin blocks equal), 1 for one
  // determinant of spin orbitals
  double spin = 2.0;
  // Hamiltonian
  double* h = nullptr;        // [M][M]
  double* L = nullptr;        // [G][M][M]
  // trial
  double* psit = nullptr;     // [N][M]   Psi_T^T
  double* Lx = nullptr;       // [(G+1)][N][M]: Psi_T^T L_g for g < G, Psi_T^T h for g = G
  // virtual space: Psi_perp, an orthonormal complement of the trial orbitals
  // ([Kv][M], one vector per row, Kv = M - N); the blocks restricted to it
  // Psi_T^T L_g Psi_perp ([(G+1)][N][Kv]) and to the trial space
  // T0_g = Psi_T^T L_g Psi_T ([(G+1)][N][N]); with Theta = Psi_T + Psi_perp
  // Theta_v, T_g = T0_g + (Psi_T^T L_g Psi_perp) Theta_v
  int Kv = 0;
  double* psiv = nullptr;
  double* Lov = nullptr;
  double* T0 = nullptr;
  double* t0tr = nullptr;     // [G] 2 tr T0_g (the trial part of ell_g)
  double* lbar = nullptr;     // [G]
  double* H1 = nullptr;       // [M][M]
  double* Bhalf = nullptr;    // [M][M] exp(-tau H1 / 2)
  double* Bm1 = nullptr;      // [M][M] exp(-tau H1 / 2) - I (expm1 form)
  double* Bfull = nullptr;    // [M][M] exp(-tau H1) (Split-1)
  double tau_b = -1.0;
  double e_const = 0.0, e_trial = 0.0;
  std::vector<double> h1_evals, h1_evecs;   // host eigendecomposition of H1
  bool trial_ready = false;
  // walkers
  double *phi_re = nullptr, *phi_im = nullptr;     // [W][N][M]
  double *phn_re = nullptr, *phn_im = nullptr;     // next-step orbitals
  double *th_re = nullptr, *th_im = nullptr;       // Theta = Phi (Psi_T^T Phi)^-1
  double *thv_re = nullptr, *thv_im = nullptr;     // [W][N][Kv] Theta_v = Psi_perp^T Theta
  double *thn_re = nullptr, *thn_im = nullptr;
  double* logdet = nullptr;   // [W][2]
  double* logdet_n = nullptr; // [W][2]
  double* weight = nullptr;   // [W]
  int* alive = nullptr;       // [W]
  int* bad = nullptr;         // [W] non-finite flag of the new state
  double* qr_logr = nullptr;  // [W] log det R of the step's reorthonormalisation
  double *ell_re = nullptr, *ell_im = nullptr;     // [W][G+1]
  double *ex_re = nullptr, *ex_im = nullptr;       // [W][G+1]
  double* eloc = nullptr;     // [W][2]
  double* ecap = nullptr;     // [W]
  double* x = nullptr;        // [W][G] fields
  double *av_re = nullptr, *av_im = nullptr;       // [W][G]: i sqrt(tau) (x - fbar)
  double* scal = nullptr;     // [W][4]: log I (re, im), s_mf (re, im)
  int* ncap = nullptr;        // [W]
  double *A_re = nullptr, *A_im = nullptr;         // [W][M][M] operator
  double *t1_re = nullptr, *t1_im = nullptr;       // [W][N][M] scratch
  double *t2_re = nullptr, *t2_im = nullptr;
  double *t3_re = nullptr, *t3_im = nullptr;
  int kmax = 0;
  double *kb_re = nullptr, *kb_im = nullptr;       // [W][N][kmax][M] Krylov basis
  // block Krylov (the basis reuses kb as [W][kmax N][M]): projected operator
  // [W][kb_k N][kb_k N], R [W][N][N], two [W][N][kb_k N] sets of the small
  // exponential, the QR flags and log det R; kb_k is the order allocated for
  int bk_k = 0;
  double *bkh_re = nullptr, *bkh_im = nullptr;
  double *bkr_re = nullptr, *bkr_im = nullptr;
  double *bkx_re = nullptr, *bkx_im = nullptr, *bky_re = nullptr, *bky_im = nullptr;
  double *bkz_re = nullptr, *bkz_im = nullptr;
  int* bk_bad = nullptr;
  double* bk_logr = nullptr;
  unsigned long long* bk_norm = nullptr;
  double* kh = nullptr;       // [W][N][kmax][kmax][2] Hessenberg
  double* kbeta = nullptr;    // [W][N]
  int* kdim = nullptr;        // [W][N]
  double* oinv = nullptr;     // [W][N][N][2]
  double* est = nullptr;      // [2] estimator scratch
  // device counters of the last propagate call: [0] walkers not frozen at
  // the last measured step, [1] capped force-bias components, [2] Krylov
  // breakdowns, [3] walkers frozen, [4] walkers with W > 0 at the last
  // measured step
  int* counters = nullptr;
  E0Dev* e0s = nullptr;       // E0 and its update history
  // generation of the walker-side buffers: bumped by every (re)allocation,
  // part of the key of a captured step graph
  uint64_t gen = 0;
  // Coulomb vector and exchange terms of a measurement-only BF16-split
  // local energy (so that it leaves the step's own arrays alone)
  double *mell_re = nullptr, *mell_im = nullptr, *mex_re = nullptr, *mex_im = nullptr;
  // population control scratch: running weight sums, source slots, flag,
  // and the gathered log-overlaps / energies [W][5]
  double* pc_cum = nullptr;
  int* pc_src = nullptr;
  int* pc_flag = nullptr;
  double* pc_small = nullptr;
  // mixed precision (BF16-split) operands
  int mx_pieces = 0;          // pieces of the current split arrays (0 = none)
  int Kp = 0;                 // K (= M) padded to a multiple of 32
  unsigned short* Lxb = nullptr;  // [P][(G+1) N][Kp] pieces of Psi_T^T L_g Psi_perp (K = Kv)
  int64_t Lxb_ps = 0;
  unsigned short* thb = nullptr;  // [P][W 2N][Kp] pieces of Theta_v
  int64_t thb_ps = 0;
  // BF16 pieces of the operator build, the one-body half-steps and the
  // operator-orbital products of the current propagate call (0 = FP64)
  int op_pieces = 0;
  // pieces of the operator, split once per step for the BF16-split
  // operator-orbital products: [P][W M][Kq], K = (re q | im q), Kq = 2M
  // padded to a multiple of 32 (allocated for three pieces on first use)
  unsigned short* Ab = nullptr;
  int64_t Ab_ps = 0;
  int Kq = 0;
  // BF16-split operator build: pieces of the Cholesky vectors transposed to
  // [P][M M][Gp] (made once, three pieces) and of the field coefficients
  // [P][2W][Gp] (per step), Gp = G padded to a multiple of 32
  // 8 x 16 blocks (p0, q0) of the operator on or above its diagonal, for the
  // FP64 build (the operator is symmetric; device table, made before the
  // first step)
  int2* op_blk = nullptr;
  int n_op_blk = 0;
  unsigned short* Ltb = nullptr;
  int64_t Ltb_ps = 0;
  unsigned short* avb = nullptr;
  int64_t avb_ps = 0;
  int Gp = 0;
  // tuned tile shape of the local-energy contraction (0 = occupancy model)
  int x_ga = 0, x_wb = 0;
  // tuned column blocks of the operator-orbital product (0 = default)
  int mv_ct = 0;
  // partial sums of the Coulomb-vector-only product (allocated on first use)
  double* coul_ws = nullptr;
  // adjoint workspace (allocated on first use, sized for the walker count)
  double* adj_ws = nullptr;
  size_t adj_ws_n = 0;        // doubles
  int adj_gchunk = 0;         // Cholesky blocks per chunk of the adjoint
  std::vector<void*> walker_allocs;
};

// Step state of a propagate call held in device memory, so that captured
// launches stay valid across replays: the fields, the reorthonormalisation
// schedule and the estimator slot read the current step from here.
struct CallState {
  uint64_t step;       // global index of the step that runs next (advanced per replay)
  uint64_t step0;      // first step of the call
  int64_t n_steps;     // steps of the call (row length of the estimator output)
  double* energies;    // [n_sys][n_steps][2] estimator output, or null
};

// One system's operands of the local-energy contraction (also one entry of
// a many-system launch): T_g^w = T0_g + Lov_g Theta_v^w over K = M - N.
// ct: column tiles of its kernel instance.
struct XSys {
  const double* Lov;
  const double* T0;
  const double* thv_re;
  const double* thv_im;
  double* ell_re;
  double* ell_im;
  double* ex_re;
  double* ex_im;
  int G1, N, K, W, GA, WB, grp, ct;
  double lscale;   // ell_g = lscale tr T_g (the spin factor)
};

// Head and exit count of a persistent launch's device work queue (zero
// between launches: the last block to leave resets it).
struct WorkQ {
  int head;
  int done;
};

// One system's operands of the per-walker back half of a step (overlap,
// QR, weight, commit) in a many-system persistent launch.
struct BackSys {
  const double* psit;
  double* phn_re;
  double* phn_im;
  double* thn_re;
  double* thn_im;
  double* logdet_n;
  int* bad;
  double* qr_logr;
  int* alive;
  double* weight;
  double* logdet;
  const double* scal;
  const E0Dev* e0s;
  int* nfrozen;
  const double* phi_re;
  const double* phi_im;
  const double* th_re;
  const double* th_im;
  double e_const;
  int N, M;
  double spin;
};

// ------------------------------------------------------------------ launchers
// Every launcher enqueues on `st` and returns hipGetLastError().

// Generic strided batched GEMM for set-up work (FP64 MFMA):
// C[b](r, c) = alpha * sum_k A(b, r, k) B(b, c, k) + beta * C[b](r, c), with
// A(b, r, k) = A[b sAb + r sAr + (k / kin) sAkb + (k % kin) sAk] and
// B(b, c, k) = B[b sBb + c sBc + (k / kin) sBkb + (k % kin) sBk].
struct GemmArgs {
  const double* A; int64_t sAb, sAr, sAk, sAkb;
  const double* B; int64_t sBb, sBc, sBk, sBkb;
  double* C; int64_t sCb, sCr, sCc;
  int R, Cn, K, kin, batch;
  double alpha, beta;
};
hipError_t launch_gemm(const GemmArgs& g, hipStream_t st);

hipError_t launch_fields(uint64_t seed, uint64_t sid, uint64_t step, int W, int G, double* out,
                         hipStream_t st, const CallState* cs = nullptr, int add = 0);
hipError_t launch_call_begin(CallState* cs, uint64_t step0, int64_t n_steps, double* energies,
                             hipStream_t st);
hipError_t launch_call_advance(CallState* cs, int n, hipStream_t st);
hipError_t launch_lbar(const SysDev& s, hipStream_t st);
hipError_t launch_axpy_L(const SysDev& s, const double* coef, double alpha, double* out,
                         hipStream_t st);
hipError_t launch_force_bias(SysDev& s, const double* x, double tau, hipStream_t st);
// Orbital-set views for the operator-orbital product: element (w, j, p) at
// w * sw + j * sj + p of the re / im planes.
struct VecRef {
  const double* re;
  const double* im;
  int64_t sw, sj;
};
struct VecOut {
  double* re;
  double* im;
  int64_t sw, sj;
};
hipError_t launch_opbuild(SysDev& s, hipStream_t st);
// out = A v over all walkers (the operator-orbital product of the exponentials).
hipError_t launch_matvec(SysDev& s, VecRef v, VecOut o, hipStream_t st);
// o = scale A v and sum += o over all walkers.
hipError_t launch_matvec_acc(SysDev& s, VecRef v, VecOut o, double scale, VecOut sum,
                             hipStream_t st);
// Chebyshev expansion out = sum_{n<=k} c_n T_n(A) in (k products); s1, s2: scratch.
hipError_t launch_chebyshev(SysDev& s, int k, const double* in_re, const double* in_im,
                            double* out_re, double* out_im, double* s1_re, double* s1_im,
                            double* s2_re, double* s2_im, hipStream_t st);
// Crank-Nicolson step out = (I - A/2)^-1 (I + A/2) in with A the current
// operator (destroyed); t: W N M scratch planes.
hipError_t launch_crank_nicolson(SysDev& s, const double* in_re, const double* in_im,
                                 double* out_re, double* out_im, double* t_re, double* t_im,
                                 hipStream_t st);
// Origins of the R x 16 blocks of an M x M symmetric matrix that hold an
// element on or above the diagonal, row blocks outermost.
void op_blocks(int M, int R, std::vector<int2>& out);
constexpr int kOpRowsFP64 = 8;
// BF16-split operator-orbital product out = A v (mode 0) or out = A v / n,
// sum += out (mode 1, a Taylor term), with the operator pieces in s.Ab.
hipError_t launch_matvec_mx(SysDev& s, VecRef v, VecOut o, int mode, double inv_n, VecOut sum,
                            hipStream_t st);
// Three pieces of L, transposed, into s.Ltb (once per system).
hipError_t launch_split_lt(SysDev& s, hipStream_t st);
// BF16-split operator build: pieces of the field coefficients, then the
// operator pieces s.Ab straight from the piece products.
hipError_t launch_opbuild_mx(SysDev& s, hipStream_t st);
// out = Bm in (FP64) for a given symmetric M x M matrix (Split-1's exp(-tau H1)).
hipError_t launch_onebody_mat(SysDev& s, const double* Bm, const double* in_re,
                              const double* in_im, double* out_re, double* out_im,
                              hipStream_t st);
// A^w += alpha D (real plane) for every walker: the refactorised operator
// A - tau H1 with D = H1, alpha = -tau.
hipError_t launch_add_real(SysDev& s, const double* D, double alpha, hipStream_t st);
hipError_t launch_onebody(SysDev& s, const double* in_re, const double* in_im, double* out_re,
                          double* out_im, hipStream_t st);
// Krylov exponential of the operator on every orbital: out = krylov_k(A, in);
// wv is a [W][N][M] scratch pair.
hipError_t launch_krylov(SysDev& s, int k, const double* in_re, const double* in_im,
                         double* out_re, double* out_im, double* wv_re, double* wv_im,
                         hipStream_t st);
// Taylor exponential: out = sum_{n<=k} A^n in / n!; s1, s2 are scratch pairs.
hipError_t launch_taylor(SysDev& s, int k, const double* in_re, const double* in_im,
                         double* out_re, double* out_im, double* s1_re, double* s1_im,
                         double* s2_re, double* s2_im, hipStream_t st);
// Overlap, log det and Theta of (phi_re, phi_im) for W walkers.
hipError_t launch_overlap(SysDev& s, int W, const double* ph_re, const double* ph_im,
                          double* logdet_out, double* th_re, double* th_im, int* bad,
                          hipStream_t st);
// Weight update; qr_logr (nullable) holds the log det R of this step's QR.
// Weight update against the system's device E0; qr_logr (nullable) holds
// the log det R of this step's QR.
hipError_t launch_weight(SysDev& s, double tau, const double* qr_logr, hipStream_t st);
// Reorthonormalisation of (ph_re, ph_im) in place; writes qr_logr[W] and
// marks walkers whose factorisation fails in s.bad.
// With cs set, the kernel itself decides from the device step whether this
// step reorthonormalises (qr_logr = 0 when it does not).
hipError_t launch_qr(SysDev& s, double* ph_re, double* ph_im, double* qr_logr, hipStream_t st,
                     const CallState* cs = nullptr, int add = 0, int every = 0);
// The same factorisation of W orbital sets at walker stride sw (doubles);
// failures are marked in bad[W] (the walker store's flags are left alone).
hipError_t launch_qr_strided(SysDev& s, double* ph_re, double* ph_im, int64_t sw, double* logr,
                             int* bad, hipStream_t st);
hipError_t launch_commit(SysDev& s, hipStream_t st);
// Back half of a step for many systems: one persistent launch over the
// items (system, walker) in the given order; QR when due (from the device
// step counter when cs is given, else qr_now).  max_n: largest N.
hipError_t launch_back_queue(const BackSys* d_sys, const int2* d_items, int n_items, int max_n,
                             WorkQ* q, double tau, const CallState* cs, int add, int every,
                             bool qr_now, hipStream_t st);
// Block-Krylov exponential (Eq. bkrylov): out = B_k exp(A_k) E_N R of every
// walker's orbital set `in`; wv is a [W][N][M] scratch pair.  Synchronises the
// stream once (the substep count of the small exponential is chosen on the
// host from the largest 1-norm of the A_k).
hipError_t launch_block_krylov(SysDev& s, int k, const double* in_re, const double* in_im,
                               double* out_re, double* out_im, double* wv_re, double* wv_im,
                               hipStream_t st);
// Theta_v = Psi_perp^T Theta of W walkers: [W][N][Kv] per plane.
hipError_t launch_project(const SysDev& s, int W, const double* th_re, const double* th_im,
                          double* thv_re, double* thv_im, hipStream_t st);
// Local energy of W walkers with Green's functions (th_re, th_im); the
// virtual-space part Theta_v goes to (thv_re, thv_im), [W][N][Kv] each.
hipError_t launch_exchange(SysDev& s, int W, const double* th_re, const double* th_im,
                           double* thv_re, double* thv_im, double* ell_re, double* ell_im,
                           double* ex_re, double* ex_im, hipStream_t st);
// Operands and grid of one system's contraction from Theta_v (tile shape from
// the tuner when set, else from the occupancy model).
hipError_t exchange_setup(const SysDev& s, int W, const double* thv_re, const double* thv_im,
                          double* ell_re, double* ell_im, double* ex_re, double* ex_im, XSys* p,
                          int* n_gt, int* n_wt);
// Tiles (gt, wt) of one system in the single-system launch order.
void exchange_tile_order(int n_gt, int n_wt, std::vector<int2>& out);
// One launch over the tiles (system, gt, wt) of systems sharing the kernel
// instance ct; d_sys and d_tiles are device tables.
hipError_t launch_exchange_group(int ct, const XSys* d_sys, const int4* d_tiles, int n_tiles,
                                 hipStream_t st);
// Column blocks of the operator-orbital product: default and largest
// admissible count (each block holds at most 8 column tiles of 16).
int matvec_default_blocks(int M);
int matvec_max_blocks(int M);
// One operator-orbital product out = A in over all walkers (tuner probe).
hipError_t launch_matvec_probe(SysDev& s, const double* in_re, const double* in_im, double* out_re,
                               double* out_im, hipStream_t st);
// Coulomb vector alone in FP64 (ell of every walker and Cholesky block into
// ell_re / ell_im [W][G + 1], the one-body entry g = G left alone), for the
// steps that do not measure the energy and after a BF16-split local energy.
// part: scratch of coulomb_slices(W, G, N M) x W x G doubles.
int coulomb_slices(int W, int G, int NM);
// The same Coulomb vector from the projected Theta_v (virtual space, K = N Kv):
// ell_g = 2 tr T0_g + 2 sum_(i,k) Lov_g[i][k] Theta_v[i][k]; part: scratch of
// coulomb_v_slices(W, G, N, Kv) x W x G doubles.
int coulomb_v_slices(int W, int G, int N, int Kv);
hipError_t launch_coulomb_v(SysDev& s, const double* thv_re, const double* thv_im, double* part,
                            double* ell_re, double* ell_im, hipStream_t st);
// t0tr[g] = 2 tr T0_g for g < G.
hipError_t launch_t0_trace(SysDev& s, hipStream_t st);
hipError_t launch_coulomb(SysDev& s, const double* th_re, const double* th_im, double* part,
                          double* ell_re, double* ell_im, hipStream_t st);
// Admissible (GA, WB) tile shapes for N, best first by the occupancy model.
void exchange_candidates(int N, std::vector<int2>& out);
hipError_t launch_energy(SysDev& s, int W, const double* ell_re, const double* ell_im,
                         const double* ex_re, const double* ex_im, double* eloc, double* ecap,
                         const E0Dev* e0s, double tau, hipStream_t st);
// With cs->energies set, out2 is replaced by row `row` of that array at the
// device step.  e0_window > 0: E0 follows the running mean of the estimates.
hipError_t launch_estimator(SysDev& s, double* out2, hipStream_t st, const CallState* cs = nullptr,
                            int add = 0, int64_t row = 0, int e0_window = 0);
hipError_t launch_set_e0(SysDev& s, double e0, hipStream_t st);
// Comb resampling of the walkers by weight after global step `step` when
// (step + 1) % every == 0 (device step under replay when cs is set).
hipError_t launch_pop_control(SysDev& s, uint64_t seed, uint64_t sid, uint64_t step, int every,
                              hipStream_t st, const CallState* cs = nullptr, int add = 0);
hipError_t launch_zero_counters(SysDev& s, hipStream_t st);
// Boundary layout (complex128 [W][M][N], interleaved) <-> planar [W][N][M].
hipError_t launch_to_planar(const double* in, int W, int M, int N, double* re, double* im,
                            hipStream_t st);
hipError_t launch_from_planar(const double* re, const double* im, int W, int M, int N,
                              double* out, hipStream_t st);
hipError_t launch_pack_complex(const double* re, const double* im, int64_t n, int64_t ld_in,
                               int64_t cols, double* out, hipStream_t st);
// BF16 pieces (see afq_device.h): rows of a float64 matrix, and Theta.
hipError_t launch_split(const double* in, int64_t R, int K, int64_t ld, int Kp, int P,
                        int64_t piece_stride, unsigned short* out, hipStream_t st);
hipError_t launch_split_theta(const double* re, const double* im, int W, int N, int M, int Kp,
                              int P, int64_t piece_stride, unsigned short* out, hipStream_t st);
// Mixed-precision local-energy contraction (pieces s.Lxb and tb).
hipError_t launch_exchange_mx(SysDev& s, int W, const unsigned short* tb, int64_t tb_ps,
                              double* ell_re, double* ell_im, double* ex_re, double* ex_im,
                              hipStream_t st);
// Adjoints (device pointers; scratch supplied by the caller):
// TH [W 2N M], Ub [gchunk N x W 2N], Db [S gchunk N M], Y [N M], ellt [G 2W];
// the Coulomb-vector adjoint uses Db as its [gchunk N M] scratch.
hipError_t launch_adjoint_into(SysDev& s, const double* dE, double* grad_h, double* grad_L,
                               double* TH, double* Ub, double* Db, double* Y, double* ellt,
                               int gchunk, hipStream_t st);
int adjoint_nsplit(int M, int N, int W, int gchunk);   // Db holds this many slices
hipError_t launch_fb_adjoint_into(SysDev& s, const double* d_ell, double* grad_L, double* TH,
                                  double* Z, int gchunk, hipStream_t st);

// Host symmetric eigensolver (cyclic Jacobi): a (n x n, row-major) is
// destroyed; evals ascending, evecs column j = eigenvector j (row-major).
void jacobi_eigh(int n, std::vector<double>& a, std::vector<double>& evals,
                 std::vector<double>& evecs);
// Orthonormal complement of the orthonormal columns of psi (m x n,
// row-major): out[(c - n) m + p], one vector per row (Householder QR).
void complement_basis(int m, int n, const std::vector<double>& psi, std::vector<double>& out);
