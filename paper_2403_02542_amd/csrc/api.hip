// C ABI of the walker-step library (declared in include/afq.h): context and
// system management, set-up of the trial, and the Split-2 step driver that
// enqueues the kernels of one walker step after another on one HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "afq.h"
#include "afq_internal.h"

struct PhaseEv {
  int phase;
  hipEvent_t a, b;
};

// Fixed device workspace of the allocation-free local energy
// (afq_local_energy_batch_noalloc): the Coulomb vector and exchange terms of
// every (walker, Cholesky block), four planes of W (G + 1) doubles.  Each
// GPU holds its own copy for the life of the process; host code uses only
// the address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchDoubles = (size_t)4 << 20;   // 32 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

struct afq_ctx {
  bool profiling = false;
  std::vector<PhaseEv> pending;
  std::vector<hipEvent_t> ev_pool;
  double ph_ms[AFQ_PH_COUNT] = {};
  int64_t ph_n[AFQ_PH_COUNT] = {};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<SysDev*> systems;
  std::vector<std::vector<void*>> sys_allocs;
  // many-system schedule: branch streams (default priority), fork/join
  // events, the device step state of graph replays, the tile tables of the
  // many-system local-energy launches and the captured step graphs
  // three branches and the context stream: the four hardware queues
  static constexpr int kBranches = 3;
  hipStream_t br[kBranches] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kBranches] = {};
  CallState* cs = nullptr;
  struct XTable {
    std::vector<char> key;
    XSys* d_sys = nullptr;
    int4* d_tiles = nullptr;
    std::vector<int> ct, begin, count;
  };
  std::vector<XTable> xtables;
  // item tables of the many-system back-half launch and its work queue
  struct BTable {
    std::vector<char> key;
    BackSys* d_sys = nullptr;
    int2* d_items = nullptr;
    int n_items = 0, max_n = 0;
  };
  std::vector<BTable> btables;
  static constexpr int kQueues = 4;
  WorkQ* wq = nullptr;
  struct GraphEntry {
    std::vector<char> key;
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
  };
  std::vector<GraphEntry> graphs;
  // this device's address of the fixed workspace `scratch`
  double* scratch_dev = nullptr;
};

namespace {

afq_status fail(afq_ctx* c, afq_status code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, AFQ_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TRY(x)                     \
  do {                             \
    afq_status s_ = (x);           \
    if (s_ != AFQ_OK) return s_;   \
  } while (0)

template <class T>
afq_status dalloc(afq_ctx* ctx, std::vector<void*>& owner, T** p, size_t n) {
  void* q = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&q, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, AFQ_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  owner.push_back(q);
  *p = (T*)q;
  return AFQ_OK;
}

void free_all(std::vector<void*>& v) {
  for (void* p : v) (void)hipFree(p);
  v.clear();
}

// Copy n doubles from a user pointer (host or device) into device memory.
afq_status copy_in(afq_ctx* ctx, double* dst, const double* src, size_t n, int is_dev) {
  HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                        is_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
  if (!is_dev) HIPCHK(hipStreamSynchronize(ctx->stream));
  return AFQ_OK;
}
afq_status copy_out(afq_ctx* ctx, void* dst, const void* src, size_t bytes, int is_dev) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, is_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        ctx->stream));
  if (!is_dev) HIPCHK(hipStreamSynchronize(ctx->stream));
  return AFQ_OK;
}

afq_status get_sys(afq_ctx* ctx, int32_t id, SysDev** s) {
  if (!ctx) return AFQ_EINVAL;
  if (id < 0 || id >= (int32_t)ctx->systems.size() || !ctx->systems[id])
    return fail(ctx, AFQ_EINVAL, "unknown system id " + std::to_string(id));
  *s = ctx->systems[id];
  return AFQ_OK;
}

// max |X[b][p][q] - X[b][q][p]| and max |X| over a batch of n x n matrices
__global__ void k_asym(const double* X, int64_t nb, int n, unsigned long long* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = nb * n * n;
  double d = 0.0, m = 0.0;
  if (e < tot) {
    const int64_t b = e / ((int64_t)n * n);
    const int r = (int)(e % ((int64_t)n * n));
    const int p = r / n, q = r % n;
    d = fabs(X[e] - X[b * n * n + (int64_t)q * n + p]);
    m = fabs(X[e]);
    if (!(d == d)) d = INFINITY;
  }
  for (int o = 32; o > 0; o >>= 1) {
    d = fmax(d, __shfl_xor(d, o, 64));
    m = fmax(m, __shfl_xor(m, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(d));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(m));
  }
}

afq_status check_symmetric(afq_ctx* ctx, const double* X, int64_t nb, int n, const char* what) {
  unsigned long long* d = nullptr;
  HIPCHK(hipMalloc(&d, 2 * sizeof(unsigned long long)));
  unsigned long long h[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(d, h, sizeof(h), hipMemcpyHostToDevice, ctx->stream);
  const int64_t tot = nb * n * n;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_asym, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, X, nb,
                       n, d);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(ctx, AFQ_EDEVICE, std::string("symmetry check: ") + hipGetErrorString(e));
  double asym, mx;
  std::memcpy(&asym, &h[0], 8);
  std::memcpy(&mx, &h[1], 8);
  if (!(asym <= 1e-12 * (mx > 1.0 ? mx : 1.0)))
    return fail(ctx, AFQ_EINVAL, std::string(what) + " is not symmetric (max asymmetry " +
                                     std::to_string(asym) + ")");
  return AFQ_OK;
}

// exp(-tau H1 / 2) from the host eigendecomposition, and B - I formed with
// expm1 (the correction the BF16-split half-step contracts, added to the
// FP64 orbitals, so that its rounding acts on the small part only).
afq_status ensure_half_step(afq_ctx* ctx, SysDev& s, double tau) {
  if (s.tau_b == tau && s.Bhalf && s.Bm1) return AFQ_OK;
  const int M = s.M;
  std::vector<double> d(M), dm(M), df(M), B((size_t)M * M, 0.0), Bm((size_t)M * M, 0.0),
      Bf((size_t)M * M, 0.0);
  for (int k = 0; k < M; ++k) {
    d[k] = std::exp(-0.5 * tau * s.h1_evals[k]);
    dm[k] = std::expm1(-0.5 * tau * s.h1_evals[k]);
    df[k] = std::exp(-tau * s.h1_evals[k]);
  }
  const double* V = s.h1_evecs.data();
  for (int p = 0; p < M; ++p)
    for (int q = p; q < M; ++q) {
      double acc = 0.0, am = 0.0, af = 0.0;
      for (int k = 0; k < M; ++k) {
        const double vv = V[(size_t)p * M + k] * V[(size_t)q * M + k];
        acc += vv * d[k];
        am += vv * dm[k];
        af += vv * df[k];
      }
      B[(size_t)p * M + q] = acc;
      B[(size_t)q * M + p] = acc;
      Bm[(size_t)p * M + q] = am;
      Bm[(size_t)q * M + p] = am;
      Bf[(size_t)p * M + q] = af;
      Bf[(size_t)q * M + p] = af;
    }
  HIPCHK(hipMemcpy(s.Bhalf, B.data(), sizeof(double) * M * M, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s.Bm1, Bm.data(), sizeof(double) * M * M, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s.Bfull, Bf.data(), sizeof(double) * M * M, hipMemcpyHostToDevice));
  s.tau_b = tau;
  return AFQ_OK;
}

afq_status ensure_krylov(afq_ctx* ctx, int32_t sid, SysDev& s, int k) {
  if (k <= s.kmax) return AFQ_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  auto& own = s.walker_allocs;
  // the Krylov arrays are re-allocated; the old ones stay owned until destroy
  const size_t WN = (size_t)s.W * s.N;
  TRY(dalloc(ctx, own, &s.kb_re, WN * k * s.M));
  TRY(dalloc(ctx, own, &s.kb_im, WN * k * s.M));
  TRY(dalloc(ctx, own, &s.kh, WN * k * k * 2));
  s.kmax = k;
  ++s.gen;
  (void)sid;
  return AFQ_OK;
}

// Split-K scratch of the FP64 Coulomb vector.
afq_status ensure_coulomb(afq_ctx* ctx, SysDev& s) {
  if (s.coul_ws) return AFQ_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  const int S1 = coulomb_slices(s.W, s.G, s.N * s.M), S2 = coulomb_v_slices(s.W, s.G, s.N, s.Kv);
  const size_t n = (size_t)(S1 > S2 ? S1 : S2) * s.W * s.G;
  TRY(dalloc(ctx, s.walker_allocs, &s.coul_ws, n));
  ++s.gen;
  return AFQ_OK;
}

// Buffers of the block-Krylov exponential of order k (kept for larger k).
afq_status ensure_bkrylov(afq_ctx* ctx, SysDev& s, int k) {
  if (k <= s.bk_k) return AFQ_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  auto& own = s.walker_allocs;
  const size_t W = s.W, N = s.N, D = (size_t)k * N;
  TRY(dalloc(ctx, own, &s.bkh_re, W * D * D));
  TRY(dalloc(ctx, own, &s.bkh_im, W * D * D));
  TRY(dalloc(ctx, own, &s.bkr_re, W * N * N));
  TRY(dalloc(ctx, own, &s.bkr_im, W * N * N));
  double** sets[] = {&s.bkx_re, &s.bkx_im, &s.bky_re, &s.bky_im, &s.bkz_re, &s.bkz_im};
  for (double** p : sets) TRY(dalloc(ctx, own, p, W * N * D));
  TRY(dalloc(ctx, own, &s.bk_bad, W));
  TRY(dalloc(ctx, own, &s.bk_logr, W));
  TRY(dalloc(ctx, own, &s.bk_norm, 1));
  s.bk_k = k;
  ++s.gen;
  return AFQ_OK;
}

// BF16 pieces of the half-rotated blocks and a Theta piece buffer.
// Block table of the symmetric FP64 operator build (made once per system,
// on the host, before any step is captured).
afq_status ensure_op_blocks(afq_ctx* ctx, int32_t sid, SysDev& s) {
  if (s.op_blk) return AFQ_OK;
  std::vector<int2> b;
  op_blocks(s.M, kOpRowsFP64, b);
  int2* d = nullptr;
  TRY(dalloc(ctx, ctx->sys_allocs[sid], &d, b.size()));
  HIPCHK(hipMemcpy(d, b.data(), sizeof(int2) * b.size(), hipMemcpyHostToDevice));
  s.op_blk = d;
  s.n_op_blk = (int)b.size();
  return AFQ_OK;
}

afq_status ensure_mixed(afq_ctx* ctx, int32_t sid, SysDev& s, int pieces) {
  if (s.mx_pieces == pieces && s.Lxb && s.thb) return AFQ_OK;
  auto& own = ctx->sys_allocs[sid];
  auto& wown = s.walker_allocs;
  s.Kp = (s.Kv + 31) / 32 * 32;
  const int64_t rows = (int64_t)(s.G + 1) * s.N;
  if (!s.Lxb || s.mx_pieces < pieces) {
    TRY(dalloc(ctx, own, &s.Lxb, (size_t)3 * rows * s.Kp));
    s.Lxb_ps = rows * s.Kp;
  }
  if (!s.thb) {
    TRY(dalloc(ctx, wown, &s.thb, (size_t)3 * s.W * 2 * s.N * s.Kp));
    s.thb_ps = (int64_t)s.W * 2 * s.N * s.Kp;
    ++s.gen;
  }
  HIPCHK(launch_split(s.Lov, rows, s.Kv, s.Kv, s.Kp, pieces, s.Lxb_ps, s.Lxb, ctx->stream));
  s.mx_pieces = pieces;
  return AFQ_OK;
}

// Local energy and Coulomb vector of the current walkers (Theta in th_*).
afq_status eval_energy(afq_ctx* ctx, SysDev& s) {
  HIPCHK(launch_exchange(s, s.W, s.th_re, s.th_im, s.thv_re, s.thv_im, s.ell_re, s.ell_im,
                         s.ex_re, s.ex_im, ctx->stream));
  HIPCHK(launch_energy(s, s.W, s.ell_re, s.ell_im, s.ex_re, s.ex_im, s.eloc, s.ecap, s.e0s, 0.0,
                       ctx->stream));
  return AFQ_OK;
}

afq_status refresh_green(afq_ctx* ctx, SysDev& s) {
  HIPCHK(launch_overlap(s, s.W, s.phi_re, s.phi_im, s.logdet, s.th_re, s.th_im, s.bad,
                        ctx->stream));
  return AFQ_OK;
}

__global__ void k_init_alive(int W, const int* bad, int* alive, double* weight, int set_weight) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  alive[w] = bad[w] ? 0 : 1;
  if (set_weight) weight[w] = 1.0;
  if (bad[w]) weight[w] = 0.0;
}

__global__ void k_fill_trial(int W, int NM, const double* psit, double* re, double* im) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)W * NM) return;
  re[e] = psit[e % NM];
  im[e] = 0.0;
}

hipEvent_t take_event(afq_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records an event pair around a phase when profiling is on.
struct Phase {
  afq_ctx* ctx;
  int ph;
  hipEvent_t a = nullptr;
  Phase(afq_ctx* c, int p) : ctx(c), ph(p) {
    if (ctx->profiling) {
      a = take_event(ctx);
      if (a) (void)hipEventRecord(a, ctx->stream);
    }
  }
  ~Phase() {
    if (a) {
      hipEvent_t b = take_event(ctx);
      if (b) {
        (void)hipEventRecord(b, ctx->stream);
        ctx->pending.push_back(PhaseEv{ph, a, b});
      } else {
        ctx->ev_pool.push_back(a);
      }
    }
  }
};

// BF16 pieces of the local-energy contraction and of the propagation
// contractions (operator build, half-steps, operator-orbital products) for a
// precision mode; 0 = FP64.
int energy_pieces(int prec) {
  return prec == AFQ_PREC_FP64 ? 0 : prec == AFQ_PREC_MIXED_FAST ? 2 : 3;
}
int op_pieces_of(int prec) {
  return prec == AFQ_PREC_MIXED ? 3 : prec == AFQ_PREC_MIXED_FAST ? 2 : 0;
}

bool reorth_due(uint64_t t, int every) { return every > 0 && ((t + 1) % (uint64_t)every) == 0; }

// Everything of one walker step up to the new Green's function: fields,
// force bias, operator, B exp(A) B, overlap and weight, reorthonormalisation
// and the commit of the new state.  With cs set (captured replays) the step
// index is read on the device, offset by `add`.
// out = exp(A) in by the step's method; t3 and `spare` (both W N M planes,
// distinct from in and out) are scratch.
afq_status exponential(afq_ctx* ctx, SysDev& s, const afq_prop_params& P, const double* in_re,
                       const double* in_im, double* out_re, double* out_im, double* spare_re,
                       double* spare_im, hipStream_t st) {
  if (P.exp_method == AFQ_EXP_KRYLOV)
    HIPCHK(launch_krylov(s, P.exp_order, in_re, in_im, out_re, out_im, s.t3_re, s.t3_im, st));
  else if (P.exp_method == AFQ_EXP_BLOCK_KRYLOV)
    HIPCHK(launch_block_krylov(s, P.exp_order, in_re, in_im, out_re, out_im, s.t3_re, s.t3_im,
                                 st));
  else if (P.exp_method == AFQ_EXP_CHEBYSHEV)
    HIPCHK(launch_chebyshev(s, P.exp_order, in_re, in_im, out_re, out_im, s.t3_re, s.t3_im,
                            spare_re, spare_im, st));
  else
    HIPCHK(launch_taylor(s, P.exp_order, in_re, in_im, out_re, out_im, s.t3_re, s.t3_im,
                           spare_re, spare_im, st));
  return AFQ_OK;
}

afq_status step_front(afq_ctx* ctx, int32_t sid, SysDev& s, const afq_prop_params& P,
                      const double* x_given, uint64_t t, const CallState* cs, int add,
                      hipStream_t st) {
  const bool half_fb = P.force_bias_at == AFQ_FB_HALF;
  if (half_fb) {
    // the force bias from Phi' = exp(-tau H1/2) Phi: Theta' and the Coulomb
    // vector at Phi' (the proposed-state buffers serve as scratch; the back
    // half of the step overwrites them)
    {
      Phase ph(ctx, AFQ_PH_ONEBODY);
      HIPCHK(launch_onebody(s, s.phi_re, s.phi_im, s.t1_re, s.t1_im, st));
    }
    {
      Phase ph(ctx, AFQ_PH_OVERLAP);
      HIPCHK(launch_overlap(s, s.W, s.t1_re, s.t1_im, s.logdet_n, s.thn_re, s.thn_im, s.bad, st));
    }
    Phase ph(ctx, AFQ_PH_COULOMB);
    HIPCHK(launch_coulomb(s, s.thn_re, s.thn_im, s.coul_ws, s.ell_re, s.ell_im, st));
  }
  const double* x = s.x;
  if (x_given) {
    x = x_given;
  } else {
    Phase ph(ctx, AFQ_PH_FIELDS);
    HIPCHK(launch_fields(P.seed, (uint64_t)sid, t, s.W, s.G, s.x, st, cs, add));
  }
  {
    Phase ph(ctx, AFQ_PH_FORCE_BIAS);
    HIPCHK(launch_force_bias(s, x, P.tau, st));
  }
  {
    Phase ph(ctx, AFQ_PH_OPBUILD);
    HIPCHK(launch_opbuild(s, st));
  }
  if (P.propagator == AFQ_PROP_CN) {
    Phase ph(ctx, AFQ_PH_EXPONENTIAL);
    HIPCHK(launch_add_real(s, s.H1, -P.tau, st));
    HIPCHK(launch_crank_nicolson(s, s.phi_re, s.phi_im, s.phn_re, s.phn_im, s.t1_re, s.t1_im, st));
    return AFQ_OK;
  }
  if (P.propagator == AFQ_PROP_TAYLOR) {
    // the refactorised operator A - tau H1, its exponential straight into
    // the proposed orbitals (t1 as scratch)
    Phase ph(ctx, AFQ_PH_EXPONENTIAL);
    HIPCHK(launch_add_real(s, s.H1, -P.tau, st));
    TRY(exponential(ctx, s, P, s.phi_re, s.phi_im, s.phn_re, s.phn_im, s.t1_re, s.t1_im, st));
    return AFQ_OK;
  }
  const double* in_re = s.phi_re;
  const double* in_im = s.phi_im;
  if (P.propagator == AFQ_PROP_SPLIT2) {
    if (!half_fb) {
      Phase ph(ctx, AFQ_PH_ONEBODY);
      HIPCHK(launch_onebody(s, s.phi_re, s.phi_im, s.t1_re, s.t1_im, st));
    }
    in_re = s.t1_re;
    in_im = s.t1_im;
  }
  {
    Phase ph(ctx, AFQ_PH_EXPONENTIAL);
    TRY(exponential(ctx, s, P, in_re, in_im, s.t2_re, s.t2_im, s.phn_re, s.phn_im, st));
  }
  {
    Phase ph(ctx, AFQ_PH_ONEBODY);
    if (P.propagator == AFQ_PROP_SPLIT2)
      HIPCHK(launch_onebody(s, s.t2_re, s.t2_im, s.phn_re, s.phn_im, st));
    else
      HIPCHK(launch_onebody_mat(s, s.Bfull, s.t2_re, s.t2_im, s.phn_re, s.phn_im, st));
  }
  return AFQ_OK;
}

// The new orbitals' host pointers become the held ones.
void swap_state(SysDev& s) {
  std::swap(s.phi_re, s.phn_re);
  std::swap(s.phi_im, s.phn_im);
  std::swap(s.th_re, s.thn_re);
  std::swap(s.th_im, s.thn_im);
}

// Back half of one system's step: overlap and Theta at the proposed
// orbitals, QR when due, weights, frozen walkers restored.
afq_status step_back(afq_ctx* ctx, SysDev& s, const afq_prop_params& P, uint64_t t,
                     const CallState* cs, int add, hipStream_t st) {
  {
    Phase ph(ctx, AFQ_PH_OVERLAP);
    HIPCHK(launch_overlap(s, s.W, s.phn_re, s.phn_im, s.logdet_n, s.thn_re, s.thn_im, s.bad, st));
  }
  bool qr;
  if (cs) {
    qr = P.reorth_every > 0;   // the kernel applies the schedule itself
    if (qr) {
      Phase ph(ctx, AFQ_PH_QR);
      HIPCHK(launch_qr(s, s.phn_re, s.phn_im, s.qr_logr, st, cs, add, P.reorth_every));
    }
  } else {
    qr = reorth_due(t, P.reorth_every);
    if (qr) {
      Phase ph(ctx, AFQ_PH_QR);
      HIPCHK(launch_qr(s, s.phn_re, s.phn_im, s.qr_logr, st));
    }
  }
  {
    Phase ph(ctx, AFQ_PH_WEIGHT);
    HIPCHK(launch_weight(s, P.tau, qr ? s.qr_logr : nullptr, st));
  }
  {
    Phase ph(ctx, AFQ_PH_WEIGHT);
    HIPCHK(launch_commit(s, st));
  }
  swap_state(s);
  return AFQ_OK;
}

// Local-energy contraction of one system (FP64 or BF16-split).
afq_status step_exchange(afq_ctx* ctx, SysDev& s, const afq_prop_params& P, hipStream_t st) {
  Phase ph(ctx, AFQ_PH_EXCHANGE);
  if (energy_pieces(P.precision) == 0) {
    HIPCHK(launch_exchange(s, s.W, s.th_re, s.th_im, s.thv_re, s.thv_im, s.ell_re, s.ell_im,
                           s.ex_re, s.ex_im, st));
  } else {
    HIPCHK(launch_project(s, s.W, s.th_re, s.th_im, s.thv_re, s.thv_im, st));
    HIPCHK(launch_split_theta(s.thv_re, s.thv_im, s.W, s.N, s.Kv, s.Kp, s.mx_pieces, s.thb_ps,
                              s.thb, st));
    HIPCHK(launch_exchange_mx(s, s.W, s.thb, s.thb_ps, s.ell_re, s.ell_im, s.ex_re, s.ex_im, st));
    // the force bias of the next step (and the Hartree term) from the FP64
    // Coulomb vector over the virtual space: the walkers follow the FP64
    // trajectory
    HIPCHK(launch_coulomb_v(s, s.thv_re, s.thv_im, s.coul_ws, s.ell_re, s.ell_im, st));
  }
  return AFQ_OK;
}

// Energies and the weighted estimator of step si (row `row` of energies_out).
afq_status step_energy(afq_ctx* ctx, SysDev& s, const afq_prop_params& P, int si, int row,
                       const CallState* cs, int add, hipStream_t st) {
  Phase ph(ctx, AFQ_PH_ENERGY);
  HIPCHK(launch_energy(s, s.W, s.ell_re, s.ell_im, s.ex_re, s.ex_im, s.eloc, s.ecap, s.e0s, P.tau,
                       st));
  double* out = (!cs && P.energies_out) ? P.energies_out + ((size_t)row * P.n_steps + si) * 2
                                        : s.est;
  HIPCHK(launch_estimator(s, out, st, cs, add, row, P.e0_window));
  return AFQ_OK;
}

// Population control after the step (comb resampling; the kernels decide
// from the step index whether it is due).
afq_status step_pop(afq_ctx* ctx, int32_t sid, SysDev& s, const afq_prop_params& P, uint64_t t,
                    const CallState* cs, int add, hipStream_t st) {
  if (P.pop_every <= 0) return AFQ_OK;
  if (!cs && (t + 1) % (uint64_t)P.pop_every != 0) return AFQ_OK;
  Phase ph(ctx, AFQ_PH_POPCTL);
  HIPCHK(launch_pop_control(s, P.seed, (uint64_t)sid, t, P.pop_every, st, cs, add));
  return AFQ_OK;
}

afq_status step_system(afq_ctx* ctx, int32_t sid, SysDev& s, const afq_prop_params& P, int si,
                       int row) {
  const uint64_t t = P.step0 + (uint64_t)si;
  const double* x = P.fields ? P.fields + (size_t)si * s.W * s.G : nullptr;
  TRY(step_front(ctx, sid, s, P, x, t, nullptr, 0, ctx->stream));
  TRY(step_back(ctx, s, P, t, nullptr, 0, ctx->stream));
  const int every = P.energy_every > 0 ? P.energy_every : 1;
  const bool measure = (si + 1) % every == 0 || si + 1 == P.n_steps;
  if (measure) {
    TRY(step_exchange(ctx, s, P, ctx->stream));
    TRY(step_energy(ctx, s, P, si, row, nullptr, 0, ctx->stream));
  } else {
    // no energy this step: the next force bias needs only ell
    Phase ph(ctx, AFQ_PH_COULOMB);
    HIPCHK(launch_coulomb(s, s.th_re, s.th_im, s.coul_ws, s.ell_re, s.ell_im, ctx->stream));
  }
  TRY(step_pop(ctx, sid, s, P, t, nullptr, 0, ctx->stream));
  return AFQ_OK;
}

// ------------------------------------------------------------ many systems

afq_status ensure_sched(afq_ctx* ctx) {
  if (ctx->cs) return AFQ_OK;
  for (int b = 0; b < afq_ctx::kBranches; ++b) {
    HIPCHK(hipStreamCreateWithFlags(&ctx->br[b], hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_join[b], hipEventDisableTiming));
  }
  HIPCHK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  HIPCHK(hipMalloc(&ctx->wq, sizeof(WorkQ) * afq_ctx::kQueues));
  HIPCHK(hipMemset(ctx->wq, 0, sizeof(WorkQ) * afq_ctx::kQueues));
  HIPCHK(hipMalloc(&ctx->cs, sizeof(CallState)));
  return AFQ_OK;
}


// Rough cost of one step of a system (flops), for branch balancing and the
// order of the many-system local-energy tiles.
double step_cost(const SysDev& s, int k) {
  const double M = s.M, N = s.N, G = s.G, W = s.W;
  return W * ((G + 1) * 4.0 * N * N * M + 4.0 * G * M * M + 8.0 * k * M * M * N);
}

// Systems to branches: longest step first, each to the least loaded branch.
std::vector<std::vector<int>> assign_branches(const std::vector<SysDev*>& ss, int k) {
  const int n = (int)ss.size();
  const int nb = n < afq_ctx::kBranches ? n : afq_ctx::kBranches;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return step_cost(*ss[a], k) > step_cost(*ss[b], k); });
  std::vector<std::vector<int>> br(nb);
  std::vector<double> load(nb, 0.0);
  for (int i : order) {
    int b = 0;
    for (int c = 1; c < nb; ++c)
      if (load[c] < load[b]) b = c;
    br[b].push_back(i);
    load[b] += step_cost(*ss[i], k);
  }
  return br;
}

// Destroys every cached step graph (the caller has waited for the stream).
void clear_graphs(afq_ctx* ctx) {
  for (auto& g : ctx->graphs) {
    (void)hipGraphExecDestroy(g.ex);
    (void)hipGraphDestroy(g.g);
  }
  ctx->graphs.clear();
}

template <class T>
void put_bytes(std::vector<char>& key, const T& v) {
  const char* p = reinterpret_cast<const char*>(&v);
  key.insert(key.end(), p, p + sizeof(T));
}

// Tile table of the many-system local-energy launch for the systems' current
// Green's-function buffers (built once per buffer state, then reused).
afq_status get_xtable(afq_ctx* ctx, const std::vector<SysDev*>& ss, afq_ctx::XTable** out) {
  const int n = (int)ss.size();
  std::vector<XSys> xs(n);
  std::vector<int> ngt(n), nwt(n);
  std::vector<char> key;
  for (int i = 0; i < n; ++i) {
    SysDev& s = *ss[i];
    const hipError_t e = exchange_setup(s, s.W, s.thv_re, s.thv_im, s.ell_re, s.ell_im, s.ex_re,
                                        s.ex_im, &xs[i], &ngt[i], &nwt[i]);
    if (e != hipSuccess) return fail(ctx, AFQ_EINVAL, "local-energy tile set-up failed");
    put_bytes(key, xs[i]);
  }
  for (auto& t : ctx->xtables)
    if (t.key == key) {
      *out = &t;
      return AFQ_OK;
    }
  afq_ctx::XTable t;
  t.key = key;
  std::vector<int4> tiles;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  // longest tiles first (K = M - N), larger systems first within equal K
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (xs[a].K != xs[b].K) return xs[a].K > xs[b].K;
    return (int64_t)ngt[a] * nwt[a] > (int64_t)ngt[b] * nwt[b];
  });
  std::vector<int2> tl;
  for (int ct : {10, 8, 7, 4}) {
    const int begin = (int)tiles.size();
    for (int i : order) {
      if (xs[i].ct != ct) continue;
      tl.clear();
      exchange_tile_order(ngt[i], nwt[i], tl);
      for (const int2& g : tl) tiles.push_back(int4{i, g.x, g.y, 0});
    }
    if ((int)tiles.size() > begin) {
      t.ct.push_back(ct);
      t.begin.push_back(begin);
      t.count.push_back((int)tiles.size() - begin);
    }
  }
  std::vector<void*> tmp;
  TRY(dalloc(ctx, tmp, &t.d_sys, (size_t)n));
  afq_status r = dalloc(ctx, tmp, &t.d_tiles, tiles.size());
  if (r != AFQ_OK) {
    free_all(tmp);
    return r;
  }
  hipError_t e = hipMemcpy(t.d_sys, xs.data(), sizeof(XSys) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(t.d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_all(tmp);
    return fail(ctx, AFQ_EDEVICE, std::string("tile table: ") + hipGetErrorString(e));
  }
  if (ctx->xtables.size() >= 16) {   // bound the cache; tables in use are waited for
    HIPCHK(hipDeviceSynchronize());
    // captured graphs hold pointers to these tables: they go with them
    clear_graphs(ctx);
    for (auto& o : ctx->xtables) {
      (void)hipFree(o.d_sys);
      (void)hipFree(o.d_tiles);
    }
    ctx->xtables.clear();
  }
  ctx->xtables.push_back(std::move(t));
  *out = &ctx->xtables.back();
  return AFQ_OK;
}

// The cache of back-half item tables is bounded; tables in use are waited
// for, and the captured graphs that hold them go with them.
constexpr size_t kMaxBTables = 16;
afq_status clear_btables(afq_ctx* ctx) {
  HIPCHK(hipDeviceSynchronize());
  clear_graphs(ctx);
  for (auto& o : ctx->btables) {
    (void)hipFree(o.d_sys);
    (void)hipFree(o.d_items);
  }
  ctx->btables.clear();
  return AFQ_OK;
}

// Item table of the many-system back half for the current buffer state:
// systems by decreasing cost of their per-walker work (M N^2), each
// system's walkers in order.
afq_status get_btable(afq_ctx* ctx, const std::vector<SysDev*>& ss, afq_ctx::BTable** out) {
  const int n = (int)ss.size();
  std::vector<BackSys> bs(n);
  std::vector<char> key;
  int max_n = 0;
  for (int i = 0; i < n; ++i) {
    const SysDev& s = *ss[i];
    bs[i] = BackSys{s.psit, s.phn_re, s.phn_im, s.thn_re, s.thn_im, s.logdet_n, s.bad,
                    s.qr_logr, s.alive, s.weight, s.logdet, s.scal, s.e0s,
                    s.counters ? s.counters + 3 : nullptr, s.phi_re, s.phi_im, s.th_re,
                    s.th_im, s.e_const, s.N, s.M, s.spin};
    put_bytes(key, bs[i]);
    put_bytes(key, s.W);
    if (s.N > max_n) max_n = s.N;
  }
  for (auto& t : ctx->btables)
    if (t.key == key) {
      *out = &t;
      return AFQ_OK;
    }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (double)ss[a]->M * ss[a]->N * ss[a]->N > (double)ss[b]->M * ss[b]->N * ss[b]->N;
  });
  std::vector<int2> items;
  for (int i : order)
    for (int w = 0; w < ss[i]->W; ++w) items.push_back(int2{i, w});
  afq_ctx::BTable t;
  t.key = key;
  t.n_items = (int)items.size();
  t.max_n = max_n;
  std::vector<void*> tmp;
  TRY(dalloc(ctx, tmp, &t.d_sys, (size_t)n));
  afq_status r = dalloc(ctx, tmp, &t.d_items, items.size());
  if (r != AFQ_OK) {
    free_all(tmp);
    return r;
  }
  hipError_t e = hipMemcpy(t.d_sys, bs.data(), sizeof(BackSys) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(t.d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_all(tmp);
    return fail(ctx, AFQ_EDEVICE, std::string("item table: ") + hipGetErrorString(e));
  }
  if (ctx->btables.size() >= kMaxBTables) TRY(clear_btables(ctx));
  ctx->btables.push_back(std::move(t));
  *out = &ctx->btables.back();
  return AFQ_OK;
}

// One step of several systems: the per-system front halves run on the branch
// streams, then (FP64) one local-energy launch per kernel instance covers all
// systems, then the energies.  Host step t / row index si are used when cs
// is null; under capture the device step state is read instead.
afq_status batch_step(afq_ctx* ctx, const int32_t* ids, const std::vector<SysDev*>& ss,
                      const std::vector<std::vector<int>>& branches, const afq_prop_params& P,
                      uint64_t t, int si, const CallState* cs, int add) {
  hipStream_t origin = ctx->stream;
  const int nb = (int)branches.size();
  HIPCHK(hipEventRecord(ctx->ev_fork, origin));
  for (int b = 0; b < nb; ++b) HIPCHK(hipStreamWaitEvent(ctx->br[b], ctx->ev_fork, 0));
  // per branch: the front halves of its systems one after the other, then
  // the per-walker back halves of all of them in one persistent launch
  const bool qr_now = !cs && reorth_due(t, P.reorth_every);
  for (int b = 0; b < nb; ++b) {
    std::vector<SysDev*> sub;
    for (int i : branches[b]) {
      TRY(step_front(ctx, ids[i], *ss[i], P, nullptr, t, cs, add, ctx->br[b]));
      sub.push_back(ss[i]);
    }
    afq_ctx::BTable* bt;
    TRY(get_btable(ctx, sub, &bt));
    HIPCHK(launch_back_queue(bt->d_sys, bt->d_items, bt->n_items, bt->max_n, ctx->wq + b, P.tau,
                             cs, add, P.reorth_every, qr_now, ctx->br[b]));
    for (SysDev* s : sub) swap_state(*s);
  }
  for (int b = 0; b < nb; ++b) {
    HIPCHK(hipEventRecord(ctx->ev_join[b], ctx->br[b]));
    HIPCHK(hipStreamWaitEvent(origin, ctx->ev_join[b], 0));
  }
  if (energy_pieces(P.precision) == 0) {
    afq_ctx::XTable* tab;
    TRY(get_xtable(ctx, ss, &tab));
    for (SysDev* s : ss) HIPCHK(launch_project(*s, s->W, s->th_re, s->th_im, s->thv_re, s->thv_im, origin));
    // the tiles of every system: one launch per kernel instance, tiles in
    // each system's XCD super-tile order (a persistent queue that hands
    // tiles to whichever compute unit frees first loses that L2 locality
    // and measured slower)
    for (size_t c = 0; c < tab->ct.size(); ++c)
      HIPCHK(launch_exchange_group(tab->ct[c], tab->d_sys, tab->d_tiles + tab->begin[c],
                                   tab->count[c], origin));
  } else {
    for (SysDev* s : ss) TRY(step_exchange(ctx, *s, P, origin));
  }
  for (int i = 0; i < (int)ss.size(); ++i) {
    TRY(step_energy(ctx, *ss[i], P, si, i, cs, add, origin));
    TRY(step_pop(ctx, ids[i], *ss[i], P, t, cs, add, origin));
  }
  return AFQ_OK;
}

// Steps of several systems as replays of a captured two-step graph (the
// buffer swaps of two steps cancel, so the captured pointers stay valid).
afq_status run_graph(afq_ctx* ctx, const int32_t* ids, const std::vector<SysDev*>& ss,
                     const std::vector<std::vector<int>>& branches, const afq_prop_params& P) {
  const int n = (int)ss.size();
  std::vector<char> key;
  for (int i = 0; i < n; ++i) {
    // the buffer generation changes with every (re)allocation of the
    // system's walker-side arrays, so a graph never outlives its buffers
    const SysDev& s = *ss[i];
    put_bytes(key, ids[i]);
    put_bytes(key, s.gen);
    put_bytes(key, s.W);
    put_bytes(key, s.N);
    put_bytes(key, s.M);
    put_bytes(key, s.th_re);
    put_bytes(key, s.phi_re);
    put_bytes(key, s.x_ga);
    put_bytes(key, s.x_wb);
    put_bytes(key, s.mv_ct);
  }
  put_bytes(key, P.tau);
  put_bytes(key, P.exp_method);
  put_bytes(key, P.exp_order);
  put_bytes(key, P.reorth_every);
  put_bytes(key, P.precision);
  put_bytes(key, P.seed);
  put_bytes(key, P.e0_window);
  put_bytes(key, P.pop_every);
  put_bytes(key, P.propagator);
  put_bytes(key, P.force_bias_at);
  afq_ctx::GraphEntry* ge = nullptr;
  for (auto& g : ctx->graphs)
    if (g.key == key) ge = &g;
  hipStream_t origin = ctx->stream;
  if (!ge) {
    // item and tile tables of both buffer states first (no allocation
    // under capture), with room for all of them in the cache
    if (ctx->btables.size() + 2 * branches.size() > kMaxBTables) TRY(clear_btables(ctx));
    for (int pass = 0; pass < 2; ++pass) {
      for (SysDev* s : ss) swap_state(*s);
      afq_status r = AFQ_OK;
      for (size_t b = 0; b < branches.size() && r == AFQ_OK; ++b) {
        std::vector<SysDev*> sub;
        for (int i : branches[b]) sub.push_back(ss[i]);
        afq_ctx::BTable* bt;
        r = get_btable(ctx, sub, &bt);
      }
      if (r == AFQ_OK && energy_pieces(P.precision) == 0) {
        afq_ctx::XTable* tab;
        r = get_xtable(ctx, ss, &tab);
      }
      if (r != AFQ_OK) {
        if (pass == 0)
          for (SysDev* s : ss) swap_state(*s);
        return r;
      }
    }
    afq_ctx::GraphEntry g;
    g.key = key;
    HIPCHK(hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed));
    afq_status r = batch_step(ctx, ids, ss, branches, P, 0, 0, ctx->cs, 0);
    if (r == AFQ_OK) r = batch_step(ctx, ids, ss, branches, P, 0, 0, ctx->cs, 1);
    if (r == AFQ_OK && launch_call_advance(ctx->cs, 2, origin) != hipSuccess)
      r = fail(ctx, AFQ_EDEVICE, "step counter launch failed");
    const hipError_t ec = hipStreamEndCapture(origin, &g.g);
    if (r != AFQ_OK) {
      if (g.g) (void)hipGraphDestroy(g.g);
      return r;
    }
    if (ec != hipSuccess) return fail(ctx, AFQ_EDEVICE, std::string("capture: ") + hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&g.ex, g.g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g.g);
      return fail(ctx, AFQ_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    if (ctx->graphs.size() >= 4) {
      HIPCHK(hipStreamSynchronize(origin));
      clear_graphs(ctx);
    }
    ctx->graphs.push_back(std::move(g));
    ge = &ctx->graphs.back();
  }
  HIPCHK(launch_call_begin(ctx->cs, P.step0, P.n_steps, P.energies_out, origin));
  for (int r = 0; r + 1 < P.n_steps; r += 2) HIPCHK(hipGraphLaunch(ge->ex, origin));
  if (P.n_steps % 2) {
    const int si = P.n_steps - 1;
    TRY(batch_step(ctx, ids, ss, branches, P, P.step0 + (uint64_t)si, si, nullptr, 0));
  }
  return AFQ_OK;
}

}  // namespace

// =========================================================================== API

extern "C" {

afq_status afq_create(afq_ctx** out, int device, void* hip_stream) {
  if (!out) return AFQ_EINVAL;
  *out = nullptr;
  afq_ctx* ctx = new (std::nothrow) afq_ctx();
  if (!ctx) return AFQ_ENOMEM;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    delete ctx;
    return AFQ_EDEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return AFQ_EDEVICE;
  }
  ctx->device = device;
  // device address of the fixed workspace on this device (set-up, once per
  // context, with the device current)
  if (hipGetSymbolAddress((void**)&ctx->scratch_dev, HIP_SYMBOL(scratch)) != hipSuccess ||
      !ctx->scratch_dev) {
    (void)hipGetLastError();
    delete ctx;
    return AFQ_EDEVICE;
  }
  if (hip_stream) {
    ctx->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return AFQ_EDEVICE;
    }
    ctx->own_stream = true;
  }
  *out = ctx;
  return AFQ_OK;
}

void afq_destroy(afq_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (size_t i = 0; i < ctx->systems.size(); ++i) {
    if (ctx->systems[i]) {
      free_all(ctx->systems[i]->walker_allocs);
      delete ctx->systems[i];
    }
    free_all(ctx->sys_allocs[i]);
  }
  for (const PhaseEv& e : ctx->pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  clear_graphs(ctx);
  for (auto& t : ctx->xtables) {
    (void)hipFree(t.d_sys);
    (void)hipFree(t.d_tiles);
  }
  for (auto& t : ctx->btables) {
    (void)hipFree(t.d_sys);
    (void)hipFree(t.d_items);
  }
  if (ctx->cs) {
    (void)hipFree(ctx->wq);
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->cs);
    (void)hipEventDestroy(ctx->ev_fork);
    for (int b = 0; b < afq_ctx::kBranches; ++b) {
      (void)hipEventDestroy(ctx->ev_join[b]);
      (void)hipStreamDestroy(ctx->br[b]);
    }
  }
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* afq_last_error(const afq_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

afq_status afq_init_hamiltonian(afq_ctx* ctx, int64_t M, int64_t n_chol, const double* h,
                                const double* L, double e_core, int ptr_is_device,
                                int32_t* sys_id) try {
  if (!ctx) return AFQ_EINVAL;
  if (!h || !L || !sys_id) return fail(ctx, AFQ_EINVAL, "null pointer");
  if (M < 1 || M > 512 || n_chol < 1 || n_chol > (int64_t)1 << 24)
    return fail(ctx, AFQ_EINVAL, "M must be in [1, 512] and n_chol >= 1");
  HIPCHK(hipSetDevice(ctx->device));
  auto* s = new SysDev();
  ctx->systems.push_back(s);
  ctx->sys_allocs.emplace_back();
  auto& own = ctx->sys_allocs.back();
  const int32_t id = (int32_t)ctx->systems.size() - 1;
  auto undo = [&](afq_status code) {
    free_all(own);
    delete s;
    ctx->systems[id] = nullptr;
    return code;
  };
  s->M = (int)M;
  s->G = (int)n_chol;
  s->e_core = e_core;
  const size_t MM = (size_t)M * M;
  afq_status r;
  if ((r = dalloc(ctx, own, &s->h, MM)) != AFQ_OK) return undo(r);
  if ((r = dalloc(ctx, own, &s->L, MM * n_chol)) != AFQ_OK) return undo(r);
  if ((r = copy_in(ctx, s->h, h, MM, ptr_is_device)) != AFQ_OK) return undo(r);
  if ((r = copy_in(ctx, s->L, L, MM * n_chol, ptr_is_device)) != AFQ_OK) return undo(r);
  if ((r = check_symmetric(ctx, s->h, 1, (int)M, "h")) != AFQ_OK) return undo(r);
  if ((r = check_symmetric(ctx, s->L, n_chol, (int)M, "L")) != AFQ_OK) return undo(r);
  *sys_id = id;
  return AFQ_OK;
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

namespace {

// Trial set-up shared by the closed-shell and the spin-orbital entry points:
// N orbitals of one determinant, spin factor `spin` (2 or 1).
afq_status init_trial(afq_ctx* ctx, SysDev& s, int32_t sys_id, int N, double spin,
                      const double* psi_t, int ptr_is_device) {
  s.spin = spin;
  const int M = s.M, G = s.G;
  std::vector<double> psi((size_t)M * N);
  if (ptr_is_device) {
    HIPCHK(hipMemcpyAsync(psi.data(), psi_t, psi.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  } else {
    std::memcpy(psi.data(), psi_t, psi.size() * 8);
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double d = 0.0;
      for (int p = 0; p < M; ++p) d += psi[(size_t)p * N + i] * psi[(size_t)p * N + j];
      if (!(std::fabs(d - (i == j ? 1.0 : 0.0)) <= 1e-10))
        return fail(ctx, AFQ_EINVAL, "psi_t columns are not orthonormal");
    }
  auto& own = ctx->sys_allocs[sys_id];
  s.N = N;
  std::vector<double> pt((size_t)N * M);
  for (int i = 0; i < N; ++i)
    for (int p = 0; p < M; ++p) pt[(size_t)i * M + p] = psi[(size_t)p * N + i];
  const size_t MM = (size_t)M * M;
  TRY(dalloc(ctx, own, &s.psit, (size_t)N * M));
  TRY(dalloc(ctx, own, &s.Lx, (size_t)(G + 1) * N * M));
  TRY(dalloc(ctx, own, &s.lbar, (size_t)G));
  TRY(dalloc(ctx, own, &s.H1, MM));
  TRY(dalloc(ctx, own, &s.Bhalf, MM));
  TRY(dalloc(ctx, own, &s.Bm1, MM));
  TRY(dalloc(ctx, own, &s.Bfull, MM));
  HIPCHK(hipMemcpy(s.psit, pt.data(), pt.size() * 8, hipMemcpyHostToDevice));
  // Psi_T^T L_g for every g, and Psi_T^T h in the last block
  GemmArgs g{};
  g.A = s.psit; g.sAb = 0; g.sAr = M; g.sAk = 1; g.sAkb = 0;
  g.B = s.L; g.sBb = (int64_t)MM; g.sBc = M; g.sBk = 1; g.sBkb = 0;
  g.C = s.Lx; g.sCb = (int64_t)N * M; g.sCr = M; g.sCc = 1;
  g.R = N; g.Cn = M; g.K = M; g.kin = M; g.batch = G; g.alpha = 1.0; g.beta = 0.0;
  HIPCHK(launch_gemm(g, ctx->stream));
  g.B = s.h; g.C = s.Lx + (size_t)G * N * M; g.batch = 1;
  HIPCHK(launch_gemm(g, ctx->stream));
  HIPCHK(launch_lbar(s, ctx->stream));
  // virtual space: Psi_perp (host Householder QR of Psi_T), the blocks
  // Psi_T^T L_g Psi_perp and T0_g = Psi_T^T L_g Psi_T (g = G: h)
  s.Kv = M - N;
  {
    std::vector<double> pv;
    complement_basis(M, N, psi, pv);
    TRY(dalloc(ctx, own, &s.psiv, pv.size()));
    TRY(dalloc(ctx, own, &s.Lov, (size_t)(G + 1) * N * s.Kv));
    TRY(dalloc(ctx, own, &s.T0, (size_t)(G + 1) * N * N));
    TRY(dalloc(ctx, own, &s.t0tr, (size_t)G));
    if (!pv.empty())
      HIPCHK(hipMemcpy(s.psiv, pv.data(), pv.size() * 8, hipMemcpyHostToDevice));
    GemmArgs q{};
    q.A = s.Lx; q.sAb = 0; q.sAr = M; q.sAk = 1; q.sAkb = 0;
    q.B = s.psiv; q.sBb = 0; q.sBc = M; q.sBk = 1; q.sBkb = 0;
    q.C = s.Lov; q.sCb = 0; q.sCr = s.Kv; q.sCc = 1;
    q.R = (G + 1) * N; q.Cn = s.Kv; q.K = M; q.kin = M; q.batch = 1; q.alpha = 1.0; q.beta = 0.0;
    HIPCHK(launch_gemm(q, ctx->stream));
    q.B = s.psit; q.C = s.T0; q.sCr = N; q.Cn = N;
    HIPCHK(launch_gemm(q, ctx->stream));
    HIPCHK(launch_t0_trace(s, ctx->stream));
  }
  // H1 = h - 1/2 sum_g L_g L_g + sum_g Lbar_g L_g
  HIPCHK(hipMemcpyAsync(s.H1, s.h, MM * 8, hipMemcpyDeviceToDevice, ctx->stream));
  // sum_g L_g L_g in chunks of 32 Cholesky vectors: shorter sequential sums
  for (int g0 = 0; g0 < G; g0 += 32) {
    const int gn = G - g0 < 32 ? G - g0 : 32;
    GemmArgs q{};
    q.A = s.L + (size_t)g0 * MM; q.sAb = 0; q.sAr = M; q.sAk = 1; q.sAkb = (int64_t)MM;
    q.B = q.A; q.sBb = 0; q.sBc = M; q.sBk = 1; q.sBkb = (int64_t)MM;
    q.C = s.H1; q.sCb = 0; q.sCr = M; q.sCc = 1;
    q.R = M; q.Cn = M; q.K = M * gn; q.kin = M; q.batch = 1; q.alpha = -0.5; q.beta = 1.0;
    HIPCHK(launch_gemm(q, ctx->stream));
  }
  HIPCHK(launch_axpy_L(s, s.lbar, 1.0, s.H1, ctx->stream));
  std::vector<double> h1(MM), lb(G);
  HIPCHK(hipMemcpyAsync(h1.data(), s.H1, MM * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipMemcpyAsync(lb.data(), s.lbar, G * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int p = 0; p < M; ++p)  // symmetrise the rounding of the product
    for (int r = p + 1; r < M; ++r) {
      const double a = 0.5 * (h1[(size_t)p * M + r] + h1[(size_t)r * M + p]);
      h1[(size_t)p * M + r] = a;
      h1[(size_t)r * M + p] = a;
    }
  jacobi_eigh(M, h1, s.h1_evals, s.h1_evecs);
  double l2 = 0.0;
  for (double v : lb) l2 += v * v;
  s.e_const = s.e_core - 0.5 * l2;
  s.tau_b = -1.0;
  // trial energy E_L(Psi_T): Theta = Psi_T for one walker
  std::vector<void*> tmp;
  double *tre, *tim, *vre, *vim, *lr, *li, *xr, *xi, *el;
  afq_status r = AFQ_OK;
  const size_t G1 = (size_t)G + 1;
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &tre, (size_t)N * M);
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &tim, (size_t)N * M);
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &vre, (size_t)N * s.Kv);
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &vim, (size_t)N * s.Kv);
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &lr, G1);
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &li, G1);
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &xr, G1);
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &xi, G1);
  if (r == AFQ_OK) r = dalloc(ctx, tmp, &el, 2);
  if (r != AFQ_OK) {
    free_all(tmp);
    return r;
  }
  hipError_t e = hipMemcpyAsync(tre, s.psit, (size_t)N * M * 8, hipMemcpyDeviceToDevice, ctx->stream);
  std::vector<double> zeros((size_t)N * M, 0.0);
  if (e == hipSuccess) e = hipMemcpy(tim, zeros.data(), zeros.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_exchange(s, 1, tre, tim, vre, vim, lr, li, xr, xi, ctx->stream);
  if (e == hipSuccess) e = launch_energy(s, 1, lr, li, xr, xi, el, nullptr, nullptr, 0.0, ctx->stream);
  double eh[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(eh, el, 16, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  free_all(tmp);
  if (e != hipSuccess) return fail(ctx, AFQ_EDEVICE, std::string("trial energy: ") + hipGetErrorString(e));
  s.e_trial = eh[0];
  s.trial_ready = true;
  return AFQ_OK;
}

}  // namespace

namespace {

// nb matrices of M x M into nb block-diagonal matrices diag(X, X) of 2M x 2M.
__global__ void k_embed_spin(int64_t nb, int M, const double* __restrict__ src,
                             double* __restrict__ dst) {
  const int64_t M2 = 2 * (int64_t)M, per = M2 * M2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nb * per;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per, r = e - b * per;
    const int64_t p = r / M2, q = r - p * M2;
    double v = 0.0;
    if ((p < M) == (q < M)) v = src[b * M * M + (p % M) * M + (q % M)];
    dst[e] = v;
  }
}

afq_status dfree(std::vector<void*>& owner, void* p) {
  for (size_t i = 0; i < owner.size(); ++i)
    if (owner[i] == p) {
      (void)hipFree(p);
      owner.erase(owner.begin() + (std::ptrdiff_t)i);
      return AFQ_OK;
    }
  return AFQ_EINVAL;
}

// Columns [c0, c0 + n) of the row-major M x ld matrix psi orthonormal to 1e-10.
bool orthonormal_cols(const std::vector<double>& psi, int M, int ld, int c0, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double d = 0.0;
      for (int p = 0; p < M; ++p) d += psi[(size_t)p * ld + c0 + i] * psi[(size_t)p * ld + c0 + j];
      if (!(std::fabs(d - (i == j ? 1.0 : 0.0)) <= 1e-10)) return false;
    }
  return true;
}

// Open shell from spatial orbitals: the system is rewritten in the 2M spin
// orbitals (h and every L_g as diag(X, X), built on the device; the M-basis
// copies are freed) and the trial becomes diag(Psi_a, Psi_b), spin factor 1.
afq_status init_trial_open_shell(afq_ctx* ctx, SysDev& s, int32_t sys_id, int na, int nb,
                                 const double* psi_t, int ptr_is_device) {
  const int M = s.M, N = na + nb, G = s.G;
  std::vector<double> psi((size_t)M * N);
  if (ptr_is_device) {
    HIPCHK(hipMemcpyAsync(psi.data(), psi_t, psi.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  } else {
    std::memcpy(psi.data(), psi_t, psi.size() * 8);
  }
  if (!orthonormal_cols(psi, M, N, 0, na) || !orthonormal_cols(psi, M, N, na, nb))
    return fail(ctx, AFQ_EINVAL, "psi_t: the alpha or the beta columns are not orthonormal");
  const int M2 = 2 * M;
  std::vector<double> psi2((size_t)M2 * N, 0.0);
  for (int p = 0; p < M; ++p) {
    for (int i = 0; i < na; ++i) psi2[(size_t)p * N + i] = psi[(size_t)p * N + i];
    for (int i = na; i < N; ++i) psi2[(size_t)(M + p) * N + i] = psi[(size_t)p * N + i];
  }
  auto& own = ctx->sys_allocs[sys_id];
  double *h2, *L2;
  TRY(dalloc(ctx, own, &h2, (size_t)M2 * M2));
  TRY(dalloc(ctx, own, &L2, (size_t)M2 * M2 * G));
  const int64_t n2 = (int64_t)M2 * M2 * G;
  const unsigned grid = (unsigned)std::min<int64_t>((n2 + 255) / 256, 65536);
  hipLaunchKernelGGL(k_embed_spin, dim3(grid), dim3(256), 0, ctx->stream, (int64_t)1, M, s.h, h2);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_embed_spin, dim3(grid), dim3(256), 0, ctx->stream, (int64_t)G, M, s.L, L2);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  (void)dfree(own, s.h);
  (void)dfree(own, s.L);
  s.h = h2;
  s.L = L2;
  s.M = M2;
  return init_trial(ctx, s, sys_id, N, 1.0, psi2.data(), 0);
}

}  // namespace

afq_status afq_init_trial(afq_ctx* ctx, int32_t sys_id, int64_t n_alpha, int64_t n_beta,
                          const double* psi_t, int ptr_is_device) try {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  if (!psi_t) return fail(ctx, AFQ_EINVAL, "null psi_t");
  if (sp->trial_ready) return fail(ctx, AFQ_ESTATE, "trial already set for this system");
  if (n_alpha != n_beta) {
    if (n_alpha < 0 || n_beta < 0 || n_alpha > sp->M || n_beta > sp->M ||
        n_alpha + n_beta > 80)
      return fail(ctx, AFQ_EINVAL,
                  "open shell: n_alpha and n_beta in [0, M], n_alpha + n_beta <= 80");
    if (2 * sp->M > 512) return fail(ctx, AFQ_EINVAL, "open shell: 2M must be <= 512");
    HIPCHK(hipSetDevice(ctx->device));
    return init_trial_open_shell(ctx, *sp, sys_id, (int)n_alpha, (int)n_beta, psi_t,
                                 ptr_is_device);
  }
  if (n_alpha < 1 || n_alpha > sp->M || n_alpha > 80)
    return fail(ctx, AFQ_EINVAL, "n_alpha must be in [1, min(M, 80)]");
  HIPCHK(hipSetDevice(ctx->device));
  return init_trial(ctx, *sp, sys_id, (int)n_alpha, 2.0, psi_t, ptr_is_device);
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_init_trial_spin_orbital(afq_ctx* ctx, int32_t sys_id, int64_t n_elec,
                                       const double* psi_t, int ptr_is_device) try {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  if (!psi_t) return fail(ctx, AFQ_EINVAL, "null psi_t");
  if (n_elec < 1 || n_elec > sp->M || n_elec > 80)
    return fail(ctx, AFQ_EINVAL, "n_elec must be in [1, min(M, 80)]");
  if (sp->trial_ready) return fail(ctx, AFQ_ESTATE, "trial already set for this system");
  HIPCHK(hipSetDevice(ctx->device));
  return init_trial(ctx, *sp, sys_id, (int)n_elec, 1.0, psi_t, ptr_is_device);
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_init_walkers(afq_ctx* ctx, int32_t sys_id, int64_t n_walkers, const void* phi0,
                            int ptr_is_device) try {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  SysDev& s = *sp;
  if (!s.trial_ready) return fail(ctx, AFQ_ESTATE, "afq_init_trial must precede afq_init_walkers");
  if (n_walkers < 1 || n_walkers > (1 << 20)) return fail(ctx, AFQ_EINVAL, "n_walkers out of range");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  // cached graphs may hold this system's buffers, which are freed here
  clear_graphs(ctx);
  free_all(s.walker_allocs);
  ++s.gen;
  s.mell_re = s.mell_im = s.mex_re = s.mex_im = nullptr;
  s.bk_k = 0;
  s.kmax = 0;
  s.kb_re = s.kb_im = s.kh = nullptr;
  s.thb = nullptr;
  s.adj_ws = nullptr;
  s.adj_ws_n = 0;
  s.coul_ws = nullptr;
  s.Ab = nullptr;
  s.avb = nullptr;
  if (s.mx_pieces) s.mx_pieces = -1;  // pieces of L stay; Theta buffer re-made
  auto& own = s.walker_allocs;
  s.W = (int)n_walkers;
  const size_t W = s.W, NM = (size_t)s.N * s.M, G1 = (size_t)s.G + 1, MM = (size_t)s.M * s.M;
  double** planes[] = {&s.phi_re, &s.phi_im, &s.phn_re, &s.phn_im, &s.th_re, &s.th_im, &s.thn_re,
                       &s.thn_im, &s.t1_re, &s.t1_im, &s.t2_re, &s.t2_im, &s.t3_re, &s.t3_im};
  for (double** p : planes) TRY(dalloc(ctx, own, p, W * NM));
  TRY(dalloc(ctx, own, &s.thv_re, W * s.N * s.Kv));
  TRY(dalloc(ctx, own, &s.thv_im, W * s.N * s.Kv));
  TRY(dalloc(ctx, own, &s.logdet, W * 2));
  TRY(dalloc(ctx, own, &s.logdet_n, W * 2));
  TRY(dalloc(ctx, own, &s.weight, W));
  TRY(dalloc(ctx, own, &s.alive, W));
  TRY(dalloc(ctx, own, &s.bad, W));
  TRY(dalloc(ctx, own, &s.qr_logr, W));
  TRY(dalloc(ctx, own, &s.ell_re, W * G1));
  TRY(dalloc(ctx, own, &s.ell_im, W * G1));
  TRY(dalloc(ctx, own, &s.ex_re, W * G1));
  TRY(dalloc(ctx, own, &s.ex_im, W * G1));
  TRY(dalloc(ctx, own, &s.eloc, W * 2));
  TRY(dalloc(ctx, own, &s.ecap, W));
  TRY(dalloc(ctx, own, &s.x, W * s.G));
  TRY(dalloc(ctx, own, &s.av_re, W * s.G));
  TRY(dalloc(ctx, own, &s.av_im, W * s.G));
  TRY(dalloc(ctx, own, &s.scal, W * 4));
  TRY(dalloc(ctx, own, &s.ncap, W));
  TRY(dalloc(ctx, own, &s.A_re, W * MM));
  TRY(dalloc(ctx, own, &s.A_im, W * MM));
  TRY(dalloc(ctx, own, &s.kbeta, W * s.N));
  TRY(dalloc(ctx, own, &s.kdim, W * s.N));
  TRY(dalloc(ctx, own, &s.est, 2));
  TRY(dalloc(ctx, own, &s.counters, kCounters));
  TRY(dalloc(ctx, own, &s.e0s, 1));
  TRY(dalloc(ctx, own, &s.pc_cum, W));
  TRY(dalloc(ctx, own, &s.pc_src, W));
  TRY(dalloc(ctx, own, &s.pc_flag, 1));
  TRY(dalloc(ctx, own, &s.pc_small, W * 5));
  HIPCHK(launch_zero_counters(s, ctx->stream));
  HIPCHK(launch_set_e0(s, s.e_trial, ctx->stream));
  if (phi0) {
    const double* src = (const double*)phi0;
    std::vector<void*> tmp;
    double* dtmp = nullptr;
    if (!ptr_is_device) {
      TRY(dalloc(ctx, tmp, &dtmp, W * NM * 2));
      hipError_t e = hipMemcpy(dtmp, phi0, W * NM * 16, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        free_all(tmp);
        HIPCHK(e);
      }
      src = dtmp;
    }
    hipError_t e = launch_to_planar(src, s.W, s.M, s.N, s.phi_re, s.phi_im, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    free_all(tmp);
    HIPCHK(e);
  } else {
    hipLaunchKernelGGL(k_fill_trial, dim3((unsigned)((W * NM + 255) / 256)), dim3(256), 0,
                       ctx->stream, s.W, (int)NM, s.psit, s.phi_re, s.phi_im);
    HIPCHK(hipGetLastError());
  }
  TRY(refresh_green(ctx, s));
  hipLaunchKernelGGL(k_init_alive, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, ctx->stream,
                     s.W, s.bad, s.alive, s.weight, 1);
  HIPCHK(hipGetLastError());
  TRY(eval_energy(ctx, s));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return AFQ_OK;
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_propagate_batch(afq_ctx* ctx, const int32_t* sys_ids, int32_t n_sys,
                               const afq_prop_params* P) try {
  if (!ctx) return AFQ_EINVAL;
  if (!sys_ids || !P || n_sys < 1) return fail(ctx, AFQ_EINVAL, "bad arguments");
  if (!(P->tau > 0.0) || !std::isfinite(P->tau)) return fail(ctx, AFQ_EINVAL, "tau must be > 0");
  if (P->exp_method != AFQ_EXP_KRYLOV && P->exp_method != AFQ_EXP_TAYLOR &&
      P->exp_method != AFQ_EXP_BLOCK_KRYLOV && P->exp_method != AFQ_EXP_CHEBYSHEV)
    return fail(ctx, AFQ_EINVAL, "unknown exp_method");
  if (P->exp_order < 1 || P->exp_order > 16) return fail(ctx, AFQ_EINVAL, "exp_order must be in [1, 16]");
  if (P->precision < AFQ_PREC_FP64 || P->precision > AFQ_PREC_MIXED_ENERGY)
    return fail(ctx, AFQ_EINVAL, "unknown precision");
  if (P->n_steps < 0) return fail(ctx, AFQ_EINVAL, "n_steps < 0");
  if (P->fields && n_sys != 1) return fail(ctx, AFQ_EINVAL, "explicit fields need a single system");
  if (P->e0_window < 0 || P->e0_window > kE0Max)
    return fail(ctx, AFQ_EINVAL, "e0_window must be in [0, 64]");
  if (P->pop_every < 0) return fail(ctx, AFQ_EINVAL, "pop_every < 0");
  if (P->propagator < AFQ_PROP_SPLIT2 || P->propagator > AFQ_PROP_CN)
    return fail(ctx, AFQ_EINVAL, "unknown propagator");
  if (P->force_bias_at != AFQ_FB_START && P->force_bias_at != AFQ_FB_HALF)
    return fail(ctx, AFQ_EINVAL, "unknown force_bias_at");
  if (P->force_bias_at == AFQ_FB_HALF && P->propagator != AFQ_PROP_SPLIT2)
    return fail(ctx, AFQ_EINVAL, "the half-step force bias belongs to the Split-2 propagator");
  if (P->propagator != AFQ_PROP_SPLIT2 && op_pieces_of(P->precision) > 0)
    return fail(ctx, AFQ_EINVAL, "Split-1, the refactorised and the Crank-Nicolson propagators "
                                 "run with FP64 propagation (precision FP64 or MIXED_ENERGY)");
  if (P->schedule < AFQ_SCHED_AUTO || P->schedule > AFQ_SCHED_GRAPH)
    return fail(ctx, AFQ_EINVAL, "unknown schedule");
  const bool batch_ok = !P->fields && P->energy_every <= 1 && !ctx->profiling;
  int mode = P->schedule;
  if (mode == AFQ_SCHED_AUTO)
    mode = n_sys > 1 && batch_ok
               ? (P->exp_method == AFQ_EXP_KRYLOV ? AFQ_SCHED_GRAPH : AFQ_SCHED_STREAMS)
               : AFQ_SCHED_SERIAL;
  if (mode != AFQ_SCHED_SERIAL && !batch_ok)
    return fail(ctx, AFQ_EINVAL, "the stream and graph schedules need library fields, the energy "
                                 "every step and profiling off");
  if (mode == AFQ_SCHED_GRAPH && P->exp_method != AFQ_EXP_KRYLOV)
    return fail(ctx, AFQ_EINVAL, "the graph schedule runs the Krylov exponential");
  HIPCHK(hipSetDevice(ctx->device));
  std::vector<SysDev*> ss(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    TRY(get_sys(ctx, sys_ids[i], &ss[i]));
    if (!ss[i]->trial_ready || ss[i]->W == 0)
      return fail(ctx, AFQ_ESTATE, "system " + std::to_string(sys_ids[i]) + " has no walkers");
    for (int j = 0; j < i; ++j)
      if (sys_ids[j] == sys_ids[i]) return fail(ctx, AFQ_EINVAL, "duplicate system id");
    if (P->exp_method == AFQ_EXP_KRYLOV && ss[i]->M > 512)
      return fail(ctx, AFQ_EINVAL, "Krylov path supports M <= 512");
    if (P->exp_method == AFQ_EXP_BLOCK_KRYLOV && P->exp_order * ss[i]->N > ss[i]->M)
      return fail(ctx, AFQ_EINVAL, "block Krylov needs exp_order * N <= M");
    TRY(ensure_half_step(ctx, *ss[i], P->tau));
    if (P->exp_method == AFQ_EXP_KRYLOV || P->exp_method == AFQ_EXP_BLOCK_KRYLOV)
      TRY(ensure_krylov(ctx, sys_ids[i], *ss[i], P->exp_order));
    if (P->exp_method == AFQ_EXP_BLOCK_KRYLOV) TRY(ensure_bkrylov(ctx, *ss[i], P->exp_order));
    if (energy_pieces(P->precision))
      TRY(ensure_mixed(ctx, sys_ids[i], *ss[i], energy_pieces(P->precision)));
    ss[i]->op_pieces = op_pieces_of(P->precision);
    TRY(ensure_op_blocks(ctx, sys_ids[i], *ss[i]));
    if (ss[i]->op_pieces > 0) {
      SysDev& s = *ss[i];
      s.Gp = (s.G + 31) / 32 * 32;
      if (!s.Ab) {
        s.Kq = (2 * s.M + 31) / 32 * 32;
        s.Ab_ps = (int64_t)s.W * s.M * s.Kq;
        TRY(dalloc(ctx, s.walker_allocs, &s.Ab, (size_t)3 * s.Ab_ps));
        // the K padding (2M..Kq) of the operator pieces is never written
        // again and must hold zeros
        HIPCHK(hipMemsetAsync(s.Ab, 0, sizeof(unsigned short) * 3 * s.Ab_ps, ctx->stream));
        s.avb_ps = (int64_t)2 * s.W * s.Gp;
        TRY(dalloc(ctx, s.walker_allocs, &s.avb, (size_t)3 * s.avb_ps));
        ++s.gen;
      }
      if (!s.Ltb) {
        s.Ltb_ps = (int64_t)s.M * s.M * s.Gp;
        TRY(dalloc(ctx, ctx->sys_allocs[sys_ids[i]], &s.Ltb, (size_t)3 * s.Ltb_ps));
        HIPCHK(launch_split_lt(s, ctx->stream));
      }
    }
    if (P->energy_every > 1 || energy_pieces(P->precision) || P->force_bias_at == AFQ_FB_HALF)
      TRY(ensure_coulomb(ctx, *ss[i]));
    HIPCHK(launch_zero_counters(*ss[i], ctx->stream));
    if (!std::isnan(P->e0)) HIPCHK(launch_set_e0(*ss[i], P->e0, ctx->stream));
  }
  if (mode == AFQ_SCHED_SERIAL) {
    for (int si = 0; si < P->n_steps; ++si)
      for (int i = 0; i < n_sys; ++i) TRY(step_system(ctx, sys_ids[i], *ss[i], *P, si, i));
    return AFQ_OK;
  }
  TRY(ensure_sched(ctx));
  const auto branches = assign_branches(ss, P->exp_order);
  if (mode == AFQ_SCHED_STREAMS) {
    for (int si = 0; si < P->n_steps; ++si)
      TRY(batch_step(ctx, sys_ids, ss, branches, *P, P->step0 + (uint64_t)si, si, nullptr, 0));
    return AFQ_OK;
  }
  return run_graph(ctx, sys_ids, ss, branches, *P);
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_autotune(afq_ctx* ctx, const int32_t* sys_ids, int32_t n_sys, int32_t reps) try {
  if (!ctx) return AFQ_EINVAL;
  if (!sys_ids || n_sys < 1) return fail(ctx, AFQ_EINVAL, "bad arguments");
  if (reps < 1) reps = 3;
  HIPCHK(hipSetDevice(ctx->device));
  hipEvent_t ea = nullptr, eb = nullptr;
  HIPCHK(hipEventCreate(&ea));
  HIPCHK(hipEventCreate(&eb));
  std::vector<void*> tmp;
  afq_status r = AFQ_OK;
  // time `reps` launches after one warm-up launch
  auto time_it = [&](auto&& launch, float* ms) -> afq_status {
    HIPCHK(launch());
    HIPCHK(hipEventRecord(ea, ctx->stream));
    for (int i = 0; i < reps; ++i) HIPCHK(launch());
    HIPCHK(hipEventRecord(eb, ctx->stream));
    HIPCHK(hipEventSynchronize(eb));
    HIPCHK(hipEventElapsedTime(ms, ea, eb));
    return AFQ_OK;
  };
  for (int i = 0; i < n_sys && r == AFQ_OK; ++i) {
    SysDev* sp;
    r = get_sys(ctx, sys_ids[i], &sp);
    if (r != AFQ_OK) break;
    SysDev& s = *sp;
    if (!s.W) {
      r = fail(ctx, AFQ_ESTATE, "system " + std::to_string(sys_ids[i]) + " has no walkers");
      break;
    }
    // local-energy contraction: the model's six best tile shapes, outputs to scratch
    const size_t n = (size_t)s.W * (s.G + 1);
    double *lr, *li, *xr, *xi;
    if ((r = dalloc(ctx, tmp, &lr, n)) != AFQ_OK) break;
    if ((r = dalloc(ctx, tmp, &li, n)) != AFQ_OK) break;
    if ((r = dalloc(ctx, tmp, &xr, n)) != AFQ_OK) break;
    if ((r = dalloc(ctx, tmp, &xi, n)) != AFQ_OK) break;
    std::vector<int2> cand;
    exchange_candidates(s.N, cand);
    if (cand.size() > 6) cand.resize(6);
    float best = 1e30f;
    int bga = 0, bwb = 0;
    for (const int2& c : cand) {
      s.x_ga = c.x;
      s.x_wb = c.y;
      float ms = 0.f;
      r = time_it([&] { return launch_exchange(s, s.W, s.th_re, s.th_im, s.thv_re, s.thv_im, lr, li,
                                               xr, xi, ctx->stream); },
                  &ms);
      if (r != AFQ_OK) break;
      if (ms < best) {
        best = ms;
        bga = c.x;
        bwb = c.y;
      }
    }
    s.x_ga = bga;
    s.x_wb = bwb;
    if (r != AFQ_OK) break;
    // operator-orbital product (Krylov or Taylor): column-block counts
    if (s.A_re) {
      const int base = matvec_default_blocks(s.M), top = matvec_max_blocks(s.M);
      std::vector<int> nct;
      for (int c = base; c < top; c *= 2) nct.push_back(c);
      nct.push_back(top);
      best = 1e30f;
      int bct = 0;
      for (int c : nct) {
        s.mv_ct = c;
        float ms = 0.f;
        r = time_it([&] { return launch_matvec_probe(s, s.phi_re, s.phi_im, s.t3_re, s.t3_im,
                                                     ctx->stream); }, &ms);
        if (r != AFQ_OK) break;
        if (ms < best) {
          best = ms;
          bct = c;
        }
      }
      s.mv_ct = bct;
    }
  }
  (void)hipStreamSynchronize(ctx->stream);
  free_all(tmp);
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  return r;
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_local_energy_batch(afq_ctx* ctx, int32_t sys_id, int32_t precision,
                                  double* eloc_out, double* ell_out, int ptr_is_device) try {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  SysDev& s = *sp;
  if (!s.W) return fail(ctx, AFQ_ESTATE, "no walkers");
  if (!eloc_out) return fail(ctx, AFQ_EINVAL, "null eloc_out");
  if (precision < AFQ_PREC_FP64 || precision > AFQ_PREC_MIXED_ENERGY)
    return fail(ctx, AFQ_EINVAL, "unknown precision");
  HIPCHK(hipSetDevice(ctx->device));
  if (energy_pieces(precision) == 0) {
    TRY(eval_energy(ctx, s));
  } else {
    TRY(ensure_mixed(ctx, sys_id, s, energy_pieces(precision)));
    // a measurement must not change the next step: the BF16-split Coulomb
    // vector goes to scratch, the force bias keeps reading the step's own
    if (!s.mell_re) {
      const size_t n = (size_t)s.W * (s.G + 1);
      TRY(dalloc(ctx, s.walker_allocs, &s.mell_re, n));
      TRY(dalloc(ctx, s.walker_allocs, &s.mell_im, n));
      TRY(dalloc(ctx, s.walker_allocs, &s.mex_re, n));
      TRY(dalloc(ctx, s.walker_allocs, &s.mex_im, n));
    }
    HIPCHK(launch_project(s, s.W, s.th_re, s.th_im, s.thv_re, s.thv_im, ctx->stream));
    HIPCHK(launch_split_theta(s.thv_re, s.thv_im, s.W, s.N, s.Kv, s.Kp, s.mx_pieces, s.thb_ps,
                              s.thb, ctx->stream));
    HIPCHK(launch_exchange_mx(s, s.W, s.thb, s.thb_ps, s.mell_re, s.mell_im, s.mex_re, s.mex_im,
                              ctx->stream));
    TRY(ensure_coulomb(ctx, s));
    HIPCHK(launch_coulomb_v(s, s.thv_re, s.thv_im, s.coul_ws, s.mell_re, s.mell_im, ctx->stream));
    HIPCHK(launch_energy(s, s.W, s.mell_re, s.mell_im, s.mex_re, s.mex_im, s.eloc, nullptr,
                         nullptr, 0.0, ctx->stream));
  }
  TRY(copy_out(ctx, eloc_out, s.eloc, (size_t)s.W * 16, ptr_is_device));
  if (ell_out) {
    std::vector<void*> tmp;
    double* d = nullptr;
    if (!ptr_is_device) TRY(dalloc(ctx, tmp, &d, (size_t)s.W * s.G * 2));
    double* dst = ptr_is_device ? ell_out : d;
    const bool mx = energy_pieces(precision) != 0;
    hipError_t e = launch_pack_complex(mx ? s.mell_re : s.ell_re, mx ? s.mell_im : s.ell_im, s.W,
                                       s.G + 1, s.G, dst, ctx->stream);
    afq_status r = AFQ_OK;
    if (e != hipSuccess) r = fail(ctx, AFQ_EDEVICE, hipGetErrorString(e));
    if (r == AFQ_OK && !ptr_is_device) r = copy_out(ctx, ell_out, d, (size_t)s.W * s.G * 16, 0);
    free_all(tmp);
    return r;
  }
  return AFQ_OK;
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_local_energy_batch_noalloc(afq_ctx* ctx, int32_t sys_id, double* eloc_out,
                                          double* ell_out) {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  SysDev& s = *sp;
  if (!s.W) return fail(ctx, AFQ_ESTATE, "no walkers");
  if (!eloc_out) return fail(ctx, AFQ_EINVAL, "null eloc_out");
  const size_t n = (size_t)s.W * (s.G + 1);
  if (4 * n > kScratchDoubles)
    return fail(ctx, AFQ_EINVAL, "n_walkers * (n_chol + 1) = " + std::to_string(n) +
                                     " exceeds the fixed workspace of the allocation-free local "
                                     "energy (" + std::to_string(kScratchDoubles / 4) + ")");
  HIPCHK(hipSetDevice(ctx->device));
  double* lr = ctx->scratch_dev;
  double* li = lr + n;
  double* xr = li + n;
  double* xi = xr + n;
  // every element of the four planes is written by the contraction: nothing
  // needs clearing between calls
  HIPCHK(launch_exchange(s, s.W, s.th_re, s.th_im, s.thv_re, s.thv_im, lr, li, xr, xi,
                         ctx->stream));
  HIPCHK(launch_energy(s, s.W, lr, li, xr, xi, eloc_out, nullptr, nullptr, 0.0, ctx->stream));
  if (ell_out) HIPCHK(launch_pack_complex(lr, li, s.W, s.G + 1, s.G, ell_out, ctx->stream));
  return AFQ_OK;
}

afq_status afq_get_walkers(afq_ctx* ctx, int32_t sys_id, void* phi, double* weight,
                           double* log_ovlp, int32_t* alive, int ptr_is_device) try {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  SysDev& s = *sp;
  if (!s.W) return fail(ctx, AFQ_ESTATE, "no walkers");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t W = s.W, NM = (size_t)s.N * s.M;
  if (phi) {
    std::vector<void*> tmp;
    double* d = nullptr;
    if (!ptr_is_device) TRY(dalloc(ctx, tmp, &d, W * NM * 2));
    double* dst = ptr_is_device ? (double*)phi : d;
    hipError_t e = launch_from_planar(s.phi_re, s.phi_im, s.W, s.M, s.N, dst, ctx->stream);
    afq_status r = AFQ_OK;
    if (e != hipSuccess) r = fail(ctx, AFQ_EDEVICE, hipGetErrorString(e));
    if (r == AFQ_OK && !ptr_is_device) r = copy_out(ctx, phi, d, W * NM * 16, 0);
    free_all(tmp);
    TRY(r);
  }
  if (weight) TRY(copy_out(ctx, weight, s.weight, W * 8, ptr_is_device));
  if (log_ovlp) TRY(copy_out(ctx, log_ovlp, s.logdet, W * 16, ptr_is_device));
  if (alive) TRY(copy_out(ctx, alive, s.alive, W * 4, ptr_is_device));
  return AFQ_OK;
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_set_walkers(afq_ctx* ctx, int32_t sys_id, const void* phi, const double* weight,
                           int ptr_is_device) try {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  SysDev& s = *sp;
  if (!s.W) return fail(ctx, AFQ_ESTATE, "no walkers");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t W = s.W, NM = (size_t)s.N * s.M;
  if (phi) {
    std::vector<void*> tmp;
    const double* src = (const double*)phi;
    if (!ptr_is_device) {
      double* d = nullptr;
      TRY(dalloc(ctx, tmp, &d, W * NM * 2));
      hipError_t e = hipMemcpy(d, phi, W * NM * 16, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        free_all(tmp);
        HIPCHK(e);
      }
      src = d;
    }
    hipError_t e = launch_to_planar(src, s.W, s.M, s.N, s.phi_re, s.phi_im, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    free_all(tmp);
    HIPCHK(e);
  }
  if (weight) TRY(copy_in(ctx, s.weight, weight, W, ptr_is_device));
  TRY(refresh_green(ctx, s));
  hipLaunchKernelGGL(k_init_alive, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, ctx->stream,
                     s.W, s.bad, s.alive, s.weight, 0);
  HIPCHK(hipGetLastError());
  TRY(eval_energy(ctx, s));
  return AFQ_OK;
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_fill_fields(afq_ctx* ctx, uint64_t seed, uint64_t sys_id, uint64_t step,
                           int64_t n_walkers, int64_t n_chol, double* out_dev) {
  if (!ctx) return AFQ_EINVAL;
  if (!out_dev || n_walkers < 1 || n_chol < 1) return fail(ctx, AFQ_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(launch_fields(seed, sys_id, step, (int)n_walkers, (int)n_chol, out_dev, ctx->stream));
  return AFQ_OK;
}

afq_status afq_get_counters(afq_ctx* ctx, int32_t sys_id, int64_t* out, int32_t n) {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  if (!out) return fail(ctx, AFQ_EINVAL, "null out");
  if (n < 1 || n > kCounters) return fail(ctx, AFQ_EINVAL, "n must be in [1, 5]");
  if (!sp->W) return fail(ctx, AFQ_ESTATE, "no walkers");
  HIPCHK(hipSetDevice(ctx->device));
  int h[kCounters];
  HIPCHK(hipMemcpyAsync(h, sp->counters, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < n; ++i) out[i] = h[i];
  return AFQ_OK;
}

afq_status afq_get_e0(afq_ctx* ctx, int32_t sys_id, double* e0_out) {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  if (!e0_out) return fail(ctx, AFQ_EINVAL, "null e0_out");
  if (!sp->W) return fail(ctx, AFQ_ESTATE, "no walkers");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipMemcpyAsync(e0_out, &sp->e0s->e0, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return AFQ_OK;
}

// Adjoint workspace of a system, carved as TH [W 2N M] | Ub [gchunk N][W 2N] |
// Db [S][gchunk N M] | Y [N M] | ellt [G][2W] | dE [W 2 G] (the larger of
// dE_dEL and d_ell).  The chunk of Cholesky blocks keeps Ub near 2 GiB (long
// products, few launches; HBM is plentiful).
afq_status ensure_adjoint(afq_ctx* ctx, SysDev& s, double** TH, double** Ub, double** Db,
                          double** Y, double** ellt, double** dE) {
  const size_t M = s.M, N = s.N, W = s.W, G = s.G;
  const size_t cols = W * 2 * N;
  size_t gchunk = (size_t)(2ull << 30) / (N * cols * 8);
  if (gchunk < 1) gchunk = 1;
  if (gchunk > G) gchunk = G;
  const size_t S = (size_t)adjoint_nsplit(s.M, s.N, s.W, (int)gchunk);
  const size_t need = cols * M + gchunk * N * cols + S * gchunk * N * M + N * M + G * 2 * W +
                      W * 2 * G;
  if (!s.adj_ws || s.adj_ws_n < need) {
    TRY(dalloc(ctx, s.walker_allocs, &s.adj_ws, need));
    s.adj_ws_n = need;
  }
  s.adj_gchunk = (int)gchunk;
  double* p = s.adj_ws;
  *TH = p; p += cols * M;
  *Ub = p; p += gchunk * N * cols;
  *Db = p; p += S * gchunk * N * M;
  *Y = p; p += N * M;
  *ellt = p; p += G * 2 * W;
  *dE = p;
  return AFQ_OK;
}

afq_status afq_local_energy_adjoint(afq_ctx* ctx, int32_t sys_id, const double* dE_dEL,
                                    double* grad_h, double* grad_L, int ptr_is_device) try {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  SysDev& s = *sp;
  if (!s.W) return fail(ctx, AFQ_ESTATE, "no walkers");
  if (!dE_dEL || !grad_h || !grad_L) return fail(ctx, AFQ_EINVAL, "null pointer");
  if (s.spin != 2.0) return fail(ctx, AFQ_EINVAL, "adjoints are for closed-shell trials only");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t M = s.M, W = s.W, G = s.G;
  double *TH, *Ub, *Db, *Y, *ellt, *dE;
  TRY(ensure_adjoint(ctx, s, &TH, &Ub, &Db, &Y, &ellt, &dE));
  std::vector<void*> tmp;
  double *gh = grad_h, *gL = grad_L;
  afq_status r = AFQ_OK;
  if (!ptr_is_device) r = dalloc(ctx, tmp, &gh, M * M);
  if (r == AFQ_OK && !ptr_is_device) r = dalloc(ctx, tmp, &gL, G * M * M);
  if (r == AFQ_OK) r = copy_in(ctx, dE, dE_dEL, W, ptr_is_device);
  if (r == AFQ_OK) {
    const hipError_t e = launch_adjoint_into(s, dE, gh, gL, TH, Ub, Db, Y, ellt, s.adj_gchunk,
                                             ctx->stream);
    if (e != hipSuccess) r = fail(ctx, AFQ_EDEVICE, std::string("adjoint: ") + hipGetErrorString(e));
  }
  if (r == AFQ_OK && !ptr_is_device) r = copy_out(ctx, grad_h, gh, M * M * 8, 0);
  if (r == AFQ_OK && !ptr_is_device) r = copy_out(ctx, grad_L, gL, G * M * M * 8, 0);
  if (!tmp.empty()) {
    (void)hipStreamSynchronize(ctx->stream);
    free_all(tmp);
  }
  return r;
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_force_bias_adjoint(afq_ctx* ctx, int32_t sys_id, const double* d_ell,
                                  double* grad_L, int ptr_is_device) try {
  SysDev* sp;
  TRY(get_sys(ctx, sys_id, &sp));
  SysDev& s = *sp;
  if (!s.W) return fail(ctx, AFQ_ESTATE, "no walkers");
  if (!d_ell || !grad_L) return fail(ctx, AFQ_EINVAL, "null pointer");
  if (s.spin != 2.0) return fail(ctx, AFQ_EINVAL, "adjoints are for closed-shell trials only");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t M = s.M, W = s.W, G = s.G;
  double *TH, *Ub, *Db, *Y, *ellt, *dl;
  TRY(ensure_adjoint(ctx, s, &TH, &Ub, &Db, &Y, &ellt, &dl));
  std::vector<void*> tmp;
  double* gL = grad_L;
  afq_status r = AFQ_OK;
  if (!ptr_is_device) r = dalloc(ctx, tmp, &gL, G * M * M);
  if (r == AFQ_OK) r = copy_in(ctx, dl, d_ell, W * G * 2, ptr_is_device);
  if (r == AFQ_OK) {
    // Z of a chunk reuses Db (gchunk N M doubles)
    const hipError_t e = launch_fb_adjoint_into(s, dl, gL, TH, Db, s.adj_gchunk, ctx->stream);
    if (e != hipSuccess) r = fail(ctx, AFQ_EDEVICE, std::string("adjoint: ") + hipGetErrorString(e));
  }
  if (r == AFQ_OK && !ptr_is_device) r = copy_out(ctx, grad_L, gL, G * M * M * 8, 0);
  if (!tmp.empty()) {
    (void)hipStreamSynchronize(ctx->stream);
    free_all(tmp);
  }
  return r;
} catch (...) {
  return fail(ctx, AFQ_ENOMEM, "host allocation failed");
}

afq_status afq_profile(afq_ctx* ctx, int enable) {
  if (!ctx) return AFQ_EINVAL;
  ctx->profiling = enable != 0;
  return AFQ_OK;
}

afq_status afq_profile_read(afq_ctx* ctx, double* ms_out, int64_t* launches_out, int n) {
  if (!ctx) return AFQ_EINVAL;
  if (n < 0 || n > AFQ_PH_COUNT) return fail(ctx, AFQ_EINVAL, "n out of range");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (const PhaseEv& e : ctx->pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      ctx->ph_ms[e.phase] += ms;
      ctx->ph_n[e.phase] += 1;
    }
    ctx->ev_pool.push_back(e.a);
    ctx->ev_pool.push_back(e.b);
  }
  ctx->pending.clear();
  for (int i = 0; i < n; ++i) {
    if (ms_out) ms_out[i] = ctx->ph_ms[i];
    if (launches_out) launches_out[i] = ctx->ph_n[i];
  }
  for (int i = 0; i < AFQ_PH_COUNT; ++i) {
    ctx->ph_ms[i] = 0.0;
    ctx->ph_n[i] = 0;
  }
  return AFQ_OK;
}

afq_status afq_sync(afq_ctx* ctx) {
  if (!ctx) return AFQ_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return AFQ_OK;
}

}  // extern "C"
