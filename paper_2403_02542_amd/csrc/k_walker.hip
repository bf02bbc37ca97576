// Per-walker kernels of the Split-2 step:
//  * auxiliary fields from Philox4x64-10 (Salmon et al., SC'11) + Box-Muller,
//  * force bias with the |f| < 1 cap, shifted fields, importance factor and
//    mean-field scalar (Eq. force_shift, heffTOT; Sec. V.C),
//  * overlap O = Psi_T^T Phi, log det O and Theta = Phi O^-1 (Eq. hyben, eloc),
//  * hybrid energy, phaseless weight and reweighting cap (Eq. hyben,
//    phaseless, theta; Sec. V.B),
//  * QR reorthonormalisation with a real positive diagonal (Sec. IV.D),
//  * local-energy assembly, window cap and weighted estimator (Eq. eloc,
//    enwin; Sec. II.A).
#include "afq_device.h"
#include "afq_internal.h"

namespace {

// ---------------------------------------------------------------- fields

struct U64x4 {
  uint64_t v[4];
};

// Philox4x64 with 10 rounds: multipliers 0xD2E7470EE14C6C93, 0xCA5A826395121157,
// Weyl increments 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B.
AFQ_DEV U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c.v[0]), lo0 = M0 * c.v[0];
    const uint64_t hi1 = __umul64hi(M1, c.v[2]), lo1 = M1 * c.v[2];
    U64x4 n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// x[w][g], block b of walker w covers g = 4b .. 4b+3.  Philox counter of the
// block: (step * W + w) * ceil(G/4) + b + 1 (the first counter value is 1).
__global__ void k_fields(uint64_t seed, uint64_t sid, uint64_t step, int W, int G,
                         double* __restrict__ out, const CallState* __restrict__ cs, int add) {
  const int nb = (G + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)W * nb) return;
  if (cs) step = cs->step + (uint64_t)add;
  const int w = (int)(t / nb), b = (int)(t % nb);
  U64x4 c;
  c.v[0] = ((uint64_t)step * W + w) * nb + b + 1;
  c.v[1] = c.v[2] = c.v[3] = 0;
  const U64x4 r = philox4x64_10(c, seed, sid);
  const double two_pi = 2.0 * 3.14159265358979323846;
  double u[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = (double)((r.v[i] >> 11) + 1) * 0x1.0p-53;
  const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
  const double th0 = two_pi * u[1], th1 = two_pi * u[3];
  const double z[4] = {r0 * cos(th0), r0 * sin(th0), r1 * cos(th1), r1 * sin(th1)};
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (4 * b + i < G) out[(int64_t)w * G + 4 * b + i] = z[i];
}

// ---------------------------------------------------------------- set-up

// Lbar_g = s tr(Psi_T^T L_g Psi_T) = s sum_{i,p} (Psi_T^T L_g)[i][p] Psi_T[p][i],
// s the spin factor
__global__ __launch_bounds__(256) void k_lbar(int N, int M, double spin, const double* __restrict__ Lx,
                                              const double* __restrict__ psit,
                                              double* __restrict__ lbar) {
  __shared__ double red[4];
  const int g = blockIdx.x;
  const double* X = Lx + (int64_t)g * N * M;
  double s = 0.0;
  for (int e = threadIdx.x; e < N * M; e += 256) s += X[e] * psit[e];
  s = block_sum(s, red);
  if (threadIdx.x == 0) lbar[g] = spin * s;
}

// out[pq] += alpha sum_g coef[g] L[g][pq]
__global__ void k_axpy_L(int G, int64_t MM, const double* __restrict__ L,
                         const double* __restrict__ coef, double alpha, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= MM) return;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += coef[g] * L[(int64_t)g * MM + e];
  out[e] += alpha * s;
}

// ---------------------------------------------------------------- force bias
// ell_g = <Lhat_g>_mixed (from the local-energy contraction); per walker:
//   f_g = -i sqrt(tau) (ell_g - Lbar_g),   fbar_g = f_g if |f_g| < 1 else 0,
//   c_g = x_g - fbar_g,  a_g = i sqrt(tau) c_g   (operator coefficients),
//   log I = sum_g x_g fbar_g - fbar_g^2 / 2,   s_mf = -i sqrt(tau) sum_g c_g Lbar_g.
__global__ __launch_bounds__(256) void k_force_bias(int G, int G1, double sqt,
                                                    const double* __restrict__ ell_re,
                                                    const double* __restrict__ ell_im,
                                                    const double* __restrict__ lbar,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ a_re,
                                                    double* __restrict__ a_im,
                                                    double* __restrict__ scal,
                                                    int* __restrict__ ncap,
                                                    int* __restrict__ ncap_total) {
  __shared__ double red[4];
  const int w = blockIdx.x;
  double li_re = 0.0, li_im = 0.0, P = 0.0, Q = 0.0, nc = 0.0;
  for (int g = threadIdx.x; g < G; g += 256) {
    const double er = ell_re[(int64_t)w * G1 + g] - lbar[g];
    const double ei = ell_im[(int64_t)w * G1 + g];
    const double fr = sqt * ei, fi = -sqt * er;
    const bool keep = hypot(fr, fi) < 1.0;
    const double br = keep ? fr : 0.0, bi = keep ? fi : 0.0;
    nc += keep ? 0.0 : 1.0;
    const double xg = x[(int64_t)w * G + g];
    const double cr = xg - br, ci = -bi;
    a_re[(int64_t)w * G + g] = -sqt * ci;
    a_im[(int64_t)w * G + g] = sqt * cr;
    li_re += xg * br - 0.5 * (br * br - bi * bi);
    li_im += xg * bi - br * bi;
    P += cr * lbar[g];
    Q += ci * lbar[g];
  }
  li_re = block_sum(li_re, red);
  li_im = block_sum(li_im, red);
  P = block_sum(P, red);
  Q = block_sum(Q, red);
  nc = block_sum(nc, red);
  if (threadIdx.x == 0) {
    scal[w * 4 + 0] = li_re;
    scal[w * 4 + 1] = li_im;
    scal[w * 4 + 2] = sqt * Q;   // s_mf = -i sqt (P + i Q)
    scal[w * 4 + 3] = -sqt * P;
    ncap[w] = (int)nc;
    if (ncap_total) atomicAdd(ncap_total, (int)nc);
  }
}

// ---------------------------------------------------------------- small dense
// Per-walker N x N work in LDS.  Tile engine of four waves with up to
// 32 T x 32 T outputs: T = 4 (128 x 128) while 2N <= 128, else T = 5; the
// smaller stage and accumulator set let two workgroups share a compute unit.
// The products accumulate over k in the same order for either T.

template <int T>
struct Sm {
  static constexpr int MT = T, NT = T;
  static constexpr int ROWS = 32 * T, COLS = 32 * T;
  static constexpr int STAGE = (ROWS + COLS) * kLDK;
};
constexpr int kSmRowsMax = Sm<5>::ROWS;
__host__ __device__ inline int sm_tiles(int N) { return 2 * N <= Sm<4>::ROWS ? 4 : 5; }

// C[r][c] = sum_k X(r, k) Y(c, k) over k < K; store(r, c, value) is called once
// per output element (r < nr, c < nc).  Ends with a workgroup barrier.
template <int T, class GX, class GY, class ST>
AFQ_DEV void small_gram(int nr, int nc, int K, GX gx, GY gy, ST store, double* stage) {
  using E = Sm<T>;
  double* As = stage;
  double* Bs = stage + E::ROWS * kLDK;
  const WaveSplit ws = wave_split<E::MT, E::NT>(nr, nc);
  TileAcc<E::MT, E::NT> acc;
  acc.zero();
  auto fa = [&](int k0, double* S) { stage_rows<E::ROWS>(S, k0, K, nr, gx); };
  auto fb = [&](int k0, double* S) { stage_rows<E::COLS>(S, k0, K, nc, gy); };
  tile_gemm<E::MT, E::NT>(K, ws, fa, fb, As, Bs, acc);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < E::MT; ++i)
#pragma unroll
    for (int j = 0; j < E::NT; ++j) {
      if (i >= ws.mtv || j >= ws.ntv) continue;
      const int c = acc_col(ws, j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = acc_row(ws, i, e);
        if (r < nr && c < nc) store(r, c, acc.c[i][j][e]);
      }
    }
  __syncthreads();
}

// out[j][p] = sum_i X[i][j] in[i][p] (complex, X in LDS as X[(i*N + j)*2 + {0,1}]).
// in and out are planar [N][M] arrays of one walker; out may alias in.
template <int T>
AFQ_DEV void apply_right(int N, int M, const double* Xl, const double* in_re, const double* in_im,
                         double* out_re, double* out_im, double* stage) {
  using E = Sm<T>;
  double* As = stage;
  double* Bs = stage + E::ROWS * kLDK;
  const int nr = 2 * N, K = 2 * N;
  auto gx = [&](int r, int k) {
    const int pl = r >= N, j = pl ? r - N : r;
    const int pk = k >= N, i = pk ? k - N : k;
    const double xr = Xl[(i * N + j) * 2], xi = Xl[(i * N + j) * 2 + 1];
    if (!pl) return pk ? -xi : xr;
    return pk ? xr : xi;
  };
  for (int p0 = 0; p0 < M; p0 += E::COLS) {
    const int nc = min(E::COLS, M - p0);
    const WaveSplit ws = wave_split<E::MT, E::NT>(nr, nc);
    TileAcc<E::MT, E::NT> acc;
    acc.zero();
    auto gy = [&](int c, int k) {
      const int pk = k >= N, i = pk ? k - N : k;
      return pk ? in_im[(int64_t)i * M + p0 + c] : in_re[(int64_t)i * M + p0 + c];
    };
    auto fa = [&](int k0, double* S) { stage_rows<E::ROWS>(S, k0, K, nr, gx); };
    auto fb = [&](int k0, double* S) { stage_rows_kmajor<E::COLS>(S, k0, K, nc, gy); };
    tile_gemm<E::MT, E::NT>(K, ws, fa, fb, As, Bs, acc);
#pragma unroll
    for (int i = 0; i < E::MT; ++i)
#pragma unroll
      for (int j = 0; j < E::NT; ++j) {
        if (i >= ws.mtv || j >= ws.ntv) continue;
        const int c = acc_col(ws, j);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = acc_row(ws, i, e);
          if (r < nr && c < nc) {
            const int pl = r >= N, jj = pl ? r - N : r;
            if (pl) out_im[(int64_t)jj * M + p0 + c] = acc.c[i][j][e];
            else out_re[(int64_t)jj * M + p0 + c] = acc.c[i][j][e];
          }
        }
      }
    __syncthreads();
  }
}

// In-place Gauss-Jordan inversion with partial pivoting of the complex N x N
// matrix X in LDS.  Returns (via *logdet) log det X; *ok = 0 if singular.
AFQ_DEV void gj_inverse(int N, double* X, double* fcol, int* perm, double* red, cplx* logdet,
                        int* ok) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  cplx ld = cmake(0.0, 0.0);
  int swaps = 0;
  int good = 1;
  for (int k = 0; k < N; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bi = k;
      for (int r = k + lane; r < N; r += 64) {
        const double a = cabs2(cmake(X[(r * N + k) * 2], X[(r * N + k) * 2 + 1]));
        if (a > best) {
          best = a;
          bi = r;
        }
      }
      // argmax over lanes; ties -> lowest row
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) perm[k] = bi;
    }
    __syncthreads();
    const int pv = perm[k];
    if (pv != k) {
      for (int j = tid; j < N; j += blockDim.x) {
        for (int c = 0; c < 2; ++c) {
          const double t = X[(k * N + j) * 2 + c];
          X[(k * N + j) * 2 + c] = X[(pv * N + j) * 2 + c];
          X[(pv * N + j) * 2 + c] = t;
        }
      }
      ++swaps;
    }
    __syncthreads();
    const cplx p = cmake(X[(k * N + k) * 2], X[(k * N + k) * 2 + 1]);
    if (!(cabs2(p) > 0.0)) good = 0;
    ld = cadd(ld, clog(p));
    const cplx ip = cdiv(cmake(1.0, 0.0), p);
    for (int r = tid; r < N; r += blockDim.x) {
      fcol[r * 2] = X[(r * N + k) * 2];
      fcol[r * 2 + 1] = X[(r * N + k) * 2 + 1];
    }
    __syncthreads();
    // row k <- row k / p, with X[k][k] = 1 / p
    for (int j = tid; j < N; j += blockDim.x) {
      const cplx v = (j == k) ? ip : cmul(cmake(X[(k * N + j) * 2], X[(k * N + j) * 2 + 1]), ip);
      X[(k * N + j) * 2] = v.re;
      X[(k * N + j) * 2 + 1] = v.im;
    }
    __syncthreads();
    for (int e = tid; e < N * N; e += blockDim.x) {
      const int r = e / N, j = e % N;
      if (r == k) continue;
      const cplx f = cmake(fcol[r * 2], fcol[r * 2 + 1]);
      const cplx a = (j == k) ? cmake(0.0, 0.0) : cmake(X[e * 2], X[e * 2 + 1]);
      const cplx v = csub(a, cmul(f, cmake(X[(k * N + j) * 2], X[(k * N + j) * 2 + 1])));
      X[e * 2] = v.re;
      X[e * 2 + 1] = v.im;
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = N - 1; k >= 0; --k) {
    const int pv = perm[k];
    if (pv != k) {
      for (int r = tid; r < N; r += blockDim.x) {
        for (int c = 0; c < 2; ++c) {
          const double t = X[(r * N + k) * 2 + c];
          X[(r * N + k) * 2 + c] = X[(r * N + pv) * 2 + c];
          X[(r * N + pv) * 2 + c] = t;
        }
      }
    }
    __syncthreads();
  }
  if (swaps & 1) ld.im += 3.14159265358979323846;
  // wrap the phase into (-pi, pi]
  const double two_pi = 2.0 * 3.14159265358979323846;
  ld.im = ld.im - two_pi * ceil((ld.im - 3.14159265358979323846) / two_pi);
  *logdet = ld;
  *ok = good;
  (void)red;
}

AFQ_DEV bool all_finite_block(bool v, double* red) {
  return block_sum(v ? 0.0 : 1.0, red) == 0.0;
}

// O = Psi_T^T Phi, log det O, Theta = Phi O^-1 of walker w (one block).
template <int T>
AFQ_DEV void overlap_one(int N, int M, const double* __restrict__ psit,
                         const double* __restrict__ ph_re, const double* __restrict__ ph_im,
                         double* __restrict__ logdet_out, double* __restrict__ th_re,
                         double* __restrict__ th_im, int* __restrict__ bad,
                         double* __restrict__ oinv_out, int w, double* smem) {
  double* stage = smem;
  double* X = stage + Sm<T>::STAGE;         // N x N complex
  double* fcol = X + 2 * N * N;             // 2N
  double* red = fcol + 2 * N;               // 8
  int* perm = (int*)(red + 8);              // N
  const int64_t off = (int64_t)w * N * M;
  const double* pr = ph_re + off;
  const double* pi = ph_im + off;
  // O[i][j] = sum_p Psi_T[p][i] Phi[p][j]: rows i, columns (plane, j)
  auto gx = [&](int r, int k) { return psit[(int64_t)r * M + k]; };
  auto gy = [&](int c, int k) { return c < N ? pr[(int64_t)c * M + k] : pi[(int64_t)(c - N) * M + k]; };
  auto st = [&](int r, int c, double v) {
    const int pl = c >= N, j = pl ? c - N : c;
    X[(r * N + j) * 2 + pl] = v;
  };
  small_gram<T>(N, 2 * N, M, gx, gy, st, stage);
  cplx ld;
  int ok;
  gj_inverse(N, X, fcol, perm, red, &ld, &ok);
  __syncthreads();
  if (oinv_out)
    for (int e = threadIdx.x; e < 2 * N * N; e += blockDim.x) oinv_out[(int64_t)w * 2 * N * N + e] = X[e];
  apply_right<T>(N, M, X, pr, pi, th_re + off, th_im + off, stage);
  __threadfence();
  __syncthreads();
  bool fin = isfinite(ld.re) && isfinite(ld.im) && ok;
  for (int e = threadIdx.x; e < N * M; e += blockDim.x)
    fin = fin && isfinite(th_re[off + e]) && isfinite(th_im[off + e]);
  fin = all_finite_block(fin, red);
  if (threadIdx.x == 0) {
    logdet_out[w * 2] = ld.re;
    logdet_out[w * 2 + 1] = ld.im;
    bad[w] = fin ? 0 : 1;
  }
}

template <int T>
__global__ __launch_bounds__(256) void k_overlap(int N, int M, const double* __restrict__ psit,
                                                 const double* __restrict__ ph_re,
                                                 const double* __restrict__ ph_im,
                                                 double* __restrict__ logdet_out,
                                                 double* __restrict__ th_re,
                                                 double* __restrict__ th_im,
                                                 int* __restrict__ bad,
                                                 double* __restrict__ oinv_out) {
  extern __shared__ double smem[];
  overlap_one<T>(N, M, psit, ph_re, ph_im, logdet_out, th_re, th_im, bad, oinv_out, blockIdx.x,
                 smem);
}

// ---------------------------------------------------------------- weights
// log R = s (logdet_new - logdet_old) + s_mf (s the spin factor: the
// log-overlap is kept per determinant);  E_H = -(log R + log I)/tau + e_const;
// dtheta = Im log R;  m = exp(-tau (Re E_H - E0)), m >= 10 -> 0;
// W <- W m max(0, cos dtheta).  A walker whose new state is non-finite is
// frozen (alive = 0, W = 0); frozen walkers are never updated again.
AFQ_DEV void weight_one(int w, double tau, double spin, const E0Dev* __restrict__ e0s,
                        double e_const,
                        const double* __restrict__ logdet_n, double* __restrict__ logdet,
                        const double* __restrict__ scal, const int* __restrict__ bad,
                        const double* __restrict__ qr_logr, int* __restrict__ alive,
                        double* __restrict__ weight, int* __restrict__ nfrozen) {
  if (!alive[w]) return;
  const double e0 = e0s->e0;
  if (bad[w]) {
    alive[w] = 0;
    weight[w] = 0.0;
    if (nfrozen) atomicAdd(nfrozen, 1);
    return;
  }
  const double lr = spin * (logdet_n[w * 2] - logdet[w * 2]) + scal[w * 4 + 2];
  const double li = spin * (logdet_n[w * 2 + 1] - logdet[w * 2 + 1]) + scal[w * 4 + 3];
  const double eh = -(lr + scal[w * 4 + 0]) / tau + e_const;
  double m = exp(-tau * (eh - e0));
  if (!(m < 10.0)) m = 0.0;
  const double c = cos(li);
  weight[w] = weight[w] * (m * (c > 0.0 ? c : 0.0));
  // the stored log-overlap belongs to the (possibly reorthonormalised) orbitals
  logdet[w * 2] = logdet_n[w * 2] - (qr_logr ? qr_logr[w] : 0.0);
  logdet[w * 2 + 1] = logdet_n[w * 2 + 1];
}

__global__ void k_weight(int W, double tau, double spin, const E0Dev* __restrict__ e0s,
                         double e_const,
                         const double* __restrict__ logdet_n, double* __restrict__ logdet,
                         const double* __restrict__ scal, const int* __restrict__ bad,
                         const double* __restrict__ qr_logr, int* __restrict__ alive,
                         double* __restrict__ weight, int* __restrict__ nfrozen) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  weight_one(w, tau, spin, e0s, e_const, logdet_n, logdet, scal, bad, qr_logr, alive, weight,
             nfrozen);
}

// ---------------------------------------------------------------- QR
// Phi = Q R with real positive diag(R) by shifted Cholesky QR3 (Fukaya,
// Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020): pass 0 factors
// S + s I = R^H R with s = 11 (M N + N (N + 1)) u tr(S), so that the
// factorisation exists for any numerically full-rank Phi, and two further
// unshifted passes restore orthonormality; after every pass Phi <- Phi R^-1.
// qr_logr[w] = sum over passes of sum_j log R_jj (so log det(Psi_T^T Phi)
// drops by qr_logr).  A failed factorisation marks the walker bad.
// Factorisation of walker w (one block); the caller skips frozen and bad walkers.
template <int T>
AFQ_DEV void qr_one(int N, int M, double* __restrict__ ph_re, double* __restrict__ ph_im,
                    double* __restrict__ qr_logr, int* __restrict__ bad, int w, int64_t sw,
                    double* smem) {
  double* stage = smem;
  double* S = stage + Sm<T>::STAGE;       // N x N complex: S, then R, then R^-1
  double* col = S + 2 * N * N;            // 2N
  double* fail = col + 2 * N;             // failure flag of the factorisation
  const int64_t off = (int64_t)w * sw;   // walker stride (N M for the walker store)
  double* pr = ph_re + off;
  double* pi = ph_im + off;
  const int tid = threadIdx.x;
  if (tid == 0) *fail = 0.0;
  __syncthreads();
  double logr = 0.0;
  for (int pass = 0; pass < 3; ++pass) {
    // S[i][j] = sum_p conj(Phi[p][i]) Phi[p][j]; K runs over (re, im) of p:
    //   Re S: [re_i, im_i] . [re_j, im_j],   Im S: [-im_i, re_i] . [re_j, im_j]
    auto gx = [&](int r, int k) {
      const int pl = r >= N, i = pl ? r - N : r;
      const int kk = k >= M, p = kk ? k - M : k;
      if (!pl) return kk ? pi[(int64_t)i * M + p] : pr[(int64_t)i * M + p];
      return kk ? pr[(int64_t)i * M + p] : -pi[(int64_t)i * M + p];
    };
    auto gy = [&](int c, int k) {
      const int kk = k >= M, p = kk ? k - M : k;
      return kk ? pi[(int64_t)c * M + p] : pr[(int64_t)c * M + p];
    };
    auto st = [&](int r, int c, double v) {
      const int pl = r >= N, i = pl ? r - N : r;
      S[(i * N + c) * 2 + pl] = v;
    };
    small_gram<T>(2 * N, N, 2 * M, gx, gy, st, stage);
    if (pass == 0) {
      double tr = 0.0;
      for (int j = 0; j < N; ++j) tr += S[(j * N + j) * 2];
      const double shift = 11.0 * ((double)M * N + (double)N * (N + 1)) * 1.1102230246251565e-16 * tr;
      __syncthreads();
      for (int j = tid; j < N; j += blockDim.x) S[(j * N + j) * 2] += shift;
      __syncthreads();
    }
    // right-looking Cholesky: S = R^H R, R upper triangular (stored in S)
    for (int j = 0; j < N; ++j) {
      const double piv = S[(j * N + j) * 2];
      if (!(piv > 0.0) || !isfinite(piv)) {
        if (tid == 0) *fail = 1.0;
      }
      const double d = sqrt(piv > 0.0 ? piv : 1.0);
      __syncthreads();
      for (int i = tid; i < N; i += blockDim.x) {
        if (i < j) {
          S[(j * N + i) * 2] = 0.0;
          S[(j * N + i) * 2 + 1] = 0.0;
        } else if (i == j) {
          S[(j * N + j) * 2] = d;
          S[(j * N + j) * 2 + 1] = 0.0;
        } else {
          S[(j * N + i) * 2] /= d;
          S[(j * N + i) * 2 + 1] /= d;
        }
      }
      __syncthreads();
      for (int e = tid; e < N * N; e += blockDim.x) {
        const int a = e / N, b = e % N;
        if (a <= j || b <= j) continue;
        const cplx ra = cmake(S[(j * N + a) * 2], S[(j * N + a) * 2 + 1]);
        const cplx rb = cmake(S[(j * N + b) * 2], S[(j * N + b) * 2 + 1]);
        const cplx u = cmulc(ra, rb);
        S[e * 2] -= u.re;
        S[e * 2 + 1] -= u.im;
      }
      __syncthreads();
    }
    if (*fail != 0.0) break;
    if (tid == 0)
      for (int j = 0; j < N; ++j) logr += log(S[(j * N + j) * 2]);
    // in-place inverse of the upper triangular R, column by column:
    // column j of R^-1 = -(R^-1)[0:j, 0:j] R[0:j, j] / R[j][j], (R^-1)[j][j] = 1 / R[j][j]
    for (int j = 0; j < N; ++j) {
      for (int i = tid; i < j; i += blockDim.x) {
        col[i * 2] = S[(i * N + j) * 2];
        col[i * 2 + 1] = S[(i * N + j) * 2 + 1];
      }
      __syncthreads();
      const double rjj = 1.0 / S[(j * N + j) * 2];
      for (int i = tid; i < j; i += blockDim.x) {
        cplx acc = cmake(0.0, 0.0);
        for (int k = i; k < j; ++k)
          acc = cadd(acc, cmul(cmake(S[(i * N + k) * 2], S[(i * N + k) * 2 + 1]),
                               cmake(col[k * 2], col[k * 2 + 1])));
        S[(i * N + j) * 2] = -acc.re * rjj;
        S[(i * N + j) * 2 + 1] = -acc.im * rjj;
      }
      __syncthreads();
      if (tid == 0) S[(j * N + j) * 2] = rjj;
      __syncthreads();
    }
    apply_right<T>(N, M, S, pr, pi, pr, pi, stage);
    __threadfence();
    __syncthreads();
  }
  if (tid == 0) {
    qr_logr[w] = logr;
    if (*fail != 0.0 || !isfinite(logr)) bad[w] = 1;
  }
}

// QR after step t when (t + 1) % every == 0 (step read from the device
// counter when cs is given; otherwise the host launches only on such steps).
AFQ_DEV bool qr_due(const CallState* cs, int add, int every) {
  const uint64_t t = cs->step + (uint64_t)add;
  return every > 0 && (t + 1) % (uint64_t)every == 0;
}

template <int T>
AFQ_DEV void qr_block(int N, int M, double* __restrict__ ph_re, double* __restrict__ ph_im,
                      double* __restrict__ qr_logr, int* __restrict__ bad,
                      const int* __restrict__ alive, const CallState* __restrict__ cs, int add,
                      int every, int64_t sw, double* smem) {
  const int w = blockIdx.x;
  if (cs && !qr_due(cs, add, every)) {
    // not this step: its log det R is 0
    if (threadIdx.x == 0) qr_logr[w] = 0.0;
    return;
  }
  if (!alive[w] || bad[w]) return;
  qr_one<T>(N, M, ph_re, ph_im, qr_logr, bad, w, sw, smem);
}

// 160 x 160 engine (2N > 128).
__global__ __launch_bounds__(256) void k_qr(int N, int M, double* __restrict__ ph_re,
                                            double* __restrict__ ph_im,
                                            double* __restrict__ qr_logr,
                                            int* __restrict__ bad,
                                            const int* __restrict__ alive,
                                            const CallState* __restrict__ cs, int add,
                                            int every, int64_t sw) {
  extern __shared__ double smem[];
  qr_block<5>(N, M, ph_re, ph_im, qr_logr, bad, alive, cs, add, every, sw, smem);
}

// 128 x 128 engine, held to two waves per SIMD (256 registers): the few
// registers it then spills cost less than running one wave per SIMD
// (c3: 3.37 -> 2.42 ms per launch).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_qr4(
    int N, int M, double* __restrict__ ph_re, double* __restrict__ ph_im,
    double* __restrict__ qr_logr, int* __restrict__ bad, const int* __restrict__ alive,
    const CallState* __restrict__ cs, int add, int every, int64_t sw) {
  extern __shared__ double smem[];
  qr_block<4>(N, M, ph_re, ph_im, qr_logr, bad, alive, cs, add, every, sw, smem);
}

// Frozen walkers keep their held state: copy it over the proposed one.
AFQ_DEV void commit_one(int N, int M, int w, const double* __restrict__ ph_re,
                        const double* __restrict__ ph_im, const double* __restrict__ th_re,
                        const double* __restrict__ th_im, double* __restrict__ phn_re,
                        double* __restrict__ phn_im, double* __restrict__ thn_re,
                        double* __restrict__ thn_im) {
  const int64_t off = (int64_t)w * N * M;
  for (int e = threadIdx.x; e < N * M; e += blockDim.x) {
    phn_re[off + e] = ph_re[off + e];
    phn_im[off + e] = ph_im[off + e];
    thn_re[off + e] = th_re[off + e];
    thn_im[off + e] = th_im[off + e];
  }
}

__global__ void k_commit(int N, int M, const int* __restrict__ alive,
                         const double* __restrict__ ph_re, const double* __restrict__ ph_im,
                         const double* __restrict__ th_re, const double* __restrict__ th_im,
                         double* __restrict__ phn_re, double* __restrict__ phn_im,
                         double* __restrict__ thn_re, double* __restrict__ thn_im) {
  const int w = blockIdx.x;
  if (alive[w]) return;
  commit_one(N, M, w, ph_re, ph_im, th_re, th_im, phn_re, phn_im, thn_re, thn_im);
}

// ---------------------------------------------------------------- work queue
// Next item of a persistent launch: one atomic per block, broadcast in LDS.
AFQ_DEV int queue_next(WorkQ* q, int* slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(&q->head, 1);
  __syncthreads();
  const int it = *slot;
  __syncthreads();
  return it;
}

// Leaving a persistent launch: the last block out resets the queue for the
// next launch (every block has taken its last item by then).
AFQ_DEV void queue_leave(WorkQ* q) {
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&q->done, 1) == (int)gridDim.x - 1) {
      atomicExch(&q->head, 0);
      atomicExch(&q->done, 0);
    }
  }
}

// The per-walker back half of a step for many systems in one persistent
// launch: item (system, walker) = overlap and Theta at the proposed
// orbitals, the QR when due, the weight update, and the held state copied
// over a frozen walker's proposal.  Items come from the queue in the host's
// order (costliest systems first).
__global__ __launch_bounds__(256) void k_back_queue(const BackSys* __restrict__ sys,
                                                    const int2* __restrict__ items, int n_items,
                                                    WorkQ* q, double tau,
                                                    const CallState* __restrict__ cs, int add,
                                                    int every, int qr_now, int ctl_off) {
  extern __shared__ double smem[];
  // two control words after the work area (all LDS is dynamic, so the
  // kernel may take the whole 160 KB)
  int& slot = ((int*)(smem + ctl_off))[0];
  int& run = ((int*)(smem + ctl_off))[1];
  const bool due = cs ? qr_due(cs, add, every) : qr_now != 0;
  for (;;) {
    const int it = queue_next(q, &slot);
    if (it >= n_items) break;
    const int2 d = items[it];
    const BackSys& S = sys[d.x];
    const int w = d.y;
    if (sm_tiles(S.N) == 4)
      overlap_one<4>(S.N, S.M, S.psit, S.phn_re, S.phn_im, S.logdet_n, S.thn_re, S.thn_im, S.bad,
                     nullptr, w, smem);
    else
      overlap_one<5>(S.N, S.M, S.psit, S.phn_re, S.phn_im, S.logdet_n, S.thn_re, S.thn_im, S.bad,
                     nullptr, w, smem);
    __syncthreads();
    if (due) {
      if (threadIdx.x == 0) run = S.alive[w] && !S.bad[w];
      __syncthreads();
      if (run) {
        if (sm_tiles(S.N) == 4)
          qr_one<4>(S.N, S.M, S.phn_re, S.phn_im, S.qr_logr, S.bad, w, (int64_t)S.N * S.M, smem);
        else
          qr_one<5>(S.N, S.M, S.phn_re, S.phn_im, S.qr_logr, S.bad, w, (int64_t)S.N * S.M, smem);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      weight_one(w, tau, S.spin, S.e0s, S.e_const, S.logdet_n, S.logdet, S.scal, S.bad,
                 due ? S.qr_logr : nullptr, S.alive, S.weight, S.nfrozen);
      run = !S.alive[w];
    }
    __syncthreads();
    if (run)
      commit_one(S.N, S.M, w, S.phi_re, S.phi_im, S.th_re, S.th_im, S.phn_re, S.phn_im, S.thn_re,
                 S.thn_im);
    __syncthreads();
  }
  queue_leave(q);
}

// ---------------------------------------------------------------- energy
// E_L = e_core + E1 + 1/2 sum_g ell_g^2 - (s / 2) sum_g X_g,  E1 = ell_G (the
// h block), X_g = tr(T_g T_g), s the spin factor (each spin block of a
// closed-shell determinant adds X_g / 2).  Capped: clamp(Re E_L, E0 -+ dE)
// if dE > 0.
__global__ __launch_bounds__(256) void k_energy(int G, int G1, double e_core, double xs,
                                                const double* __restrict__ ell_re,
                                                const double* __restrict__ ell_im,
                                                const double* __restrict__ ex_re,
                                                const double* __restrict__ ex_im,
                                                double* __restrict__ eloc,
                                                double* __restrict__ ecap,
                                                const E0Dev* __restrict__ e0s, double dE) {
  __shared__ double red[4];
  const int w = blockIdx.x;
  const double* lr = ell_re + (int64_t)w * G1;
  const double* li = ell_im + (int64_t)w * G1;
  const double* xr = ex_re + (int64_t)w * G1;
  const double* xi = ex_im + (int64_t)w * G1;
  double sr = 0.0, si = 0.0;
  for (int g = threadIdx.x; g < G; g += 256) {
    sr += 0.5 * (lr[g] * lr[g] - li[g] * li[g]) - xs * xr[g];
    si += lr[g] * li[g] - xs * xi[g];
  }
  sr = block_sum(sr, red);
  si = block_sum(si, red);
  if (threadIdx.x == 0) {
    const double er = e_core + lr[G] + sr, ei = li[G] + si;
    eloc[w * 2] = er;
    eloc[w * 2 + 1] = ei;
    if (ecap) {
      double c = er;
      if (dE > 0.0) {
        const double e0 = e0s->e0;
        if (!(c >= e0 - dE)) c = e0 - dE;   // NaN goes to the lower edge
        if (c > e0 + dE) c = e0 + dE;
      }
      ecap[w] = c;
    }
  }
}

// (sum_w W_w Ebar_w, sum_w W_w) over live walkers, fixed order.  counts[0]:
// walkers not frozen, counts[4]: walkers with W > 0.  With window > 0, E0
// for the next step becomes the mean of the last `window` per-step estimates
// with sum W > 0 (oldest first), the running best estimate of Sec. II.A.
__global__ __launch_bounds__(256) void k_estimator(int W, const double* __restrict__ weight,
                                                   const double* __restrict__ ecap,
                                                   const int* __restrict__ alive,
                                                   double* __restrict__ out2, int* __restrict__ counts,
                                                   const CallState* __restrict__ cs, int add,
                                                   int64_t row, E0Dev* __restrict__ e0s,
                                                   int window) {
  __shared__ double red[4];
  if (cs && cs->energies)
    out2 = cs->energies + (row * cs->n_steps + (int64_t)(cs->step + (uint64_t)add - cs->step0)) * 2;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int w = threadIdx.x; w < W; w += 256) {
    if (alive[w]) {
      a += weight[w] * ecap[w];
      b += weight[w];
      c += 1.0;
      d += weight[w] > 0.0 ? 1.0 : 0.0;
    }
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  c = block_sum(c, red);
  d = block_sum(d, red);
  if (threadIdx.x == 0) {
    out2[0] = a;
    out2[1] = b;
    if (counts) {
      counts[0] = (int)c;
      counts[4] = (int)d;
    }
    if (window > 0 && b > 0.0) {
      const double e = a / b;
      if (isfinite(e)) {
        const int win = window < kE0Max ? window : kE0Max;
        e0s->ring[e0s->head] = e;
        e0s->head = (e0s->head + 1) % win;
        if (e0s->count < win) ++e0s->count;
        double tot = 0.0;
        for (int i = 0; i < e0s->count; ++i)
          tot += e0s->ring[(e0s->head - e0s->count + i + win) % win];
        e0s->e0 = tot / e0s->count;
      }
    }
  }
}

__global__ void k_zero_counters(int* c) {
  if (threadIdx.x < kCounters) c[threadIdx.x] = 0;
}

__global__ void k_set_e0(E0Dev* e0s, double e0) {
  e0s->e0 = e0;
  e0s->count = 0;
  e0s->head = 0;
}

// ---------------------------------------------------------------- population control
// Comb resampling (not described in the paper): with T = sum_w W_w and the
// running sums C_i (both added left to right by one thread), slot j copies
// walker src[j] = min{i : C_i > (j + u) T / n}, u from Philox4x64-10 under
// the key (seed, sid + 2^32), counter step + 1, word 0.  Due after global step
// t when (t + 1) % every == 0 (read from the device step under replay);
// T = 0 leaves the population alone.  flag[0] = 1 when the copies run.
__global__ __launch_bounds__(256) void k_comb_select(int W, const double* __restrict__ weight,
                                                     uint64_t seed, uint64_t sid, uint64_t step,
                                                     const CallState* __restrict__ cs, int add,
                                                     int every, double* __restrict__ csum,
                                                     int* __restrict__ src, int* __restrict__ flag) {
  __shared__ double tot_s;
  if (cs) step = cs->step + (uint64_t)add;
  const bool due = every > 0 && (step + 1) % (uint64_t)every == 0;
  if (threadIdx.x == 0) {
    double t = 0.0;
    if (due)
      for (int i = 0; i < W; ++i) {
        t += weight[i];
        csum[i] = t;
      }
    tot_s = t;
    flag[0] = due && t > 0.0 ? 1 : 0;
  }
  __syncthreads();
  const double T = tot_s;
  if (!(due && T > 0.0)) return;
  U64x4 c;
  c.v[0] = step + 1;
  c.v[1] = c.v[2] = c.v[3] = 0;
  const U64x4 r = philox4x64_10(c, seed, sid + (1ull << 32));
  const double u = (double)(r.v[0] >> 11) * 0x1.0p-53;
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    const double z = ((double)j + u) * T / (double)W;
    int lo = 0, hi = W - 1;   // first i with csum[i] > z (the last if none)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (csum[mid] > z) hi = mid;
      else lo = mid + 1;
    }
    src[j] = lo;
  }
}

// dst[j] = src-walker copy of every per-walker array (orbital planes NM,
// Coulomb vector G1, log-overlap 2, energies 3).
__global__ void k_comb_gather(int NM, int G1, const int* __restrict__ flag, const int* __restrict__ src,
                              const double* __restrict__ ph_re, const double* __restrict__ ph_im,
                              const double* __restrict__ th_re, const double* __restrict__ th_im,
                              const double* __restrict__ ell_re, const double* __restrict__ ell_im,
                              const double* __restrict__ logdet, const double* __restrict__ eloc,
                              const double* __restrict__ ecap, double* __restrict__ dph_re,
                              double* __restrict__ dph_im, double* __restrict__ dth_re,
                              double* __restrict__ dth_im, double* __restrict__ dell_re,
                              double* __restrict__ dell_im, double* __restrict__ small) {
  if (!flag[0]) return;
  const int j = blockIdx.x;
  const int i = src[j];
  const int64_t o = (int64_t)i * NM, d = (int64_t)j * NM;
  for (int e = threadIdx.x; e < NM; e += blockDim.x) {
    dph_re[d + e] = ph_re[o + e];
    dph_im[d + e] = ph_im[o + e];
    dth_re[d + e] = th_re[o + e];
    dth_im[d + e] = th_im[o + e];
  }
  for (int e = threadIdx.x; e < G1; e += blockDim.x) {
    dell_re[(int64_t)j * G1 + e] = ell_re[(int64_t)i * G1 + e];
    dell_im[(int64_t)j * G1 + e] = ell_im[(int64_t)i * G1 + e];
  }
  if (threadIdx.x == 0) {
    small[j * 5 + 0] = logdet[i * 2];
    small[j * 5 + 1] = logdet[i * 2 + 1];
    small[j * 5 + 2] = eloc[i * 2];
    small[j * 5 + 3] = eloc[i * 2 + 1];
    small[j * 5 + 4] = ecap[i];
  }
}

// The gathered copies back into the walker store, weights 1.
__global__ void k_comb_commit(int NM, int G1, const int* __restrict__ flag,
                              const double* __restrict__ dph_re, const double* __restrict__ dph_im,
                              const double* __restrict__ dth_re, const double* __restrict__ dth_im,
                              const double* __restrict__ dell_re, const double* __restrict__ dell_im,
                              const double* __restrict__ small, double* __restrict__ ph_re,
                              double* __restrict__ ph_im, double* __restrict__ th_re,
                              double* __restrict__ th_im, double* __restrict__ ell_re,
                              double* __restrict__ ell_im, double* __restrict__ logdet,
                              double* __restrict__ eloc, double* __restrict__ ecap,
                              double* __restrict__ weight, int* __restrict__ alive) {
  if (!flag[0]) return;
  const int j = blockIdx.x;
  const int64_t d = (int64_t)j * NM;
  for (int e = threadIdx.x; e < NM; e += blockDim.x) {
    ph_re[d + e] = dph_re[d + e];
    ph_im[d + e] = dph_im[d + e];
    th_re[d + e] = dth_re[d + e];
    th_im[d + e] = dth_im[d + e];
  }
  for (int e = threadIdx.x; e < G1; e += blockDim.x) {
    ell_re[(int64_t)j * G1 + e] = dell_re[(int64_t)j * G1 + e];
    ell_im[(int64_t)j * G1 + e] = dell_im[(int64_t)j * G1 + e];
  }
  if (threadIdx.x == 0) {
    logdet[j * 2] = small[j * 5 + 0];
    logdet[j * 2 + 1] = small[j * 5 + 1];
    eloc[j * 2] = small[j * 5 + 2];
    eloc[j * 2 + 1] = small[j * 5 + 3];
    ecap[j] = small[j * 5 + 4];
    weight[j] = 1.0;
    alive[j] = 1;
  }
}

// ---------------------------------------------------------------- layouts

__global__ void k_to_planar(const double* __restrict__ in, int W, int M, int N,
                            double* __restrict__ re, double* __restrict__ im) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)W * M * N;
  if (e >= tot) return;
  const int64_t w = e / ((int64_t)M * N);
  const int rem = (int)(e % ((int64_t)M * N));
  const int j = rem / M, p = rem % M;
  const int64_t src = (w * M + p) * N + j;
  re[e] = in[src * 2];
  im[e] = in[src * 2 + 1];
}

__global__ void k_from_planar(const double* __restrict__ re, const double* __restrict__ im, int W,
                              int M, int N, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)W * M * N;
  if (e >= tot) return;
  const int64_t w = e / ((int64_t)M * N);
  const int rem = (int)(e % ((int64_t)M * N));
  const int p = rem / N, j = rem % N;
  const int64_t src = (w * N + j) * M + p;
  out[e * 2] = re[src];
  out[e * 2 + 1] = im[src];
}

// out[r][c] (interleaved) = (re[r * ld + c], im[r * ld + c]) for c < cols.
__global__ void k_pack_complex(const double* __restrict__ re, const double* __restrict__ im,
                               int64_t n, int64_t ld, int64_t cols, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * cols) return;
  const int64_t r = e / cols, c = e % cols;
  out[e * 2] = re[r * ld + c];
  out[e * 2 + 1] = im[r * ld + c];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int sm_stage(int N) { return sm_tiles(N) == 4 ? Sm<4>::STAGE : Sm<5>::STAGE; }
size_t overlap_lds(int N) {
  return sizeof(double) * (sm_stage(N) + 2 * N * N + 2 * N + 8) + sizeof(int) * N;
}
size_t qr_lds(int N) { return sizeof(double) * (sm_stage(N) + 2 * N * N + 2 * N + 1); }

// Allow a kernel the whole 160 KiB of LDS of a gfx950 CU (once per kernel).
hipError_t allow_full_lds(const void* fn, bool& done) {
  if (done) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess) done = true;
  return e;
}
bool g_lds_overlap[2] = {false, false}, g_lds_qr[2] = {false, false};

// k_qr<T> over all walkers of a system (strides sw between walkers).
hipError_t run_qr(const SysDev& s, double* ph_re, double* ph_im, double* logr, int* bad,
                  const CallState* cs, int add, int every, int64_t sw, hipStream_t st) {
  if (2 * s.N > kSmRowsMax) return hipErrorInvalidValue;
  const size_t lds = qr_lds(s.N);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const bool t4 = sm_tiles(s.N) == 4;
  const void* fn = t4 ? (const void*)k_qr4 : (const void*)k_qr;
  hipError_t e = allow_full_lds(fn, g_lds_qr[t4 ? 0 : 1]);
  if (e != hipSuccess) return e;
  if (t4)
    hipLaunchKernelGGL(k_qr4, dim3(s.W), dim3(256), lds, st, s.N, s.M, ph_re, ph_im, logr, bad,
                       s.alive, cs, add, every, sw);
  else
    hipLaunchKernelGGL(k_qr, dim3(s.W), dim3(256), lds, st, s.N, s.M, ph_re, ph_im, logr, bad,
                       s.alive, cs, add, every, sw);
  return hipGetLastError();
}

}  // namespace

// ==================================================================== launchers

hipError_t launch_fields(uint64_t seed, uint64_t sid, uint64_t step, int W, int G, double* out,
                         hipStream_t st, const CallState* cs, int add) {
  const int64_t n = (int64_t)W * ((G + 3) / 4);
  hipLaunchKernelGGL(k_fields, dim3(nblk(n, 256)), dim3(256), 0, st, seed, sid, step, W, G, out,
                     cs, add);
  return hipGetLastError();
}

__global__ void k_call_begin(CallState* cs, uint64_t step0, int64_t n_steps, double* energies) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    cs->step = step0;
    cs->step0 = step0;
    cs->n_steps = n_steps;
    cs->energies = energies;
  }
}

__global__ void k_call_advance(CallState* cs, int n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) cs->step += (uint64_t)n;
}

hipError_t launch_call_begin(CallState* cs, uint64_t step0, int64_t n_steps, double* energies,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_call_begin, dim3(1), dim3(64), 0, st, cs, step0, n_steps, energies);
  return hipGetLastError();
}

hipError_t launch_call_advance(CallState* cs, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_call_advance, dim3(1), dim3(64), 0, st, cs, n);
  return hipGetLastError();
}

hipError_t launch_lbar(const SysDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_lbar, dim3(s.G), dim3(256), 0, st, s.N, s.M, s.spin, s.Lx, s.psit,
                     s.lbar);
  return hipGetLastError();
}

hipError_t launch_axpy_L(const SysDev& s, const double* coef, double alpha, double* out,
                         hipStream_t st) {
  const int64_t MM = (int64_t)s.M * s.M;
  hipLaunchKernelGGL(k_axpy_L, dim3(nblk(MM, 256)), dim3(256), 0, st, s.G, MM, s.L, coef, alpha,
                     out);
  return hipGetLastError();
}

hipError_t launch_force_bias(SysDev& s, const double* x, double tau, hipStream_t st) {
  hipLaunchKernelGGL(k_force_bias, dim3(s.W), dim3(256), 0, st, s.G, s.G + 1, sqrt(tau), s.ell_re,
                     s.ell_im, s.lbar, x, s.av_re, s.av_im, s.scal, s.ncap,
                     s.counters ? s.counters + 1 : nullptr);
  return hipGetLastError();
}

hipError_t launch_overlap(SysDev& s, int W, const double* ph_re, const double* ph_im,
                          double* logdet_out, double* th_re, double* th_im, int* bad,
                          hipStream_t st) {
  if (2 * s.N > kSmRowsMax) return hipErrorInvalidValue;
  const size_t lds = overlap_lds(s.N);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const bool t4 = sm_tiles(s.N) == 4;
  const void* fn = t4 ? (const void*)k_overlap<4> : (const void*)k_overlap<5>;
  hipError_t e = allow_full_lds(fn, g_lds_overlap[t4 ? 0 : 1]);
  if (e != hipSuccess) return e;
  if (t4)
    hipLaunchKernelGGL(k_overlap<4>, dim3(W), dim3(256), lds, st, s.N, s.M, s.psit, ph_re, ph_im,
                       logdet_out, th_re, th_im, bad, (double*)nullptr);
  else
    hipLaunchKernelGGL(k_overlap<5>, dim3(W), dim3(256), lds, st, s.N, s.M, s.psit, ph_re, ph_im,
                       logdet_out, th_re, th_im, bad, (double*)nullptr);
  return hipGetLastError();
}

hipError_t launch_weight(SysDev& s, double tau, const double* qr_logr, hipStream_t st) {
  hipLaunchKernelGGL(k_weight, dim3(nblk(s.W, 256)), dim3(256), 0, st, s.W, tau, s.spin, s.e0s,
                     s.e_const,
                     s.logdet_n, s.logdet, s.scal, s.bad, qr_logr, s.alive, s.weight,
                     s.counters ? s.counters + 3 : nullptr);
  return hipGetLastError();
}

hipError_t launch_qr(SysDev& s, double* ph_re, double* ph_im, double* qr_logr, hipStream_t st,
                     const CallState* cs, int add, int every) {
  return run_qr(s, ph_re, ph_im, qr_logr, s.bad, cs, add, every, (int64_t)s.N * s.M, st);
}

hipError_t launch_qr_strided(SysDev& s, double* ph_re, double* ph_im, int64_t sw, double* logr,
                             int* bad, hipStream_t st) {
  return run_qr(s, ph_re, ph_im, logr, bad, nullptr, 0, 0, sw, st);
}

size_t back_lds(int N) {
  const size_t a = overlap_lds(N), b = qr_lds(N);
  return a > b ? a : b;
}

hipError_t launch_back_queue(const BackSys* d_sys, const int2* d_items, int n_items, int max_n,
                             WorkQ* q, double tau, const CallState* cs, int add, int every,
                             bool qr_now, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (2 * max_n > kSmRowsMax) return hipErrorInvalidValue;
  const size_t work = back_lds(max_n);
  const int ctl_off = (int)((work + 7) / 8);        // in doubles
  const size_t lds = sizeof(double) * (ctl_off + 1);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static bool g_lds_back = false;
  hipError_t e = allow_full_lds((const void*)k_back_queue, g_lds_back);
  if (e != hipSuccess) return e;
  // blocks resident at once: LDS-limited, at most 8 per compute unit
  int per_cu = (int)((160 * 1024) / (lds + 64));
  if (per_cu > 8) per_cu = 8;
  if (per_cu < 1) per_cu = 1;
  int grid = 256 * per_cu;
  if (grid > n_items) grid = n_items;
  hipLaunchKernelGGL(k_back_queue, dim3(grid), dim3(256), lds, st, d_sys, d_items, n_items, q,
                     tau, cs, add, every, qr_now ? 1 : 0, ctl_off);
  return hipGetLastError();
}

hipError_t launch_commit(SysDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_commit, dim3(s.W), dim3(256), 0, st, s.N, s.M, s.alive, s.phi_re, s.phi_im,
                     s.th_re, s.th_im, s.phn_re, s.phn_im, s.thn_re, s.thn_im);
  return hipGetLastError();
}

hipError_t launch_energy(SysDev& s, int W, const double* ell_re, const double* ell_im,
                         const double* ex_re, const double* ex_im, double* eloc, double* ecap,
                         const E0Dev* e0s, double tau, hipStream_t st) {
  double dE = 0.0;
  if (tau > 0.0) {
    const double ne = s.spin * s.N;   // electrons
    dE = 0.5 * sqrt(ne / tau) + sqrt(ne * tau);
  }
  hipLaunchKernelGGL(k_energy, dim3(W), dim3(256), 0, st, s.G, s.G + 1, s.e_core, 0.5 * s.spin,
                     ell_re, ell_im,
                     ex_re, ex_im, eloc, ecap, e0s, dE);
  return hipGetLastError();
}

hipError_t launch_estimator(SysDev& s, double* out2, hipStream_t st, const CallState* cs, int add,
                            int64_t row, int e0_window) {
  hipLaunchKernelGGL(k_estimator, dim3(1), dim3(256), 0, st, s.W, s.weight, s.ecap, s.alive, out2,
                     s.counters, cs, add, row, s.e0s, e0_window);
  return hipGetLastError();
}

hipError_t launch_zero_counters(SysDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, s.counters);
  return hipGetLastError();
}

hipError_t launch_set_e0(SysDev& s, double e0, hipStream_t st) {
  hipLaunchKernelGGL(k_set_e0, dim3(1), dim3(1), 0, st, s.e0s, e0);
  return hipGetLastError();
}

hipError_t launch_pop_control(SysDev& s, uint64_t seed, uint64_t sid, uint64_t step, int every,
                              hipStream_t st, const CallState* cs, int add) {
  const int NM = s.N * s.M, G1 = s.G + 1;
  hipLaunchKernelGGL(k_comb_select, dim3(1), dim3(256), 0, st, s.W, s.weight, seed, sid, step, cs,
                     add, every, s.pc_cum, s.pc_src, s.pc_flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the next-step buffers (phn, thn) and the exchange-term arrays are free
  // between steps: they stage the copies
  hipLaunchKernelGGL(k_comb_gather, dim3(s.W), dim3(256), 0, st, NM, G1, s.pc_flag, s.pc_src,
                     s.phi_re, s.phi_im, s.th_re, s.th_im, s.ell_re, s.ell_im, s.logdet, s.eloc,
                     s.ecap, s.phn_re, s.phn_im, s.thn_re, s.thn_im, s.ex_re, s.ex_im, s.pc_small);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_comb_commit, dim3(s.W), dim3(256), 0, st, NM, G1, s.pc_flag, s.phn_re,
                     s.phn_im, s.thn_re, s.thn_im, s.ex_re, s.ex_im, s.pc_small, s.phi_re, s.phi_im,
                     s.th_re, s.th_im, s.ell_re, s.ell_im, s.logdet, s.eloc, s.ecap, s.weight,
                     s.alive);
  return hipGetLastError();
}

hipError_t launch_to_planar(const double* in, int W, int M, int N, double* re, double* im,
                            hipStream_t st) {
  const int64_t n = (int64_t)W * M * N;
  hipLaunchKernelGGL(k_to_planar, dim3(nblk(n, 256)), dim3(256), 0, st, in, W, M, N, re, im);
  return hipGetLastError();
}

hipError_t launch_from_planar(const double* re, const double* im, int W, int M, int N,
                              double* out, hipStream_t st) {
  const int64_t n = (int64_t)W * M * N;
  hipLaunchKernelGGL(k_from_planar, dim3(nblk(n, 256)), dim3(256), 0, st, re, im, W, M, N, out);
  return hipGetLastError();
}

hipError_t launch_pack_complex(const double* re, const double* im, int64_t n, int64_t ld_in,
                               int64_t cols, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_complex, dim3(nblk(n * cols, 256)), dim3(256), 0, st, re, im, n,
                     ld_in, cols, out);
  return hipGetLastError();
}
