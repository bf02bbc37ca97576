// Dense contractions of the walker step on the FP64 matrix cores:
//  * generic strided GEMM (set-up work: Psi_T^T L_g, sum_g L_g L_g, ...),
//  * the exact one-body half-step Phi <- exp(-tau H1/2) Phi (Sec. III.B),
//  * the operator build A^w = i sqrt(tau) sum_g (x_g - fbar_g) L_g (Eq. heffTOT),
//  * the operator-orbital product A^w psi that every exponential method
//    repeats k times (Sec. IV), with the Taylor and Krylov drivers.
#include <algorithm>

#include "afq_device.h"
#include "afq_internal.h"

namespace {

// Map a linear block id to (outer, inner) so that the inner_n blocks that
// share an outer index are dispatched to the same XCD (block ids are handed
// to the 8 XCDs round-robin) and share its L2.  Grid = ceil(outer_n/8)*8*inner_n.
AFQ_DEV bool xcd_swizzle(int id, int inner_n, int outer_n, int& outer, int& inner) {
  const int xcd = id & 7, slot = id >> 3;
  const int grp = slot / inner_n;
  inner = slot - grp * inner_n;
  outer = grp * 8 + xcd;
  return outer < outer_n;
}
inline int xcd_grid(int outer_n, int inner_n) { return ((outer_n + 7) / 8) * 8 * inner_n; }

// ------------------------------------------------------------ generic GEMM

template <int MT, int NT>
__global__ __launch_bounds__(256) void k_gemm_generic(GemmArgs g) {
  constexpr int ROWS = 32 * MT, COLS = 32 * NT;
  __shared__ double As[ROWS * kLDK];
  __shared__ double Bs[COLS * kLDK];
  const int nct = (g.Cn + COLS - 1) / COLS;
  const int rt = blockIdx.x / nct, ct = blockIdx.x % nct;
  const int64_t b = blockIdx.y;
  const int r0 = rt * ROWS, c0 = ct * COLS;
  const int nr = min(ROWS, g.R - r0), nc = min(COLS, g.Cn - c0);
  const WaveSplit ws = wave_split<MT, NT>(nr, nc);
  TileAcc<MT, NT> acc;
  acc.zero();
  const double* A = g.A + b * g.sAb;
  const double* B = g.B + b * g.sBb;
  auto getA = [&](int r, int k) {
    return A[(int64_t)(r0 + r) * g.sAr + (int64_t)(k / g.kin) * g.sAkb + (int64_t)(k % g.kin) * g.sAk];
  };
  auto getB = [&](int c, int k) {
    return B[(int64_t)(c0 + c) * g.sBc + (int64_t)(k / g.kin) * g.sBkb + (int64_t)(k % g.kin) * g.sBk];
  };
  auto fa = [&](int k0, double* S) {
    if (g.sAk == 1) stage_rows<ROWS>(S, k0, g.K, nr, getA);
    else stage_rows_kmajor<ROWS>(S, k0, g.K, nr, getA);
  };
  auto fb = [&](int k0, double* S) {
    if (g.sBk == 1) stage_rows<COLS>(S, k0, g.K, nc, getB);
    else stage_rows_kmajor<COLS>(S, k0, g.K, nc, getB);
  };
  tile_gemm<MT, NT>(g.K, ws, fa, fb, As, Bs, acc);
  double* C = g.C + b * g.sCb;
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      if (i >= ws.mtv || j >= ws.ntv) continue;
      const int c = acc_col(ws, j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = acc_row(ws, i, e);
        if (r < nr && c < nc) {
          const int64_t idx = (int64_t)(r0 + r) * g.sCr + (int64_t)(c0 + c) * g.sCc;
          double v = g.alpha * acc.c[i][j][e];
          if (g.beta != 0.0) v += g.beta * C[idx];
          C[idx] = v;
        }
      }
    }
}

// Same strided contraction on the pipelined engine (128 x 128 tiles of 8
// waves) for the large set-up and adjoint products.  KB: K is a sequence of
// blocks of kin elements (stride sAkb / sBkb between blocks).
using GPP = Pipe<4, 2, 2, 4>;

template <bool AKM, bool BKM, bool KB>
__global__ __launch_bounds__(GPP::NT) void k_gemm_pipe(GemmArgs g, int nct) {
  extern __shared__ double smem[];
  const int rt = blockIdx.x / nct, ct = blockIdx.x % nct;
  const int64_t b = blockIdx.y;
  const int r0 = rt * GPP::ROWS, c0 = ct * GPP::COLS;
  const int nr = min(GPP::ROWS, g.R - r0), nc = min(GPP::COLS, g.Cn - c0);
  const double* A = g.A + b * g.sAb + (int64_t)r0 * g.sAr;
  const double* B = g.B + b * g.sBb + (int64_t)c0 * g.sBc;
  auto koff = [&](int k, int64_t sk, int64_t skb) {
    if (!KB) return (int64_t)k * sk;
    const int kb = k / g.kin;
    return (int64_t)kb * skb + (int64_t)(k - kb * g.kin) * sk;
  };
  auto ga = [&](int r, int k) { return A[(int64_t)r * g.sAr + koff(k, g.sAk, g.sAkb)]; };
  auto gb = [&](int c, int k) { return B[(int64_t)c * g.sBc + koff(k, g.sBk, g.sBkb)]; };
  d4_t acc[2][4];
  const PipeSplit sp = pipe_gemm<4, 2, 2, 4, AKM, BKM>(g.K, nr, nc, ga, gb, smem, acc);
  double* C = g.C + b * g.sCb;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (i >= sp.mtv || j >= sp.ntv) continue;
      const int c = pipe_col(sp, j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = pipe_row(sp, i, e);
        if (r < nr && c < nc) {
          const int64_t idx = (int64_t)(r0 + r) * g.sCr + (int64_t)(c0 + c) * g.sCc;
          double v = g.alpha * acc[i][j][e];
          if (g.beta != 0.0) v += g.beta * C[idx];
          C[idx] = v;
        }
      }
    }
}

// ------------------------------------------------------------ one-body step
// out[(plane, w, j)][p] = sum_q in[(plane, w, j)][q] B[p][q]   (B symmetric)

using OBP = Pipe<4, 2, 2, 5>;

template <int PC>
__global__ __launch_bounds__(OBP::NT) void k_onebody(int WN, int M, int n_ct,
                                                     const double* __restrict__ in_re,
                                                     const double* __restrict__ in_im,
                                                     const double* __restrict__ Bm,
                                                     double* __restrict__ out_re,
                                                     double* __restrict__ out_im) {
  extern __shared__ double smem[];
  const int rt = blockIdx.x / n_ct, ct = blockIdx.x % n_ct;
  const int r0 = rt * OBP::ROWS, c0 = ct * OBP::COLS;
  const int R = 2 * WN;
  const int nr = min(OBP::ROWS, R - r0), nc = min(OBP::COLS, M - c0);
  auto ga = [&](int r, int k) {
    const int64_t rr = r0 + r;
    return rr < WN ? in_re[rr * M + k] : in_im[(rr - WN) * M + k];
  };
  auto gb = [&](int c, int k) { return Bm[(int64_t)(c0 + c) * M + k]; };
  // FP64: Bm = B.  BF16-split: Bm = B - I and the FP64 input is added back.
  pipe_run<4, 2, 2, 5, PC, false, false>(M, nr, nc, ga, gb, smem, [&](int r, int c, double v) {
    if (r < nr && c < nc) {
      const int64_t rr = r0 + r;
      if (rr < WN) {
        if (PC) v += in_re[rr * M + c0 + c];
        out_re[rr * M + c0 + c] = v;
      } else {
        if (PC) v += in_im[(rr - WN) * M + c0 + c];
        out_im[(rr - WN) * M + c0 + c] = v;
      }
    }
  });
}

// ------------------------------------------------------------ operator build
// A_plane[w][p][q] = sum_g a_plane[w][g] L[g][p][q],  a = i sqrt(tau) (x - fbar)
// (FP64; the BF16-split build is k_opbuild_mx).  A is symmetric, so only
// the column blocks of (p, q) that hold an element on or above the diagonal
// are formed (the packed triangle, M(M+1)/2 of the M^2 columns, padded to
// whole blocks); each element with q >= p is written to A[p][q] and A[q][p].
// Row tiles of 128 (RT = 2) or, from 2W = 512 rows on, of 256 (RT = 4: twice
// the MFMAs per staged operand and half the reads of L per column block).

template <int RT_>
struct OpTile {
  static constexpr int WR = 4, WC = 2, RT = RT_, CT = 4;
  static constexpr int ROWS = WR * RT * 16, COLS = WC * CT * 16, NT = WR * WC * 64;
};
static_assert(OpTile<2>::COLS == kOpRowsFP64 * 16, "a column tile is one 8 x 16 block of (p, q)");

template <int RT_>
__global__ __launch_bounds__(OpTile<RT_>::NT) void k_opbuild(int W, int G, int M,
                                                     const double* __restrict__ a_re,
                                                     const double* __restrict__ a_im,
                                                     const double* __restrict__ L,
                                                     double* __restrict__ A_re,
                                                     double* __restrict__ A_im,
                                                     const int2* __restrict__ blk, int n_rt,
                                                     int n_ct) {
  using T = OpTile<RT_>;
  extern __shared__ double smem[];
  int ct, rt;
  if (!xcd_swizzle(blockIdx.x, n_rt, n_ct, ct, rt)) return;
  const int r0 = rt * T::ROWS;
  const int2 b0 = blk[ct];
  const int p0 = b0.x, q0 = b0.y;
  const int64_t MM = (int64_t)M * M;
  const int R = 2 * W;
  const int nr = min(T::ROWS, R - r0);
  auto ga = [&](int r, int k) {
    const int rr = r0 + r;
    return rr < W ? a_re[(int64_t)rr * G + k] : a_im[(int64_t)(rr - W) * G + k];
  };
  auto gb = [&](int c, int k) {
    const int p = p0 + (c >> 4), q = q0 + (c & 15);
    return (p < M && q < M) ? L[(int64_t)k * MM + (int64_t)p * M + q] : 0.0;
  };
  pipe_run<T::WR, T::WC, T::RT, T::CT, 0, false, true>(G, nr, T::COLS, ga, gb, smem,
                                                        [&](int r, int c, double v) {
    const int p = p0 + (c >> 4), q = q0 + (c & 15);
    if (r < nr && p < M && q < M && q >= p) {
      const int rr = r0 + r;
      double* A = rr < W ? A_re + (int64_t)rr * MM : A_im + (int64_t)(rr - W) * MM;
      A[(int64_t)p * M + q] = v;
      if (q != p) A[(int64_t)q * M + p] = v;
    }
  });
}

// ------------------------------------------------------------ A^w psi
// For walker w and orbitals j < N: out[j][p] = sum_q A^w[p][q] v[j][q]
// (complex).  Real form: rows r = (plane, j), r < 2N, and K = (plane', q)
// in two halves of M:
//   half 0 (A_re): row (re, j) takes v_re[j][q], row (im, j) takes v_im[j][q],
//   half 1 (A_im): row (re, j) takes -v_im[j][q], row (im, j) takes v_re[j][q].
// mode 0: out = A v.   mode 1 (Taylor term n): out = A v / n and sum += out.
// mode 2 (Chebyshev T_1): out = A v and sum += c out (c = inv_n).
// mode 3 (Chebyshev T_n): out = 2 A v - out (out holds T_{n-2} on entry, v
// is T_{n-1}) and sum += c out.
//
// A workgroup of MV_W waves covers up to MV_W column tiles (16 values of p
// each) of one walker, one per wave, and all TR = ceil(2N / 16) row tiles.
// Each wave is the only reader of its 16 operator rows, so it loads them
// straight from global memory into its MFMA B fragments (lane (lr, lk) holds
// A[p0 + lr][q0 + 4 s + lk] for k-step s), the next chunk's while the current
// one runs; the orbital rows, read by every wave, go through two LDS stages.
// Each half of K runs in chunks of MV_BK with the last chunk padded with
// zeros, so the products accumulate in the groups of four consecutive q of a
// plain ordered sum.  Signs are applied when a chunk is staged, after the
// MFMAs that hide its loads.  (The BF16-split product is k_matvec_mx.)
constexpr int MV_W = 4;          // waves (column tiles) per workgroup
constexpr int MV_BK = 32;
constexpr int MV_LDK = MV_BK + 1;

template <int TR>
constexpr size_t matvec_lds_bytes() {
  return (size_t)2 * TR * 16 * MV_LDK * sizeof(double);
}

template <int TR>
__global__ __launch_bounds__(MV_W * 64) void k_matvec(int W, int N, int M, VecRef v,
                                                      const double* __restrict__ A_re,
                                                      const double* __restrict__ A_im,
                                                      VecOut o, int mode, double inv_n,
                                                      VecOut sum, int n_ct) {
  constexpr int NT = MV_W * 64;
  constexpr int ROWS = TR * 16;
  constexpr int RSTEP = NT / MV_BK;                       // staged rows per pass
  constexpr int PF = (ROWS + RSTEP - 1) / RSTEP;          // staged elements per thread
  constexpr int STAGE = ROWS * MV_LDK;
  extern __shared__ double smem[];
  int w, ct;
  if (!xcd_swizzle(blockIdx.x, n_ct, W, w, ct)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int TC = (M + 15) / 16;
  const int tpb = (TC + n_ct - 1) / n_ct;   // column tiles of this block (<= MV_W)
  const int tile = ct * tpb + wave;
  const bool active = wave < tpb && tile < TC;
  const int p = tile * 16 + lr;
  const bool p_ok = active && p < M;
  const int64_t MM = (int64_t)M * M;
  const double* Ar = A_re + (int64_t)w * MM + (int64_t)(p_ok ? p : 0) * M;
  const double* Ai = A_im + (int64_t)w * MM + (int64_t)(p_ok ? p : 0) * M;
  const double* vre = v.re + (int64_t)w * v.sw;
  const double* vim = v.im + (int64_t)w * v.sw;
  const int nr = 2 * N;
  const int sk = tid % MV_BK, srow0 = tid / MV_BK;
  const int nch = (M + MV_BK - 1) / MV_BK, nchunk = 2 * nch;

  double pv[PF], bn[8], bc[8];
  auto fetch_b = [&](int c) {
    const int h = c >= nch;
    const int q0 = (h ? c - nch : c) * MV_BK;
    const double* Ah = h ? Ai : Ar;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int q = q0 + 4 * s + lk;
      bn[s] = (p_ok && q < M) ? Ah[q] : 0.0;
    }
  };
  auto fetch_v = [&](int c) {
    const int h = c >= nch;
    const int q = (h ? c - nch : c) * MV_BK + sk;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int r = srow0 + i * RSTEP;
      double x = 0.0;
      if (r < nr && r < ROWS && q < M) {
        const bool im_row = r >= N;
        const int j = im_row ? r - N : r;
        const double* src = (im_row != (h != 0)) ? vim : vre;
        x = src[(int64_t)j * v.sj + q];
      }
      pv[i] = x;
    }
  };
  auto store = [&](double* S, int c) {
    const int h = c >= nch;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int r = srow0 + i * RSTEP;
      if (r < ROWS) S[r * MV_LDK + sk] = (h && r < N) ? -pv[i] : pv[i];
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) bc[s] = bn[s];
  };

  d4_t acc[TR];
#pragma unroll
  for (int i = 0; i < TR; ++i) acc[i] = d4_t{0.0, 0.0, 0.0, 0.0};
  fetch_b(0);
  fetch_v(0);
  store(smem, 0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const double* As = smem + (c & 1) * STAGE;
    const bool more = c + 1 < nchunk;
    if (active) {
      // the next chunk's loads are issued between the MFMAs of this one
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        double a[TR];
#pragma unroll
        for (int i = 0; i < TR; ++i) a[i] = As[(i * 16 + lr) * MV_LDK + 4 * s + lk];
#pragma unroll
        for (int i = 0; i < TR; ++i) acc[i] = mfma_f64(a[i], bc[s], acc[i]);
        if (s == 0 && more) fetch_b(c + 1);
        if (s == 4 && more) fetch_v(c + 1);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else if (more) {
      fetch_b(c + 1);
      fetch_v(c + 1);
    }
    if (more) store(smem + ((c + 1) & 1) * STAGE, c + 1);
    __syncthreads();
  }
  if (!p_ok) return;
  // accumulator element e of tile i: row i 16 + 4 e + lk, column p
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = i * 16 + 4 * e + lk;
      if (r >= nr) continue;
      const bool im_row = r >= N;
      const int j = im_row ? r - N : r;
      double val = acc[i][e];
      const int64_t off = (int64_t)w * o.sw + (int64_t)j * o.sj + p;
      if (mode == 3) val = 2.0 * val - (im_row ? o.im[off] : o.re[off]);
      if (mode >= 1) {
        const double add = mode == 1 ? (val *= inv_n) : inv_n * val;
        const int64_t soff = (int64_t)w * sum.sw + (int64_t)j * sum.sj + p;
        if (im_row) sum.im[soff] += add;
        else sum.re[soff] += add;
      }
      if (im_row) o.im[off] = val;
      else o.re[off] = val;
    }
}

int matvec_col_blocks(int M) {
  const int TC = (M + 15) / 16;
  return (TC + MV_W - 1) / MV_W;
}

template <int TR>
hipError_t matvec_tr(SysDev& s, VecRef v, VecOut o, int mode, double inv_n, VecOut sum,
                     hipStream_t st) {
  constexpr size_t lds = matvec_lds_bytes<TR>();
  static bool lds_ok = false;
  if (!lds_ok) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_matvec<TR>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  // a tuned count below the minimum would leave column tiles out
  const int n_ct = max(s.mv_ct, matvec_col_blocks(s.M));
  hipLaunchKernelGGL((k_matvec<TR>), dim3(xcd_grid(s.W, n_ct)), dim3(MV_W * 64), lds, st, s.W,
                     s.N, s.M, v, s.A_re, s.A_im, o, mode, inv_n, sum, n_ct);
  return hipGetLastError();
}

// The operator-orbital product in the system's current precision.
hipError_t run_matvec(SysDev& s, VecRef v, VecOut o, int mode, double inv_n, VecOut sum,
                      hipStream_t st) {
  if (s.op_pieces > 0) return launch_matvec_mx(s, v, o, mode, inv_n, sum, st);
  switch ((2 * s.N + 15) / 16) {
    case 1: return matvec_tr<1>(s, v, o, mode, inv_n, sum, st);
    case 2: return matvec_tr<2>(s, v, o, mode, inv_n, sum, st);
    case 3: return matvec_tr<3>(s, v, o, mode, inv_n, sum, st);
    case 4: return matvec_tr<4>(s, v, o, mode, inv_n, sum, st);
    case 5: return matvec_tr<5>(s, v, o, mode, inv_n, sum, st);
    case 6: return matvec_tr<6>(s, v, o, mode, inv_n, sum, st);
    case 7: return matvec_tr<7>(s, v, o, mode, inv_n, sum, st);
    case 8: return matvec_tr<8>(s, v, o, mode, inv_n, sum, st);
    case 9: return matvec_tr<9>(s, v, o, mode, inv_n, sum, st);
    case 10: return matvec_tr<10>(s, v, o, mode, inv_n, sum, st);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------ Krylov pieces
// One 64-lane wave per (walker, orbital).  M <= 64 * KV_R.

constexpr int KV_R = 8;

// b_0 = psi / ||psi||, beta = ||psi||, dim = k (0 if psi == 0).
__global__ __launch_bounds__(256) void k_krylov_init(int WN, int M, int kmax, int k,
                                                     const double* __restrict__ in_re,
                                                     const double* __restrict__ in_im,
                                                     double* __restrict__ kb_re,
                                                     double* __restrict__ kb_im,
                                                     double* __restrict__ kbeta,
                                                     int* __restrict__ kdim) {
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (o >= WN) return;
  const double* xr = in_re + (int64_t)o * M;
  const double* xi = in_im + (int64_t)o * M;
  double s = 0.0;
  for (int p = lane; p < M; p += 64) s += xr[p] * xr[p] + xi[p] * xi[p];
  s = wave_sum(s);
  const double beta = sqrt(s);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  double* br = kb_re + (int64_t)o * kmax * M;
  double* bi = kb_im + (int64_t)o * kmax * M;
  for (int p = lane; p < M; p += 64) {
    br[p] = xr[p] * inv;
    bi[p] = xi[p] * inv;
  }
  if (lane == 0) {
    kbeta[o] = beta;
    kdim[o] = beta > 0.0 ? k : 0;
  }
}

// Arnoldi step m: w = A b_m (in wv) is orthogonalised against b_0..b_m by
// modified Gram-Schmidt (each b_i is read once into registers for both its
// projection and the update), with one more pass when the norm drops below
// 1/sqrt(2) of its value before the pass (Daniel-Gragg-Kaufman-Stewart);
// H[0..m][m] accumulates the projections, H[m+1][m] = ||w|| and
// b_{m+1} = w / ||w|| unless the residual vanishes against ||A b_m||
// (happy breakdown: dim = m + 1, b_{m+1} = 0).
__global__ __launch_bounds__(256) void k_krylov_orth(int WN, int M, int kmax, int k, int m,
                                                     const double* __restrict__ wv_re,
                                                     const double* __restrict__ wv_im,
                                                     double* __restrict__ kb_re,
                                                     double* __restrict__ kb_im,
                                                     double* __restrict__ kh,
                                                     int* __restrict__ kdim,
                                                     double breakdown_rel) {
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (o >= WN) return;
  if (m >= kdim[o]) return;
  double wr[KV_R], wi[KV_R];
  const double* xr = wv_re + (int64_t)o * M;
  const double* xi = wv_im + (int64_t)o * M;
#pragma unroll
  for (int t = 0; t < KV_R; ++t) {
    const int p = lane + 64 * t;
    wr[t] = p < M ? xr[p] : 0.0;
    wi[t] = p < M ? xi[p] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < KV_R; ++t) s += wr[t] * wr[t] + wi[t] * wi[t];
  const double wnorm2 = wave_sum(s);
  double* br = kb_re + (int64_t)o * kmax * M;
  double* bi = kb_im + (int64_t)o * kmax * M;
  double* H = kh + (int64_t)o * kmax * kmax * 2;
  double before2 = wnorm2, after2 = wnorm2;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1 && !(after2 < 0.5 * before2)) break;
    before2 = after2;
    for (int i = 0; i <= m; ++i) {
      double b_r[KV_R], b_i[KV_R];
      double ar = 0.0, ai = 0.0;
#pragma unroll
      for (int t = 0; t < KV_R; ++t) {
        const int p = lane + 64 * t;
        b_r[t] = p < M ? br[i * M + p] : 0.0;
        b_i[t] = p < M ? bi[i * M + p] : 0.0;
        ar += b_r[t] * wr[t] + b_i[t] * wi[t];
        ai += b_r[t] * wi[t] - b_i[t] * wr[t];
      }
      const double cr = wave_sum(ar), ci = wave_sum(ai);
#pragma unroll
      for (int t = 0; t < KV_R; ++t) {
        wr[t] -= cr * b_r[t] - ci * b_i[t];
        wi[t] -= cr * b_i[t] + ci * b_r[t];
      }
      if (lane == 0) {
        double* h = H + (i * kmax + m) * 2;
        if (pass == 0) {
          h[0] = cr;
          h[1] = ci;
        } else {
          h[0] += cr;
          h[1] += ci;
        }
      }
    }
    s = 0.0;
#pragma unroll
    for (int t = 0; t < KV_R; ++t) s += wr[t] * wr[t] + wi[t] * wi[t];
    after2 = wave_sum(s);
  }
  if (m + 1 >= k) return;
  const double hn = sqrt(after2);
  const bool brk = !(hn > breakdown_rel * sqrt(wnorm2)) || hn == 0.0;
  const double inv = brk ? 0.0 : 1.0 / hn;
#pragma unroll
  for (int t = 0; t < KV_R; ++t) {
    const int p = lane + 64 * t;
    if (p < M) {
      br[(m + 1) * M + p] = wr[t] * inv;
      bi[(m + 1) * M + p] = wi[t] * inv;
    }
  }
  if (lane == 0) {
    H[((m + 1) * kmax + m) * 2 + 0] = brk ? 0.0 : hn;
    H[((m + 1) * kmax + m) * 2 + 1] = 0.0;
    if (brk) kdim[o] = m + 1;
  }
}

// out = beta * B_d exp(H_d) e_1 with d = dim <= 16.  exp(H_d) e_1 by s
// Taylor substeps of 18 terms each, s = ceil(||H_d||_1 / 0.5), so that every
// substep has a norm of at most 1/2.  Lane i < d owns row i of H_d and
// component i of the vector; the vector is broadcast lane by lane through the
// scalar registers.
__global__ __launch_bounds__(256) void k_krylov_combine(int WN, int M, int kmax, int k,
                                                        const double* __restrict__ kb_re,
                                                        const double* __restrict__ kb_im,
                                                        const double* __restrict__ kh,
                                                        const double* __restrict__ kbeta,
                                                        const int* __restrict__ kdim,
                                                        double* __restrict__ out_re,
                                                        double* __restrict__ out_im,
                                                        int* __restrict__ nbreak) {
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (o >= WN) return;
  const int d = kdim[o];
  const double beta = kbeta[o];
  const double* H = kh + (int64_t)o * kmax * kmax * 2;
  double hr[16], hi[16];
#pragma unroll
  for (int l = 0; l < 16; ++l) {
    // upper Hessenberg: only entries on or above the subdiagonal exist
    const bool v = lane < d && l < d && lane <= l + 1;
    hr[l] = v ? H[(lane * kmax + l) * 2 + 0] : 0.0;
    hi[l] = v ? H[(lane * kmax + l) * 2 + 1] : 0.0;
  }
  // 1-norm: max over columns l of sum_i |H[i][l]| (column sums via shuffles)
  double nrm = 0.0;
#pragma unroll
  for (int l = 0; l < 16; ++l) {
    const double c = wave_sum(sqrt(hr[l] * hr[l] + hi[l] * hi[l]));
    nrm = fmax(nrm, c);
  }
  int nsub = (int)ceil(nrm / 0.5);
  if (nsub < 1) nsub = 1;
  const double sc = 1.0 / nsub;
  double yr = (lane == 0) ? 1.0 : 0.0, yi = 0.0;
  for (int sub = 0; sub < nsub; ++sub) {
    double tr = yr, ti = yi;
    double acr = yr, aci = yi;
    for (int n = 1; n <= 18; ++n) {
      double nr = 0.0, ni = 0.0;
#pragma unroll
      for (int l = 0; l < 16; ++l) {
        const double u = lane_bcast(tr, l), v = lane_bcast(ti, l);
        nr += hr[l] * u - hi[l] * v;
        ni += hr[l] * v + hi[l] * u;
      }
      const double f = sc / n;
      tr = nr * f;
      ti = ni * f;
      acr += tr;
      aci += ti;
    }
    yr = lane < d ? acr : 0.0;
    yi = lane < d ? aci : 0.0;
  }
  double ur[16], ui[16];
#pragma unroll
  for (int l = 0; l < 16; ++l) {
    ur[l] = lane_bcast(yr, l) * beta;
    ui[l] = lane_bcast(yi, l) * beta;
  }
  const double* br = kb_re + (int64_t)o * kmax * M;
  const double* bi = kb_im + (int64_t)o * kmax * M;
  double* xr = out_re + (int64_t)o * M;
  double* xi = out_im + (int64_t)o * M;
  for (int p = lane; p < M; p += 64) {
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int mm = 0; mm < 16; ++mm) {
      if (mm < d) {
        const double b_r = br[mm * M + p], b_i = bi[mm * M + p];
        ar += ur[mm] * b_r - ui[mm] * b_i;
        ai += ur[mm] * b_i + ui[mm] * b_r;
      }
    }
    xr[p] = ar;
    xi[p] = ai;
  }
  if (lane == 0 && d < k && d > 0 && nbreak) atomicAdd(nbreak, 1);
}

}  // namespace

int matvec_default_blocks(int M) { return matvec_col_blocks(M); }

int matvec_max_blocks(int M) { return (M + 15) / 16; }

hipError_t launch_matvec(SysDev& s, VecRef v, VecOut o, hipStream_t st) {
  return run_matvec(s, v, o, 0, 1.0, o, st);
}

hipError_t launch_matvec_acc(SysDev& s, VecRef v, VecOut o, double scale, VecOut sum,
                             hipStream_t st) {
  return run_matvec(s, v, o, 1, scale, sum, st);
}

hipError_t launch_matvec_probe(SysDev& s, const double* in_re, const double* in_im, double* out_re,
                               double* out_im, hipStream_t st) {
  const int64_t sw = (int64_t)s.N * s.M;
  VecRef v{in_re, in_im, sw, s.M};
  VecOut o{out_re, out_im, sw, s.M};
  return run_matvec(s, v, o, 0, 1.0, o, st);
}

// ==================================================================== launchers

template <bool AKM, bool BKM, bool KB>
hipError_t run_gemm_pipe(const GemmArgs& g, hipStream_t st) {
  static bool lds_ok = false;
  if (!lds_ok) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_gemm_pipe<AKM, BKM, KB>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)GPP::LDS_BYTES);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  const int nrt = (g.R + GPP::ROWS - 1) / GPP::ROWS;
  const int nct = (g.Cn + GPP::COLS - 1) / GPP::COLS;
  hipLaunchKernelGGL((k_gemm_pipe<AKM, BKM, KB>), dim3(nrt * nct, g.batch), dim3(GPP::NT),
                     GPP::LDS_BYTES, st, g, nct);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t st) {
  if (g.R <= 0 || g.Cn <= 0 || g.batch <= 0) return hipSuccess;
  // Large products go to the pipelined engine; small ones (a few tiles) to
  // the plain kernel, whose 64 x 64 tiles waste less on ragged edges.
  if ((double)g.R * g.Cn * g.K * g.batch >= (double)(1 << 24) && g.R >= 64 && g.Cn >= 64) {
    const bool akm = g.sAk != 1, bkm = g.sBk != 1, kb = g.kin < g.K;
    if (akm) {
      if (bkm) return kb ? run_gemm_pipe<true, true, true>(g, st) : run_gemm_pipe<true, true, false>(g, st);
      return kb ? run_gemm_pipe<true, false, true>(g, st) : run_gemm_pipe<true, false, false>(g, st);
    }
    if (bkm) return kb ? run_gemm_pipe<false, true, true>(g, st) : run_gemm_pipe<false, true, false>(g, st);
    return kb ? run_gemm_pipe<false, false, true>(g, st) : run_gemm_pipe<false, false, false>(g, st);
  }
  constexpr int MT = 2, NT = 2;
  const int nrt = (g.R + 32 * MT - 1) / (32 * MT);
  const int nct = (g.Cn + 32 * NT - 1) / (32 * NT);
  hipLaunchKernelGGL((k_gemm_generic<MT, NT>), dim3(nrt * nct, g.batch), dim3(256), 0, st, g);
  return hipGetLastError();
}

namespace {

template <int PC>
hipError_t onebody_p(SysDev& s, const double* in_re, const double* in_im, double* out_re,
                     double* out_im, hipStream_t st, const double* Bmat = nullptr) {
  constexpr size_t lds = pipe_lds_bytes<4, 2, 2, 5, PC>();
  static bool lds_ok = false;
  if (!lds_ok) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_onebody<PC>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  const int WN = s.W * s.N;
  const int nrt = (2 * WN + OBP::ROWS - 1) / OBP::ROWS;
  const int nct = (s.M + OBP::COLS - 1) / OBP::COLS;
  hipLaunchKernelGGL(k_onebody<PC>, dim3(nrt * nct), dim3(OBP::NT), lds, st, WN, s.M, nct, in_re,
                     in_im, Bmat ? Bmat : PC ? s.Bm1 : s.Bhalf, out_re, out_im);
  return hipGetLastError();
}

template <int RT_>
hipError_t opbuild_rt(SysDev& s, hipStream_t st) {
  using T = OpTile<RT_>;
  constexpr size_t lds = pipe_lds_bytes<T::WR, T::WC, T::RT, T::CT, 0>();
  static bool lds_ok = false;
  if (!lds_ok) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_opbuild<RT_>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  if (!s.op_blk || s.n_op_blk < 1) return hipErrorInvalidValue;
  const int n_rt = (2 * s.W + T::ROWS - 1) / T::ROWS;
  const int n_ct = s.n_op_blk;
  hipLaunchKernelGGL(k_opbuild<RT_>, dim3(xcd_grid(n_ct, n_rt)), dim3(T::NT), lds, st, s.W, s.G,
                     s.M, s.av_re, s.av_im, s.L, s.A_re, s.A_im, s.op_blk, n_rt, n_ct);
  return hipGetLastError();
}

hipError_t opbuild_fp64(SysDev& s, hipStream_t st) {
  return 2 * s.W >= 512 ? opbuild_rt<4>(s, st) : opbuild_rt<2>(s, st);
}

}  // namespace

__global__ void k_add_real(int64_t MM, int W, const double* __restrict__ D, double alpha,
                           double* __restrict__ A) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < MM * W;
       e += (int64_t)gridDim.x * blockDim.x)
    A[e] = fma(alpha, D[e % MM], A[e]);
}

hipError_t launch_add_real(SysDev& s, const double* D, double alpha, hipStream_t st) {
  const int64_t MM = (int64_t)s.M * s.M, n = MM * s.W;
  const int64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_add_real, dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, st, MM,
                     s.W, D, alpha, s.A_re);
  return hipGetLastError();
}

hipError_t launch_onebody_mat(SysDev& s, const double* Bm, const double* in_re,
                              const double* in_im, double* out_re, double* out_im,
                              hipStream_t st) {
  return onebody_p<0>(s, in_re, in_im, out_re, out_im, st, Bm);
}

hipError_t launch_onebody(SysDev& s, const double* in_re, const double* in_im, double* out_re,
                          double* out_im, hipStream_t st) {
  if (s.op_pieces == 3) return onebody_p<3>(s, in_re, in_im, out_re, out_im, st);
  if (s.op_pieces == 2) return onebody_p<2>(s, in_re, in_im, out_re, out_im, st);
  return onebody_p<0>(s, in_re, in_im, out_re, out_im, st);
}

void op_blocks(int M, int R, std::vector<int2>& out) {
  out.clear();
  for (int p0 = 0; p0 < M; p0 += R)
    for (int q0 = 0; q0 < M; q0 += 16)
      if (std::min(M, q0 + 16) - 1 >= p0) out.push_back(make_int2(p0, q0));
}

hipError_t launch_opbuild(SysDev& s, hipStream_t st) {
  if (s.op_pieces == 0) return opbuild_fp64(s, st);
  return launch_opbuild_mx(s, st);   // operator pieces for the BF16-split products
}

// out = a in, y = in (the first term of the Chebyshev sum and T_0).
__global__ void k_cheb_init(int64_t n, double a, const double* __restrict__ ire,
                            const double* __restrict__ iim, double* __restrict__ ore,
                            double* __restrict__ oim, double* __restrict__ yre,
                            double* __restrict__ yim) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double r = ire[e], i = iim[e];
    ore[e] = a * r;
    oim[e] = a * i;
    yre[e] = r;
    yim[e] = i;
  }
}

// Coefficients of the Chebyshev expansion of the exponential (Sec. IV.B):
// c_0 = J_0(i), c_n = 2 i^n J_n(-i).  With J_n(i z) = i^n I_n(z) both are
// real: c_0 = I_0(1), c_n = 2 I_n(1), from the power series
// I_n(1) = sum_m (1/2)^(2m + n) / (m! (m + n)!).
double cheb_coef(int n) {
  double term = 1.0;
  for (int q = 1; q <= n; ++q) term *= 0.5 / q;   // (1/2)^n / n!
  double sum = 0.0;
  for (int m = 0; m < 40; ++m) {
    sum += term;
    term *= 0.25 / ((m + 1.0) * (m + 1.0 + n));
  }
  return n == 0 ? sum : 2.0 * sum;
}

hipError_t launch_chebyshev(SysDev& s, int k, const double* in_re, const double* in_im,
                            double* out_re, double* out_im, double* s1_re, double* s1_im,
                            double* s2_re, double* s2_im, hipStream_t st) {
  const int64_t sw = (int64_t)s.N * s.M, sj = s.M, n = sw * s.W;
  const int64_t g = (n + 255) / 256;
  // out = c_0 T_0, s2 = T_0
  hipLaunchKernelGGL(k_cheb_init, dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, st, n,
                     cheb_coef(0), in_re, in_im, out_re, out_im, s2_re, s2_im);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || k < 1) return e;
  // s1 = T_1 = A T_0, out += c_1 T_1
  VecOut sum{out_re, out_im, sw, sj};
  e = run_matvec(s, VecRef{in_re, in_im, sw, sj}, VecOut{s1_re, s1_im, sw, sj}, 2, cheb_coef(1),
                 sum, st);
  if (e != hipSuccess) return e;
  // T_n = 2 A T_{n-1} - T_{n-2} over the older buffer, out += c_n T_n
  double* cur_re = s1_re;
  double* cur_im = s1_im;
  double* old_re = s2_re;
  double* old_im = s2_im;
  for (int m = 2; m <= k; ++m) {
    e = run_matvec(s, VecRef{cur_re, cur_im, sw, sj}, VecOut{old_re, old_im, sw, sj}, 3,
                   cheb_coef(m), sum, st);
    if (e != hipSuccess) return e;
    std::swap(cur_re, old_re);
    std::swap(cur_im, old_im);
  }
  return hipSuccess;
}

hipError_t launch_taylor(SysDev& s, int k, const double* in_re, const double* in_im,
                         double* out_re, double* out_im, double* s1_re, double* s1_im,
                         double* s2_re, double* s2_im, hipStream_t st) {
  const size_t bytes = sizeof(double) * (size_t)s.W * s.N * s.M;
  hipError_t e = hipMemcpyAsync(out_re, in_re, bytes, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(out_im, in_im, bytes, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  const int64_t sw = (int64_t)s.N * s.M, sj = s.M;
  const double* cur_re = in_re;
  const double* cur_im = in_im;
  double* bufs_re[2] = {s1_re, s2_re};
  double* bufs_im[2] = {s1_im, s2_im};
  for (int n = 1; n <= k; ++n) {
    VecRef v{cur_re, cur_im, sw, sj};
    VecOut o{bufs_re[n & 1], bufs_im[n & 1], sw, sj};
    VecOut sum{out_re, out_im, sw, sj};
    e = run_matvec(s, v, o, 1, 1.0 / n, sum, st);
    if (e != hipSuccess) return e;
    cur_re = bufs_re[n & 1];
    cur_im = bufs_im[n & 1];
  }
  return hipSuccess;
}

hipError_t launch_krylov(SysDev& s, int k, const double* in_re, const double* in_im,
                         double* out_re, double* out_im, double* wv_re, double* wv_im,
                         hipStream_t st) {
  if (k > s.kmax || k > 16 || s.M > 64 * KV_R) return hipErrorInvalidValue;
  const int WN = s.W * s.N;
  const int nb = (WN + 3) / 4;
  hipLaunchKernelGGL(k_krylov_init, dim3(nb), dim3(256), 0, st, WN, s.M, s.kmax, k, in_re, in_im,
                     s.kb_re, s.kb_im, s.kbeta, s.kdim);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t sw = (int64_t)s.N * s.M;
  for (int m = 0; m < k; ++m) {
    VecRef v{s.kb_re + (int64_t)m * s.M, s.kb_im + (int64_t)m * s.M, (int64_t)s.N * s.kmax * s.M,
             (int64_t)s.kmax * s.M};
    VecOut o{wv_re, wv_im, sw, s.M};
    e = run_matvec(s, v, o, 0, 1.0, o, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_krylov_orth, dim3(nb), dim3(256), 0, st, WN, s.M, s.kmax, k, m, wv_re,
                       wv_im, s.kb_re, s.kb_im, s.kh, s.kdim, 1e-12);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_krylov_combine, dim3(nb), dim3(256), 0, st, WN, s.M, s.kmax, k, s.kb_re,
                     s.kb_im, s.kh, s.kbeta, s.kdim, out_re, out_im,
                     s.counters ? s.counters + 2 : nullptr);
  return hipGetLastError();
}
