// Adjoint of the local energy and of the Coulomb vector with respect to h
// and L_g at fixed walkers and fixed Psi_T (derivatives of Eq. eloc).
//
// With Theta^w = Phi^w (Psi_T^T Phi^w)^-1 stored orbital-major (th[w][i][q] =
// Theta^w[q][i]), T_g^w = (Psi_T^T L_g) Theta^w and ell_g^w = 2 tr T_g^w,
//   E_L = e_core + 2 tr(Psi_T^T h Theta) + 1/2 sum_g ell_g^2 - sum_g tr(T_g T_g)
// gives, for weights d_w on Re E_L^w,
//   dE/dh[p][q]   = 2 sum_i Psi_T[p][i] Y[i][q],     Y = sum_w d_w Re Theta^w (orbital-major)
//   dE/dL_g[p][q] = 2 sum_i Psi_T[p][i] D_g[i][q],
//   D_g[i][q] = sum_w d_w Re( ell_g^w th_w[i][q] - sum_j T_g^w[j][i] th_w[j][q] ).
// D_g is evaluated as one contraction over (w, plane, j): D = U TH with the
// stacked rows TH[(w, plane, j)][q] = th_plane[w][j][q] and
//   U_g[i][(w, re, j)] = d_w ( Re ell_g^w delta_ij - Re T_g^w[j][i]),
//   U_g[i][(w, im, j)] = d_w (-Im ell_g^w delta_ij + Im T_g^w[j][i]).
// All T_g^w of a chunk of Cholesky blocks come from one product of TH with the
// half-rotated blocks Psi_T^T L_g, written out directly as U; ell_g^w comes
// from one product over K = (i, p).
#include "afq_device.h"
#include "afq_internal.h"

namespace {

// TH[(w, plane, j)][q] from the planar Green's functions.
__global__ void k_stack_theta(const double* __restrict__ re, const double* __restrict__ im, int W,
                              int NM, double* __restrict__ TH) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)W * 2 * NM;
  if (e >= tot) return;
  const int64_t w = e / (2 * NM);
  const int64_t r = e - w * 2 * NM;
  TH[e] = r < NM ? re[w * NM + r] : im[w * NM + (r - NM)];
}

// U of a chunk of Cholesky blocks straight from the contraction that forms
// T_g^w: rows r = (w, pl, i) of TH against rows c = (g, j) of the half-rotated
// blocks give T_g^w[j][i] (plane pl) = sum_p Lx[(g, j)][p] th_pl[w][i][p],
// stored at U[(g, i)][(w, pl, j)] (consecutive j contiguous) with the Coulomb
// term on the diagonal and the walker weight applied.
using UP = Pipe<4, 2, 2, 4>;

__global__ __launch_bounds__(UP::NT) void k_adj_t(int W, int N, int M, int gn, int n_ct,
                                                  const double* __restrict__ TH,
                                                  const double* __restrict__ Lx,
                                                  const double* __restrict__ dE,
                                                  const double* __restrict__ ellt,
                                                  double* __restrict__ U) {
  extern __shared__ double smem[];
  const int rt = blockIdx.x / n_ct, ct = blockIdx.x % n_ct;
  const int R = W * 2 * N, Cn = gn * N;
  const int r0 = rt * UP::ROWS, c0 = ct * UP::COLS;
  const int nr = min(UP::ROWS, R - r0), nc = min(UP::COLS, Cn - c0);
  auto ga = [&](int r, int k) { return TH[(int64_t)(r0 + r) * M + k]; };
  auto gb = [&](int c, int k) { return Lx[(int64_t)(c0 + c) * M + k]; };
  d4_t acc[2][4];
  const PipeSplit sp = pipe_gemm<4, 2, 2, 4, false, false>(M, nr, nc, ga, gb, smem, acc);
  const int64_t cols = (int64_t)R;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (a >= sp.mtv || b >= sp.ntv) continue;
      const int c = pipe_col(sp, b);
      if (c >= nc) continue;
      const int cc = c0 + c, g = cc / N, j = cc - g * N;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = pipe_row(sp, a, e);
        if (r >= nr) continue;
        const int rr = r0 + r, w = rr / (2 * N), rem = rr - w * 2 * N;
        const int pl = rem >= N, i = rem - pl * N;
        const double t = acc[a][b][e];
        double v = pl ? t : -t;
        if (i == j) {
          const double l = ellt[(int64_t)g * 2 * W + 2 * w + pl];
          v += pl ? -l : l;
        }
        U[((int64_t)g * N + i) * cols + (int64_t)w * 2 * N + pl * N + j] = dE[w] * v;
      }
    }
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// Slices of the D contraction: enough (tiles x slices >= ~1024 workgroups)
// to fill 256 compute units, each slice at least 512 long, S dividing 2 W N.
int adjoint_nsplit(int M, int N, int W, int gchunk) {
  const int64_t cols = (int64_t)W * 2 * N;
  const int64_t tiles = (((int64_t)gchunk * N + 127) / 128) * ((M + 127) / 128);
  int S = 1;
  while (S < 16 && tiles * S < 1024 && cols % (2 * S) == 0 && cols / (2 * S) >= 512) S *= 2;
  return S;
}

// grad_h and grad_L (device pointers, M x M and G x M x M).  dE on device.
// Uses s.ell_* of the current walkers (filled by the caller).
hipError_t launch_adjoint_into(SysDev& s, const double* dE, double* grad_h, double* grad_L,
                               double* TH, double* Ub, double* Db, double* Y, double* ellt,
                               int gchunk, hipStream_t st) {
  const int M = s.M, N = s.N, W = s.W, G = s.G;
  const int NM = N * M;
  const int64_t cols = (int64_t)W * 2 * N;
  hipLaunchKernelGGL(k_stack_theta, dim3(nb((int64_t)W * 2 * NM)), dim3(256), 0, st, s.th_re,
                     s.th_im, W, NM, TH);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Y[c] = sum_w dE[w] th_re[w][c]
  GemmArgs y{};
  y.A = dE; y.sAb = 0; y.sAr = 0; y.sAk = 1; y.sAkb = 0;
  y.B = TH; y.sBb = 0; y.sBc = 1; y.sBk = 2 * (int64_t)NM; y.sBkb = 0;
  y.C = Y; y.sCb = 0; y.sCr = 0; y.sCc = 1;
  y.R = 1; y.Cn = NM; y.K = W; y.kin = W; y.batch = 1; y.alpha = 1.0; y.beta = 0.0;
  if ((e = launch_gemm(y, st)) != hipSuccess) return e;
  // grad_h[p][q] = 2 sum_i psit[i][p] Y[i][q]
  GemmArgs gh{};
  gh.A = s.psit; gh.sAb = 0; gh.sAr = 1; gh.sAk = M; gh.sAkb = 0;
  gh.B = Y; gh.sBb = 0; gh.sBc = 1; gh.sBk = M; gh.sBkb = 0;
  gh.C = grad_h; gh.sCb = 0; gh.sCr = M; gh.sCc = 1;
  gh.R = M; gh.Cn = M; gh.K = N; gh.kin = N; gh.batch = 1; gh.alpha = 2.0; gh.beta = 0.0;
  if ((e = launch_gemm(gh, st)) != hipSuccess) return e;
  // Coulomb vector of every (g, walker, plane): ellt[g][(w, pl)] = 2 tr T_g^w
  GemmArgs el{};
  el.A = s.Lx; el.sAb = 0; el.sAr = NM; el.sAk = 1; el.sAkb = 0;
  el.B = TH; el.sBb = 0; el.sBc = NM; el.sBk = 1; el.sBkb = 0;
  el.C = ellt; el.sCb = 0; el.sCr = 2 * (int64_t)W; el.sCc = 1;
  el.R = G; el.Cn = 2 * W; el.K = NM; el.kin = NM; el.batch = 1; el.alpha = 2.0; el.beta = 0.0;
  if ((e = launch_gemm(el, st)) != hipSuccess) return e;
  static bool lds_ok = false;
  if (!lds_ok) {
    e = hipFuncSetAttribute((const void*)k_adj_t, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)UP::LDS_BYTES);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  const int S = adjoint_nsplit(M, N, W, gchunk);
  const int64_t kc = cols / S;
  const int64_t dstride = (int64_t)gchunk * NM;
  for (int g0 = 0; g0 < G; g0 += gchunk) {
    const int gn = G - g0 < gchunk ? G - g0 : gchunk;
    const int n_rt = (int)((cols + UP::ROWS - 1) / UP::ROWS);
    const int n_ct = (gn * N + UP::COLS - 1) / UP::COLS;
    hipLaunchKernelGGL(k_adj_t, dim3(n_rt * n_ct), dim3(UP::NT), UP::LDS_BYTES, st, W, N, M, gn,
                       n_ct, TH, s.Lx + (int64_t)g0 * NM, dE, ellt + (int64_t)g0 * 2 * W, Ub);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // D = U TH: the long contraction over (w, pl, j) is cut into S equal
    // slices (one batch entry each, partial sums D_s[(g, i)][q]) so that the
    // few output tiles still fill the chip; the slices are summed in the next
    // product, deterministically.
    GemmArgs d{};
    d.A = Ub; d.sAb = kc; d.sAr = cols; d.sAk = 1; d.sAkb = 0;
    d.B = TH; d.sBb = kc * M; d.sBc = 1; d.sBk = M; d.sBkb = 0;
    d.C = Db; d.sCb = dstride; d.sCr = M; d.sCc = 1;
    d.R = gn * N; d.Cn = M; d.K = (int)kc; d.kin = (int)kc; d.batch = S; d.alpha = 1.0;
    d.beta = 0.0;
    if ((e = launch_gemm(d, st)) != hipSuccess) return e;
    // grad_L[g0 + g][p][q] = 2 sum_{s, i} psit[i][p] D_s[(g, i)][q]
    GemmArgs gl{};
    gl.A = s.psit; gl.sAb = 0; gl.sAr = 1; gl.sAk = M; gl.sAkb = 0;
    gl.B = Db; gl.sBb = NM; gl.sBc = 1; gl.sBk = M; gl.sBkb = dstride;
    gl.C = grad_L + (int64_t)g0 * M * M; gl.sCb = (int64_t)M * M; gl.sCr = M; gl.sCc = 1;
    gl.R = M; gl.Cn = M; gl.K = N * S; gl.kin = N; gl.batch = gn; gl.alpha = 2.0; gl.beta = 0.0;
    if ((e = launch_gemm(gl, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Force-bias (Coulomb vector) adjoint: grad_L[g] = 2 psit^T Z_g with
// Z_g[(i, q)] = sum_w Re d_ell[w][g] th_re[w][i][q] + Im d_ell[w][g] th_im[w][i][q].
hipError_t launch_fb_adjoint_into(SysDev& s, const double* d_ell, double* grad_L, double* TH,
                                  double* Z, int gchunk, hipStream_t st) {
  const int M = s.M, N = s.N, W = s.W, G = s.G;
  const int NM = N * M;
  hipLaunchKernelGGL(k_stack_theta, dim3(nb((int64_t)W * 2 * NM)), dim3(256), 0, st, s.th_re,
                     s.th_im, W, NM, TH);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int g0 = 0; g0 < G; g0 += gchunk) {
    const int gn = G - g0 < gchunk ? G - g0 : gchunk;
    // Z[g][c] = sum_{k = (w, pl)} d_ell[w][g0 + g].{re, im} TH[w][pl][c]
    GemmArgs z{};
    z.A = d_ell + 2 * (int64_t)g0; z.sAb = 0; z.sAr = 2; z.sAk = 1; z.sAkb = 2 * (int64_t)G;
    z.B = TH; z.sBb = 0; z.sBc = 1; z.sBk = NM; z.sBkb = 2 * (int64_t)NM;
    z.C = Z; z.sCb = 0; z.sCr = NM; z.sCc = 1;
    z.R = gn; z.Cn = NM; z.K = 2 * W; z.kin = 2; z.batch = 1; z.alpha = 1.0; z.beta = 0.0;
    if ((e = launch_gemm(z, st)) != hipSuccess) return e;
    GemmArgs gl{};
    gl.A = s.psit; gl.sAb = 0; gl.sAr = 1; gl.sAk = M; gl.sAkb = 0;
    gl.B = Z; gl.sBb = NM; gl.sBc = 1; gl.sBk = M; gl.sBkb = 0;
    gl.C = grad_L + (int64_t)g0 * M * M; gl.sCb = (int64_t)M * M; gl.sCr = M; gl.sCc = 1;
    gl.R = M; gl.Cn = M; gl.K = N; gl.kin = N; gl.batch = gn; gl.alpha = 2.0; gl.beta = 0.0;
    if ((e = launch_gemm(gl, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}
