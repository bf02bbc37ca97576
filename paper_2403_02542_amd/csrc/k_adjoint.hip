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
// All T_g^w of a chunk of Cholesky blocks come from one GEMM C = (Psi_T^T L) TH^T.
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

// U rows (g, i) of the chunk from C rows (g, j): U[(g,i)][(w,pl,j)] as above.
__global__ void k_adj_u(int gn, int N, int W, int G1, int g0, const double* __restrict__ C,
                        const double* __restrict__ dE, const double* __restrict__ ell_re,
                        const double* __restrict__ ell_im, double* __restrict__ U) {
  const int64_t cols = (int64_t)W * 2 * N;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)gn * N * cols) return;
  const int64_t row = e / cols;
  const int64_t col = e - row * cols;
  const int g = (int)(row / N), i = (int)(row % N);
  const int w = (int)(col / (2 * N));
  const int rem = (int)(col % (2 * N));
  const int pl = rem >= N, j = pl ? rem - N : rem;
  // T_g^w[j][i] (plane pl) = C[(g, j)][(w, pl, i)]
  const double t = C[((int64_t)g * N + j) * cols + (int64_t)w * 2 * N + pl * N + i];
  const int64_t o = (int64_t)w * G1 + g0 + g;
  double v;
  if (!pl) v = (i == j ? ell_re[o] : 0.0) - t;
  else v = (i == j ? -ell_im[o] : 0.0) + t;
  U[e] = dE[w] * v;
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// grad_h and grad_L (device pointers, M x M and G x M x M).  dE on device.
// Uses s.ell_* of the current walkers (filled by the caller).
hipError_t launch_adjoint_into(SysDev& s, const double* dE, double* grad_h, double* grad_L,
                               double* TH, double* Cb, double* Ub, double* Db, double* Y,
                               int gchunk, hipStream_t st) {
  const int M = s.M, N = s.N, W = s.W, G = s.G, G1 = G + 1;
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
  for (int g0 = 0; g0 < G; g0 += gchunk) {
    const int gn = G - g0 < gchunk ? G - g0 : gchunk;
    // C[(g, i)][(w, pl, j)] = sum_p Lx[(g0 + g, i)][p] TH[(w, pl, j)][p]
    GemmArgs c{};
    c.A = s.Lx + (int64_t)g0 * NM; c.sAb = 0; c.sAr = M; c.sAk = 1; c.sAkb = 0;
    c.B = TH; c.sBb = 0; c.sBc = M; c.sBk = 1; c.sBkb = 0;
    c.C = Cb; c.sCb = 0; c.sCr = cols; c.sCc = 1;
    c.R = gn * N; c.Cn = (int)cols; c.K = M; c.kin = M; c.batch = 1; c.alpha = 1.0; c.beta = 0.0;
    if ((e = launch_gemm(c, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_u, dim3(nb((int64_t)gn * N * cols)), dim3(256), 0, st, gn, N, W, G1,
                       g0, Cb, dE, s.ell_re, s.ell_im, Ub);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // D[(g, i)][q] = sum_{(w,pl,j)} U[(g, i)][(w,pl,j)] TH[(w,pl,j)][q]
    GemmArgs d{};
    d.A = Ub; d.sAb = 0; d.sAr = cols; d.sAk = 1; d.sAkb = 0;
    d.B = TH; d.sBb = 0; d.sBc = 1; d.sBk = M; d.sBkb = 0;
    d.C = Db; d.sCb = 0; d.sCr = M; d.sCc = 1;
    d.R = gn * N; d.Cn = M; d.K = (int)cols; d.kin = (int)cols; d.batch = 1; d.alpha = 1.0;
    d.beta = 0.0;
    if ((e = launch_gemm(d, st)) != hipSuccess) return e;
    // grad_L[g0 + g][p][q] = 2 sum_i psit[i][p] D[(g, i)][q]
    GemmArgs gl{};
    gl.A = s.psit; gl.sAb = 0; gl.sAr = 1; gl.sAk = M; gl.sAkb = 0;
    gl.B = Db; gl.sBb = NM; gl.sBc = 1; gl.sBk = M; gl.sBkb = 0;
    gl.C = grad_L + (int64_t)g0 * M * M; gl.sCb = (int64_t)M * M; gl.sCr = M; gl.sCc = 1;
    gl.R = M; gl.Cn = M; gl.K = N; gl.kin = N; gl.batch = gn; gl.alpha = 2.0; gl.beta = 0.0;
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
