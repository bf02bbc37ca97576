// Local-energy contraction (Eq. eloc, Cholesky form) on the FP64 matrix cores.
//
// For every walker w and Cholesky block g (g < G: Psi_T^T L_g; g = G:
// Psi_T^T h), T_g^w = (Psi_T^T L_g) Theta^w is an N x N complex matrix.
// The kernel never stores T: a workgroup computes the T blocks of GA
// consecutive g-blocks and WB consecutive walkers as one MFMA tile
//   rows (g, i) = GA N,   columns (w, plane, j) = WB 2N,   K = M,
// stages the tile in LDS walker by walker and reduces each N x N block to
//   ell_g = 2 tr T_g        (the mixed <Lhat_g>, also the next force bias)
//   X_g   = tr(T_g T_g)     (exchange term)
// The h block gives ell_G = 2 tr(Psi_T^T h Theta), the one-body energy.
#include "afq_device.h"
#include "afq_internal.h"

namespace {

constexpr int EX_MT = 4, EX_NT = 5;
constexpr int EX_ROWS = 32 * EX_MT, EX_COLS = 32 * EX_NT;
constexpr int EX_STAGE = (EX_ROWS + EX_COLS) * kLDK;
constexpr int EX_SUPER = 8;   // super-tile: 8 g-tiles x 8 walker tiles per XCD

__global__ __launch_bounds__(256) void k_exchange(int G1, int N, int M, int W, int GA, int WB,
                                                  int n_gt, int n_wt,
                                                  const double* __restrict__ Lx,
                                                  const double* __restrict__ th_re,
                                                  const double* __restrict__ th_im,
                                                  double* __restrict__ ell_re,
                                                  double* __restrict__ ell_im,
                                                  double* __restrict__ ex_re,
                                                  double* __restrict__ ex_im) {
  extern __shared__ double smem[];
  double* As = smem;
  double* Bs = smem + EX_ROWS * kLDK;
  // XCD-aware order: blocks of one 8 x 8 super-tile share an XCD and its L2.
  const int id = blockIdx.x;
  const int xcd = id & 7, slot = id >> 3;
  const int per = EX_SUPER * EX_SUPER;
  const int sidx = (slot / per) * 8 + xcd, local = slot % per;
  const int n_sw = (n_wt + EX_SUPER - 1) / EX_SUPER;
  const int gt = (sidx / n_sw) * EX_SUPER + local / EX_SUPER;
  const int wt = (sidx % n_sw) * EX_SUPER + local % EX_SUPER;
  if (gt >= n_gt || wt >= n_wt) return;
  const int g0 = gt * GA, w0 = wt * WB;
  const int ga = min(GA, G1 - g0), wb = min(WB, W - w0);
  const int nr = ga * N, twoN = 2 * N, nc = wb * twoN;
  const WaveSplit ws = wave_split<EX_MT, EX_NT>(nr, nc);
  TileAcc<EX_MT, EX_NT> acc;
  acc.zero();
  const double* A0 = Lx + (int64_t)g0 * N * M;
  auto getA = [&](int r, int k) { return A0[(int64_t)r * M + k]; };
  auto getB = [&](int c, int k) {
    const int wl = c / twoN, rem = c - wl * twoN;
    const int pl = rem >= N, j = pl ? rem - N : rem;
    const int64_t row = ((int64_t)(w0 + wl) * N + j) * M;
    return pl ? th_im[row + k] : th_re[row + k];
  };
  auto fa = [&](int k0, double* S) { stage_rows<EX_ROWS>(S, k0, M, nr, getA); };
  auto fb = [&](int k0, double* S) { stage_rows<EX_COLS>(S, k0, M, nc, getB); };
  tile_gemm<EX_MT, EX_NT>(M, ws, fa, fb, As, Bs, acc);

  double* Ts = smem;
  const int ldt = twoN + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int wl = 0; wl < wb; ++wl) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EX_MT; ++i)
#pragma unroll
      for (int j = 0; j < EX_NT; ++j) {
        if (i >= ws.mtv || j >= ws.ntv) continue;
        const int c = acc_col(ws, j) - wl * twoN;
        if (c < 0 || c >= twoN) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = acc_row(ws, i, e);
          if (r < nr) Ts[r * ldt + c] = acc.c[i][j][e];
        }
      }
    __syncthreads();
    for (int gl = wave; gl < ga; gl += 4) {
      const double* T = Ts + (int64_t)gl * N * ldt;
      double xr = 0.0, xi = 0.0, tr = 0.0, ti = 0.0;
      for (int e = lane; e < N * N; e += 64) {
        const int i = e / N, j = e - (e / N) * N;
        const double ar = T[i * ldt + j], ai = T[i * ldt + N + j];
        const double br = T[j * ldt + i], bi = T[j * ldt + N + i];
        xr += ar * br - ai * bi;
        xi += ar * bi + ai * br;
        if (i == j) {
          tr += ar;
          ti += ai;
        }
      }
      xr = wave_sum(xr);
      xi = wave_sum(xi);
      tr = wave_sum(tr);
      ti = wave_sum(ti);
      if (lane == 0) {
        const int64_t o = (int64_t)(w0 + wl) * G1 + g0 + gl;
        ell_re[o] = 2.0 * tr;
        ell_im[o] = 2.0 * ti;
        ex_re[o] = xr;
        ex_im[o] = xi;
      }
    }
  }
}

// Choose GA (g-blocks per tile) and WB (walkers per tile) for N: maximise the
// useful fraction of the MFMA work of the busiest wave.
void exchange_tile(int N, int& GA, int& WB) {
  double best = -1.0;
  GA = 1;
  WB = 1;
  for (int ga = 1; ga * N <= EX_ROWS; ++ga)
    for (int wb = 1; wb * 2 * N <= EX_COLS; ++wb) {
      const int TR = (ga * N + 15) / 16, TC = (wb * 2 * N + 15) / 16;
      const int hr = (TR + 1) / 2, hc = (TC + 1) / 2;
      if (hr > EX_MT || hc > EX_NT) continue;
      const double useful = (double)ga * N * wb * 2 * N;
      const double work = 4.0 * hr * hc * 256.0;
      const double eff = useful / work + 1e-6 * ga * wb;
      if (eff > best) {
        best = eff;
        GA = ga;
        WB = wb;
      }
    }
}

}  // namespace

hipError_t launch_exchange(SysDev& s, int W, const double* th_re, const double* th_im,
                           double* ell_re, double* ell_im, double* ex_re, double* ex_im,
                           hipStream_t st) {
  const int N = s.N, G1 = s.G + 1;
  if (2 * N > EX_COLS || N > EX_ROWS) return hipErrorInvalidValue;
  int GA, WB;
  exchange_tile(N, GA, WB);
  const int n_gt = (G1 + GA - 1) / GA, n_wt = (W + WB - 1) / WB;
  const int n_sg = (n_gt + EX_SUPER - 1) / EX_SUPER, n_sw = (n_wt + EX_SUPER - 1) / EX_SUPER;
  const int n_super = n_sg * n_sw;
  const int grid = ((n_super + 7) / 8) * 8 * EX_SUPER * EX_SUPER;
  size_t lds = sizeof(double) * EX_STAGE;
  const size_t lds_t = sizeof(double) * (size_t)GA * N * (2 * N + 1);
  if (lds_t > lds) lds = lds_t;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static bool lds_ok = false;
  if (!lds_ok) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_exchange,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  hipLaunchKernelGGL(k_exchange, dim3(grid), dim3(256), lds, st, G1, N, s.M, W, GA, WB, n_gt,
                     n_wt, s.Lx, th_re, th_im, ell_re, ell_im, ex_re, ex_im);
  return hipGetLastError();
}
