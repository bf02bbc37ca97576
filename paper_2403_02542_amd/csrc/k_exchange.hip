// Local-energy contraction (Eq. eloc, Cholesky form) on the FP64 matrix cores.
//
// For every walker w and Cholesky block g (g < G: Psi_T^T L_g; g = G:
// Psi_T^T h), T_g^w = (Psi_T^T L_g) Theta^w is an N x N complex matrix.
// The kernel never stores T: a 512-thread workgroup computes the T blocks
// of GA consecutive g-blocks and WB consecutive walkers as one MFMA tile
//   rows (g, i): GA N,   columns (w, plane, j): WB 2N,   K = M,
// then stages the tile in LDS a few g-blocks at a time and reduces every
// N x N block to
//   ell_g = 2 tr T_g        (the mixed <Lhat_g>, also the next force bias)
//   X_g   = tr(T_g T_g)     (exchange term)
// The h block gives ell_G = 2 tr(Psi_T^T h Theta), the one-body energy.
//
// Main loop: the eight waves split the 16-row MFMA tiles of the tile rows
// evenly (ceil(TR / 8) each) and all hold every column tile, so a 250-row
// tile at N = 50 keeps all waves equally busy.  K is consumed in chunks of
// 16; chunk c+1 is fetched from global memory into registers while the MFMAs
// of chunk c run from the other half of a double-buffered LDS stage.
#include "afq_device.h"
#include "afq_internal.h"

namespace {

constexpr int XW = 8;                      // waves per workgroup
constexpr int XT = XW * 64;                // threads
constexpr int X_RT = 2;                    // max row tiles per wave
constexpr int X_CTMAX = 10;                // max column tiles (all waves): 2N <= 160
constexpr int X_ROWS = XW * X_RT * 16;     // 256
constexpr int X_COLS = X_CTMAX * 16;       // 160
constexpr int X_STAGE = (X_ROWS + X_COLS) * kLDK;   // LDS stage (doubles), largest CT
constexpr int X_SUPER_G = 4, X_SUPER_W = 8;         // super-tile per XCD

// CT: column tiles held by every wave (compile-time, >= ceil(WB 2N / 16)).
template <int CT>
__global__ __launch_bounds__(XT) void k_exchange(int G1, int N, int M, int W, int GA, int WB,
                                                 int n_gt, int n_wt, int grp,
                                                 const double* __restrict__ Lx,
                                                 const double* __restrict__ th_re,
                                                 const double* __restrict__ th_im,
                                                 double* __restrict__ ell_re,
                                                 double* __restrict__ ell_im,
                                                 double* __restrict__ ex_re,
                                                 double* __restrict__ ex_im) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // XCD-aware order: the blocks of one super-tile (X_SUPER_G g-tiles x
  // X_SUPER_W walker tiles) run on one XCD and share its L2.
  const int id = blockIdx.x;
  const int xcd = id & 7, slot = id >> 3;
  const int per = X_SUPER_G * X_SUPER_W;
  const int sidx = (slot / per) * 8 + xcd, local = slot % per;
  const int n_sw = (n_wt + X_SUPER_W - 1) / X_SUPER_W;
  const int gt = (sidx / n_sw) * X_SUPER_G + local / X_SUPER_W;
  const int wt = (sidx % n_sw) * X_SUPER_W + local % X_SUPER_W;
  if (gt >= n_gt || wt >= n_wt) return;
  const int g0 = gt * GA, w0 = wt * WB;
  const int ga = min(GA, G1 - g0), wb = min(WB, W - w0);
  const int nr = ga * N, twoN = 2 * N, nc = wb * twoN;
  const int TR = (nr + 15) >> 4, TC = (nc + 15) >> 4;
  const int rpw = (TR + XW - 1) / XW;            // row tiles per wave (<= X_RT)
  const int rt0 = wave * rpw;
  const int mtv = max(0, min(rpw, TR - rt0));
  const double* A0 = Lx + (int64_t)g0 * N * M;

  // ---- staging: element e of a chunk is (row r, k) of A for e < X_ROWS*16,
  // then (col c, k) of B.  Fetch into registers, store into an LDS stage.
  constexpr int TOT = (X_ROWS + CT * 16) * kBK;
  constexpr int PF = (TOT + XT - 1) / XT;
  double pf[PF];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * XT;
      double v = 0.0;
      if (e >= TOT) {
      } else if (e < X_ROWS * kBK) {
        const int r = e >> 4, k = k0 + (e & 15);
        if (r < nr && k < M) v = A0[(int64_t)r * M + k];
      } else {
        const int e2 = e - X_ROWS * kBK;
        const int c = e2 >> 4, k = k0 + (e2 & 15);
        if (c < nc && k < M) {
          const int wl = c / twoN, rem = c - wl * twoN;
          const int pl = rem >= N, j = pl ? rem - N : rem;
          const int64_t row = ((int64_t)(w0 + wl) * N + j) * M;
          v = pl ? th_im[row + k] : th_re[row + k];
        }
      }
      pf[i] = v;
    }
  };
  auto store = [&](double* S) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + i * XT;
      const int r = e >> 4, k = e & 15;   // B rows follow A rows in the stage
      if (e < TOT) S[r * kLDK + k] = pf[i];
    }
  };

  d4_t acc[X_RT][CT];
#pragma unroll
  for (int i = 0; i < X_RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int nchunk = (M + kBK - 1) / kBK;
  const int lr = lane & 15, lk = lane >> 4;
  fetch(0);
  store(smem);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const double* S = smem + (ch & 1) * X_STAGE;
    if (ch + 1 < nchunk) fetch((ch + 1) * kBK);
    const double* As = S;
    const double* Bs = S + X_ROWS * kLDK;
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      double a[X_RT], b[CT];
#pragma unroll
      for (int i = 0; i < X_RT; ++i) a[i] = As[((rt0 + i) * 16 + lr) * kLDK + kk + lk];
#pragma unroll
      for (int j = 0; j < CT; ++j) b[j] = j < TC ? Bs[(j * 16 + lr) * kLDK + kk + lk] : 0.0;
#pragma unroll
      for (int i = 0; i < X_RT; ++i) {
        if (i < mtv) {
#pragma unroll
          for (int j = 0; j < CT; ++j)
            if (j < TC) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
        }
      }
    }
    if (ch + 1 < nchunk) store(smem + ((ch + 1) & 1) * X_STAGE);
    __syncthreads();
  }

  // ---- epilogue: per walker, groups of `grp` g-blocks staged in LDS
  double* Ts = smem;
  double* red = smem + 2 * X_STAGE - 4 * XW * 32;  // partial sums [gl][wave][4]
  const int ldt = twoN + 1;
  for (int wl = 0; wl < wb; ++wl) {
    for (int gb = 0; gb < ga; gb += grp) {
      const int gn = min(grp, ga - gb);
      const int rlo = gb * N, rhi = (gb + gn) * N;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < X_RT; ++i) {
        if (i >= mtv) continue;
#pragma unroll
        for (int j = 0; j < CT; ++j) {
          if (j >= TC) continue;
          const int c = j * 16 + lr - wl * twoN;
          if (c < 0 || c >= twoN) continue;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = (rt0 + i) * 16 + 4 * e + lk;
            if (r >= rlo && r < rhi) Ts[(r - rlo) * ldt + c] = acc[i][j][e];
          }
        }
      }
      __syncthreads();
      for (int gl = 0; gl < gn; ++gl) {
        const double* T = Ts + (int64_t)gl * N * ldt;
        double xr = 0.0, xi = 0.0, tr = 0.0, ti = 0.0;
        for (int e = tid; e < N * N; e += XT) {
          const int i = e / N, j = e - i * N;
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
          double* rr = red + (gl * XW + wave) * 4;
          rr[0] = xr;
          rr[1] = xi;
          rr[2] = tr;
          rr[3] = ti;
        }
      }
      __syncthreads();
      if (tid < gn) {
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int v = 0; v < XW; ++v)
          for (int q = 0; q < 4; ++q) s[q] += red[(tid * XW + v) * 4 + q];
        const int64_t o = (int64_t)(w0 + wl) * G1 + g0 + gb + tid;
        ex_re[o] = s[0];
        ex_im[o] = s[1];
        ell_re[o] = 2.0 * s[2];
        ell_im[o] = 2.0 * s[3];
      }
    }
  }
}

// Choose GA (g-blocks per tile) and WB (walkers per tile) for N: maximise
// the useful fraction of the MFMA work of the busiest wave.
void exchange_tile(int N, int& GA, int& WB) {
  double best = -1.0;
  GA = 1;
  WB = 1;
  for (int ga = 1; ga * N <= X_ROWS; ++ga)
    for (int wb = 1; wb * 2 * N <= X_COLS; ++wb) {
      const int TR = (ga * N + 15) / 16, TC = (wb * 2 * N + 15) / 16;
      const int rpw = (TR + XW - 1) / XW;
      if (rpw > X_RT || TC > X_CTMAX) continue;
      const double useful = (double)ga * N * wb * 2 * N;
      const double work = (double)XW * rpw * TC * 256.0;
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
  if (2 * N > X_COLS) return hipErrorInvalidValue;
  int GA, WB;
  exchange_tile(N, GA, WB);
  const int n_gt = (G1 + GA - 1) / GA, n_wt = (W + WB - 1) / WB;
  const int n_sg = (n_gt + X_SUPER_G - 1) / X_SUPER_G;
  const int n_sw = (n_wt + X_SUPER_W - 1) / X_SUPER_W;
  const int n_super = n_sg * n_sw;
  const int grid = ((n_super + 7) / 8) * 8 * X_SUPER_G * X_SUPER_W;
  // LDS: two stages; the epilogue reuses them for T (grp g-blocks at a time)
  // and keeps the partial sums at the end.
  const size_t lds = sizeof(double) * 2 * X_STAGE;
  const int red_d = 4 * XW * 32;
  const int avail = 2 * X_STAGE - red_d;
  int grp = avail / (N * (2 * N + 1));
  if (grp > 32) grp = 32;
  if (grp < 1) return hipErrorInvalidValue;
  const int TC = (WB * 2 * N + 15) / 16;
  const void* fn;
  if (TC <= 4) fn = (const void*)k_exchange<4>;
  else if (TC <= 7) fn = (const void*)k_exchange<7>;
  else if (TC <= 8) fn = (const void*)k_exchange<8>;
  else fn = (const void*)k_exchange<10>;
  static bool lds_ok[4] = {false, false, false, false};
  const int slot = TC <= 4 ? 0 : TC <= 7 ? 1 : TC <= 8 ? 2 : 3;
  if (!lds_ok[slot]) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_ok[slot] = true;
  }
  void* args[] = {(void*)&G1, (void*)&N, (void*)&s.M, (void*)&W, (void*)&GA, (void*)&WB,
                  (void*)&n_gt, (void*)&n_wt, (void*)&grp, (void*)&s.Lx, (void*)&th_re,
                  (void*)&th_im, (void*)&ell_re, (void*)&ell_im, (void*)&ex_re, (void*)&ex_im};
  const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(XT), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}
