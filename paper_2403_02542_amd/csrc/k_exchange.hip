// Local-energy contraction (Eq. eloc, Cholesky form) on the FP64 matrix cores.
//
// For every walker w and Cholesky block g (g < G: L_g; g = G: h),
// T_g^w = Psi_T^T L_g Theta^w is an N x N complex matrix.  Since
// Psi_T^T Theta = I, Theta = Psi_T + Psi_perp Theta_v with Psi_perp an
// orthonormal complement of the trial orbitals, and
//   T_g^w = T0_g + (Psi_T^T L_g Psi_perp) Theta_v^w,  T0_g = Psi_T^T L_g Psi_T,
// a product over the virtual space only (K = M - N).
// The kernel never stores T: a 512-thread workgroup computes the T blocks
// of GA consecutive g-blocks and WB consecutive walkers as one MFMA tile
//   rows (g, i): GA N,   columns (w, j, plane): WB 2N,   K = M - N,
// the epilogue adding T0 (real, symmetric),
// then stages the tile in LDS a few blocks at a time and reduces every
// N x N block (exchange_epilogue) to
//   ell_g = s tr T_g        (the mixed <Lhat_g>, also the next force bias)
//   X_g   = tr(T_g T_g)     (exchange term)
// with s the spin factor (2 for a closed-shell determinant of spatial
// orbitals, 1 for spin orbitals).  The h block gives ell_G = s tr(Psi_T^T h
// Theta), the one-body energy.
//
// Main loop: the eight waves split the 16-row MFMA tiles of the tile rows
// evenly (ceil(TR / 8) each) and all hold every column tile, so a 250-row
// tile at N = 50 keeps all waves equally busy.  K is consumed in chunks of
// 16; chunk c+1 is fetched from global memory into registers while the MFMAs
// of chunk c run from the other half of a double-buffered LDS stage.
#include <algorithm>
#include <vector>

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
// The workgroup takes the whole 160 KB of LDS (one workgroup per compute unit
// anyway): two stages for the main loop, then as many staged g-blocks as fit
// for the epilogue, with the partial sums at the end.
constexpr int X_LDS = 160 * 1024 / 8;                // doubles
constexpr int X_RED = 4 * XW * 32;                   // partial sums [gl][wave][4]
static_assert(2 * X_STAGE <= X_LDS - X_RED, "LDS budget");
constexpr int X_SUPER_G = 4, X_SUPER_W = 8;         // super-tile per XCD

// CT: column tiles held by every wave (compile-time, >= ceil(WB 2N / 16)).
// One tile (g-tile gt, walker tile wt) of one system.
template <int CT>
__device__ __forceinline__ void exchange_tile_run(const XSys& p, int gt, int wt, double* smem) {
  const int G1 = p.G1, N = p.N, M = p.K, W = p.W, GA = p.GA, WB = p.WB, grp = p.grp;
  const double* __restrict__ Lx = p.Lov;
  const double* __restrict__ th_re = p.thv_re;
  const double* __restrict__ th_im = p.thv_im;
  double* __restrict__ ell_re = p.ell_re;
  double* __restrict__ ell_im = p.ell_im;
  double* __restrict__ ex_re = p.ex_re;
  double* __restrict__ ex_im = p.ex_im;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
          const int pl = rem & 1, j = rem >> 1;
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

  const int lr = lane & 15, lk = lane >> 4;
  d4_t acc[X_RT][CT];
#pragma unroll
  for (int i = 0; i < X_RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int nchunk = (M + kBK - 1) / kBK;
  // (the widest instance keeps the generic loop: the unconditional copy would
  // not fit its registers)
  // (column tiles TC..CT-1 of the stage hold zeros, so their MFMAs are wasted
  // but harmless; the occupancy model prices them in)
  const bool full = CT < 10 && mtv == X_RT;
  fetch(0);
  store(smem);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const double* S = smem + (ch & 1) * X_STAGE;
    if (ch + 1 < nchunk) fetch((ch + 1) * kBK);
    const double* As = S;
    const double* Bs = S + X_ROWS * kLDK;
    if (full) {
      // every wave holds X_RT row tiles: no per-MFMA conditions, so loads and
      // MFMAs interleave freely
#pragma unroll
      for (int kk = 0; kk < kBK; kk += 4) {
        double a[X_RT], b[CT];
#pragma unroll
        for (int i = 0; i < X_RT; ++i) a[i] = As[((rt0 + i) * 16 + lr) * kLDK + kk + lk];
#pragma unroll
        for (int j = 0; j < CT; ++j) b[j] = Bs[(j * 16 + lr) * kLDK + kk + lk];
#pragma unroll
        for (int i = 0; i < X_RT; ++i)
#pragma unroll
          for (int j = 0; j < CT; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
      }
    } else {
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
    }
    if (ch + 1 < nchunk) store(smem + ((ch + 1) & 1) * X_STAGE);
    __syncthreads();
  }

  // ---- epilogue: the rows of `grp` g-blocks at a time staged in LDS
  exchange_epilogue<double, CT * 16 + 2, 4>(
      acc, [&](int i, int e) { return (rt0 + i) * 16 + 4 * e + lk; }, mtv, N, ga, wb, g0, w0, G1,
      smem, grp, smem + X_LDS - X_RED, p.T0, p.lscale, ell_re, ell_im, ex_re, ex_im);
}

template <int CT>
__global__ __launch_bounds__(XT) void k_exchange(XSys p, int n_gt, int n_wt) {
  extern __shared__ double smem[];
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
  exchange_tile_run<CT>(p, gt, wt, smem);
}

// Many systems in one launch: block b runs tile tiles[b] = (system, gt, wt).
// The host orders the tiles by decreasing cost, so the hardware dispatcher,
// which hands out blocks in index order as compute units free up, packs the
// small systems' tiles around the large ones.
template <int CT>
__global__ __launch_bounds__(XT) void k_exchange_group(const XSys* __restrict__ sys,
                                                       const int4* __restrict__ tiles) {
  extern __shared__ double smem[];
  const int4 t = tiles[blockIdx.x];
  exchange_tile_run<CT>(sys[t.x], t.y, t.z, smem);
}

// Choose GA (g-blocks per tile) and WB (walkers per tile) for N: maximise
// the useful fraction of the MFMA work of the busiest wave.
// Column tiles of the kernel instance that serves TC.
int exchange_ct(int TC) { return TC <= 4 ? 4 : TC <= 7 ? 7 : TC <= 8 ? 8 : 10; }

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
      const double work = (double)XW * rpw * exchange_ct(TC) * 256.0;
      const double eff = useful / work + 1e-6 * ga * wb;
      if (eff > best) {
        best = eff;
        GA = ga;
        WB = wb;
      }
    }
}

}  // namespace

hipError_t exchange_setup(const SysDev& s, int W, const double* thv_re, const double* thv_im,
                          double* ell_re, double* ell_im, double* ex_re, double* ex_im, XSys* p,
                          int* n_gt, int* n_wt) {
  const int N = s.N, G1 = s.G + 1;
  if (2 * N > X_COLS) return hipErrorInvalidValue;
  int GA, WB;
  exchange_tile(N, GA, WB);
  if (s.x_ga > 0 && s.x_wb > 0) {   // tuned choice
    GA = s.x_ga;
    WB = s.x_wb;
  }
  if (GA * N > X_ROWS || WB * 2 * N > X_COLS || (GA * N + 15) / 16 > XW * X_RT) return hipErrorInvalidValue;
  // LDS: the epilogue stages the rows of grp g-blocks at a time (pitch
  // 16 CT + 2 doubles).
  const int TC = (WB * 2 * N + 15) / 16;
  const int ct = exchange_ct(TC);
  const int avail = X_LDS - X_RED;
  int grp = avail / (N * (16 * ct + 2));
  if (grp > 32) grp = 32;
  if (grp < 1) return hipErrorInvalidValue;
  *p = XSys{s.Lov, s.T0, thv_re, thv_im, ell_re, ell_im, ex_re, ex_im, G1, N, s.Kv, W, GA, WB,
            grp, ct, s.spin};
  *n_gt = (G1 + GA - 1) / GA;
  *n_wt = (W + WB - 1) / WB;
  return hipSuccess;
}

namespace {

template <int CT>
hipError_t allow_exchange_lds() {
  static bool ok = false;
  if (ok) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_exchange<CT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_exchange_group<CT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  ok = e == hipSuccess;
  return e;
}

template <int CT>
hipError_t run_exchange(const XSys& p, int n_gt, int n_wt, hipStream_t st) {
  hipError_t e = allow_exchange_lds<CT>();
  if (e != hipSuccess) return e;
  const int n_sg = (n_gt + X_SUPER_G - 1) / X_SUPER_G;
  const int n_sw = (n_wt + X_SUPER_W - 1) / X_SUPER_W;
  const int grid = ((n_sg * n_sw + 7) / 8) * 8 * X_SUPER_G * X_SUPER_W;
  hipLaunchKernelGGL(k_exchange<CT>, dim3(grid), dim3(XT), sizeof(double) * X_LDS, st, p,
                     n_gt, n_wt);
  return hipGetLastError();
}

template <int CT>
hipError_t run_exchange_group(const XSys* d_sys, const int4* d_tiles, int n_tiles, hipStream_t st) {
  hipError_t e = allow_exchange_lds<CT>();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_exchange_group<CT>, dim3(n_tiles), dim3(XT), sizeof(double) * X_LDS,
                     st, d_sys, d_tiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_project(const SysDev& s, int W, const double* th_re, const double* th_im,
                          double* thv_re, double* thv_im, hipStream_t st) {
  if (s.Kv == 0) return hipSuccess;
  // rows (w, j) of Theta (K = M) times the complement vectors
  const double* in[2] = {th_re, th_im};
  double* out[2] = {thv_re, thv_im};
  for (int pl = 0; pl < 2; ++pl) {
    GemmArgs g{};
    g.A = in[pl]; g.sAb = 0; g.sAr = s.M; g.sAk = 1; g.sAkb = 0;
    g.B = s.psiv; g.sBb = 0; g.sBc = s.M; g.sBk = 1; g.sBkb = 0;
    g.C = out[pl]; g.sCb = 0; g.sCr = s.Kv; g.sCc = 1;
    g.R = W * s.N; g.Cn = s.Kv; g.K = s.M; g.kin = s.M; g.batch = 1; g.alpha = 1.0; g.beta = 0.0;
    const hipError_t e = launch_gemm(g, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_exchange(SysDev& s, int W, const double* th_re, const double* th_im,
                           double* thv_re, double* thv_im, double* ell_re, double* ell_im,
                           double* ex_re, double* ex_im, hipStream_t st) {
  hipError_t e = launch_project(s, W, th_re, th_im, thv_re, thv_im, st);
  if (e != hipSuccess) return e;
  XSys p;
  int n_gt, n_wt;
  e = exchange_setup(s, W, thv_re, thv_im, ell_re, ell_im, ex_re, ex_im, &p, &n_gt, &n_wt);
  if (e != hipSuccess) return e;
  switch (p.ct) {
    case 4: return run_exchange<4>(p, n_gt, n_wt, st);
    case 7: return run_exchange<7>(p, n_gt, n_wt, st);
    case 8: return run_exchange<8>(p, n_gt, n_wt, st);
    default: return run_exchange<10>(p, n_gt, n_wt, st);
  }
}

void exchange_tile_order(int n_gt, int n_wt, std::vector<int2>& out) {
  // the single-system kernel's XCD super-tile order, invalid slots dropped
  const int n_sg = (n_gt + X_SUPER_G - 1) / X_SUPER_G;
  const int n_sw = (n_wt + X_SUPER_W - 1) / X_SUPER_W;
  const int per = X_SUPER_G * X_SUPER_W;
  const int grid = ((n_sg * n_sw + 7) / 8) * 8 * per;
  for (int id = 0; id < grid; ++id) {
    const int xcd = id & 7, slot = id >> 3;
    const int sidx = (slot / per) * 8 + xcd, local = slot % per;
    const int gt = (sidx / n_sw) * X_SUPER_G + local / X_SUPER_W;
    const int wt = (sidx % n_sw) * X_SUPER_W + local % X_SUPER_W;
    if (gt < n_gt && wt < n_wt) out.push_back(int2{gt, wt});
  }
}

hipError_t launch_exchange_group(int ct, const XSys* d_sys, const int4* d_tiles, int n_tiles,
                                 hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  switch (ct) {
    case 4: return run_exchange_group<4>(d_sys, d_tiles, n_tiles, st);
    case 7: return run_exchange_group<7>(d_sys, d_tiles, n_tiles, st);
    case 8: return run_exchange_group<8>(d_sys, d_tiles, n_tiles, st);
    case 10: return run_exchange_group<10>(d_sys, d_tiles, n_tiles, st);
    default: return hipErrorInvalidValue;
  }
}

// Tile shapes the model admits for N, best first (candidates of the tuner).
void exchange_candidates(int N, std::vector<int2>& out) {
  struct C { double eff; int ga, wb; };
  std::vector<C> cs;
  for (int ga = 1; ga * N <= X_ROWS; ++ga)
    for (int wb = 1; wb * 2 * N <= X_COLS; ++wb) {
      const int TR = (ga * N + 15) / 16, TC = (wb * 2 * N + 15) / 16;
      const int rpw = (TR + XW - 1) / XW;
      if (rpw > X_RT || TC > X_CTMAX) continue;
      const double useful = (double)ga * N * wb * 2 * N;
      const double work = (double)XW * rpw * exchange_ct(TC) * 256.0;
      cs.push_back(C{useful / work + 1e-6 * ga * wb, ga, wb});
    }
  std::sort(cs.begin(), cs.end(), [](const C& a, const C& b) { return a.eff > b.eff; });
  for (const C& c : cs) out.push_back(int2{c.ga, c.wb});
}

// ------------------------------------------------------------ Coulomb vector only
// ell_g^w = s tr T_g^w = s sum_(i,p) (Psi_T^T L_g)[i][p] Theta^w[p][i] (s the
// spin factor): one
// product [W x NM] x [NM x G] per plane, for the steps that do not measure the
// energy (the force bias needs ell every step; the exchange term only when the
// energy is measured).  K = NM is cut into S slices (batch entries writing
// partial sums), summed in slice order into ell.

namespace {

__global__ void k_sum_slices(const double* __restrict__ part, int S, int W, int G, int G1,
                             double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)W * G;
  if (e >= n) return;
  double v = 0.0;
  for (int q = 0; q < S; ++q) v += part[q * n + e];
  const int64_t w = e / G, g = e - w * G;
  out[w * G1 + g] = v;
}

}  // namespace

int coulomb_slices(int W, int G, int NM) {
  const int tiles = ((W + 127) / 128) * ((G + 127) / 128);
  int S = 1;
  while (S < 16 && tiles * S < 512 && NM % (2 * S) == 0 && NM / (2 * S) >= 256) S *= 2;
  return S;
}

hipError_t launch_coulomb(SysDev& s, const double* th_re, const double* th_im, double* part,
                          double* ell_re, double* ell_im, hipStream_t st) {
  const int W = s.W, G = s.G, G1 = G + 1;
  const int NM = s.N * s.M;
  const int S = coulomb_slices(W, G, NM);
  const int kc = NM / S;
  const double* planes[2] = {th_re, th_im};
  double* outs[2] = {ell_re, ell_im};
  for (int pl = 0; pl < 2; ++pl) {
    GemmArgs c{};
    c.A = planes[pl]; c.sAb = kc; c.sAr = NM; c.sAk = 1; c.sAkb = 0;
    c.B = s.Lx; c.sBb = kc; c.sBc = NM; c.sBk = 1; c.sBkb = 0;
    c.C = part; c.sCb = (int64_t)W * G; c.sCr = G; c.sCc = 1;
    c.R = W; c.Cn = G; c.K = kc; c.kin = kc; c.batch = S; c.alpha = s.spin; c.beta = 0.0;
    hipError_t e = launch_gemm(c, st);
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)W * G;
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, S,
                       W, G, G1, outs[pl]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}
