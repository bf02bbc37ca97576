// Mixed-precision forms of the dense contractions: BF16-split operands on
// the BF16 matrix cores with FP32 accumulation (see afq_device.h).  FP64
// stays for everything else: overlap, inverse, QR, weights and the energy
// sums.
//
//  * k_split: float64 planes -> P bfloat16 piece planes, rows padded to Kp.
//  * k_exchange_mx: the local-energy contraction of k_exchange.hip with the
//    virtual-space part of the T_g blocks formed from BF16-split
//    (Psi_T^T L_g Psi_perp) and Theta_v on top of T0_g; the N x N blocks are
//    reduced by the FP64 kernel's epilogue.
//  * k_split_lt / k_split_av / k_opbuild_mx: the operator build A^w =
//    sum_g a_g^w L_g from pieces of L (split once, transposed) and of the
//    field coefficients a (split per step), writing the operator's pieces.
//  * k_matvec_mx: the operator-orbital product A^w psi of the exponential
//    from those operator pieces, with the orbitals split while they are
//    staged.
#include "afq_device.h"
#include "afq_internal.h"

namespace {

// out[p][r][k] (bf16 bits), r < R, k < Kp: pieces of in[r * ld + k] (0 for k >= K).
__global__ void k_split(const double* __restrict__ in, int64_t R, int K, int64_t ld, int Kp, int P,
                        int64_t piece_stride, unsigned short* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= R * Kp) return;
  const int64_t r = e / Kp;
  const int k = (int)(e - r * Kp);
  double x = k < K ? in[r * ld + k] : 0.0;
  for (int p = 0; p < P; ++p) {
    const unsigned short b = bf16_bits_rn((float)x);
    out[p * piece_stride + e] = b;
    x -= (double)bf16_bits_to_f(b);
  }
}

// Theta planes [W][N][M] -> pieces of rows (w, j, plane) x Kp.
__global__ void k_split_theta(const double* __restrict__ re, const double* __restrict__ im, int W,
                              int N, int M, int Kp, int P, int64_t piece_stride,
                              unsigned short* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = (int64_t)W * 2 * N;
  if (e >= rows * Kp) return;
  const int64_t r = e / Kp;
  const int k = (int)(e - r * Kp);
  const int64_t w = r / (2 * N);
  const int rem = (int)(r - w * 2 * N);
  const int pl = rem & 1, j = rem >> 1;
  const double* src = pl ? im : re;
  double x = k < M ? src[(w * N + j) * M + k] : 0.0;
  for (int p = 0; p < P; ++p) {
    const unsigned short b = bf16_bits_rn((float)x);
    out[p * piece_stride + e] = b;
    x -= (double)bf16_bits_to_f(b);
  }
}

constexpr int MW = 8;                      // waves
constexpr int MT_ = MW * 64;               // threads
constexpr int M_RT = 2;                    // row tiles per wave
constexpr int M_ROWS = MW * M_RT * 16;     // 256
constexpr int M_KC = 32;                   // K per chunk (one MFMA k-step)
constexpr int M_PITCH = 40;                // bf16 per staged row (32 + 8 pad)
constexpr int M_SUPER_G = 4, M_SUPER_W = 8;
// Up to 13 column tiles (208 columns): two walkers per tile up to N = 52, so
// every row fragment loaded from HBM feeds both walkers' products.
constexpr int M_CTMAX = 13;
constexpr int M_JG = 4;                    // column tiles per MFMA group
inline int mx_ct(int TC) { return TC <= 4 ? 4 : TC <= 7 ? 7 : TC <= 10 ? 10 : 13; }

template <int P>
struct MxProds;
template <>
struct MxProds<2> {
  static constexpr int N = 3;
  static constexpr int a[3] = {0, 0, 1};
  static constexpr int b[3] = {0, 1, 0};
};
template <>
struct MxProds<3> {
  static constexpr int N = 6;
  static constexpr int a[6] = {0, 0, 1, 1, 0, 2};
  static constexpr int b[6] = {0, 1, 0, 1, 2, 0};
};

// Lb: P pieces of the (G+1) N x Kp blocks Psi_T^T L_g Psi_perp; tb: P
// pieces of Theta_v as rows (w, j, plane) x Kp; T0: the trial-space blocks
// the epilogue adds.
//
// Each wave owns its row tiles outright, so their fragments are loaded from
// global memory straight into registers (next chunk prefetched); only the
// column operand, which every wave reads, is staged in LDS (double buffer,
// register prefetch, one barrier per chunk).
template <int CT, int P>
__global__ __launch_bounds__(MT_) void k_exchange_mx(int G1, int N, int Kp, int W, int GA, int WB,
                                                     int n_gt, int n_wt, int grp, int red_off,
                                                     const unsigned short* __restrict__ Lb,
                                                     int64_t Lb_ps,
                                                     const unsigned short* __restrict__ tb,
                                                     int64_t tb_ps, double* __restrict__ ell_re,
                                                     double* __restrict__ ell_im,
                                                     double* __restrict__ ex_re,
                                                     double* __restrict__ ex_im,
                                                     const double* __restrict__ T0,
                                                     double lscale) {
  extern __shared__ double smem[];
  unsigned short* lds = (unsigned short*)smem;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int id = blockIdx.x;
  const int xcd = id & 7, slot = id >> 3;
  const int per = M_SUPER_G * M_SUPER_W;
  const int sidx = (slot / per) * 8 + xcd, local = slot % per;
  const int n_sw = (n_wt + M_SUPER_W - 1) / M_SUPER_W;
  const int gt = (sidx / n_sw) * M_SUPER_G + local / M_SUPER_W;
  const int wt = (sidx % n_sw) * M_SUPER_W + local % M_SUPER_W;
  if (gt >= n_gt || wt >= n_wt) return;
  const int g0 = gt * GA, w0 = wt * WB;
  const int ga = min(GA, G1 - g0), wb = min(WB, W - w0);
  const int nr = ga * N, twoN = 2 * N, nc = wb * twoN;
  const int TR = (nr + 15) >> 4, TC = (nc + 15) >> 4;
  const int rpw = (TR + MW - 1) / MW;
  const int rt0 = wave * rpw;
  const int mtv = max(0, min(rpw, TR - rt0));
  const int lr = lane & 15, lk = (lane >> 4) * 8;

  // ---- row operand: this lane's fragment rows, straight from global memory
  const int64_t a_row0 = (int64_t)g0 * N;
  bool arow_ok[M_RT];
  const unsigned short* aptr[M_RT];
#pragma unroll
  for (int i = 0; i < M_RT; ++i) {
    const int r = (rt0 + i) * 16 + lr;
    arow_ok[i] = (i < mtv) && (r < nr);
    aptr[i] = Lb + (a_row0 + (arow_ok[i] ? r : 0)) * Kp + lk;
  }
  uint4 afr[M_RT][P];
  auto fetch_a = [&](int k0, uint4 (&dst)[M_RT][P]) {
#pragma unroll
    for (int i = 0; i < M_RT; ++i)
#pragma unroll
      for (int p = 0; p < P; ++p)
        dst[i][p] = arow_ok[i] ? *(const uint4*)(aptr[i] + p * Lb_ps + k0) : make_uint4(0, 0, 0, 0);
  };

  // ---- column operand: staged in LDS, [stage][p][col][M_PITCH]
  constexpr int BROWS = CT * 16;
  constexpr int BSTAGE = P * BROWS * M_PITCH;      // bf16 per stage
  constexpr int UNITS = BROWS * P * (M_KC / 8);    // 16-byte units per chunk
  constexpr int PFU = (UNITS + MT_ - 1) / MT_;
  const int64_t b_row0 = (int64_t)w0 * twoN;
  uint4 pf[PFU];
  auto fetch_b = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PFU; ++i) {
      const int u = tid + i * MT_;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (u < UNITS) {
        // consecutive lanes walk k, then columns, within one piece plane
        // (lanes of one LDS store then hit distinct banks)
        const int k8 = u & 3, rp = u >> 2, p = rp / BROWS, c = rp - p * BROWS;
        if (c < nc) v = *(const uint4*)(tb + p * tb_ps + (b_row0 + c) * Kp + k0 + k8 * 8);
      }
      pf[i] = v;
    }
  };
  auto store_b = [&](unsigned short* S) {
#pragma unroll
    for (int i = 0; i < PFU; ++i) {
      const int u = tid + i * MT_;
      if (u < UNITS) {
        const int k8 = u & 3, rp = u >> 2, p = rp / BROWS, c = rp - p * BROWS;
        *(uint4*)(S + ((size_t)p * BROWS + c) * M_PITCH + k8 * 8) = pf[i];
      }
    }
  };

  f4_t acc[M_RT][CT];
#pragma unroll
  for (int i = 0; i < M_RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int nchunk = Kp / M_KC;
  const bool full = mtv == M_RT;   // column tiles TC..CT-1 of the stage are zeros
  fetch_a(0, afr);
  fetch_b(0);
  store_b(lds);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const unsigned short* Bs = lds + (ch & 1) * BSTAGE;
    uint4 anx[M_RT][P];
    const bool more = ch + 1 < nchunk;
    if (more) {
      fetch_a((ch + 1) * M_KC, anx);
      fetch_b((ch + 1) * M_KC);
    }
    if (full) {
      // all row tiles present: no per-MFMA conditions.  Column tiles go in
      // groups of M_JG with the piece product outermost, so consecutive
      // MFMAs feed M_RT * M_JG different accumulators.
#pragma unroll
      for (int j0 = 0; j0 < CT; j0 += M_JG) {
        bf8_t b[M_JG][P];
#pragma unroll
        for (int jj = 0; jj < M_JG; ++jj)
#pragma unroll
          for (int p = 0; p < P; ++p)
            if (j0 + jj < CT)
              b[jj][p] = *(const bf8_t*)(Bs + ((size_t)p * BROWS + (j0 + jj) * 16 + lr) * M_PITCH + lk);
#pragma unroll
        for (int q = 0; q < MxProds<P>::N; ++q)
#pragma unroll
          for (int jj = 0; jj < M_JG; ++jj)
#pragma unroll
            for (int i = 0; i < M_RT; ++i)
              if (j0 + jj < CT) {
                const uint4 av = afr[i][MxProds<P>::a[q]];
                acc[i][j0 + jj] =
                    mfma_bf16(*(const bf8_t*)&av, b[jj][MxProds<P>::b[q]], acc[i][j0 + jj]);
              }
      }
    } else {
#pragma unroll
      for (int j = 0; j < CT; ++j) {
        if (j >= TC) continue;
        bf8_t b[P];
#pragma unroll
        for (int p = 0; p < P; ++p)
          b[p] = *(const bf8_t*)(Bs + ((size_t)p * BROWS + j * 16 + lr) * M_PITCH + lk);
#pragma unroll
        for (int i = 0; i < M_RT; ++i) {
          if (i >= mtv) continue;
#pragma unroll
          for (int q = 0; q < MxProds<P>::N; ++q) {
            const uint4 av = afr[i][MxProds<P>::a[q]];
            acc[i][j] = mfma_bf16(*(const bf8_t*)&av, b[MxProds<P>::b[q]], acc[i][j]);
          }
        }
      }
    }
    if (more) {
      store_b(lds + ((ch + 1) & 1) * BSTAGE);
#pragma unroll
      for (int i = 0; i < M_RT; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p) afr[i][p] = anx[i][p];
    }
    __syncthreads();
  }

  // ---- epilogue (shared with the FP64 kernel), T staged in FP32 (its
  // precision)
  exchange_epilogue<float, CT * 16 + 2, 6>(
      acc, [&](int i, int e) { return (rt0 + i) * 16 + (lane >> 4) * 4 + e; }, mtv, N, ga, wb, g0,
      w0, G1, (float*)smem, grp, smem + red_off, T0, lscale, ell_re, ell_im, ex_re, ex_im);
}

void exchange_mx_tile(int N, int& GA, int& WB) {
  double best = -1.0;
  GA = 1;
  WB = 1;
  for (int ga = 1; ga * N <= M_ROWS; ++ga)
    for (int wb = 1; wb * 2 * N <= 16 * M_CTMAX; ++wb) {
      const int TR = (ga * N + 15) / 16, TC = (wb * 2 * N + 15) / 16;
      const int rpw = (TR + MW - 1) / MW;
      if (rpw > M_RT || TC > M_CTMAX) continue;
      const double useful = (double)ga * N * wb * 2 * N;
      const int ct = mx_ct(TC);   // width of the kernel instance
      const double work = (double)MW * rpw * ct * 256.0;
      const double eff = useful / work + 1e-6 * ga * wb;
      if (eff > best) {
        best = eff;
        GA = ga;
        WB = wb;
      }
    }
}

template <int CT, int P>
hipError_t launch_mx(SysDev& s, int W, const unsigned short* tb, int64_t tb_ps, double* ell_re,
                     double* ell_im, double* ex_re, double* ex_im, int GA, int WB, hipStream_t st) {
  const int N = s.N, G1 = s.G + 1;
  const int n_gt = (G1 + GA - 1) / GA, n_wt = (W + WB - 1) / WB;
  const int n_sg = (n_gt + M_SUPER_G - 1) / M_SUPER_G;
  const int n_sw = (n_wt + M_SUPER_W - 1) / M_SUPER_W;
  const int grid = ((n_sg * n_sw + 7) / 8) * 8 * M_SUPER_G * M_SUPER_W;
  // LDS: the whole 160 KB (one workgroup per compute unit): two B stages for
  // the main loop, then as many FP32 T blocks as fit for the epilogue, with
  // the partial sums at the end
  const int red_d = 4 * MW * 32;
  const size_t stage_doubles = ((size_t)2 * P * CT * 16 * M_PITCH * 2 + 7) / 8;
  const size_t lds_doubles = 160 * 1024 / 8;
  if (stage_doubles > lds_doubles - red_d) return hipErrorInvalidValue;
  // the epilogue stages the rows of grp g-blocks at a time (FP32, pitch
  // 16 CT + 2)
  int grp = (int)((lds_doubles - red_d) * 2 / ((size_t)N * (16 * CT + 2)));
  if (grp > 32) grp = 32;
  if (grp < 1) return hipErrorInvalidValue;
  const int red_off = (int)(lds_doubles - red_d);
  static bool lds_ok = false;
  if (!lds_ok) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_exchange_mx<CT, P>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  hipLaunchKernelGGL((k_exchange_mx<CT, P>), dim3(grid), dim3(MT_), lds_doubles * 8, st, G1, N,
                     s.Kp, W, GA, WB, n_gt, n_wt, grp, red_off, s.Lxb, s.Lxb_ps, tb, tb_ps, ell_re, ell_im,
                     ex_re, ex_im, s.T0, s.spin);
  return hipGetLastError();
}

// ---------------------------------------------------------------- operator build
// Ltb[p][pq][g] = piece p of L[g][pq] (0 for g >= G): 64 x 64 tiles
// transposed through LDS so that both the reads and the writes run along
// memory.
__global__ __launch_bounds__(256) void k_split_lt(const double* __restrict__ L, int G, int64_t MM,
                                                  int Gp, int64_t piece_stride,
                                                  unsigned short* __restrict__ out) {
  __shared__ double t[64][65];
  const int64_t pq0 = (int64_t)blockIdx.x * 64;
  const int g0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int g = g0 + r;
    const int64_t pq = pq0 + tx;
    t[r][tx] = (g < G && pq < MM) ? L[(int64_t)g * MM + pq] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t pq = pq0 + r;
    const int g = g0 + tx;
    if (pq < MM && g < Gp) {
      double x = t[tx][r];
      for (int p = 0; p < 3; ++p) {
        const unsigned short b = bf16_bits_rn((float)x);
        out[p * piece_stride + pq * Gp + g] = b;
        x -= (double)bf16_bits_to_f(b);
      }
    }
  }
}

// avb[p][r][g]: pieces of the field coefficients, rows r < W the real plane
// of walker r, rows W + w the imaginary plane; 0 for g >= G.
__global__ void k_split_av(const double* __restrict__ are, const double* __restrict__ aim, int W,
                           int G, int Gp, int P, int64_t piece_stride,
                           unsigned short* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)2 * W * Gp) return;
  const int r = (int)(e / Gp), g = (int)(e - (int64_t)r * Gp);
  double x = g < G ? (r < W ? are[(int64_t)r * G + g] : aim[(int64_t)(r - W) * G + g]) : 0.0;
  for (int p = 0; p < P; ++p) {
    const unsigned short b = bf16_bits_rn((float)x);
    out[p * piece_stride + e] = b;
    x -= (double)bf16_bits_to_f(b);
  }
}

// Tile: rows (plane, w) of the coefficients (256, loaded by each wave straight
// into registers) times 208 columns pq of L (staged in LDS), K = Gp.  The
// FP32 sums are the operator elements A_plane^w[p][q]; the epilogue splits
// each into P pieces at Ab[piece][w M + p][plane M + q], the layout of the
// operator-orbital product.  Tiles are dealt to the XCDs in contiguous
// ranges, row blocks fastest, so the row blocks of one column block share
// their L chunks in one L2.
constexpr int O_CT = 13;

template <int P>
__global__ __launch_bounds__(MT_) void k_opbuild_mx(int W, int M, int Gp, int Kq, int n_rb,
                                                    int n_tiles, int per_xcd,
                                                    const unsigned short* __restrict__ avb,
                                                    int64_t avb_ps,
                                                    const unsigned short* __restrict__ Ltb,
                                                    int64_t Ltb_ps, unsigned short* __restrict__ Ab,
                                                    int64_t Ab_ps) {
  extern __shared__ double smem[];
  unsigned short* lds = (unsigned short*)smem;
  constexpr int CT = O_CT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (tile >= n_tiles) return;
  const int cb = tile / n_rb, rb = tile - cb * n_rb;
  const int64_t MM = (int64_t)M * M;
  const int64_t pq0 = (int64_t)cb * CT * 16;
  const int R = 2 * W, r0 = rb * M_ROWS;
  const int nr = min(M_ROWS, R - r0);
  const int nc = (int)min((int64_t)CT * 16, MM - pq0);
  const int TR = (nr + 15) >> 4;
  const int rpw = (TR + MW - 1) / MW;
  const int rt0 = wave * rpw;
  const int mtv = max(0, min(rpw, TR - rt0));
  const int lr = lane & 15, lk = (lane >> 4) * 8;

  // ---- row operand: coefficient pieces straight from global memory
  bool arow_ok[M_RT];
  const unsigned short* aptr[M_RT];
#pragma unroll
  for (int i = 0; i < M_RT; ++i) {
    const int r = (rt0 + i) * 16 + lr;
    arow_ok[i] = (i < mtv) && (r < nr);
    aptr[i] = avb + (int64_t)(r0 + (arow_ok[i] ? r : 0)) * Gp + lk;
  }
  uint4 afr[M_RT][P];
  auto fetch_a = [&](int k0, uint4 (&dst)[M_RT][P]) {
#pragma unroll
    for (int i = 0; i < M_RT; ++i)
#pragma unroll
      for (int p = 0; p < P; ++p)
        dst[i][p] = arow_ok[i] ? *(const uint4*)(aptr[i] + p * avb_ps + k0) : make_uint4(0, 0, 0, 0);
  };

  // ---- column operand: L pieces, staged in LDS [stage][p][col][M_PITCH]
  constexpr int BROWS = CT * 16;
  constexpr int BSTAGE = P * BROWS * M_PITCH;
  constexpr int UNITS = BROWS * P * (M_KC / 8);
  constexpr int PFU = (UNITS + MT_ - 1) / MT_;
  uint4 pf[PFU];
  auto fetch_b = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PFU; ++i) {
      const int u = tid + i * MT_;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (u < UNITS) {
        const int k8 = u & 3, rp = u >> 2, p = rp / BROWS, c = rp - p * BROWS;
        if (c < nc) v = *(const uint4*)(Ltb + p * Ltb_ps + (pq0 + c) * Gp + k0 + k8 * 8);
      }
      pf[i] = v;
    }
  };
  auto store_b = [&](unsigned short* S) {
#pragma unroll
    for (int i = 0; i < PFU; ++i) {
      const int u = tid + i * MT_;
      if (u < UNITS) {
        const int k8 = u & 3, rp = u >> 2, p = rp / BROWS, c = rp - p * BROWS;
        *(uint4*)(S + ((size_t)p * BROWS + c) * M_PITCH + k8 * 8) = pf[i];
      }
    }
  };

  f4_t acc[M_RT][CT];
#pragma unroll
  for (int i = 0; i < M_RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  // invalid row fragments and columns beyond nc hold zeros
  const bool active = mtv > 0;
  const int nchunk = Gp / M_KC;
  fetch_a(0, afr);
  fetch_b(0);
  store_b(lds);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const unsigned short* Bs = lds + (ch & 1) * BSTAGE;
    uint4 anx[M_RT][P];
    const bool more = ch + 1 < nchunk;
    if (more) {
      fetch_a((ch + 1) * M_KC, anx);
      fetch_b((ch + 1) * M_KC);
    }
    if (active) {
#pragma unroll
      for (int j0 = 0; j0 < CT; j0 += M_JG) {
        bf8_t b[M_JG][P];
#pragma unroll
        for (int jj = 0; jj < M_JG; ++jj)
#pragma unroll
          for (int p = 0; p < P; ++p)
            if (j0 + jj < CT)
              b[jj][p] = *(const bf8_t*)(Bs + ((size_t)p * BROWS + (j0 + jj) * 16 + lr) * M_PITCH + lk);
#pragma unroll
        for (int q = 0; q < MxProds<P>::N; ++q)
#pragma unroll
          for (int jj = 0; jj < M_JG; ++jj)
#pragma unroll
            for (int i = 0; i < M_RT; ++i)
              if (j0 + jj < CT) {
                const uint4 av = afr[i][MxProds<P>::a[q]];
                acc[i][j0 + jj] =
                    mfma_bf16(*(const bf8_t*)&av, b[jj][MxProds<P>::b[q]], acc[i][j0 + jj]);
              }
      }
    }
    if (more) {
      store_b(lds + ((ch + 1) & 1) * BSTAGE);
#pragma unroll
      for (int i = 0; i < M_RT; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p) afr[i][p] = anx[i][p];
    }
    __syncthreads();
  }

  // ---- epilogue: element e of tile (i, j) is row 4 (lane / 16) + e, column
  // lane % 16; each value goes out as its P pieces
#pragma unroll
  for (int i = 0; i < M_RT; ++i) {
    if (i >= mtv) continue;
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int c = j * 16 + lr;
      if (c >= nc) continue;
      const int64_t pq = pq0 + c;
      const int pr = (int)(pq / M), qc = (int)(pq - (int64_t)pr * M);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = (rt0 + i) * 16 + (lane >> 4) * 4 + e;
        if (r >= nr) continue;
        const int rg = r0 + r;
        const bool im = rg >= W;
        const int w = im ? rg - W : rg;
        const int64_t off = ((int64_t)w * M + pr) * Kq + (im ? M : 0) + qc;
        float x = acc[i][j][e];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const unsigned short b = bf16_bits_rn(x);
          Ab[p * Ab_ps + off] = b;
          x -= bf16_bits_to_f(b);
        }
      }
    }
  }
}

template <int P>
hipError_t launch_opb_mx(SysDev& s, hipStream_t st) {
  const int n_rb = (2 * s.W + M_ROWS - 1) / M_ROWS;
  const int64_t MM = (int64_t)s.M * s.M;
  const int64_t n_cb = (MM + O_CT * 16 - 1) / (O_CT * 16);
  const int64_t n_tiles = n_cb * n_rb;
  if (n_tiles > (1 << 28)) return hipErrorInvalidValue;
  const int per_xcd = (int)((n_tiles + 7) / 8);
  const size_t lds = (size_t)2 * P * O_CT * 16 * M_PITCH * 2;
  static bool lds_ok = false;
  if (!lds_ok) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_opbuild_mx<P>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  hipLaunchKernelGGL(k_opbuild_mx<P>, dim3(per_xcd * 8), dim3(MT_), lds, st, s.W, s.M, s.Gp, s.Kq,
                     n_rb, (int)n_tiles, per_xcd, s.avb, s.avb_ps, s.Ltb, s.Ltb_ps, s.Ab, s.Ab_ps);
  return hipGetLastError();
}

// ---------------------------------------------------------------- A^w psi
// For walker w: out[j][p] = sum_q A^w[p][q] v[j][q] (complex) as one real
// product of K = 2M: rows p of [A_re | A_im] (the pre-split operator, loaded
// by each wave straight into registers) times columns (plane, j) of the real
// form of the orbitals, [v_re | -v_im] and [v_im | v_re], which are split
// while they are staged in LDS.  One workgroup per walker and block of up to
// 8 RT row tiles; all 2N columns in one tile (CT >= ceil(2N / 16)).
constexpr int V_JG = 2;                    // column tiles per MFMA group

template <int CT, int P, int RT>
__global__ __launch_bounds__(MT_) void k_matvec_mx(int W, int N, int M, int Kq, int nrb,
                                                   const unsigned short* __restrict__ Ab,
                                                   int64_t Ab_ps, VecRef v, VecOut o, int mode,
                                                   double inv_n, VecOut sum) {
  extern __shared__ double smem[];
  unsigned short* lds = (unsigned short*)smem;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int w = blockIdx.x / nrb, rb = blockIdx.x - w * nrb;
  if (w >= W) return;
  const int TR_all = (M + 15) >> 4;
  const int tpb = (TR_all + nrb - 1) / nrb;
  const int tr0 = rb * tpb;
  const int TR = min(tpb, TR_all - tr0);
  if (TR <= 0) return;
  const int row0 = tr0 * 16;
  const int nr = min(TR * 16, M - row0), nc = 2 * N;
  const int rpw = (TR + MW - 1) / MW;
  const int rt0 = wave * rpw;
  const int mtv = max(0, min(rpw, TR - rt0));
  const int lr = lane & 15, lk = (lane >> 4) * 8;

  // ---- row operand: this lane's operator rows, straight from global memory
  const unsigned short* Aw = Ab + ((int64_t)w * M + row0) * Kq;
  bool arow_ok[RT];
  const unsigned short* aptr[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    const int r = (rt0 + i) * 16 + lr;
    arow_ok[i] = (i < mtv) && (r < nr);
    aptr[i] = Aw + (int64_t)(arow_ok[i] ? r : 0) * Kq + lk;
  }
  uint4 afr[RT][P];
  auto fetch_a = [&](int k0, uint4 (&dst)[RT][P]) {
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int p = 0; p < P; ++p)
        dst[i][p] = arow_ok[i] ? *(const uint4*)(aptr[i] + p * Ab_ps + k0) : make_uint4(0, 0, 0, 0);
  };

  // ---- column operand: float64 orbitals, split into the LDS stage
  // [stage][p][col][M_PITCH] in units of four k (eight units per column)
  constexpr int BROWS = CT * 16;
  constexpr int BSTAGE = P * BROWS * M_PITCH;
  constexpr int UNITS = BROWS * (M_KC / 4);
  constexpr int PFU = (UNITS + MT_ - 1) / MT_;
  const double* vre = v.re + (int64_t)w * v.sw;
  const double* vim = v.im + (int64_t)w * v.sw;
  auto vget = [&](int c, int k) -> double {
    const bool im_row = c >= N;
    const int j = im_row ? c - N : c;
    if (k < M) return im_row ? vim[j * v.sj + k] : vre[j * v.sj + k];
    const int q = k - M;
    if (q >= M) return 0.0;
    // -v_im of the real rows: the sign is applied in store_b, so that no
    // prefetch is waited for before the chunk's MFMAs
    return im_row ? vre[j * v.sj + q] : vim[j * v.sj + q];
  };
  double pf[PFU][4];
  auto fetch_b = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PFU; ++i) {
      const int u = tid + i * MT_;
      const int c = u >> 3, k = k0 + (u & 7) * 4;
#pragma unroll
      for (int t = 0; t < 4; ++t) pf[i][t] = (u < UNITS && c < nc) ? vget(c, k + t) : 0.0;
    }
  };
  auto store_b = [&](unsigned short* S, int k0) {
#pragma unroll
    for (int i = 0; i < PFU; ++i) {
      const int u = tid + i * MT_;
      if (u < UNITS) {
        const int c = u >> 3, k = (u & 7) * 4;
        double x[4] = {pf[i][0], pf[i][1], pf[i][2], pf[i][3]};
        if (c < N) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (k0 + k + t >= M) x[t] = -x[t];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
          unsigned short b[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            b[t] = bf16_bits_rn((float)x[t]);
            x[t] -= (double)bf16_bits_to_f(b[t]);
          }
          uint2 q;
          q.x = (unsigned)b[0] | ((unsigned)b[1] << 16);
          q.y = (unsigned)b[2] | ((unsigned)b[3] << 16);
          *(uint2*)(S + ((size_t)p * BROWS + c) * M_PITCH + k) = q;
        }
      }
    }
  };

  f4_t acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  // invalid row fragments and the columns beyond 2N hold zeros, so a wave
  // with any valid row tile runs the loop without per-MFMA conditions
  const bool active = mtv > 0;
  const int nchunk = Kq / M_KC;
  fetch_a(0, afr);
  fetch_b(0);
  store_b(lds, 0);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const unsigned short* Bs = lds + (ch & 1) * BSTAGE;
    uint4 anx[RT][P];
    const bool more = ch + 1 < nchunk;
    if (more) {
      fetch_a((ch + 1) * M_KC, anx);
      fetch_b((ch + 1) * M_KC);
    }
    if (active) {
#pragma unroll
      for (int j0 = 0; j0 < CT; j0 += V_JG) {
        bf8_t b[V_JG][P];
#pragma unroll
        for (int jj = 0; jj < V_JG; ++jj)
#pragma unroll
          for (int p = 0; p < P; ++p)
            if (j0 + jj < CT)
              b[jj][p] = *(const bf8_t*)(Bs + ((size_t)p * BROWS + (j0 + jj) * 16 + lr) * M_PITCH + lk);
#pragma unroll
        for (int q = 0; q < MxProds<P>::N; ++q)
#pragma unroll
          for (int jj = 0; jj < V_JG; ++jj)
#pragma unroll
            for (int i = 0; i < RT; ++i)
              if (j0 + jj < CT) {
                const uint4 av = afr[i][MxProds<P>::a[q]];
                acc[i][j0 + jj] =
                    mfma_bf16(*(const bf8_t*)&av, b[jj][MxProds<P>::b[q]], acc[i][j0 + jj]);
              }
      }
    }
    if (more) {
      store_b(lds + ((ch + 1) & 1) * BSTAGE, (ch + 1) * M_KC);
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p) afr[i][p] = anx[i][p];
    }
    __syncthreads();
  }

  // ---- epilogue: element e of tile (i, j) is operator row 4 (lane / 16) + e,
  // column lane % 16 of the tile
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    if (i >= mtv) continue;
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int c = j * 16 + lr;
      if (c >= nc) continue;
      const bool im_row = c >= N;
      const int jo = im_row ? c - N : c;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = (rt0 + i) * 16 + (lane >> 4) * 4 + e;
        if (r >= nr) continue;
        double val = (double)acc[i][j][e];
        const int64_t pcol = row0 + r;
        const int64_t off = (int64_t)w * o.sw + (int64_t)jo * o.sj + pcol;
        // modes as in the FP64 product (k_matvec)
        if (mode == 3) val = 2.0 * val - (im_row ? o.im[off] : o.re[off]);
        if (mode >= 1) {
          const double add = mode == 1 ? (val *= inv_n) : inv_n * val;
          const int64_t soff = (int64_t)w * sum.sw + (int64_t)jo * sum.sj + pcol;
          if (im_row) sum.im[soff] += add;
          else sum.re[soff] += add;
        }
        if (im_row) o.im[off] = val;
        else o.re[off] = val;
      }
    }
  }
}

template <int CT, int P>
hipError_t launch_mv_mx(SysDev& s, VecRef v, VecOut o, int mode, double inv_n, VecOut sum,
                        hipStream_t st) {
  constexpr int RT = CT <= 7 ? 3 : 2;   // registers: accumulators + fragments
  const int TR_all = (s.M + 15) / 16;
  const int nrb = (TR_all + MW * RT - 1) / (MW * RT);
  const size_t lds = (size_t)2 * P * CT * 16 * M_PITCH * 2;
  static bool lds_ok = false;
  if (!lds_ok) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_matvec_mx<CT, P, RT>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    lds_ok = true;
  }
  hipLaunchKernelGGL((k_matvec_mx<CT, P, RT>), dim3(s.W * nrb), dim3(MT_), lds, st, s.W, s.N, s.M,
                     s.Kq, nrb, s.Ab, s.Ab_ps, v, o, mode, inv_n, sum);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_split(const double* in, int64_t R, int K, int64_t ld, int Kp, int P,
                        int64_t piece_stride, unsigned short* out, hipStream_t st) {
  const int64_t n = R * Kp;
  hipLaunchKernelGGL(k_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, R, K, ld, Kp,
                     P, piece_stride, out);
  return hipGetLastError();
}

hipError_t launch_split_theta(const double* re, const double* im, int W, int N, int M, int Kp,
                              int P, int64_t piece_stride, unsigned short* out, hipStream_t st) {
  const int64_t n = (int64_t)W * 2 * N * Kp;
  hipLaunchKernelGGL(k_split_theta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, re, im, W,
                     N, M, Kp, P, piece_stride, out);
  return hipGetLastError();
}

hipError_t launch_exchange_mx(SysDev& s, int W, const unsigned short* tb, int64_t tb_ps,
                              double* ell_re, double* ell_im, double* ex_re, double* ex_im,
                              hipStream_t st) {
  if (2 * s.N > 160 || !s.Lxb) return hipErrorInvalidValue;
  int GA, WB;
  exchange_mx_tile(s.N, GA, WB);
  const int TC = (WB * 2 * s.N + 15) / 16;
  if (s.mx_pieces == 3) {
    if (TC <= 4) return launch_mx<4, 3>(s, W, tb, tb_ps, ell_re, ell_im, ex_re, ex_im, GA, WB, st);
    if (TC <= 7) return launch_mx<7, 3>(s, W, tb, tb_ps, ell_re, ell_im, ex_re, ex_im, GA, WB, st);
    if (TC <= 10) return launch_mx<10, 3>(s, W, tb, tb_ps, ell_re, ell_im, ex_re, ex_im, GA, WB, st);
    return launch_mx<13, 3>(s, W, tb, tb_ps, ell_re, ell_im, ex_re, ex_im, GA, WB, st);
  }
  if (TC <= 4) return launch_mx<4, 2>(s, W, tb, tb_ps, ell_re, ell_im, ex_re, ex_im, GA, WB, st);
  if (TC <= 7) return launch_mx<7, 2>(s, W, tb, tb_ps, ell_re, ell_im, ex_re, ex_im, GA, WB, st);
  if (TC <= 10) return launch_mx<10, 2>(s, W, tb, tb_ps, ell_re, ell_im, ex_re, ex_im, GA, WB, st);
  return launch_mx<13, 2>(s, W, tb, tb_ps, ell_re, ell_im, ex_re, ex_im, GA, WB, st);
}

hipError_t launch_split_lt(SysDev& s, hipStream_t st) {
  if (!s.Ltb || s.Gp < s.G || s.Gp % 32) return hipErrorInvalidValue;
  const int64_t MM = (int64_t)s.M * s.M;
  const dim3 grid((unsigned)((MM + 63) / 64), (unsigned)((s.Gp + 63) / 64));
  hipLaunchKernelGGL(k_split_lt, grid, dim3(256), 0, st, s.L, s.G, MM, s.Gp, s.Ltb_ps, s.Ltb);
  return hipGetLastError();
}

hipError_t launch_opbuild_mx(SysDev& s, hipStream_t st) {
  if (!s.Ab || !s.avb || !s.Ltb || s.op_pieces < 2 || s.op_pieces > 3) return hipErrorInvalidValue;
  const int64_t n = (int64_t)2 * s.W * s.Gp;
  hipLaunchKernelGGL(k_split_av, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s.av_re,
                     s.av_im, s.W, s.G, s.Gp, s.op_pieces, s.avb_ps, s.avb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return s.op_pieces == 3 ? launch_opb_mx<3>(s, st) : launch_opb_mx<2>(s, st);
}

hipError_t launch_matvec_mx(SysDev& s, VecRef v, VecOut o, int mode, double inv_n, VecOut sum,
                            hipStream_t st) {
  if (!s.Ab || 2 * s.N > 160) return hipErrorInvalidValue;
  const int TC = (2 * s.N + 15) / 16;
  if (s.op_pieces == 3) {
    if (TC <= 4) return launch_mv_mx<4, 3>(s, v, o, mode, inv_n, sum, st);
    if (TC <= 7) return launch_mv_mx<7, 3>(s, v, o, mode, inv_n, sum, st);
    return launch_mv_mx<10, 3>(s, v, o, mode, inv_n, sum, st);
  }
  if (s.op_pieces == 2) {
    if (TC <= 4) return launch_mv_mx<4, 2>(s, v, o, mode, inv_n, sum, st);
    if (TC <= 7) return launch_mv_mx<7, 2>(s, v, o, mode, inv_n, sum, st);
    return launch_mv_mx<10, 2>(s, v, o, mode, inv_n, sum, st);
  }
  return hipErrorInvalidValue;
}
