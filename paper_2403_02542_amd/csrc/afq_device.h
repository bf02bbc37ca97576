// Device-side building blocks shared by the walker-step kernels (gfx950).
//
//  * complex helpers on (re, im) double pairs,
//  * wavefront (64-lane) and workgroup reductions in a fixed order, so every
//    run of a kernel gives bitwise the same sums,
//  * an LDS-staged tile engine around the FP64 matrix-core instruction
//    v_mfma_f64_16x16x4f64.  Operand layout of that instruction on gfx950
//    (measured): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
//    accumulator element i of lane l is C[4 i + l / 16][l % 16].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define AFQ_DEV __device__ __forceinline__

typedef double d4_t __attribute__((ext_vector_type(4)));

struct cplx {
  double re, im;
};

AFQ_DEV cplx cmake(double r, double i) { return cplx{r, i}; }
AFQ_DEV cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
AFQ_DEV cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
AFQ_DEV cplx cmul(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
AFQ_DEV cplx cmulc(cplx a, cplx b) {
  return cplx{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
AFQ_DEV cplx cscale(cplx a, double s) { return cplx{a.re * s, a.im * s}; }
AFQ_DEV double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
AFQ_DEV cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return cplx{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    double r = b.re / b.im, d = b.re * r + b.im;
    return cplx{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}
AFQ_DEV cplx clog(cplx a) { return cplx{0.5 * log(cabs2(a)), atan2(a.im, a.re)}; }

// ---------------------------------------------------------------- reductions

// Wave sum on the VALU's data-parallel lane moves (no LDS): pairs, quads,
// half rows and rows of 16 lanes by quad permutations and mirrors, then rows
// 0+1 and 2+3 by the broadcast of lane 15 into the next row, and the total
// by the broadcast of lane 31 into rows 2 and 3; lane 63 holds it and every
// lane gets it back.  The order of the additions is fixed.
template <int CTRL, int ROWS>
AFQ_DEV double dpp_move(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xf, false);
  return __hiloint2double(h2, l2);
}
AFQ_DEV double wave_sum(double v) {   // every lane of the wave must be active
  v += dpp_move<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_move<0x140, 0xf>(v);   // row_mirror
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
// wave_sum of K values at once, every step taken for all values before the
// next (independent DPP chains interleave instead of queueing behind one
// another); the same additions in the same order as wave_sum.  The sums are
// complete in lane 63 only.
template <int K>
AFQ_DEV void wave_sum_n(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_move<0xB1, 0xf>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_move<0x4E, 0xf>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_move<0x141, 0xf>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_move<0x140, 0xf>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_move<0x142, 0xa>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_move<0x143, 0xc>(v[k]);
}
// Value of lane l (a compile-time constant after unrolling) in every lane,
// through the scalar registers.
AFQ_DEV double lane_bcast(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
AFQ_DEV double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the workgroup; every thread gets the result.  `red` holds at
// least blockDim.x / 64 doubles of LDS.  Fixed order: waves, then slots.
AFQ_DEV double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- MFMA tiles

AFQ_DEV d4_t mfma_f64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Tile engine: a 256-thread workgroup computes C[r][c] = sum_k A[r][k] B[c][k]
// for r < 32 MT, c < 32 NT.  The four waves form a 2 x 2 grid over the 16 x 16
// MFMA tiles (see wave_split); each wave holds at most MT x NT of them.
// K is consumed in chunks of BK = 16 staged in LDS as As[r][k], Bs[c][k] with
// a row pitch of 17 doubles (conflict-free fragment reads).
constexpr int kBK = 16;
constexpr int kLDK = kBK + 1;

template <int MT, int NT>
struct TileAcc {
  d4_t c[MT][NT];
  AFQ_DEV void zero() {
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) c[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
  }
};

template <int MT, int NT>
struct TileShape {
  static constexpr int ROWS = 32 * MT;
  static constexpr int COLS = 32 * NT;
  static constexpr int LDS_DOUBLES = (ROWS + COLS) * kLDK;
};

// Work split of a tile among the four waves (2 x 2 grid): the TR valid row
// tiles are divided as evenly as possible between the two wave rows, and the
// TC valid column tiles between the two wave columns.
struct WaveSplit {
  int rt0, mtv, ct0, ntv;
};
template <int MT, int NT>
AFQ_DEV WaveSplit wave_split(int nrows, int ncols) {
  const int wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int TR = (nrows + 15) >> 4, TC = (ncols + 15) >> 4;
  const int hr = (TR + 1) >> 1, hc = (TC + 1) >> 1;
  WaveSplit s;
  s.rt0 = wr * hr;
  s.mtv = min(MT, max(0, min(hr, TR - s.rt0)));
  s.ct0 = wc * hc;
  s.ntv = min(NT, max(0, min(hc, TC - s.ct0)));
  return s;
}

// One BK chunk of MFMAs from LDS.
template <int MT, int NT>
AFQ_DEV void tile_mma_chunk(const double* As, const double* Bs, TileAcc<MT, NT>& acc,
                            const WaveSplit& ws) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < kBK; kk += 4) {
    double a[MT], b[NT];
#pragma unroll
    for (int i = 0; i < MT; ++i) a[i] = As[((ws.rt0 + i) * 16 + lr) * kLDK + kk + lk];
#pragma unroll
    for (int j = 0; j < NT; ++j) b[j] = Bs[((ws.ct0 + j) * 16 + lr) * kLDK + kk + lk];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      if (i < ws.mtv) {
#pragma unroll
        for (int j = 0; j < NT; ++j)
          if (j < ws.ntv) acc.c[i][j] = mfma_f64(a[i], b[j], acc.c[i][j]);
      }
    }
  }
}

// Row / column (within the tile) of accumulator element e of tile (i, j).
AFQ_DEV int acc_row(const WaveSplit& ws, int i, int e) {
  return (ws.rt0 + i) * 16 + 4 * e + ((threadIdx.x & 63) >> 4);
}
AFQ_DEV int acc_col(const WaveSplit& ws, int j) {
  return (ws.ct0 + j) * 16 + (threadIdx.x & 15);
}

// Full K loop.  fillA(k0, As) / fillB(k0, Bs) stage one chunk (zero beyond
// the valid ranges); both are called by all threads.  Requires
// ceil(nrows / 16) <= 2 MT and ceil(ncols / 16) <= 2 NT.
template <int MT, int NT, class FillA, class FillB>
AFQ_DEV void tile_gemm(int K, const WaveSplit& ws, FillA fillA, FillB fillB, double* As,
                       double* Bs, TileAcc<MT, NT>& acc) {
  for (int k0 = 0; k0 < K; k0 += kBK) {
    __syncthreads();
    fillA(k0, As);
    fillB(k0, Bs);
    __syncthreads();
    tile_mma_chunk<MT, NT>(As, Bs, acc, ws);
  }
}

// Staging helper: element (r, k) of a tile with ROWS rows from a functor
// get(r, k) (only called for r < nvalid, k < K); zero elsewhere.  Consecutive
// threads take consecutive k (operands stored with k contiguous).
template <int ROWS, class Get>
AFQ_DEV void stage_rows(double* S, int k0, int K, int nvalid, Get get) {
  for (int e = threadIdx.x; e < ROWS * kBK; e += blockDim.x) {
    const int r = e >> 4, k = e & 15;
    double v = 0.0;
    if (r < nvalid && k0 + k < K) v = get(r, k0 + k);
    S[r * kLDK + k] = v;
  }
}
// Same, but consecutive threads take consecutive r (operands stored with r
// contiguous, k outer).
template <int ROWS, class Get>
AFQ_DEV void stage_rows_kmajor(double* S, int k0, int K, int nvalid, Get get) {
  for (int e = threadIdx.x; e < ROWS * kBK; e += blockDim.x) {
    const int k = e / ROWS, r = e - k * ROWS;
    double v = 0.0;
    if (r < nvalid && k0 + k < K) v = get(r, k0 + k);
    S[r * kLDK + k] = v;
  }
}

// ---------------------------------------------------------------- pipelined engine
// Workgroup of WR x WC waves computing C[r][c] = sum_k A(r, k) B(c, k) for
// r < WR*RT*16, c < WC*CT*16.  The TR valid row tiles are split evenly over
// the WR wave rows (at most RT each) and the TC valid column tiles over the
// WC wave columns (at most CT each).  K runs in chunks of BK through two LDS
// stages: chunk c+1 is fetched from global memory into registers while the
// MFMAs of chunk c run, then stored into the other stage (one barrier per
// chunk).  A_KM / B_KM: the operand is stored k-major (consecutive r
// contiguous); consecutive threads then walk r instead of k.  The getters
// should return plain loads: arithmetic on a loaded value makes the compiler
// wait for that prefetch before the chunk's MFMAs are issued.

template <int WR, int WC, int RT, int CT, int BK = 16>
struct Pipe {
  static constexpr int NW = WR * WC;
  static constexpr int NT = NW * 64;
  static constexpr int ROWS = WR * RT * 16;
  static constexpr int COLS = WC * CT * 16;
  static constexpr int LDK = BK + 1;
  static constexpr int STAGE = (ROWS + COLS) * LDK;   // doubles per stage
  static constexpr int TOT = (ROWS + COLS) * BK;
  static constexpr int PF = (TOT + NT - 1) / NT;
  static constexpr size_t LDS_BYTES = 2 * STAGE * sizeof(double);
};

struct PipeSplit {
  int rt0, mtv, ct0, ntv;
};

template <int WR, int WC, int RT, int CT, bool A_KM, bool B_KM, int BK = 16, class GA, class GB>
AFQ_DEV PipeSplit pipe_gemm(int K, int nr, int nc, GA ga, GB gb, double* smem,
                            d4_t (&acc)[RT][CT]) {
  using P = Pipe<WR, WC, RT, CT, BK>;
  constexpr int LDK = P::LDK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int TR = (nr + 15) >> 4, TC = (nc + 15) >> 4;
  const int rpw = (TR + WR - 1) / WR, cpw = (TC + WC - 1) / WC;
  PipeSplit sp;
  sp.rt0 = wr * rpw;
  sp.mtv = max(0, min(min(rpw, RT), TR - sp.rt0));
  sp.ct0 = wc * cpw;
  sp.ntv = max(0, min(min(cpw, CT), TC - sp.ct0));
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
  double pf[P::PF];
  auto slot = [&](int e, int& row, int& k) {   // staging element -> (stage row, k)
    if (e < P::ROWS * BK) {
      if (A_KM) {
        k = e / P::ROWS;
        row = e - k * P::ROWS;
      } else {
        row = e / BK;
        k = e - row * BK;
      }
    } else {
      const int e2 = e - P::ROWS * BK;
      int c;
      if (B_KM) {
        k = e2 / P::COLS;
        c = e2 - k * P::COLS;
      } else {
        c = e2 / BK;
        k = e2 - c * BK;
      }
      row = P::ROWS + c;
    }
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < P::PF; ++i) {
      const int e = tid + i * P::NT;
      double v = 0.0;
      if (e < P::TOT) {
        int row, k;
        slot(e, row, k);
        const int kg = k0 + k;
        if (kg < K) {
          if (row < P::ROWS) {
            if (row < nr) v = ga(row, kg);
          } else if (row - P::ROWS < nc) {
            v = gb(row - P::ROWS, kg);
          }
        }
      }
      pf[i] = v;
    }
  };
  auto store = [&](double* S) {
#pragma unroll
    for (int i = 0; i < P::PF; ++i) {
      const int e = tid + i * P::NT;
      if (e < P::TOT) {
        int row, k;
        slot(e, row, k);
        S[row * LDK + k] = pf[i];
      }
    }
  };
  const int nchunk = (K + BK - 1) / BK;
  const int lr = lane & 15, lk = lane >> 4;
  // tiles beyond the valid ones hold zeros in the stage, so a wave with any
  // valid tile runs the condition-free loop over all RT x CT (the extra
  // products are discarded by the caller's bounds)
  const bool full = sp.mtv > 0 && sp.ntv > 0;
  fetch(0);
  store(smem);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const double* As = smem + (ch & 1) * P::STAGE;
    const double* Bs = As + P::ROWS * LDK;
    if (ch + 1 < nchunk) fetch((ch + 1) * BK);
    if (full) {
      // no per-MFMA conditions
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double a[RT], b[CT];
#pragma unroll
        for (int i = 0; i < RT; ++i) a[i] = As[((sp.rt0 + i) * 16 + lr) * LDK + kk + lk];
#pragma unroll
        for (int j = 0; j < CT; ++j) b[j] = Bs[((sp.ct0 + j) * 16 + lr) * LDK + kk + lk];
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < CT; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double a[RT], b[CT];
#pragma unroll
        for (int i = 0; i < RT; ++i)
          a[i] = i < sp.mtv ? As[((sp.rt0 + i) * 16 + lr) * LDK + kk + lk] : 0.0;
#pragma unroll
        for (int j = 0; j < CT; ++j)
          b[j] = j < sp.ntv ? Bs[((sp.ct0 + j) * 16 + lr) * LDK + kk + lk] : 0.0;
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          if (i < sp.mtv) {
#pragma unroll
            for (int j = 0; j < CT; ++j)
              if (j < sp.ntv) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
          }
        }
      }
    }
    if (ch + 1 < nchunk) store(smem + ((ch + 1) & 1) * P::STAGE);
    __syncthreads();
  }
  return sp;
}

// Row / column (within the tile) of accumulator element e of tile (i, j).
AFQ_DEV int pipe_row(const PipeSplit& sp, int i, int e) {
  return (sp.rt0 + i) * 16 + 4 * e + ((threadIdx.x & 63) >> 4);
}
AFQ_DEV int pipe_col(const PipeSplit& sp, int j) { return (sp.ct0 + j) * 16 + (threadIdx.x & 15); }

// ---------------------------------------------------------------- BF16 split
// A float64 value x is carried as P bfloat16 pieces x = x0 + x1 (+ x2) + r,
// x_{i+1} = bf16(x - x0 - ... - x_i) (round to nearest even); two pieces keep
// 16 significand bits, three keep 24.  Products a b are formed from the
// piece products that matter at that precision (3 for two pieces: a0b0,
// a0b1, a1b0; 6 for three: + a1b1, a0b2, a2b0) on the BF16 matrix cores,
// accumulated in FP32.
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

AFQ_DEV unsigned short bf16_bits_rn(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
AFQ_DEV float bf16_bits_to_f(unsigned short b) { return __uint_as_float((unsigned int)b << 16); }

// v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) .. +7] and
// B[8 (l / 16) .. +7][l % 16]; accumulator element i of lane l is
// C[4 (l / 16) + i][l % 16].
AFQ_DEV f4_t mfma_bf16(const bf8_t& a, const bf8_t& b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- BF16-split pipelined engine
// The FP64 engine's contract (C[r][c] = sum_k A(r, k) B(c, k), float64
// getters) on the BF16 matrix cores: operands are read as float64, split into
// P bfloat16 pieces while they are staged in LDS ([piece][row][k], pitch 40),
// and the piece products (3 for P = 2, 6 for P = 3) accumulate in FP32.  K
// runs in chunks of 32 (one MFMA k-step) through two LDS stages with the next
// chunk prefetched into registers.  Each thread stages units of four
// consecutive k of one row (one 8-byte LDS store per piece).
template <int P>
struct SplitProds;
template <>
struct SplitProds<2> {
  static constexpr int N = 3;
  static constexpr int a[3] = {0, 0, 1};
  static constexpr int b[3] = {0, 1, 0};
};
template <>
struct SplitProds<3> {
  static constexpr int N = 6;
  static constexpr int a[6] = {0, 0, 1, 1, 0, 2};
  static constexpr int b[6] = {0, 1, 0, 1, 2, 0};
};

template <int WR, int WC, int RT, int CT, int P>
struct PipeMx {
  static constexpr int NW = WR * WC;
  static constexpr int NT = NW * 64;
  static constexpr int ROWS = WR * RT * 16;
  static constexpr int COLS = WC * CT * 16;
  static constexpr int KC = 32;
  static constexpr int PITCH = 40;                        // bf16 per staged row
  static constexpr int STAGE = P * (ROWS + COLS) * PITCH; // bf16 per stage
  static constexpr int UNITS = (ROWS + COLS) * (KC / 4);  // 4-k units per chunk
  static constexpr int PF = (UNITS + NT - 1) / NT;
  static constexpr size_t LDS_BYTES = 2 * (size_t)STAGE * 2;
};

template <int WR, int WC, int RT, int CT, int P, bool A_KM, bool B_KM, class GA, class GB>
AFQ_DEV PipeSplit pipe_gemm_mx(int K, int nr, int nc, GA ga, GB gb, unsigned short* smem,
                               f4_t (&acc)[RT][CT]) {
  using Q = PipeMx<WR, WC, RT, CT, P>;
  constexpr int KU = Q::KC / 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int TR = (nr + 15) >> 4, TC = (nc + 15) >> 4;
  const int rpw = (TR + WR - 1) / WR, cpw = (TC + WC - 1) / WC;
  PipeSplit sp;
  sp.rt0 = wr * rpw;
  sp.mtv = max(0, min(min(rpw, RT), TR - sp.rt0));
  sp.ct0 = wc * cpw;
  sp.ntv = max(0, min(min(cpw, CT), TC - sp.ct0));
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  double pf[Q::PF][4];
  // unit u -> (stage row, first k of the unit)
  auto slot = [&](int u, int& row, int& k) {
    if (u < Q::ROWS * KU) {
      if (A_KM) {
        k = (u / Q::ROWS) * 4;
        row = u % Q::ROWS;
      } else {
        row = u / KU;
        k = (u % KU) * 4;
      }
    } else {
      const int u2 = u - Q::ROWS * KU;
      int c;
      if (B_KM) {
        k = (u2 / Q::COLS) * 4;
        c = u2 % Q::COLS;
      } else {
        c = u2 / KU;
        k = (u2 % KU) * 4;
      }
      row = Q::ROWS + c;
    }
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < Q::PF; ++i) {
      const int u = tid + i * Q::NT;
#pragma unroll
      for (int t = 0; t < 4; ++t) pf[i][t] = 0.0;
      if (u < Q::UNITS) {
        int row, k;
        slot(u, row, k);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int kg = k0 + k + t;
          if (kg < K) {
            if (row < Q::ROWS) {
              if (row < nr) pf[i][t] = ga(row, kg);
            } else if (row - Q::ROWS < nc) {
              pf[i][t] = gb(row - Q::ROWS, kg);
            }
          }
        }
      }
    }
  };
  auto store = [&](unsigned short* S) {
#pragma unroll
    for (int i = 0; i < Q::PF; ++i) {
      const int u = tid + i * Q::NT;
      if (u < Q::UNITS) {
        int row, k;
        slot(u, row, k);
        double x[4] = {pf[i][0], pf[i][1], pf[i][2], pf[i][3]};
#pragma unroll
        for (int p = 0; p < P; ++p) {
          unsigned short b[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            b[t] = bf16_bits_rn((float)x[t]);
            x[t] -= (double)bf16_bits_to_f(b[t]);
          }
          uint2 v;
          v.x = (unsigned)b[0] | ((unsigned)b[1] << 16);
          v.y = (unsigned)b[2] | ((unsigned)b[3] << 16);
          *(uint2*)(S + ((size_t)p * (Q::ROWS + Q::COLS) + row) * Q::PITCH + k) = v;
        }
      }
    }
  };
  const bool full = sp.mtv == RT && sp.ntv == CT;
  const int nchunk = (K + Q::KC - 1) / Q::KC;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  fetch(0);
  store(smem);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const unsigned short* S = smem + (size_t)(ch & 1) * Q::STAGE;
    if (ch + 1 < nchunk) fetch((ch + 1) * Q::KC);
    bf8_t a[RT][P], b[CT][P];
    if (full) {
      // the wave holds RT x CT tiles: no per-MFMA conditions
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p)
          a[i][p] = *(const bf8_t*)(S + ((size_t)p * (Q::ROWS + Q::COLS) + (sp.rt0 + i) * 16 + lr) *
                                            Q::PITCH + lk);
#pragma unroll
      for (int j = 0; j < CT; ++j)
#pragma unroll
        for (int p = 0; p < P; ++p)
          b[j][p] = *(const bf8_t*)(S + ((size_t)p * (Q::ROWS + Q::COLS) + Q::ROWS +
                                         (sp.ct0 + j) * 16 + lr) * Q::PITCH + lk);
#pragma unroll
      for (int q = 0; q < SplitProds<P>::N; ++q)
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < CT; ++j)
            acc[i][j] = mfma_bf16(a[i][SplitProds<P>::a[q]], b[j][SplitProds<P>::b[q]], acc[i][j]);
    } else {
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int p = 0; p < P; ++p)
          if (i < sp.mtv)
            a[i][p] = *(const bf8_t*)(S + ((size_t)p * (Q::ROWS + Q::COLS) + (sp.rt0 + i) * 16 + lr) *
                                              Q::PITCH + lk);
#pragma unroll
      for (int j = 0; j < CT; ++j)
#pragma unroll
        for (int p = 0; p < P; ++p)
          if (j < sp.ntv)
            b[j][p] = *(const bf8_t*)(S + ((size_t)p * (Q::ROWS + Q::COLS) + Q::ROWS +
                                           (sp.ct0 + j) * 16 + lr) * Q::PITCH + lk);
#pragma unroll
      for (int q = 0; q < SplitProds<P>::N; ++q)
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          if (i >= sp.mtv) continue;
#pragma unroll
          for (int j = 0; j < CT; ++j)
            if (j < sp.ntv)
              acc[i][j] = mfma_bf16(a[i][SplitProds<P>::a[q]], b[j][SplitProds<P>::b[q]], acc[i][j]);
        }
    }
    if (ch + 1 < nchunk) store(smem + (size_t)((ch + 1) & 1) * Q::STAGE);
    __syncthreads();
  }
  return sp;
}

// Row / column (within the tile) of FP32 accumulator element e of tile (i, j).
AFQ_DEV int pipe_mx_row(const PipeSplit& sp, int i, int e) {
  return (sp.rt0 + i) * 16 + 4 * ((threadIdx.x & 63) >> 4) + e;
}
AFQ_DEV int pipe_mx_col(const PipeSplit& sp, int j) { return (sp.ct0 + j) * 16 + (threadIdx.x & 15); }

// Visit every valid accumulator element of an engine tile: f(row, col, value)
// in tile coordinates (rows / columns beyond the tile's extent are skipped
// by the caller's bounds in f).
template <int RT, int CT, class F>
AFQ_DEV void pipe_emit(const PipeSplit& sp, d4_t (&acc)[RT][CT], F f) {
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      if (i >= sp.mtv || j >= sp.ntv) continue;
      const int c = pipe_col(sp, j);
#pragma unroll
      for (int e = 0; e < 4; ++e) f(pipe_row(sp, i, e), c, acc[i][j][e]);
    }
}
template <int RT, int CT, class F>
AFQ_DEV void pipe_emit(const PipeSplit& sp, f4_t (&acc)[RT][CT], F f) {
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      if (i >= sp.mtv || j >= sp.ntv) continue;
      const int c = pipe_mx_col(sp, j);
#pragma unroll
      for (int e = 0; e < 4; ++e) f(pipe_mx_row(sp, i, e), c, (double)acc[i][j][e]);
    }
}

// C tile of the FP64 engine (PC = 0) or of the BF16-split engine with PC
// pieces, then f(row, col, value) for every element.
template <int WR, int WC, int RT, int CT, int PC, bool A_KM, bool B_KM, int BK = 16, class GA,
          class GB, class F>
AFQ_DEV void pipe_run(int K, int nr, int nc, GA ga, GB gb, double* smem, F f) {
  if constexpr (PC == 0) {
    d4_t acc[RT][CT];
    const PipeSplit sp = pipe_gemm<WR, WC, RT, CT, A_KM, B_KM, BK>(K, nr, nc, ga, gb, smem, acc);
    pipe_emit(sp, acc, f);
  } else {
    f4_t acc[RT][CT];
    const PipeSplit sp = pipe_gemm_mx<WR, WC, RT, CT, PC, A_KM, B_KM>(
        K, nr, nc, ga, gb, reinterpret_cast<unsigned short*>(smem), acc);
    pipe_emit(sp, acc, f);
  }
}

// Dynamic LDS bytes of either engine.
template <int WR, int WC, int RT, int CT, int PC, int BK = 16>
constexpr size_t pipe_lds_bytes() {
  if constexpr (PC == 0) return Pipe<WR, WC, RT, CT, BK>::LDS_BYTES;
  else return PipeMx<WR, WC, RT, CT, PC>::LDS_BYTES;
}

// ---------------------------------------------------------------- exchange epilogue
// Reduction of the T_g^w = (Psi_T^T L_g) Theta^w blocks of one local-energy
// tile, shared by the FP64 and the BF16-split kernels.  The tile holds rows
// (g, i) of ga Cholesky blocks and columns (w, j, plane) of wb walkers, the
// real and imaginary parts of T_ij side by side.  The rows of `gpp`
// consecutive Cholesky blocks (a phase) are staged in LDS in the tile's own
// layout, Ts[row][col] with the compile-time pitch PITCH, so that every
// accumulator element is stored at a lane base plus a constant offset.  Then
// every block (Cholesky block, walker) of the phase is reduced to
//   X_g = sum_ij T_ij T_ji = 2 sum_{i<j} T_ij T_ji + sum_i T_ii^2,
//   ell_g = 2 sum_i T_ii,
// where T = (staged product) + T0_g, T0_g the real symmetric trial-space
// block shared by the walkers,
// with a fixed cut: thread t takes the pairs i < j of index
// p = t + nthreads k (row by row) in the order of k, and thread t < N the
// diagonal element t; wave sums, then the waves' partial sums in wave order.
// The products are formed in MT (float64, or float32 when T itself is a
// float32 result) and summed per thread in MT, the wave and workgroup sums in
// float64.  The cut depends on N and the workgroup size only, so the sums do
// not depend on the tile shape.  row_of(i, e) is the tile row of accumulator
// element e of row tile i; the columns of tile j are j * 16 + (lane & 15).
// The blocks of a phase are reduced up to NBMAX at a time (red holds
// 4 NBMAX nwaves doubles).
template <typename TS, int NB, int PITCH>
AFQ_DEV void exchange_reduce(const TS* Ts, const int* boff_in, const double* const* t0_in, int N,
                             double* red) {
  typedef typename std::conditional<sizeof(TS) == 8, double2, float2>::type TS2;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
  const int P = N * (N - 1) / 2, twoN1 = 2 * N - 1;
  int boff[NB];
  const double* t0[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    boff[b] = boff_in[b];
    t0[b] = t0_in[b];
  }
  TS xr[NB], xi[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) xr[b] = xi[b] = (TS)0;
  for (int p = tid; p < P; p += nthr) {
    // row i of pair p: C(i) = i (2N - 1 - i) / 2 pairs precede row i
    int i = (int)(0.5f * ((float)twoN1 - sqrtf((float)(twoN1 * twoN1 - 8 * p))));
    i = max(0, min(i, N - 2));
    while (i > 0 && i * (twoN1 - i) / 2 > p) --i;
    while ((i + 1) * (twoN1 - i - 1) / 2 <= p) ++i;
    const int j = i + 1 + p - i * (twoN1 - i) / 2;
    const int oij = i * PITCH + 2 * j, oji = j * PITCH + 2 * i;
    TS2 a[NB], c[NB];
    TS s[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) s[b] = (TS)t0[b][i * N + j];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      a[b] = *(const TS2*)(Ts + boff[b] + oij);
      c[b] = *(const TS2*)(Ts + boff[b] + oji);
    }
    // explicit fused multiply-adds: every instance rounds alike
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const TS ar = a[b].x + s[b], br = c[b].x + s[b];
      xr[b] = fma(ar, br, xr[b]);
      xr[b] = fma(-a[b].y, c[b].y, xr[b]);
      xi[b] = fma(ar, c[b].y, xi[b]);
      xi[b] = fma(a[b].y, br, xi[b]);
    }
  }
  double dr[NB], di[NB], tr[NB], ti[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) dr[b] = di[b] = tr[b] = ti[b] = 0.0;
  if (tid < N) {
    const int o = tid * PITCH + 2 * tid;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const TS2 d = *(const TS2*)(Ts + boff[b] + o);
      const double x = (double)d.x + t0[b][tid * N + tid], y = d.y;
      dr[b] = fma(x, x, -(y * y));
      di[b] = 2.0 * (x * y);
      tr[b] = x;
      ti[b] = y;
    }
  }
  double v[4 * NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    v[4 * b] = fma(2.0, (double)xr[b], dr[b]);
    v[4 * b + 1] = fma(2.0, (double)xi[b], di[b]);
    v[4 * b + 2] = tr[b];
    v[4 * b + 3] = ti[b];
  }
  wave_sum_n(v);
  if (lane == 63) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double* rr = red + (b * nwaves + wave) * 4;
      rr[0] = v[4 * b];
      rr[1] = v[4 * b + 1];
      rr[2] = v[4 * b + 2];
      rr[3] = v[4 * b + 3];
    }
  }
}

template <typename TS, int PITCH, int NBMAX, typename ACC, int RT, int CT, class RowOf>
AFQ_DEV void exchange_epilogue(ACC (&acc)[RT][CT], RowOf row_of, int mtv, int N, int ga, int wb,
                               int g0, int w0, int G1, TS* Ts, int gpp, double* red,
                               const double* __restrict__ T0, double lscale,
                               double* __restrict__ ell_re, double* __restrict__ ell_im,
                               double* __restrict__ ex_re, double* __restrict__ ex_im) {
  static_assert(PITCH >= CT * 16, "pitch");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  const int twoN = 2 * N;
  TS* lane_base = Ts + (lane & 15);
  for (int gb0 = 0; gb0 < ga; gb0 += gpp) {
    const int ngl = min(gpp, ga - gb0), nb = ngl * wb;
    const int p0 = gb0 * N, p1 = p0 + ngl * N;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = row_of(i, e);
        if (i < mtv && r >= p0 && r < p1) {
          TS* d = lane_base + (r - p0) * PITCH;
#pragma unroll
          for (int j = 0; j < CT; ++j) d[j * 16] = (TS)acc[i][j][e];
        }
      }
    __syncthreads();
    for (int bb0 = 0; bb0 < nb; bb0 += NBMAX) {
      const int nbb = min(NBMAX, nb - bb0);
      int boff[NBMAX];
      const double* t0[NBMAX];
#pragma unroll
      for (int b = 0; b < NBMAX; ++b) {
        const int bq = b < nbb ? bb0 + b : bb0;
        const int gl = bq / wb, wl = bq - gl * wb;
        boff[b] = gl * N * PITCH + wl * twoN;
        t0[b] = T0 + (int64_t)(g0 + gb0 + gl) * N * N;
      }
      // exactly nbb blocks: one instance per count
      switch (nbb) {
#define AFQ_REDUCE_CASE(K)                                          \
  case K:                                                           \
    if constexpr (K <= NBMAX) exchange_reduce<TS, K, PITCH>(Ts, boff, t0, N, red); \
    break;
        AFQ_REDUCE_CASE(1)
        AFQ_REDUCE_CASE(2)
        AFQ_REDUCE_CASE(3)
        AFQ_REDUCE_CASE(4)
        AFQ_REDUCE_CASE(5)
        AFQ_REDUCE_CASE(6)
        AFQ_REDUCE_CASE(7)
        AFQ_REDUCE_CASE(8)
#undef AFQ_REDUCE_CASE
        default: break;
      }
      __syncthreads();
      if (tid < nbb) {
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int w = 0; w < nwaves; ++w)
          for (int k = 0; k < 4; ++k) s[k] += red[(tid * nwaves + w) * 4 + k];
        const int gl = (bb0 + tid) / wb, wl = bb0 + tid - gl * wb;
        const int64_t o = (int64_t)(w0 + wl) * G1 + g0 + gb0 + gl;
        ex_re[o] = s[0];
        ex_im[o] = s[1];
        ell_re[o] = lscale * s[2];
        ell_im[o] = lscale * s[3];
      }
      __syncthreads();
    }
  }
}
