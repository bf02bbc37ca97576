// Block-Krylov exponential of the one-body operator (Sec. IV.D, Eq.
// bkrylovsub, bkrylov): one Krylov space of dimension kN per walker for all
// its orbitals together,
//   Psi = B_1 R,  W = A B_j,  H_ij = B_i^dag W,  W -= B_i H_ij  (i <= j),
//   W = B_{j+1} H_{j+1,j}  (QR, j < k),
//   bkrylov_k{A, Psi} = B_k exp(A_k) E_N R,   A_k = [H_ij] (kN x kN).
// The k operator-orbital products A B_j run on the MFMA product of the
// per-orbital Krylov (k_matvec); the block orthonormalisations on the
// shifted Cholesky-QR3 kernel of the reorthonormalisation (positive real
// diag R, so H_{j+1,j} = B_{j+1}^dag W); the small complex products
// (H_ij, the block Gram-Schmidt updates, R, the Taylor terms of the small
// exponential and the final B_k X) as batched FP64 GEMMs over walkers, four
// real products per complex one.  exp(A_k) E_N R is a Taylor series of 18
// terms in s substeps, s = ceil(max_w ||A_k||_1), read on the host.
#include <cmath>
#include <cstring>
#include <utility>

#include "afq_device.h"
#include "afq_internal.h"

namespace {

constexpr int kTaylorTerms = 18;     // per substep of norm <= 1: error < 1 / 19!

// Planar complex operand of a batched product: element (b, r, k) at
// b sb + r sr + k sk of the re / im arrays.
struct CIn {
  const double* re;
  const double* im;
  int64_t sb, sr, sk;
};
struct COut {
  double* re;
  double* im;
  int64_t sb, sr, sc;
};

// C(b, r, c) = alpha sum_k A(b, r, k) B(b, c, k) + beta C(b, r, c), complex;
// conjA takes the complex conjugate of A.
hipError_t cgemm(int batch, int R, int Cn, int K, CIn a, bool conjA, CIn b, COut c, double alpha,
                 double beta, hipStream_t st) {
  const double sa = conjA ? -1.0 : 1.0;
  auto one = [&](const double* A, const double* B, double* C, double al, double be) {
    GemmArgs g{};
    g.A = A; g.sAb = a.sb; g.sAr = a.sr; g.sAk = a.sk; g.sAkb = 0;
    g.B = B; g.sBb = b.sb; g.sBc = b.sr; g.sBk = b.sk; g.sBkb = 0;
    g.C = C; g.sCb = c.sb; g.sCr = c.sr; g.sCc = c.sc;
    g.R = R; g.Cn = Cn; g.K = K; g.kin = K; g.batch = batch; g.alpha = al; g.beta = be;
    return launch_gemm(g, st);
  };
  hipError_t e;
  // Re C = alpha (Ar Br - sa Ai Bi) + beta Re C
  if ((e = one(a.re, b.re, c.re, alpha, beta)) != hipSuccess) return e;
  if ((e = one(a.im, b.im, c.re, -sa * alpha, 1.0)) != hipSuccess) return e;
  // Im C = alpha (Ar Bi + sa Ai Br) + beta Im C
  if ((e = one(a.re, b.im, c.im, alpha, beta)) != hipSuccess) return e;
  return one(a.im, b.re, c.im, sa * alpha, 1.0);
}

// dst[b][r][p] = src[b][r][p] for W sets of `rows` rows of M (strides in doubles).
__global__ void k_copy_sets(int rows, int M, const double* __restrict__ sre,
                            const double* __restrict__ sim, int64_t ssb, double* __restrict__ dre,
                            double* __restrict__ dim, int64_t dsb) {
  const int b = blockIdx.y;
  const int64_t n = (int64_t)rows * M;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    dre[b * dsb + e] = sre[b * ssb + e];
    dim[b * dsb + e] = sim[b * ssb + e];
  }
}

__global__ void k_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_zero2(int64_t n, double* __restrict__ a, double* __restrict__ b) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    a[e] = 0.0;
    b[e] = 0.0;
  }
}

// max over walkers (alive, factorised, finite) of ||A_k||_1 =
// max_c sum_r |A_k[r][c]|, as the bit pattern of a non-negative double.  A
// walker whose block factorisation failed is poisoned afterwards; its A_k
// must not set the substep count of the others.
__global__ __launch_bounds__(256) void k_norm1(int D, const double* __restrict__ hre,
                                               const double* __restrict__ him,
                                               const int* __restrict__ alive,
                                               const int* __restrict__ bad,
                                               unsigned long long* __restrict__ out) {
  const int b = blockIdx.x;
  if (!alive[b] || bad[b]) return;
  const double* r0 = hre + (int64_t)b * D * D;
  const double* i0 = him + (int64_t)b * D * D;
  double m = 0.0;
  for (int c = threadIdx.x; c < D; c += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < D; ++r) s += sqrt(r0[r * D + c] * r0[r * D + c] + i0[r * D + c] * i0[r * D + c]);
    m = fmax(m, s);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0 && isfinite(m)) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

// X^T[b][n][q] = (E_N R)[q][n] = R[q][n] for q < N, 0 for N <= q < D.
__global__ void k_enr(int N, int D, const double* __restrict__ rre, const double* __restrict__ rim,
                      double* __restrict__ xre, double* __restrict__ xim) {
  const int b = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * D) return;
  const int n = e / D, q = e - n * D;
  const double vr = q < N ? rre[(int64_t)b * N * N + q * N + n] : 0.0;
  const double vi = q < N ? rim[(int64_t)b * N * N + q * N + n] : 0.0;
  xre[(int64_t)b * N * D + e] = vr;
  xim[(int64_t)b * N * D + e] = vi;
}

// x += y over n doubles per plane.
__global__ void k_axpy2(int64_t n, const double* __restrict__ yre, const double* __restrict__ yim,
                        double* __restrict__ xre, double* __restrict__ xim) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    xre[e] += yre[e];
    xim[e] += yim[e];
  }
}

// Walkers whose block factorisation failed get a non-finite result, so the
// overlap marks them and the weight update freezes them.
__global__ void k_poison(int NM, const int* __restrict__ bad, double* __restrict__ ore,
                         double* __restrict__ oim) {
  const int b = blockIdx.y;
  if (!bad[b]) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NM; e += gridDim.x * blockDim.x) {
    ore[(int64_t)b * NM + e] = NAN;
    oim[(int64_t)b * NM + e] = NAN;
  }
}

inline unsigned blocks_for(int64_t n, int b) {
  const int64_t g = (n + b - 1) / b;
  return (unsigned)(g < 4096 ? g : 4096);
}

}  // namespace

hipError_t launch_block_krylov(SysDev& s, int k, const double* in_re, const double* in_im,
                               double* out_re, double* out_im, double* wv_re, double* wv_im,
                               hipStream_t st) {
  const int W = s.W, N = s.N, M = s.M, D = k * N;
  if (k < 1 || k > s.kmax || k > s.bk_k || D > M) return hipErrorInvalidValue;
  const int64_t NM = (int64_t)N * M, sbB = (int64_t)s.kmax * NM, DD = (int64_t)D * D;
  hipError_t e;
  hipLaunchKernelGGL(k_zero_int, dim3((W + 255) / 256), dim3(256), 0, st, s.bk_bad, W);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // A_k from zero: the blocks below its first block subdiagonal stay zero
  hipLaunchKernelGGL(k_zero2, dim3(blocks_for(DD * W, 256)), dim3(256), 0, st, DD * W, s.bkh_re,
                     s.bkh_im);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // B_1 R = Psi
  hipLaunchKernelGGL(k_copy_sets, dim3(blocks_for(NM, 256), W), dim3(256), 0, st, N, M, in_re,
                     in_im, NM, s.kb_re, s.kb_im, sbB);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_qr_strided(s, s.kb_re, s.kb_im, sbB, s.bk_logr, s.bk_bad, st)) != hipSuccess)
    return e;
  // R = B_1^dag Psi
  e = cgemm(W, N, N, M, CIn{s.kb_re, s.kb_im, sbB, M, 1}, true, CIn{in_re, in_im, NM, M, 1},
            COut{s.bkr_re, s.bkr_im, (int64_t)N * N, N, 1}, 1.0, 0.0, st);
  if (e != hipSuccess) return e;
  for (int j = 0; j < k; ++j) {
    // W = A B_j
    const VecRef v{s.kb_re + (int64_t)j * NM, s.kb_im + (int64_t)j * NM, sbB, M};
    const VecOut o{wv_re, wv_im, NM, M};
    if ((e = launch_matvec(s, v, o, st)) != hipSuccess) return e;
    for (int i = 0; i <= j; ++i) {
      // H_ij = B_i^dag W, then W -= B_i H_ij
      const CIn Bi{s.kb_re + (int64_t)i * NM, s.kb_im + (int64_t)i * NM, sbB, M, 1};
      double* hr = s.bkh_re + (int64_t)i * N * D + (int64_t)j * N;
      double* hi = s.bkh_im + (int64_t)i * N * D + (int64_t)j * N;
      e = cgemm(W, N, N, M, Bi, true, CIn{wv_re, wv_im, NM, M, 1}, COut{hr, hi, DD, D, 1}, 1.0,
                0.0, st);
      if (e != hipSuccess) return e;
      e = cgemm(W, N, M, N, CIn{hr, hi, DD, 1, D}, false, CIn{Bi.re, Bi.im, sbB, 1, M},
                COut{wv_re, wv_im, NM, M, 1}, -1.0, 1.0, st);
      if (e != hipSuccess) return e;
    }
    if (j + 1 == k) break;
    // B_{j+1} H_{j+1,j} = W
    double* br = s.kb_re + (int64_t)(j + 1) * NM;
    double* bi = s.kb_im + (int64_t)(j + 1) * NM;
    hipLaunchKernelGGL(k_copy_sets, dim3(blocks_for(NM, 256), W), dim3(256), 0, st, N, M, wv_re,
                       wv_im, NM, br, bi, sbB);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_qr_strided(s, br, bi, sbB, s.bk_logr, s.bk_bad, st)) != hipSuccess) return e;
    double* hr = s.bkh_re + (int64_t)(j + 1) * N * D + (int64_t)j * N;
    double* hi = s.bkh_im + (int64_t)(j + 1) * N * D + (int64_t)j * N;
    e = cgemm(W, N, N, M, CIn{br, bi, sbB, M, 1}, true, CIn{wv_re, wv_im, NM, M, 1},
              COut{hr, hi, DD, D, 1}, 1.0, 0.0, st);
    if (e != hipSuccess) return e;
  }
  // substeps of the small exponential from the largest ||A_k||_1
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, s.bk_norm);
  hipLaunchKernelGGL(k_norm1, dim3(W), dim3(256), 0, st, D, s.bkh_re, s.bkh_im, s.alive, s.bk_bad,
                     s.bk_norm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  unsigned long long nb = 0;
  if ((e = hipMemcpyAsync(&nb, s.bk_norm, sizeof(nb), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  double nrm;
  std::memcpy(&nrm, &nb, sizeof(nrm));
  int nsub = (int)std::ceil(nrm);
  if (nsub < 1) nsub = 1;
  if (nsub > 1024) nsub = 1024;
  // X = E_N R (stored transposed, [n][q]); per substep Y = X, then
  // Y <- (A_k / nsub) Y / t and X += Y for t = 1..18
  const int64_t ND = (int64_t)N * D;
  hipLaunchKernelGGL(k_enr, dim3((unsigned)((ND + 255) / 256), W), dim3(256), 0, st, N, D,
                     s.bkr_re, s.bkr_im, s.bkx_re, s.bkx_im);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int sub = 0; sub < nsub; ++sub) {
    hipLaunchKernelGGL(k_copy_sets, dim3(blocks_for(ND, 256), W), dim3(256), 0, st, N, D, s.bkx_re,
                       s.bkx_im, ND, s.bky_re, s.bky_im, ND);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double *yr = s.bky_re, *yi = s.bky_im, *zr = s.bkz_re, *zi = s.bkz_im;
    for (int t = 1; t <= kTaylorTerms; ++t) {
      e = cgemm(W, N, D, D, CIn{yr, yi, ND, D, 1}, false, CIn{s.bkh_re, s.bkh_im, DD, D, 1},
                COut{zr, zi, ND, D, 1}, 1.0 / ((double)nsub * t), 0.0, st);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_axpy2, dim3(blocks_for(ND * W, 256)), dim3(256), 0, st, ND * W, zr, zi,
                         s.bkx_re, s.bkx_im);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      std::swap(yr, zr);
      std::swap(yi, zi);
    }
  }
  // out = B_k X
  e = cgemm(W, N, M, D, CIn{s.bkx_re, s.bkx_im, ND, D, 1}, false, CIn{s.kb_re, s.kb_im, sbB, 1, M},
            COut{out_re, out_im, NM, M, 1}, 1.0, 0.0, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_poison, dim3(blocks_for(NM, 256), W), dim3(256), 0, st, (int)NM, s.bk_bad,
                     out_re, out_im);
  return hipGetLastError();
}
