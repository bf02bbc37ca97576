// Crank-Nicolson propagator (Sec. III.D): per walker,
//   X = (I - A_T / 2)^-1 (I + A_T / 2) Phi,   A_T = A - tau H1,
// the (1,1) Pade form of exp(A_T) on the orbitals.  The right-hand sides
// R = Phi + A_T Phi / 2 come from one operator-orbital product on the matrix
// cores; the operator, no longer needed, is turned into I - A_T / 2 in place
// and solved against R by Gauss-Jordan elimination with partial pivoting,
// one workgroup per walker (the M x M system streams through L2; M <= a few
// hundred).
#include <cmath>

#include "afq_device.h"
#include "afq_internal.h"

namespace {

__global__ void k_cn_copy(int64_t n, const double* __restrict__ sre,
                          const double* __restrict__ sim, double* __restrict__ dre,
                          double* __restrict__ dim) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    dre[e] = sre[e];
    dim[e] = sim[e];
  }
}

// A <- I - A / 2 over every walker's M x M operator.
__global__ void k_cn_prep(int64_t MM, int M, int W, double* __restrict__ are,
                          double* __restrict__ aim) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < MM * W;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % MM;
    const int p = (int)(r / M), q = (int)(r - (int64_t)p * M);
    are[e] = (p == q ? 1.0 : 0.0) - 0.5 * are[e];
    aim[e] = -0.5 * aim[e];
  }
}

constexpr int CN_T = 256;

// Solve C X = R in place for walker blockIdx.x: C = [W][M][M] row-major
// (C[p][q] at p M + q), R = X = [W][N][M] (orbital j, entry p at j M + p).
// Columns left of the pivot are never read again, so only columns right of
// it are updated.
__global__ __launch_bounds__(CN_T) void k_cn_solve(int M, int N, double* __restrict__ cre,
                                                   double* __restrict__ cim,
                                                   double* __restrict__ xre,
                                                   double* __restrict__ xim) {
  __shared__ double s_v[CN_T];
  __shared__ int s_i[CN_T];
  __shared__ double s_pr, s_pi;
  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  double* Cr = cre + w * M * M;
  double* Ci = cim + w * M * M;
  double* Xr = xre + w * N * M;
  double* Xi = xim + w * N * M;
  for (int k = 0; k < M; ++k) {
    // pivot: the largest |C[i][k]|, i >= k (first index among equals)
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < M; i += CN_T) {
      const double v = Cr[(int64_t)i * M + k] * Cr[(int64_t)i * M + k] +
                       Ci[(int64_t)i * M + k] * Ci[(int64_t)i * M + k];
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    s_v[tid] = best;
    s_i[tid] = bi;
    __syncthreads();
    for (int o = CN_T / 2; o > 0; o >>= 1) {
      if (tid < o) {
        const double a = s_v[tid], b = s_v[tid + o];
        if (b > a || (b == a && s_i[tid + o] < s_i[tid])) {
          s_v[tid] = b;
          s_i[tid] = s_i[tid + o];
        }
      }
      __syncthreads();
    }
    const int p = s_i[0];
    if (p != k) {
      for (int c = k + tid; c < M; c += CN_T) {
        const double tr = Cr[(int64_t)k * M + c], ti = Ci[(int64_t)k * M + c];
        Cr[(int64_t)k * M + c] = Cr[(int64_t)p * M + c];
        Ci[(int64_t)k * M + c] = Ci[(int64_t)p * M + c];
        Cr[(int64_t)p * M + c] = tr;
        Ci[(int64_t)p * M + c] = ti;
      }
      for (int j = tid; j < N; j += CN_T) {
        const double tr = Xr[(int64_t)j * M + k], ti = Xi[(int64_t)j * M + k];
        Xr[(int64_t)j * M + k] = Xr[(int64_t)j * M + p];
        Xi[(int64_t)j * M + k] = Xi[(int64_t)j * M + p];
        Xr[(int64_t)j * M + p] = tr;
        Xi[(int64_t)j * M + p] = ti;
      }
    }
    __syncthreads();
    if (tid == 0) {
      // 1 / C[k][k]
      const double ar = Cr[(int64_t)k * M + k], ai = Ci[(int64_t)k * M + k];
      const double d = ar * ar + ai * ai;
      s_pr = ar / d;
      s_pi = -ai / d;
    }
    __syncthreads();
    const double ir = s_pr, ii = s_pi;
    // scale the pivot row right of the pivot, and the right-hand sides' entry k
    for (int c = k + 1 + tid; c < M + N; c += CN_T) {
      double* pr = c < M ? Cr + (int64_t)k * M + c : Xr + (int64_t)(c - M) * M + k;
      double* pi = c < M ? Ci + (int64_t)k * M + c : Xi + (int64_t)(c - M) * M + k;
      const double vr = *pr, vi = *pi;
      *pr = vr * ir - vi * ii;
      *pi = vr * ii + vi * ir;
    }
    __syncthreads();
    // eliminate column k from every other row
    const int width = M - k - 1 + N;
    for (int64_t e = tid; e < (int64_t)M * width; e += CN_T) {
      const int i = (int)(e / width), c = (int)(e - (int64_t)i * width);
      if (i == k) continue;
      const double fr = Cr[(int64_t)i * M + k], fi = Ci[(int64_t)i * M + k];
      double *tr, *ti;
      double sr, si;
      if (c < M - k - 1) {
        const int col = k + 1 + c;
        tr = Cr + (int64_t)i * M + col;
        ti = Ci + (int64_t)i * M + col;
        sr = Cr[(int64_t)k * M + col];
        si = Ci[(int64_t)k * M + col];
      } else {
        const int j = c - (M - k - 1);
        tr = Xr + (int64_t)j * M + i;
        ti = Xi + (int64_t)j * M + i;
        sr = Xr[(int64_t)j * M + k];
        si = Xi[(int64_t)j * M + k];
      }
      *tr -= fr * sr - fi * si;
      *ti -= fr * si + fi * sr;
    }
    __syncthreads();
  }
}

inline unsigned grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 8192 ? g : 8192);
}

}  // namespace

hipError_t launch_crank_nicolson(SysDev& s, const double* in_re, const double* in_im,
                                 double* out_re, double* out_im, double* t_re, double* t_im,
                                 hipStream_t st) {
  const int64_t NM = (int64_t)s.N * s.M, MM = (int64_t)s.M * s.M;
  // out = Phi + A_T Phi / 2
  hipLaunchKernelGGL(k_cn_copy, dim3(grid_for(NM * s.W)), dim3(256), 0, st, NM * s.W, in_re, in_im,
                     out_re, out_im);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_matvec_acc(s, VecRef{in_re, in_im, NM, s.M}, VecOut{t_re, t_im, NM, s.M}, 0.5,
                        VecOut{out_re, out_im, NM, s.M}, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cn_prep, dim3(grid_for(MM * s.W)), dim3(256), 0, st, MM, s.M, s.W, s.A_re,
                     s.A_im);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cn_solve, dim3(s.W), dim3(CN_T), 0, st, s.M, s.N, s.A_re, s.A_im, out_re,
                     out_im);
  return hipGetLastError();
}
