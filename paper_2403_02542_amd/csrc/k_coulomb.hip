// The Coulomb vector ell_g = s tr T_g over the virtual space (the FP64
// companion of the BF16-split local energy; s the spin factor, 2 for a
// closed-shell determinant): with Theta = Psi_T + Psi_perp Theta_v,
//   ell_g = s tr T0_g + s sum_(i,k) (Psi_T^T L_g Psi_perp)[i][k] Theta_v[k][i],
// one product [W x N Kv] x [N Kv x G] per plane on the FP64 matrix cores,
// cut into S slices of whole orbitals (batch entries writing partial sums)
// and summed in slice order with the trial part s tr T0_g.
#include "afq_device.h"
#include "afq_internal.h"

namespace {

__global__ void k_sum_slices_t0(const double* __restrict__ part, int S, int W, int G, int G1,
                                const double* __restrict__ t0tr, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)W * G;
  if (e >= n) return;
  const int64_t w = e / G, g = e - w * G;
  double v = t0tr ? t0tr[g] : 0.0;
  for (int q = 0; q < S; ++q) v += part[q * n + e];
  out[w * G1 + g] = v;
}

__global__ void k_t0_trace(int G, int N, double spin, const double* __restrict__ T0,
                           double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  double t = 0.0;
  for (int i = 0; i < N; ++i) t += T0[(int64_t)g * N * N + (int64_t)i * N + i];
  out[g] = spin * t;
}

}  // namespace

int coulomb_v_slices(int W, int G, int N, int Kv) {
  // slices of whole orbitals (S divides N), enough blocks to fill the chip
  const int tiles = ((W + 127) / 128) * ((G + 127) / 128);
  int best = 1;
  for (int S = 1; S <= N && S <= 64; ++S)
    if (N % S == 0 && (N / S) * Kv >= 256 && tiles * S <= 768) best = S;
  return best;
}

hipError_t launch_t0_trace(SysDev& s, hipStream_t st) {
  hipLaunchKernelGGL(k_t0_trace, dim3((s.G + 255) / 256), dim3(256), 0, st, s.G, s.N, s.spin,
                     s.T0, s.t0tr);
  return hipGetLastError();
}

hipError_t launch_coulomb_v(SysDev& s, const double* thv_re, const double* thv_im, double* part,
                            double* ell_re, double* ell_im, hipStream_t st) {
  const int W = s.W, G = s.G, G1 = G + 1, NK = s.N * s.Kv;
  if (s.Kv == 0) {
    // Psi_T spans the orbital space: ell is the trial part alone
    hipLaunchKernelGGL(k_sum_slices_t0, dim3((unsigned)(((int64_t)W * G + 255) / 256)), dim3(256),
                       0, st, part, 0, W, G, G1, s.t0tr, ell_re);
    hipLaunchKernelGGL(k_sum_slices_t0, dim3((unsigned)(((int64_t)W * G + 255) / 256)), dim3(256),
                       0, st, part, 0, W, G, G1, (const double*)nullptr, ell_im);
    return hipGetLastError();
  }
  const int S = coulomb_v_slices(W, G, s.N, s.Kv);
  const int kc = NK / S;
  const double* planes[2] = {thv_re, thv_im};
  double* outs[2] = {ell_re, ell_im};
  for (int pl = 0; pl < 2; ++pl) {
    GemmArgs c{};
    c.A = planes[pl]; c.sAb = kc; c.sAr = NK; c.sAk = 1; c.sAkb = 0;
    c.B = s.Lov; c.sBb = kc; c.sBc = NK; c.sBk = 1; c.sBkb = 0;
    c.C = part; c.sCb = (int64_t)W * G; c.sCr = G; c.sCc = 1;
    c.R = W; c.Cn = G; c.K = kc; c.kin = kc; c.batch = S; c.alpha = s.spin; c.beta = 0.0;
    hipError_t e = launch_gemm(c, st);
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)W * G;
    hipLaunchKernelGGL(k_sum_slices_t0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part,
                       S, W, G, G1, pl == 0 ? (const double*)s.t0tr : nullptr, outs[pl]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

