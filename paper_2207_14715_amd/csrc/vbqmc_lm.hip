// gfx950 sample sums of the linear optimisation method (Sec. 2.2, Eqs.
// geneigeq; Sec. 2.3.1, Eqs. Hi0, H0j, Hij, Sij).
//
// Every average those estimators need is an entry of three weighted
// products over the samples k (walkers) of the augmented per-sample rows
//   X_k = [1 | O_k1 .. O_kP]   (O_kj = Psi_j / Psi_0 = d ln|Psi| / dp_j)
//   Y_k = [E_k^2 | D_k1 .. D_kP]   (D_kj = E_L,j = d E_L / dp_j):
//   S'[i][j] += sum_k w_k X_ki X_kj
//   H'[i][j] += sum_k w_k E_k X_ki X_kj
//   D'[i][j] += sum_k w_k X_ki Y_kj
// (row 0 holds sum w, sum w O_j, sum w E, sum w E O_j, sum w E^2 and
// sum w D_j).  Each is a dense (P+1) x W by W x (P+1) product, here on FP64
// MFMA: a 256-thread workgroup owns a 64 x 64 block of one matrix, wavefront
// g rows 16 g .. 16 g + 15 of it as four 16 x 16 tiles, and walks the
// samples four at a time (one 16x16x4 k-step).  Operands come straight from
// the row-major per-sample arrays (16 consecutive doubles per sample row per
// lane quarter); the sample sum runs in one fixed order, so the sums are
// reproducible, and each block adds its result to the accumulator it owns.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vbqmc {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kLmB = 64;   // block edge
constexpr int kLmT = 256;  // threads per workgroup

// mat 0: S', 1: H', 2: D'.  acc: three (P+1) x (P+1) row-major matrices.
__global__ __launch_bounds__(kLmT) void k_lm_accumulate(int P, int64_t W, const double* __restrict__ O,
                                                         const double* __restrict__ D, const double* __restrict__ E,
                                                         const double* __restrict__ wt, double* __restrict__ acc) {
  const int P1 = P + 1;
  const int mat = blockIdx.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int i = blockIdx.y * kLmB + 16 * wave + m;  // A row (X column)
  const int j0 = blockIdx.x * kLmB;
  v4d c[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) c[t][r] = 0.0;
  const bool iin = i < P1;
  for (int64_t k0 = 0; k0 < W; k0 += 4) {
    const int64_t k = k0 + kq;
    const bool kin = k < W;
    const int64_t kk = kin ? k : 0;
    const double w = kin ? (wt ? wt[kk] : 1.0) : 0.0;
    const double e = E[kk];
    const double* Ok = O + kk * P;
    // A: X_ki
    const double a = (iin && i > 0) ? Ok[i - 1] : (iin ? 1.0 : 0.0);
    const double s = mat == 1 ? w * e : w;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = j0 + 16 * t + m;
      double z;
      if (mat < 2) z = (j < P1 && j > 0) ? Ok[j - 1] : (j == 0 ? 1.0 : 0.0);
      else z = (j < P1 && j > 0) ? D[kk * P + j - 1] : (j == 0 ? e * e : 0.0);
      c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, z * s, c[t], 0, 0, 0);
    }
  }
  // register q of lane l holds row 4 q + l / 16, column l % 16 of a tile
  double* out = acc + (size_t)mat * P1 * P1;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = blockIdx.y * kLmB + 16 * wave + 4 * q + kq;
      const int col = j0 + 16 * t + m;
      if (row < P1 && col < P1) out[(size_t)row * P1 + col] += c[t][q];
    }
}

hipError_t launch_lm_accumulate(int P, int64_t W, const double* O, const double* D, const double* E,
                                const double* w, double* acc, hipStream_t s) {
  const int nb = (P + 1 + kLmB - 1) / kLmB;
  hipLaunchKernelGGL(k_lm_accumulate, dim3(nb, nb, 3), dim3(kLmT), 0, s, P, W, O, D, E, w, acc);
  return hipGetLastError();
}

// Orbital-rotation derivatives (Sec. 2.2, Eq. PsiJVBp) from the orbital
// coefficient derivatives of the adjoint.  To first order the rotation
// exp(kappa_kl E_kl) adds kappa_kl phi_k to orbital l, i.e. lambda_l +=
// kappa_kl lambda_k, so d/d kappa_kl = sum_mu lambda_k,mu d/d lambda_l,mu; a
// pair tied by kappa_lk = -kappa_kl (kind 1) takes the difference of its two
// directions.  One workgroup per walker and array (blockIdx.y 0: d lnPsi,
// 1: d E_L), one thread per pair; a pair whose orbitals or kind are out of
// range gives NaN (nothing is read for it).
constexpr int kRotT = 256;

__global__ __launch_bounds__(kRotT) void k_rotation_grad(int P, int lam_off, int M, int nop, int norb, int npair,
                                                        const int* __restrict__ pairs,
                                                        const double* __restrict__ lamT,
                                                        const double* __restrict__ dl, const double* __restrict__ de,
                                                        double* __restrict__ odl, double* __restrict__ ode) {
  const int64_t w = blockIdx.x;
  const double* src = (blockIdx.y == 0 ? dl : de) + w * P + lam_off;
  double* dst = (blockIdx.y == 0 ? odl : ode) + w * npair;
  for (int q = threadIdx.x; q < npair; q += kRotT) {
    const int k = pairs[3 * q], l = pairs[3 * q + 1], kind = pairs[3 * q + 2];
    if ((unsigned)k >= (unsigned)norb || (unsigned)l >= (unsigned)norb || (unsigned)kind > 1u) {
      dst[q] = __builtin_nan("");
      continue;
    }
    const double* rl = src + (size_t)l * M;
    double a = 0.0;
    for (int mu = 0; mu < M; ++mu) a += lamT[(size_t)mu * nop + k] * rl[mu];
    if (kind == 1) {
      const double* rk = src + (size_t)k * M;
      double b = 0.0;
      for (int mu = 0; mu < M; ++mu) b += lamT[(size_t)mu * nop + l] * rk[mu];
      a -= b;
    }
    dst[q] = a;
  }
}

hipError_t launch_rotation_grad(int P, int lam_off, int M, int nop, int norb, int64_t W, int npair,
                                const int* pairs, const double* lamT, const double* dl, const double* de,
                                double* odl, double* ode, hipStream_t s) {
  hipLaunchKernelGGL(k_rotation_grad, dim3((unsigned)W, 2), dim3(kRotT), 0, s, P, lam_off, M, nop, norb, npair,
                     pairs, lamT, dl, de, odl, ode);
  return hipGetLastError();
}

}  // namespace vbqmc
