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
// MFMA: a 512-thread workgroup owns a 128 x 128 block of one matrix, each
// wavefront a 32 x 64 part of it as 2 x 4 tiles of 16 x 16 (two wavefronts
// per SIMD), and walks the samples four at a time (one 16x16x4 k-step: six
// operand loads per lane for eight MFMAs), the operands of the next two
// k-steps in flight.  S' and H' are symmetric: only the blocks on and above
// the diagonal are formed, each element also written to its mirror.
// Operands come straight from the row-major per-sample arrays (16
// consecutive doubles per sample row per lane quarter); the sample sum runs
// in one fixed order, so the sums are reproducible, and each block adds its
// result to the elements it owns.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vbqmc {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kLmB = 128;  // block edge
constexpr int kLmRT = 2;   // 16-row tiles per wavefront (a wavefront owns 16 kLmRT x 64)
constexpr int kLmT = 64 * (kLmB / (16 * kLmRT)) * (kLmB / 64);  // threads per workgroup

// mat 0: S', 1: H', 2: D'.  acc: three (P+1) x (P+1) row-major matrices.
__global__ __launch_bounds__(kLmT) void k_lm_accumulate(int P, int64_t W, const double* __restrict__ O,
                                                         const double* __restrict__ D, const double* __restrict__ E,
                                                         const double* __restrict__ wt, double* __restrict__ acc) {
  const int P1 = P + 1;
  const int mat = blockIdx.z;
  // the symmetric products: blocks below the diagonal come from their mirrors
  if (mat < 2 && blockIdx.y > blockIdx.x) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int i0 = blockIdx.y * kLmB + 16 * kLmRT * (wave >> 1);  // rows of this wavefront's part
  const int j0 = blockIdx.x * kLmB + 64 * (wave & 1);           // columns
  v4d c[kLmRT][4];
#pragma unroll
  for (int rt = 0; rt < kLmRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) c[rt][ct][r] = 0.0;
  // operands of k-step k0 (samples k0 .. k0 + 3): the raw row entries and
  // the sample's weight and energy; the next step's are loaded while the
  // current step's MFMAs run
  auto load = [&](int64_t k0, double (&a)[kLmRT], double (&z)[4], double& w, double& e) {
    const int64_t k = k0 + kq;
    const bool kin = k < W;
    const int64_t kk = kin ? k : 0;
    w = kin ? (wt ? wt[kk] : 1.0) : 0.0;
    e = E[kk];
    const double* Ok = O + kk * P;
#pragma unroll
    for (int rt = 0; rt < kLmRT; ++rt) {  // A: X_ki
      const int i = i0 + 16 * rt + m;
      a[rt] = i < P1 ? (i > 0 ? Ok[i - 1] : 1.0) : 0.0;
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {  // B before scaling: X_kj or Y_kj (E_k^2 in column 0)
      const int j = j0 + 16 * ct + m;
      if (mat < 2) z[ct] = j < P1 ? (j > 0 ? Ok[j - 1] : 1.0) : 0.0;
      else z[ct] = j < P1 && j > 0 ? D[kk * P + j - 1] : 0.0;
    }
  };
  // two k-steps per pass, the next pass's operands in flight meanwhile
  double an[2][kLmRT], zn[2][4], wn[2], en[2];
  load(0, an[0], zn[0], wn[0], en[0]);
  load(4, an[1], zn[1], wn[1], en[1]);
  for (int64_t k0 = 0; k0 < W; k0 += 8) {
    double a[2][kLmRT], z[2][4], w[2], e[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int r = 0; r < kLmRT; ++r) a[h][r] = an[h][r];
#pragma unroll
      for (int r = 0; r < 4; ++r) z[h][r] = zn[h][r];
      w[h] = wn[h];
      e[h] = en[h];
    }
    if (k0 + 8 < W) load(k0 + 8, an[0], zn[0], wn[0], en[0]);
    if (k0 + 12 < W) load(k0 + 12, an[1], zn[1], wn[1], en[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (k0 + 4 * h >= W) break;  // (the same in every lane)
      const double sc = mat == 1 ? w[h] * e[h] : w[h];
      double b[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int j = j0 + 16 * ct + m;
        b[ct] = (mat == 2 && j == 0 ? e[h] * e[h] : z[h][ct]) * sc;
      }
#pragma unroll
      for (int rt = 0; rt < kLmRT; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          c[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][rt], b[ct], c[rt][ct], 0, 0, 0);
    }
  }
  // register q of lane l holds row 4 q + l / 16, column l % 16 of a tile
  double* out = acc + (size_t)mat * P1 * P1;
  const bool mirror = mat < 2 && blockIdx.y < blockIdx.x;
#pragma unroll
  for (int rt = 0; rt < kLmRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = i0 + 16 * rt + 4 * q + kq;
        const int col = j0 + 16 * ct + m;
        if (row < P1 && col < P1) {
          out[(size_t)row * P1 + col] += c[rt][ct][q];
          if (mirror) out[(size_t)col * P1 + row] += c[rt][ct][q];
        }
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
