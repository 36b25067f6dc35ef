// Device building blocks shared by the walker kernels and the adjoint kernel
// of the JVB library (gfx950).  See vbqmc_kernels.hip for the design notes.
#pragma once
#include <type_traits>

#include "vbqmc_internal.h"

namespace vbqmc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the counter layout of the walks:
// key = seed, counter = (walker slot, step, 4 * electron + purpose, draw).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox_pair(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                            uint32_t c3, double& u0, double& u1) {
  uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
    uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
    uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  const double s = 1.0 / 9007199254740992.0;
  u0 = (double)((((uint64_t)x1 << 32) | x0) >> 11) * s;
  u1 = (double)((((uint64_t)x3 << 32) | x2) >> 11) * s;
}

// ---------------------------------------------------------------------------
// block reductions (fixed order: identical results in every lane)
// ---------------------------------------------------------------------------
template <int NT, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  if constexpr (NT > 64) {
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int k = 0; k < K; ++k) red[(threadIdx.x >> 6) * K + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[w * K + k];
      v[k] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Jastrow pair function u(r) = a R/(1 + b R) + sum_{p=2..5} q_p R^p with
// R = r/(1 + kappa r); returns u, u' and u'' in r.  Coefficients travel by
// value so that a loop mixing electron and nucleus partners reads them from
// registers rather than through a per-lane pointer.
// ---------------------------------------------------------------------------
struct PairCoef {
  double a, b, q0, q1, q2, q3;
};

__device__ __forceinline__ PairCoef ee_coef(const DevWF& wf, bool anti) {
  return {anti ? wf.ee[0] : wf.ee[1], anti ? wf.ee[2] : wf.ee[3], wf.ee[4], wf.ee[5], wf.ee[6], wf.ee[7]};
}

__device__ __forceinline__ PairCoef en_coef(const double* e) { return {e[0], e[1], e[2], e[3], e[4], e[5]}; }

// 1 + bR = (den + b r) / den with den = 1 + kappa r, so the two reciprocals
// below are independent (they overlap instead of chaining).  K0: kappa is 0,
// so den = 1 and the first reciprocal is 1 (the same values, one division
// fewer).
template <bool K0 = false>
__device__ __forceinline__ void pair_fn(double r, double kappa, const PairCoef& c, double& u, double& u1,
                                        double& u2) {
  double den = K0 ? 1.0 : 1.0 + kappa * r;
  double iden = K0 ? 1.0 : 1.0 / den;
  double id2 = 1.0 / (den + c.b * r);
  double R = r * iden, R1 = iden * iden, R2 = -2.0 * kappa * R1 * iden;
  double ib = den * id2;
  u = c.a * R * ib;
  double uR = c.a * ib * ib;
  double uRR = -2.0 * c.a * c.b * ib * ib * ib;
  const double q[4] = {c.q0, c.q1, c.q2, c.q3};
  double Rp2 = 1.0;  // R^(p-2)
#pragma unroll
  for (int p = 2; p <= 5; ++p) {
    double cp = q[p - 2];
    uRR += p * (p - 1) * cp * Rp2;
    uR += p * cp * Rp2 * R;
    u += cp * Rp2 * R * R;
    Rp2 *= R;
  }
  u1 = uR * R1;
  u2 = uRR * R1 * R1 + uR * R2;
}

template <bool K0 = false>
__device__ __forceinline__ double pair_val(double r, double kappa, const PairCoef& c) {
  double den = K0 ? 1.0 : 1.0 + kappa * r;
  double R = K0 ? r : r / den;
  double u = c.a * r / (den + c.b * r);  // a R / (1 + b R), independent of the division above
  double R2 = R * R;
  return u + R2 * (c.q0 + R * (c.q1 + R * (c.q2 + R * c.q3)));
}

// ---------------------------------------------------------------------------
// Three-body Jastrow f_een (Sec. 2.1).  Term t of nucleus alpha adds, for
// every electron pair i < j,
//   c_t Rbar_ij^k (Rbar_ia^l + Rbar_ja^l) (Rbar_ia Rbar_ja)^m,  Rbar(r) = 1/(1 + kappa r),
// over the (k, l, m) with p = k + l + 2m from 2 to 5, k < p and l at most
// p - k (p - k - 2 when k = 0), listed by p, then k, then l.
// ---------------------------------------------------------------------------
constexpr int kEenK[kEenTerms] = {0, 1, 0, 1, 1, 2, 0, 0, 1, 1, 2, 2, 3, 0, 0, 1, 1, 1, 2, 2, 3, 3, 4};
constexpr int kEenL[kEenTerms] = {0, 1, 1, 0, 2, 1, 0, 2, 1, 3, 0, 2, 1, 1, 3, 0, 2, 4, 1, 3, 0, 2, 1};
constexpr int kEenM[kEenTerms] = {1, 0, 1, 1, 0, 0, 2, 1, 1, 0, 1, 0, 0, 2, 1, 2, 1, 0, 1, 0, 1, 0, 0};

// One (i, j, alpha) triple: F = sum_t c_t a^k B_t with a = Rbar_ij,
// B_t = b^(l+m) c^m + b^m c^(l+m), b = Rbar_ia, c = Rbar_ja, and (DERIV) its
// first and second partial derivatives in a and b (c does not depend on
// electron i).  cf: the 23 coefficients of nucleus alpha.
struct EenTriple {
  double F, Fa, Fb, Faa, Fbb, Fab;
};

template <bool DERIV>
__device__ __forceinline__ EenTriple een_triple(const double* __restrict__ cf, double a, double b, double c) {
  double pa[5], pb[6], pc[6];
  pa[0] = pb[0] = pc[0] = 1.0;
#pragma unroll
  for (int q = 1; q < 6; ++q) {
    if (q < 5) pa[q] = pa[q - 1] * a;
    pb[q] = pb[q - 1] * b;
    pc[q] = pc[q - 1] * c;
  }
  EenTriple o = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < kEenTerms; ++t) {
    const int k = kEenK[t], l = kEenL[t], m = kEenM[t], n = l + m;
    const double ct = cf[t];
    const double B = pb[n] * pc[m] + pb[m] * pc[n];
    o.F += ct * pa[k] * B;
    if (DERIV) {
      const double B1 = (n > 0 ? n * pb[n > 0 ? n - 1 : 0] * pc[m] : 0.0) +
                        (m > 0 ? m * pb[m > 0 ? m - 1 : 0] * pc[n] : 0.0);
      const double B2 = (n > 1 ? n * (n - 1) * pb[n > 1 ? n - 2 : 0] * pc[m] : 0.0) +
                        (m > 1 ? m * (m - 1) * pb[m > 1 ? m - 2 : 0] * pc[n] : 0.0);
      const double A1 = k > 0 ? k * pa[k > 0 ? k - 1 : 0] : 0.0;
      const double A2 = k > 1 ? k * (k - 1) * pa[k > 1 ? k - 2 : 0] : 0.0;
      o.Fa += ct * A1 * B;
      o.Faa += ct * A2 * B;
      o.Fb += ct * pa[k] * B1;
      o.Fbb += ct * pa[k] * B2;
      o.Fab += ct * A1 * B1;
    }
  }
  return o;
}

// f_een of electron i with one partner electron j, summed over the nuclei
// (nuc: [nnuc][4] x, y, z, Z): MODE 0 the value; 1 also the gradient in r_i;
// 2 also the Laplacian in r_i.  With a(r) = Rbar(r): a' = -kappa a^2,
// a'' = 2 kappa^2 a^3, grad_i a = a' d/|d| (d = r_i - r_j), lap_i a =
// a'' + 2 a'/|d|, and likewise b with e = r_i - R_alpha; the Laplacian of F
// adds the cross term 2 F_ab a' b' (d . e)/(|d| |e|).
template <int MODE>
__device__ __forceinline__ void een_partner(const DevWF& wf, const double* nuc, double xi, double yi, double zi,
                                            double xj, double yj, double zj, double& u, double* g, double& lap) {
  const double kap = wf.kappa;
  const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  const double rij = sqrt(dx * dx + dy * dy + dz * dz), irij = 1.0 / rij;
  const double a = 1.0 / (1.0 + kap * rij), a1 = -kap * a * a, a2 = 2.0 * kap * kap * a * a * a;
#pragma unroll 1
  for (int al = 0; al < wf.nnuc; ++al) {
    const double* A = nuc + 4 * al;
    const double ex = xi - A[0], ey = yi - A[1], ez = zi - A[2];
    const double fx = xj - A[0], fy = yj - A[1], fz = zj - A[2];
    const double ria = sqrt(ex * ex + ey * ey + ez * ez), iria = 1.0 / ria;
    const double b = 1.0 / (1.0 + kap * ria);
    const double c = 1.0 / (1.0 + kap * sqrt(fx * fx + fy * fy + fz * fz));
    const EenTriple T = een_triple<MODE >= 1>(wf.een + kEenTerms * al, a, b, c);
    u += T.F;
    if (MODE >= 1) {
      const double b1 = -kap * b * b;
      const double sa = T.Fa * a1 * irij, sb = T.Fb * b1 * iria;
      g[0] += sa * dx + sb * ex;
      g[1] += sa * dy + sb * ey;
      g[2] += sa * dz + sb * ez;
      if (MODE >= 2) {
        const double b2 = 2.0 * kap * kap * b * b * b;
        const double cosde = (dx * ex + dy * ey + dz * ez) * irij * iria;
        lap += T.Faa * a1 * a1 + T.Fa * (a2 + 2.0 * a1 * irij) + T.Fbb * b1 * b1 + T.Fb * (b2 + 2.0 * b1 * iria) +
               2.0 * T.Fab * a1 * b1 * cosde;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// basis functions: radial sums and the angular set
// ---------------------------------------------------------------------------
// e^{-t}, t >= 0, by Tang's table-driven method (ACM TOMS 15, 1989): with
// n = rint(-64 t / ln 2) = 64 m + j (0 <= j < 64), e^{-t} = 2^m 2^{j/64} e^r
// where r = -t - n ln2/64 (Cody-Waite, ln 2/64 in two parts) lies in
// [-ln2/128, ln2/128]; 2^{j/64} comes from the staged 64-entry table and
// e^r - 1 from its degree-5 Taylor polynomial (truncation below 4e-17
// relative), about 1.3 ulp in all.  Arguments past the range of a 32-bit n
// give 0 and NaN gives NaN; the table index always lies in 0..63.
template <typename T> __device__ __forceinline__ T exp_neg(T t, const double* etab);
template <> __device__ __forceinline__ double exp_neg<double>(double t, const double* etab) {
  const double n = __builtin_rint(t * -92.33248261689366);  // -64 / ln 2
  double r = __builtin_fma(-n, 0.010830424696249145, -t);  // ln 2 / 64, high part
  r = __builtin_fma(-n, 3.623510646634843e-19, r);          // low part
  const int k = (int)n;
  const double T2 = etab[k & 63];
  double q = __builtin_fma(r, 1.0 / 120.0, 1.0 / 24.0);
  q = __builtin_fma(q, r, 1.0 / 6.0);
  q = __builtin_fma(q, r, 0.5);
  q = __builtin_fma(q, r, 1.0);
  return __builtin_ldexp(__builtin_fma(T2, q * r, T2), k >> 6);
}
template <> __device__ __forceinline__ float exp_neg<float>(float t, const double*) { return expf(-t); }

// Two independent exp_neg evaluations with the same operations, arranged so
// that both table reads are in flight before either polynomial needs them.
template <typename T>
__device__ __forceinline__ void exp_neg2(T t0, T t1, const double* etab, T& e0, T& e1) {
  e0 = exp_neg<T>(t0, etab);
  e1 = exp_neg<T>(t1, etab);
}
template <>
__device__ __forceinline__ void exp_neg2<double>(double t0, double t1, const double* etab, double& e0, double& e1) {
  const double n0 = __builtin_rint(t0 * -92.33248261689366), n1 = __builtin_rint(t1 * -92.33248261689366);
  const int k0 = (int)n0, k1 = (int)n1;
  const double T0 = etab[k0 & 63], T1 = etab[k1 & 63];
  double r0 = __builtin_fma(-n0, 0.010830424696249145, -t0), r1 = __builtin_fma(-n1, 0.010830424696249145, -t1);
  r0 = __builtin_fma(-n0, 3.623510646634843e-19, r0);
  r1 = __builtin_fma(-n1, 3.623510646634843e-19, r1);
  double q0 = __builtin_fma(r0, 1.0 / 120.0, 1.0 / 24.0), q1 = __builtin_fma(r1, 1.0 / 120.0, 1.0 / 24.0);
  q0 = __builtin_fma(q0, r0, 1.0 / 6.0);
  q1 = __builtin_fma(q1, r1, 1.0 / 6.0);
  q0 = __builtin_fma(q0, r0, 0.5);
  q1 = __builtin_fma(q1, r1, 0.5);
  q0 = __builtin_fma(q0, r0, 1.0);
  q1 = __builtin_fma(q1, r1, 1.0);
  const double p0 = q0 * r0, p1 = q1 * r1;
  e0 = __builtin_ldexp(__builtin_fma(T0, p0, T0), k0 >> 6);
  e1 = __builtin_ldexp(__builtin_fma(T1, p1, T1), k1 >> 6);
}

// Radial sums of a shell: Gaussian (kind 0) g = sum c e^{-a r^2} with
// g1 = dg/d(r^2), g2 = d2g/d(r^2)^2; Slater (kind 1) g = sum c e^{-a r} with
// g1 = dg/dr, g2 = d2g/dr2.  Primitives whose exponent argument exceeds 50 are
// below 2e-22 of their coefficient and are skipped.

// channels of one basis function: 0 value, 1..3 gradient, 4 Laplacian
template <typename T>
__device__ __forceinline__ void channels(int kind, int l, int m, T x, T y, T z, T r2, T r, T g, T g1,
                                         T g2, int nch, T* out) {
  T P, Px = T(0), Py = T(0), Pz = T(0);
  if (l == 0) {
    P = T(1);
  } else if (l == 1) {
    P = m == 0 ? x : (m == 1 ? y : z);
    Px = m == 0 ? T(1) : T(0);
    Py = m == 1 ? T(1) : T(0);
    Pz = m == 2 ? T(1) : T(0);
  } else {
    switch (m) {
      case 0: P = x * y; Px = y; Py = x; break;
      case 1: P = y * z; Py = z; Pz = y; break;
      case 2: P = z * x; Px = z; Pz = x; break;
      case 3: P = x * x - y * y; Px = T(2) * x; Py = T(-2) * y; break;
      default: P = T(2) * z * z - x * x - y * y; Px = T(-2) * x; Py = T(-2) * y; Pz = T(4) * z;
    }
  }
  out[0] = P * g;
  if (nch == 1) return;
  // grad g = fr * d
  T fr = kind == 0 ? T(2) * g1 : g1 / r;
  out[1] = Px * g + P * fr * x;
  out[2] = Py * g + P * fr * y;
  out[3] = Pz * g + P * fr * z;
  if (nch < 5) return;
  // lap chi = P lap g + 2 grad P . grad g  (lap P = 0, d . grad P = l P)
  if (kind == 0)
    out[4] = P * (T(2 * (2 * l + 3)) * g1 + T(4) * r2 * g2);
  else
    out[4] = P * (g2 + T(2 * (l + 1)) * g1 / r);
}

// ---------------------------------------------------------------------------
// small e x e determinant algebra (e <= 3), matrices row-major with stride 3
// ---------------------------------------------------------------------------
__device__ __forceinline__ double det_e(int e, const double* m) {
  if (e == 0) return 1.0;
  if (e == 1) return m[0];
  if (e == 2) return m[0] * m[4] - m[1] * m[3];
  return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
         m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// y^T adj(m) b
__device__ __forceinline__ double adj_e(int e, const double* m, const double* y, const double* b) {
  if (e == 0) return 0.0;
  if (e == 1) return y[0] * b[0];
  if (e == 2) return y[0] * (m[4] * b[0] - m[1] * b[1]) + y[1] * (-m[3] * b[0] + m[0] * b[1]);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    int r1 = r == 0 ? 1 : 0, r2 = r == 2 ? 1 : 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int c1 = c == 0 ? 1 : 0, c2 = c == 2 ? 1 : 2;
      double cof = m[r1 * 3 + c1] * m[r2 * 3 + c2] - m[r1 * 3 + c2] * m[r2 * 3 + c1];
      if ((r + c) & 1) cof = -cof;
      s += y[c] * cof * b[r];  // adj[c][r] = cofactor[r][c]
    }
  }
  return s;
}

// gather T[J, Q] (+ optional rank-1 term bJ yQ / rho) of determinant u into m
// (stride 3).  Loops run to 3 with guards so that m stays in registers.
__device__ __forceinline__ int gather_u(const int* ui, const double* T, int nP, double* m,
                                        const double* bc, const double* y, double irho) {
  int e = ui[0];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (r < e && c < e) {
        double v = T[ui[1 + r] * nP + ui[4 + c]];
        if (bc) v += bc[ui[1 + r]] * y[ui[4 + c]] * irho;
        m[r * 3 + c] = v;
      }
  return e;
}

// ---------------------------------------------------------------------------
// LDS views.  The constant tables (basis, orbital coefficients when they fit,
// determinant tables) are staged once per block; the walker state and the
// scratch of each phase follow.
// ---------------------------------------------------------------------------
struct Ld {
  double* L;
  const DevWF& wf;
  double* bk = nullptr;  // backup area of the walker record (all-electron moves)
  __device__ Ld(double* l, const DevWF& w) : L(l), wf(w) {}
  // constant tables
  __device__ const int* fn() const { return (const int*)(L + wf.l_fn); }      // [Mpad][2], see FnInfo
  __device__ const int* sh() const { return (const int*)(L + wf.l_sh); }      // [nshell][8]
  __device__ const double* pe() const { return L + wf.l_pe; }
  __device__ const double* pc() const { return L + wf.l_pc; }
  __device__ const double* nuc() const { return L + wf.l_nuc; }
  __device__ const double* en() const { return L + wf.l_en; }
  __device__ const int* psh() const { return (const int*)(L + wf.l_psh); }
  __device__ const int* ref(int s) const { return (const int*)(L + wf.l_ref[s]); }
  __device__ const int* porb(int s) const { return (const int*)(L + wf.l_porb[s]); }
  __device__ const int* ui(int s) const { return (const int*)(L + wf.l_ui[s]); }
  __device__ const int* wrow(int s) const { return (const int*)(L + wf.l_wrow[s]); }
  __device__ const int* woth(int s) const { return (const int*)(L + wf.l_woth[s]); }
  __device__ const double* wcoef(int s) const { return L + wf.l_wcoef[s]; }
  __device__ const int* srow() const { return (const int*)(L + wf.l_srow); }
  __device__ const int* slu() const { return (const int*)(L + wf.l_slu); }
  __device__ const double* slc() const { return L + wf.l_slc; }
  template <typename T> __device__ const T* lam() const;
  // walker state
  __device__ double* R() const { return L + wf.l_R; }
  __device__ double* B(int s) const { return L + wf.l_B[s]; }
  __device__ double* T(int s) const { return L + wf.l_T[s]; }
  __device__ double* PP(int s) const { return L + wf.l_PP[s]; }
  __device__ double* Ru(int s) const { return L + wf.l_Ru[s]; }
  __device__ double* Wu(int s) const { return L + wf.l_Wu[s]; }
  __device__ double* Qu() const { return L + wf.l_Qu; }
  __device__ double* sc() const { return L + wf.l_sc; }
  __device__ double* red() const { return L + wf.l_red; }
  __device__ int* ipiv() const { return (int*)(L + wf.l_ipiv); }
  __device__ double* f() const { return L + wf.l_f; }
  __device__ double* gU() const { return L + wf.l_gU; }
  __device__ double* lU() const { return L + wf.l_lU; }
  __device__ double* gD() const { return L + wf.l_gD; }
  __device__ double* lD() const { return L + wf.l_lD; }
  __device__ double* disp() const { return L + wf.l_disp; }
  __device__ double* gtab() const { return L + wf.l_gtab; }
  __device__ double* pt() const { return L + wf.l_pt; }
  __device__ double* Phi() const { return L + wf.l_Phi; }
  __device__ double* part() const { return L + wf.l_part; }
  __device__ double* chi() const { return L + wf.l_chi; }
  __device__ double* v() const { return L + wf.l_v; }
  __device__ double* y() const { return L + wf.l_y; }
  __device__ double* bcol() const { return L + wf.l_bcol; }
  __device__ double* z() const { return L + wf.l_z; }
  __device__ double* yb() const { return L + wf.l_yb; }
  __device__ double* sij() const { return L + wf.l_sij; }
  __device__ double* ratio() const { return L + wf.l_ratio; }
  __device__ double* Rp() const { return L + wf.l_Rp; }
  __device__ double* ua() const { return L + wf.l_ua; }
  __device__ double* Vn() const { return L + wf.l_Vn; }
};
// basis function mu of the staged function table: shell (-1 for padding),
// angular index m, l, kind (0 Gaussian, 1 Slater) and center, from one load
struct FnInfo {
  int sh, m, lq, kind, nuc;
};
__device__ __forceinline__ FnInfo fn_decode(int2 w) { return {w.x, w.y & 15, (w.y >> 4) & 3, (w.y >> 6) & 1, w.y >> 8}; }
__device__ __forceinline__ int2 fn_word(const Ld& l, int mu) { return ((const int2*)l.fn())[mu]; }
__device__ __forceinline__ FnInfo fn_info(const Ld& l, int mu) { return fn_decode(fn_word(l, mu)); }

template <> __device__ const double* Ld::lam<double>() const {
  return wf.lam_in_lds ? (const double*)(L + wf.l_lam) : wf.lamT;
}
template <> __device__ const float* Ld::lam<float>() const {
  return wf.lam_in_lds ? (const float*)(L + wf.l_lam) : wf.lamT32;
}
template <> __device__ const uint16_t* Ld::lam<uint16_t>() const {
  return wf.lam_in_lds ? (const uint16_t*)(L + wf.l_lam) : wf.lamT16;
}

__device__ __forceinline__ int spin_of(const DevWF& wf, int i) { return i < wf.nup ? 0 : 1; }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int NT, typename T>
__device__ __forceinline__ void stage(T* dst, const T* src, int n) {
  for (int k = threadIdx.x; k < n; k += NT) dst[k] = src[k];
}

// copy the constant tables into LDS (once per block): one contiguous image
// laid out as the LDS table region, in the context's precision
template <int NT, int PREC>
__device__ void stage_tables(const DevWF& wf, const Ld& l) {
  const double* __restrict__ src = wf.timg;
  double* dst = l.L;
  const int n = wf.timg_len;
  int k = threadIdx.x;
  for (; k + 3 * NT < n; k += 4 * NT) {
    double a0 = src[k], a1 = src[k + NT], a2 = src[k + 2 * NT], a3 = src[k + 3 * NT];
    dst[k] = a0; dst[k + NT] = a1; dst[k + 2 * NT] = a2; dst[k + 3 * NT] = a3;
  }
  for (; k < n; k += NT) dst[k] = src[k];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// AO -> orbital contraction for a tile of up to 16 electrons on MFMA.
// group_radial fills, per electron of the tile, the displacement to every
// nucleus and the radial sums of every shell; group_channel then builds the
// A operand (basis channel c at electron e, function mu) on the fly from those
// tables and contracts it with lambda^T, one 16x16 output tile at a time,
// writing Phi[e][p] (FP64) for channel c.
// ---------------------------------------------------------------------------
// Row strides of the tile tables, odd so that the 16 rows of a tile fall in
// distinct LDS banks.
__device__ __forceinline__ int disp_stride(const DevWF& wf) { return 4 * wf.nnuc + 1; }
template <int GS>
__device__ __forceinline__ int gtab_stride(const DevWF& wf) { return (GS * wf.nshell) | 1; }

// Radial sums of a row tile on one 64-lane block, from a staged radial
// schedule of NB bins: lane l takes electron l % (64 / NB) and bin
// l / (64 / NB) and walks the bin's primitives two at a time in a loop of
// fixed length (16 electrons per pass with four bins; eight bins serve a tile
// of at most 8 rows in about half the steps).  The two exponentials of a step
// are independent (arguments past the cutoff are clamped and their terms
// dropped afterwards), and the schedule entries and operands of the next step
// are loaded while they are evaluated.  Each shell's sum is accumulated in the
// order of its primitives, restarting at its first one, whatever the bin, and
// the running sum is stored at every entry, so that the loop body has no
// branch: the last store of a shell holds its whole sum (padding entries
// repeat the bin's last shell and add nothing).  Rows past the electrons of
// the pass hold sums the tile passes never read (their basis values are set
// to zero, or their outputs dropped, by the passes themselves).
template <int PREC, int GS, bool STO, int NB>
__device__ __forceinline__ void radial_bins(const DevWF& wf, const Ld& l) {
  // each term is rounded before it is added, in every kernel: the value rows
  // of an inverse refresh and of the local energy then agree bit for bit
#pragma clang fp contract(off)
  typedef typename std::conditional<PREC == 0, double, float>::type T;
  constexpr int EP = 64 / NB;  // electrons per pass
  const int e = threadIdx.x & (EP - 1);
  const T* de = (const T*)l.disp() + e * disp_stride(wf);
  T* o = (T*)l.gtab() + e * gtab_stride<GS>(wf);
  const unsigned* sc = (const unsigned*)(l.L + (NB == 4 ? wf.l_rsched : wf.l_rsched8)) + (threadIdx.x / EP);
  const int len = NB == 4 ? wf.rsched_len : wf.rsched_len8;
  const double* pe = l.pe();
  const double* pc = l.pc();
  const double* etab = l.L + wf.l_etab;
  auto nuc = [](unsigned f) { return (int)((f >> kRsNucShift) & kRsNucMask); };
  unsigned n0 = sc[0], n1 = sc[NB], m0 = sc[2 * NB], m1 = sc[3 * NB];
  double a0 = pe[n0 & kRsPrim], c0 = pc[n0 & kRsPrim];
  double a1 = pe[n1 & kRsPrim], c1 = pc[n1 & kRsPrim];
  T d0 = de[4 * nuc(n0) + 3], d1 = de[4 * nuc(n1) + 3];
  T g = 0, g1 = 0, g2 = 0;
  auto add = [&](T ex, T a, unsigned f) {
    const bool first = f & kRsFirst;
    g = (first ? T(0) : g) + ex;
    if constexpr (GS == 3) {
      g1 = (first ? T(0) : g1) - a * ex;
      g2 = (first ? T(0) : g2) + a * a * ex;
    }
    T* q = o + GS * (int)((f >> kRsShift) & kRsShMask);
    q[0] = g;
    if constexpr (GS == 3) {
      q[1] = g1;
      q[2] = g2;
    }
  };
#pragma unroll 2
  for (int j = 0; j < len; j += 2) {
    const unsigned f0 = n0, f1 = n1;
    const T A0 = (T)a0, C0 = (T)c0, R0 = d0, A1 = (T)a1, C1 = (T)c1, R1 = d1;
    n0 = m0;
    n1 = m1;
    m0 = sc[NB * (j + 4)];
    m1 = sc[NB * (j + 5)];
    a0 = pe[n0 & kRsPrim];
    c0 = pc[n0 & kRsPrim];
    a1 = pe[n1 & kRsPrim];
    c1 = pc[n1 & kRsPrim];
    d0 = de[4 * nuc(n0) + 3];
    d1 = de[4 * nuc(n1) + 3];
    T t0 = A0 * R0, t1 = A1 * R1;
    if constexpr (STO) {
      if (f0 & kRsSto) t0 = A0 * (T)sqrt(R0);
      if (f1 & kRsSto) t1 = A1 * (T)sqrt(R1);
    }
    T ex0, ex1;
    exp_neg2<T>(fmin(t0, T(64)), fmin(t1, T(64)), etab, ex0, ex1);
    const T x0 = C0 * ex0, x1 = C1 * ex1;
    add(((f0 & kRsLive) && t0 < T(50)) ? x0 : T(0), A0, f0);
    add(((f1 & kRsLive) && t1 < T(50)) ? x1 : T(0), A1, f1);
  }
}

template <int NT, int PREC, int GS = 3>
__device__ void group_radial(const DevWF& wf, const Ld& l, const double* Rsrc, int g0, int ne) {
  typedef typename std::conditional<PREC == 0, double, float>::type T;
  T* disp = (T*)l.disp();  // [16][stride]: per nucleus x, y, z, r2
  T* gt = (T*)l.gtab();    // [16][stride]: per shell g (and g1, g2 when GS = 3)
  const int ds = disp_stride(wf), gs = gtab_stride<GS>(wf);
  for (int idx = threadIdx.x; idx < kGroup * wf.nnuc; idx += NT) {
    int e = idx / wf.nnuc, a = idx - e * wf.nnuc;
    T x = 0, y = 0, z = 0;
    if (e < ne) {
      x = (T)(Rsrc[3 * (g0 + e)] - l.nuc()[4 * a]);
      y = (T)(Rsrc[3 * (g0 + e) + 1] - l.nuc()[4 * a + 1]);
      z = (T)(Rsrc[3 * (g0 + e) + 2] - l.nuc()[4 * a + 2]);
    }
    T* d = disp + e * ds + 4 * a;
    d[0] = x; d[1] = y; d[2] = z;
    d[3] = x * x + y * y + z * z;
  }
  __syncthreads();
  if constexpr (NT == 64) {
    if (wf.rsched_len > 0 && wf.l_rsched < wf.timg_len) {
      if (ne <= 8 && wf.rsched_len8 > 0) {
        if (wf.rsched_sto) radial_bins<PREC, GS, true, 8>(wf, l);
        else radial_bins<PREC, GS, false, 8>(wf, l);
      } else {
        if (wf.rsched_sto) radial_bins<PREC, GS, true, 4>(wf, l);
        else radial_bins<PREC, GS, false, 4>(wf, l);
      }
      __syncthreads();
      return;
    }
  }
  {
#pragma clang fp contract(off)
    for (int idx = threadIdx.x; idx < kGroup * wf.nshell; idx += NT) {
      int e = idx / wf.nshell, sh = idx - e * wf.nshell;
      const int* si = l.sh() + 8 * sh;
      T r2 = disp[e * ds + 4 * si[0] + 3], r = sqrt(r2);
      T g = 0, g1 = 0, g2 = 0;
      if (e < ne) {
#pragma unroll 2
        for (int k = 0; k < si[5]; ++k) {
          T a = (T)l.pe()[si[4] + k];
          T t = si[1] == 0 ? a * r2 : a * r;
          if (t < T(50)) {
            T ex = (T)l.pc()[si[4] + k] * exp_neg<T>(t, l.L + wf.l_etab);
            g += ex;
            if constexpr (GS == 3) {
              g1 -= a * ex;
              g2 += a * a * ex;
            }
          }
        }
      }
      T* o = gt + e * gs + GS * sh;
      o[0] = g;
      if constexpr (GS == 3) {
        o[1] = g1;
        o[2] = g2;
      }
    }
  }
  __syncthreads();
}

// operands of basis function fi at electron e of the tile: displacement from
// its center and the radial sums of its shell (padding functions read shell 0
// and evaluate to zero), loaded apart from the arithmetic so that a pass can
// issue the loads of all its functions first
template <typename T>
struct ChanIn {
  T x, y, z, r2, g, g1, g2;
};
template <typename T, int GS = 3>
__device__ __forceinline__ ChanIn<T> chan_load(const DevWF& wf, const Ld& l, int e, const FnInfo& fi) {
  const T* d = (const T*)l.disp() + e * disp_stride(wf) + 4 * fi.nuc;
  const T* gg = (const T*)l.gtab() + e * gtab_stride<GS>(wf) + GS * max(fi.sh, 0);
  ChanIn<T> in{d[0], d[1], d[2], d[3], gg[0], T(0), T(0)};
  if constexpr (GS == 3) {
    in.g1 = gg[1];
    in.g2 = gg[2];
  }
  return in;
}

// basis channel c (0 value, 1..3 gradient, 4 Laplacian) of function fi from
// its operands
template <typename T>
__device__ __forceinline__ T chan_eval(const FnInfo& fi, const ChanIn<T>& in, int c) {
  const int m = fi.m, kind = fi.kind, lq = fi.lq;
  const T x = in.x, y = in.y, z = in.z, r2 = in.r2, g = in.g, g1 = in.g1, g2 = in.g2;
  if (c == 0) {
    // the value by selects, without a branch: angular factor 1 (s); x, y, z
    // (p); xy, yz, zx, x^2 - y^2, 2z^2 - x^2 - y^2 (d) as u v (doubled for
    // m = 4) less the squares that apply
    const T p1 = m == 0 ? x : (m == 1 ? y : z);
    const T u = m == 1 ? y : ((m == 2 || m == 4) ? z : x);
    const T v = m == 0 ? y : ((m == 1 || m == 4) ? z : x);
    T p2 = m == 4 ? T(2) * (u * v) : u * v;
    p2 = p2 - (m == 4 ? x * x : T(0));
    p2 = p2 - (m >= 3 ? y * y : T(0));
    const T P = lq == 0 ? T(1) : (lq == 1 ? p1 : p2);
    return fi.sh < 0 ? T(0) : P * g;
  }
  if (fi.sh < 0) return T(0);
  T P, Px = T(0), Py = T(0), Pz = T(0);
  if (lq == 0) {
    P = T(1);
  } else if (lq == 1) {
    P = m == 0 ? x : (m == 1 ? y : z);
    Px = m == 0 ? T(1) : T(0);
    Py = m == 1 ? T(1) : T(0);
    Pz = m == 2 ? T(1) : T(0);
  } else {
    switch (m) {
      case 0: P = x * y; Px = y; Py = x; break;
      case 1: P = y * z; Py = z; Pz = y; break;
      case 2: P = z * x; Px = z; Pz = x; break;
      case 3: P = x * x - y * y; Px = T(2) * x; Py = T(-2) * y; break;
      default: P = T(2) * z * z - x * x - y * y; Px = T(-2) * x; Py = T(-2) * y; Pz = T(4) * z;
    }
  }
  if (kind == 0) {
    if (c == 4) return P * (T(2 * (2 * lq + 3)) * g1 + T(4) * r2 * g2);
    T fr = T(2) * g1;
    if (c == 1) return Px * g + P * fr * x;
    if (c == 2) return Py * g + P * fr * y;
    return Pz * g + P * fr * z;
  }
  T r = sqrt(r2);
  if (c == 4) return P * (g2 + T(2 * (lq + 1)) * g1 / r);
  T fr = g1 / r;
  if (c == 1) return Px * g + P * fr * x;
  if (c == 2) return Py * g + P * fr * y;
  return Pz * g + P * fr * z;
}

// basis channel c of function fi at electron e of the tile
template <typename T, int GS = 3>
__device__ __forceinline__ T chan_value_fi(const DevWF& wf, const Ld& l, int e, const FnInfo& fi, int c) {
  if (fi.sh < 0) return T(0);
  return chan_eval<T>(fi, chan_load<T, GS>(wf, l, e, fi), c);
}

template <typename T, int GS = 3>
__device__ __forceinline__ T chan_value(const DevWF& wf, const Ld& l, int e, int mu, int c) {
  return chan_value_fi<T, GS>(wf, l, e, fn_info(l, mu), c);
}

// Writes rows e < nout_rows of the tile (all 16 by default).  With a column
// map (cmap[spin][orbital] = position or -1, rows grow0 + e below rsplit of
// spin 0) only the mapped columns are stored, row e at out + e * ostride.
template <int NT, int PREC, int GS = 3>
__device__ void group_channel(const DevWF& wf, const Ld& l, int ne, int c, double* out = nullptr,
                              int nout_rows = kGroup, const int* cmap = nullptr, int ostride = 0, int grow0 = 0,
                              int rsplit = 0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  const int nct = wf.nop / 16;
  double* Phi = out ? out : l.Phi();
  for (int ct = wave; ct < nct; ct += NW) {
    const int col = ct * 16 + (lane & 15);
    const int e = lane & 15;
    const bool live = e < ne;
    auto put = [&](int row, double v) {
      if (row >= nout_rows) return;
      if (cmap) {
        const int p = cmap[(grow0 + row < rsplit ? 0 : wf.nop) + col];
        if (p >= 0) Phi[row * ostride + p] = v;
      } else {
        Phi[row * wf.nop + col] = v;
      }
    };
    if constexpr (PREC == 0) {
      const double* lam = l.lam<double>();
      v4d acc = {0, 0, 0, 0};
      // Mpad is a multiple of 16: four k-steps per pass, their table lookups
      // and coefficient loads issued before the MFMAs (same accumulation
      // order); the function words of the next pass are loaded one pass ahead
      int2 wd[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) wd[u] = fn_word(l, 4 * u + (lane >> 4));
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        double a[4], b[4];
        FnInfo fi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          fi[u] = fn_decode(wd[u]);
          wd[u] = fn_word(l, min(k0 + 16, wf.Mpad - 16) + 4 * u + (lane >> 4));
        }
        ChanIn<double> in[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * u + (lane >> 4);
          in[u] = chan_load<double, GS>(wf, l, e, fi[u]);
          b[u] = lam[(size_t)k * wf.nop + col];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = live ? chan_eval<double>(fi[u], in[u], c) : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
      }
      // f64 16x16x4 output: register r of lane l holds row 4r + l/16
#pragma unroll
      for (int r = 0; r < 4; ++r) put(4 * r + (lane >> 4), acc[r]);
    } else if constexpr (PREC == 1) {
      const float* lam = l.lam<float>();
      v4f acc = {0, 0, 0, 0};
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        float a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * u + (lane >> 4);
          a[u] = live ? chan_value<float, GS>(wf, l, e, k, c) : 0.f;
          b[u] = lam[(size_t)k * wf.nop + col];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
      }
      // f32 output: register r of lane l holds row 4(l/16) + r
#pragma unroll
      for (int r = 0; r < 4; ++r) put(4 * (lane >> 4) + r, (double)acc[r]);
    } else {
      const uint16_t* lam = l.lam<uint16_t>();
      v4f acc = {0, 0, 0, 0};
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        int kb = k0 + 4 * (lane >> 4);
        v4s a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          a[j] = (short)(live ? f2bf(chan_value<float, GS>(wf, l, e, kb + j, c)) : (uint16_t)0);
          b[j] = (short)lam[(size_t)(kb + j) * wf.nop + col];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) put(4 * (lane >> 4) + r, (double)acc[r]);
    }
  }
  __syncthreads();
}

// Channels 1..4 (gradient x, y, z and Laplacian) of function fi from its
// operands (radial sums with both derivatives).
template <typename T>
__device__ __forceinline__ void chan_eval4(const FnInfo& fi, const ChanIn<T>& in, T (&o)[4]) {
  if (fi.sh < 0) {
    o[0] = o[1] = o[2] = o[3] = T(0);
    return;
  }
  const int m = fi.m, kind = fi.kind, lq = fi.lq;
  const T x = in.x, y = in.y, z = in.z, r2 = in.r2, g = in.g, g1 = in.g1, g2 = in.g2;
  T P, Px = T(0), Py = T(0), Pz = T(0);
  if (lq == 0) {
    P = T(1);
  } else if (lq == 1) {
    P = m == 0 ? x : (m == 1 ? y : z);
    Px = m == 0 ? T(1) : T(0);
    Py = m == 1 ? T(1) : T(0);
    Pz = m == 2 ? T(1) : T(0);
  } else {
    switch (m) {
      case 0: P = x * y; Px = y; Py = x; break;
      case 1: P = y * z; Py = z; Pz = y; break;
      case 2: P = z * x; Px = z; Pz = x; break;
      case 3: P = x * x - y * y; Px = T(2) * x; Py = T(-2) * y; break;
      default: P = T(2) * z * z - x * x - y * y; Px = T(-2) * x; Py = T(-2) * y; Pz = T(4) * z;
    }
  }
  T fr, lap;
  if (kind == 0) {
    fr = T(2) * g1;
    lap = P * (T(2 * (2 * lq + 3)) * g1 + T(4) * r2 * g2);
  } else {
    T r = sqrt(r2);
    fr = g1 / r;
    lap = P * (g2 + T(2 * (lq + 1)) * g1 / r);
  }
  o[0] = Px * g + P * fr * x;
  o[1] = Py * g + P * fr * y;
  o[2] = Pz * g + P * fr * z;
  o[3] = lap;
}
template <typename T>
__device__ __forceinline__ void chan_value4_fi(const DevWF& wf, const Ld& l, int e, const FnInfo& fi, T (&o)[4]) {
  if (fi.sh < 0) {
    o[0] = o[1] = o[2] = o[3] = T(0);
    return;
  }
  chan_eval4<T>(fi, chan_load<T, 3>(wf, l, e, fi), o);
}

template <typename T>
__device__ __forceinline__ void chan_value4(const DevWF& wf, const Ld& l, int e, int mu, T (&o)[4]) {
  chan_value4_fi<T>(wf, l, e, fn_info(l, mu), o);
}

// All four derivative channels of a tile in one pass: out[c][e][p] for
// c = 0..3 (gradient x, y, z, Laplacian), rows e < ne.
template <int NT, int PREC>
__device__ void group_channels4(const DevWF& wf, const Ld& l, int ne, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  const int nct = wf.nop / 16;
  const size_t cst = (size_t)kGroup * wf.nop;
  for (int ct = wave; ct < nct; ct += NW) {
    const int col = ct * 16 + (lane & 15);
    const int e = lane & 15;
    const bool live = e < ne;
    if constexpr (PREC == 0) {
      const double* lam = l.lam<double>();
      v4d acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = v4d{0, 0, 0, 0};
      int2 wd[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) wd[u] = fn_word(l, 4 * u + (lane >> 4));
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        double a[4][4], b[4];
        FnInfo fi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          fi[u] = fn_decode(wd[u]);
          wd[u] = fn_word(l, min(k0 + 16, wf.Mpad - 16) + 4 * u + (lane >> 4));
        }
        ChanIn<double> in[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * u + (lane >> 4);
          in[u] = chan_load<double, 3>(wf, l, e, fi[u]);
          b[u] = lam[(size_t)k * wf.nop + col];
        }
        // (rows past ne are evaluated too: their outputs are not stored)
#pragma unroll
        for (int u = 0; u < 4; ++u) chan_eval4<double>(fi[u], in[u], a[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][c], b[u], acc[c], 0, 0, 0);
      }
      // f64 16x16x4 output: register r of lane l holds row 4r + l/16
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * r + (lane >> 4) < ne) out[c * cst + (4 * r + (lane >> 4)) * wf.nop + col] = acc[c][r];
    } else if constexpr (PREC == 1) {
      const float* lam = l.lam<float>();
      v4f acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = v4f{0, 0, 0, 0};
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        float a[4][4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * u + (lane >> 4);
          a[u][0] = a[u][1] = a[u][2] = a[u][3] = 0.f;
          if (live) chan_value4<float>(wf, l, e, k, a[u]);
          b[u] = lam[(size_t)k * wf.nop + col];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][c], b[u], acc[c], 0, 0, 0);
      }
      // f32 output: register r of lane l holds row 4(l/16) + r
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * (lane >> 4) + r < ne) out[c * cst + (4 * (lane >> 4) + r) * wf.nop + col] = (double)acc[c][r];
    } else {
      const uint16_t* lam = l.lam<uint16_t>();
      v4f acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = v4f{0, 0, 0, 0};
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        int kb = k0 + 4 * (lane >> 4);
        v4s a[4], b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float v[4] = {0.f, 0.f, 0.f, 0.f};
          if (live) chan_value4<float>(wf, l, e, kb + j, v);
#pragma unroll
          for (int c = 0; c < 4; ++c) a[c][j] = (short)f2bf(v[c]);
          b[j] = (short)lam[(size_t)(kb + j) * wf.nop + col];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[c], b, acc[c], 0, 0, 0);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * (lane >> 4) + r < ne) out[c * cst + (4 * (lane >> 4) + r) * wf.nop + col] = (double)acc[c][r];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// In-place Gauss-Jordan inverse with partial pivoting of the n x n matrix A
// (rows electrons, columns reference slots) -> A^{-1} (rows slots, columns
// electrons).  Returns false if a pivot is exactly zero.
// ---------------------------------------------------------------------------
template <int NT>
__device__ bool gj_invert(const Ld& l, double* A, int n, double& logdet, double& sgn) {
  int* piv = l.ipiv();
  double* f = l.f();
  double* sc = l.sc();
  logdet = 0.0;
  sgn = 1.0;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x < 64) {
      int lane = threadIdx.x;
      double best = -1.0;
      int bi = n;
      for (int i = k + lane; i < n; i += 64) {
        double v = fabs(A[i * n + k]);
        if (v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        double ob = __shfl_xor(best, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        piv[k] = bi;
        sc[SC_TMP3] = best;
      }
    }
    __syncthreads();
    int p = piv[k];
    if (!(sc[SC_TMP3] > 0.0)) {
      __syncthreads();
      return false;
    }
    if (p != k)
      for (int j = threadIdx.x; j < n; j += NT) {
        double t = A[k * n + j];
        A[k * n + j] = A[p * n + j];
        A[p * n + j] = t;
      }
    __syncthreads();
    double pv = A[k * n + k];
    logdet += log(fabs(pv));
    if (pv < 0) sgn = -sgn;
    if (p != k) sgn = -sgn;
    for (int i = threadIdx.x; i < n; i += NT) f[i] = A[i * n + k];
    __syncthreads();
    double ip = 1.0 / pv;
    for (int j = threadIdx.x; j < n; j += NT) A[k * n + j] = (j == k ? 1.0 : A[k * n + j]) * ip;
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * n; idx += NT) {
      int i = idx / n, j = idx - i * n;
      if (i != k) A[idx] = (j == k ? 0.0 : A[idx]) - f[i] * A[k * n + j];
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    int p = piv[k];
    if (p != k)
      for (int i = threadIdx.x; i < n; i += NT) {
        double t = A[i * n + k];
        A[i * n + k] = A[i * n + p];
        A[i * n + p] = t;
      }
    __syncthreads();
  }
  return true;
}

// ---------------------------------------------------------------------------
// Determinant-table bookkeeping: R_u = det(T[J,Q]), W_u = sum over the pairs
// holding u of w_k R_{other}, S = sum_k w_k R_up R_dn = sum_u R_u W_u.
// ---------------------------------------------------------------------------
template <int NT>
__device__ void update_R(const DevWF& wf, const Ld& l, int s) {
  const SpinTab& st = wf.sp[s];
  for (int u = threadIdx.x; u < st.nU; u += NT) {
    double m[9];
    int e = gather_u(l.ui(s) + 8 * u, l.T(s), st.nP, m, nullptr, nullptr, 0.0);
    l.Ru(s)[u] = det_e(e, m);
  }
}

template <int NT>
__device__ void update_W(const DevWF& wf, const Ld& l, int s) {
  const SpinTab& st = wf.sp[s];
  const double* Ro = l.Ru(1 - s);
  const int* wr = l.wrow(s);
  const int* wo = l.woth(s);
  const double* wc = l.wcoef(s);
  for (int u = threadIdx.x; u < st.nU; u += NT) {
    double w = 0.0;
    for (int k = wr[u]; k < wr[u + 1]; ++k) w += wc[k] * Ro[wo[k]];
    l.Wu(s)[u] = w;
  }
}

template <int NT>
__device__ void update_S(const DevWF& wf, const Ld& l) {
  double v[1] = {0.0};
  for (int u = threadIdx.x; u < wf.sp[0].nU; u += NT) v[0] += l.Ru(0)[u] * l.Wu(0)[u];
  block_sum<NT, 1>(v, l.red());
  if (threadIdx.x == 0) l.sc()[SC_S] = v[0];
  __syncthreads();
}

template <int NT>
__device__ void compute_RWS(const DevWF& wf, const Ld& l) {
  update_R<NT>(wf, l, 0);
  update_R<NT>(wf, l, 1);
  __syncthreads();
  update_W<NT>(wf, l, 0);
  update_W<NT>(wf, l, 1);
  __syncthreads();
  update_S<NT>(wf, l);
}

// Invert the staged reference matrices (in B) and form T = B PP, per spin.
template <int NT>
__device__ bool finish_state(const DevWF& wf, const Ld& l) {
  bool ok = true;
  for (int s = 0; s < 2; ++s) {
    const SpinTab& st = wf.sp[s];
    double ld = 0.0, sg = 1.0;
    if (st.n > 0 && !gj_invert<NT>(l, l.B(s), st.n, ld, sg)) ok = false;
    if (threadIdx.x == 0) {
      l.sc()[SC_LOGDET0 + s] = ld;
      l.sc()[SC_SGN0 + s] = sg;
      l.sc()[SC_NUPD0 + s] = 0.0;
    }
    for (int idx = threadIdx.x; idx < st.n * st.nP; idx += NT) {
      int j = idx / st.nP, q = idx - j * st.nP;
      double a = 0.0;
      for (int i = 0; i < st.n; ++i) a += l.B(s)[j * st.n + i] * l.PP(s)[i * st.nP + q];
      l.T(s)[idx] = a;
    }
    __syncthreads();
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Fresh reference inverses and tables from positions Rsrc (values pass on
// MFMA + Gauss-Jordan).  Returns false on an exactly singular reference.
// ---------------------------------------------------------------------------
template <int NT, int PREC, int GS = 3>
__device__ bool build_state(const DevWF& wf, const Ld& l, const double* Rsrc, double* rows = nullptr) {
  double* Phi = rows ? rows : l.Phi();  // 16 x nop scratch rows
  for (int g0 = 0; g0 < wf.N; g0 += kGroup) {
    int ne = min(kGroup, wf.N - g0);
    group_radial<NT, PREC, GS>(wf, l, Rsrc, g0, ne);
    group_channel<NT, PREC, GS>(wf, l, ne, 0, Phi, ne);
    for (int s = 0; s < 2; ++s) {
      const SpinTab& st = wf.sp[s];
      int w = st.n + st.nP;
      for (int idx = threadIdx.x; idx < ne * w; idx += NT) {
        int e = idx / w, j = idx - e * w, i = g0 + e;
        if (spin_of(wf, i) != s) continue;
        int il = i - st.e0;
        if (j < st.n)
          l.B(s)[il * st.n + j] = Phi[e * wf.nop + l.ref(s)[j]];
        else
          l.PP(s)[il * st.nP + (j - st.n)] = Phi[e * wf.nop + l.porb(s)[j - st.n]];
      }
    }
    __syncthreads();
  }
  return finish_state<NT>(wf, l);
}

// ---------------------------------------------------------------------------
// Jastrow factor and potential for all electrons: U, grad_i U, lap_i U, V
// (EEN: with the three-body term f_een).
// ---------------------------------------------------------------------------
template <int NT, bool EEN = false>
__device__ void jastrow_full(const DevWF& wf, const Ld& l, const double* Rsrc) {
  double part[2] = {0.0, 0.0};  // U, V
  const double* nuc = l.nuc();
  for (int i = threadIdx.x; i < wf.N; i += NT) {
    double xi = Rsrc[3 * i], yi = Rsrc[3 * i + 1], zi = Rsrc[3 * i + 2];
    double gx = 0, gy = 0, gz = 0, lap = 0, Ui = 0, Vi = 0;
    for (int a = 0; a < wf.nnuc; ++a) {
      double dx = xi - nuc[4 * a], dy = yi - nuc[4 * a + 1], dz = zi - nuc[4 * a + 2];
      double r = sqrt(dx * dx + dy * dy + dz * dz), ir = 1.0 / r, u, u1, u2;
      const double* ja = l.en() + 6 * a;
      pair_fn(r, wf.kappa, en_coef(ja), u, u1, u2);
      Ui += u;
      double f = u1 * ir;
      gx += f * dx; gy += f * dy; gz += f * dz;
      lap += u2 + 2.0 * f;
      Vi -= nuc[4 * a + 3] * ir;
    }
    int si = spin_of(wf, i);
    for (int j = 0; j < wf.N; ++j) {
      if (j == i) continue;
      double dx = xi - Rsrc[3 * j], dy = yi - Rsrc[3 * j + 1], dz = zi - Rsrc[3 * j + 2];
      double r = sqrt(dx * dx + dy * dy + dz * dz), ir = 1.0 / r, u, u1, u2;
      bool anti = si != spin_of(wf, j);
      pair_fn(r, wf.kappa, ee_coef(wf, anti), u, u1, u2);
      Ui += 0.5 * u;
      double f = u1 * ir;
      gx += f * dx; gy += f * dy; gz += f * dz;
      lap += u2 + 2.0 * f;
      Vi += 0.5 * ir;
      if constexpr (EEN) {
        // f_een of the pair (i, j) with every nucleus (each pair seen twice)
        double ue = 0.0, ge[3] = {0.0, 0.0, 0.0}, le = 0.0;
        een_partner<2>(wf, nuc, xi, yi, zi, Rsrc[3 * j], Rsrc[3 * j + 1], Rsrc[3 * j + 2], ue, ge, le);
        Ui += 0.5 * ue;
        gx += ge[0]; gy += ge[1]; gz += ge[2];
        lap += le;
      }
    }
    l.gU()[3 * i] = gx; l.gU()[3 * i + 1] = gy; l.gU()[3 * i + 2] = gz;
    l.lU()[i] = lap;
    part[0] += Ui;
    part[1] += Vi;
  }
  block_sum<NT, 2>(part, l.red());
  if (threadIdx.x == 0) {
    l.sc()[SC_U] = part[0];
    l.sc()[SC_V] = part[1] + wf.vnn;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Row-operator ratio of one electron: sum_u (rho R_u + y^T adj(T_JQ) B_J,i) W_u
// for a row w (length nop) of electron il of spin s.  B, T, Ru, Wu may live in
// LDS or in a walker record in HBM.
// ---------------------------------------------------------------------------
// B[j * bstride + bcol] is B[j][il]: the full inverse (bstride = n, bcol = il)
// or a staged copy of its column il (bstride = 1, bcol = 0).
__device__ double row_op_sum_p(const DevWF& wf, const Ld& l, int s, const double* w, double* ybuf,
                               const double* B, int bstride, int bcol, const double* T, const double* Ru,
                               const double* Wu) {
  const SpinTab& st = wf.sp[s];
  const int* ref = l.ref(s);
  const int* porb = l.porb(s);
  double rho = 0.0;
#pragma unroll 4
  for (int j = 0; j < st.n; ++j) rho += w[ref[j]] * B[j * bstride + bcol];
  for (int q = 0; q < st.nP; ++q) {
    double a = w[porb[q]];
#pragma unroll 4
    for (int k = 0; k < st.n; ++k) a -= w[ref[k]] * T[k * st.nP + q];
    ybuf[q] = a;
  }
  double tot = 0.0;
  const int* uit = l.ui(s);
  for (int u = 0; u < st.nU; ++u) {
    const int* ui = uit + 8 * u;
    double m[9], yy[3], bb[3];
    int e = gather_u(ui, T, st.nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < e) {
        yy[r] = ybuf[ui[4 + r]];
        bb[r] = B[ui[1 + r] * bstride + bcol];
      }
    tot += (rho * Ru[u] + adj_e(e, m, yy, bb)) * Wu[u];
  }
  return tot;
}

// row_op_sum_p for spins of at most NE electrons, with every load of the
// reference part issued before the sums (same sums, same order)
template <int NE>
__device__ double row_op_sum_r(const DevWF& wf, const Ld& l, int s, const double* w, double* ybuf,
                               const double* B, int bstride, int bcol, const double* T, const double* Ru,
                               const double* Wu) {
  const SpinTab& st = wf.sp[s];
  const int n = st.n;
  const int* ref = l.ref(s);
  const int* porb = l.porb(s);
  double wv[NE], bv[NE];
#pragma unroll
  for (int j = 0; j < NE; ++j) {
    const int jj = j < n ? j : 0;
    wv[j] = j < n ? w[ref[jj]] : 0.0;
    bv[j] = j < n ? B[jj * bstride + bcol] : 0.0;
  }
  double rho = 0.0;
#pragma unroll
  for (int j = 0; j < NE; ++j)
    if (j < n) rho += wv[j] * bv[j];
  for (int q = 0; q < st.nP; ++q) {
    double a = w[porb[q]];
#pragma unroll
    for (int k = 0; k < NE; ++k)
      if (k < n) a -= wv[k] * T[k * st.nP + q];
    ybuf[q] = a;
  }
  double tot = 0.0;
  const int* uit = l.ui(s);
  for (int u = 0; u < st.nU; ++u) {
    const int* ui = uit + 8 * u;
    double m[9], yy[3], bb[3];
    int e = gather_u(ui, T, st.nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < e) {
        yy[r] = ybuf[ui[4 + r]];
        bb[r] = B[ui[1 + r] * bstride + bcol];
      }
    tot += (rho * Ru[u] + adj_e(e, m, yy, bb)) * Wu[u];
  }
  return tot;
}

__device__ __forceinline__ double row_op_sum(const DevWF& wf, const Ld& l, int s, int il, const double* w,
                                             double* ybuf) {
  return row_op_sum_p(wf, l, s, w, ybuf, l.B(s), wf.sp[s].n, il, l.T(s), l.Ru(s), l.Wu(s));
}

// ---------------------------------------------------------------------------
// Local energy pass: per tile of electrons, MFMA channels 1..4 (gradient and
// Laplacian rows), row-operator ratios, then the Jastrow and potential.
// Fills gD, lD, gU, lU and SC_ELOC, SC_LOGPSI, SC_SIGN.  gc (the DMC
// gradient cache in the walker record) may be null.
// ---------------------------------------------------------------------------
template <int NT, int PREC, bool EEN = false>
__device__ void local_energy(const DevWF& wf, const Ld& l, double* gc) {
  const double* R = l.R();
  const double S = l.sc()[SC_S];
  const int nPmax = max(wf.sp[0].nP, wf.sp[1].nP);
  for (int g0 = 0; g0 < wf.N; g0 += kGroup) {
    int ne = min(kGroup, wf.N - g0);
    group_radial<NT, PREC>(wf, l, R, g0, ne);
    for (int c = 1; c <= 4; ++c) {
      group_channel<NT, PREC>(wf, l, ne, c);
      const double* Phi = l.Phi();
      for (int e = threadIdx.x; e < ne; e += NT) {
        int i = g0 + e;
        int s = spin_of(wf, i), il = i - wf.sp[s].e0;
        double tot = row_op_sum(wf, l, s, il, Phi + e * wf.nop, l.yb() + e * (nPmax + 1));
        if (c < 4)
          l.gD()[3 * i + c - 1] = tot / S;
        else
          l.lD()[i] = tot / S;
      }
      if (gc && c < 4)
        for (int idx = threadIdx.x; idx < ne * wf.nop; idx += NT) {
          int e = idx / wf.nop, p = idx - e * wf.nop;
          gc[((g0 + e) * 3 + c - 1) * wf.nop + p] = Phi[idx];
        }
      __syncthreads();
    }
  }
  jastrow_full<NT, EEN>(wf, l, R);
  double part[1] = {0.0};
  for (int i = threadIdx.x; i < wf.N; i += NT) {
    double t = l.lU()[i] + l.lD()[i];
    for (int x = 0; x < 3; ++x) {
      double gu = l.gU()[3 * i + x];
      t += gu * gu + 2.0 * gu * l.gD()[3 * i + x];
    }
    part[0] += -0.5 * t;
  }
  block_sum<NT, 1>(part, l.red());
  if (threadIdx.x == 0) {
    double* sc = l.sc();
    sc[SC_ELOC] = part[0] + sc[SC_V];
    sc[SC_LOGPSI] = sc[SC_U] + sc[SC_LOGDET0] + sc[SC_LOGDET1] + log(fabs(S));
    sc[SC_SIGN] = sc[SC_SGN0] * sc[SC_SGN1] * (S > 0 ? 1.0 : (S < 0 ? -1.0 : 0.0));
  }
  __syncthreads();
}

// structure ratios r_I = sum_links d' R_up R_dn / S into l.ratio()
template <int NT>
__device__ void structure_ratios(const DevWF& wf, const Ld& l) {
  double S = l.sc()[SC_S];
  const int* srow = l.srow();
  const int* slu = l.slu();
  const double* slc = l.slc();
  for (int I = threadIdx.x; I < wf.nstruct; I += NT) {
    double a = 0.0;
    for (int k = srow[I]; k < srow[I + 1]; ++k) a += slc[k] * l.Ru(0)[slu[2 * k]] * l.Ru(1)[slu[2 * k + 1]];
    l.ratio()[I] = a / S;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Basis values (+ gradients if nch = 4) at one point and their contraction to
// orbital rows v[c][p] on the VALU.  One lane per primitive forms the
// exponentials, one lane per basis function sums its shell's primitives and
// applies the angular factor, then lanes split the basis sum of each output
// and reduce with cross-lane shuffles.
// ---------------------------------------------------------------------------
template <int NT, int PREC>
__device__ void point_orbitals(const DevWF& wf, const Ld& l, double px, double py, double pz, int nch) {
  typedef typename std::conditional<PREC == 0, double, float>::type T;
  T* chi = (T*)l.chi();
  T* pt = (T*)l.pt();  // [nprim][2] primitive terms
  const double* nuc = l.nuc();
  const int* psh = l.psh();
  for (int q = threadIdx.x; q < wf.nprim; q += NT) {
    const int* si = l.sh() + 8 * psh[q];
    int a = si[0];
    T x = (T)(px - nuc[4 * a]), y = (T)(py - nuc[4 * a + 1]), z = (T)(pz - nuc[4 * a + 2]);
    T r2 = x * x + y * y + z * z;
    T al = (T)l.pe()[q];
    T t = si[1] == 0 ? al * r2 : al * sqrt(r2);
    T ex = t < T(50) ? (T)l.pc()[q] * exp_neg<T>(t, l.L + wf.l_etab) : T(0);
    pt[2 * q] = ex;
    pt[2 * q + 1] = -al * ex;
  }
  __syncthreads();
  for (int mu = threadIdx.x; mu < wf.Mpad; mu += NT) {
    int sh = l.fn()[2 * mu];
    if (sh < 0) {
      for (int c = 0; c < nch; ++c) chi[c * wf.Mpad + mu] = T(0);
      continue;
    }
    const int* si = l.sh() + 8 * sh;
    int a = si[0], kind = si[1], lq = si[2], p0 = si[4], np = si[5];
    T x = (T)(px - nuc[4 * a]), y = (T)(py - nuc[4 * a + 1]), z = (T)(pz - nuc[4 * a + 2]);
    T r2 = x * x + y * y + z * z, r = sqrt(r2);
    T g = 0, g1 = 0;
#pragma unroll 4
    for (int k = 0; k < np; ++k) {
      g += pt[2 * (p0 + k)];
      g1 += pt[2 * (p0 + k) + 1];
    }
    T o[5];
    channels<T>(kind, lq, l.fn()[2 * mu + 1] & 15, x, y, z, r2, r, g, g1, T(0), nch, o);
    for (int c = 0; c < nch; ++c) chi[c * wf.Mpad + mu] = o[c];
  }
  __syncthreads();
  typedef typename std::conditional<PREC == 0, double, float>::type LT;
  const LT* lam = l.lam<LT>();
  const int nout = nch * wf.nop;
  if (nout <= 64) {
    // one wave: lane = part * nout + o, parts reduced with shuffles
    if (threadIdx.x < 64) {
      // lane = o * nparts + part (nparts a power of two): adjacent lanes
      // split one output's basis sum and are combined with xor shuffles
      int lg = 0;
      while ((2 << lg) * nout <= 64) ++lg;
      const int nparts = 1 << lg;
      const int lane = threadIdx.x, o = lane >> lg, pt_ = lane & (nparts - 1);
      const int chunk = wf.Mpad >> lg;  // Mpad is a multiple of 16 and nparts <= 64 / 16
      T acc = T(0);
      if (o < nout) {
        int c = (o >= wf.nop) + (o >= 2 * wf.nop) + (o >= 3 * wf.nop);
        int p = o - c * wf.nop;
        const T* ch = chi + c * wf.Mpad + pt_ * chunk;
        const LT* lp = lam + (size_t)pt_ * chunk * wf.nop + p;
#pragma unroll 4
        for (int k = 0; k < chunk; ++k) acc += ch[k] * (T)lp[(size_t)k * wf.nop];
      }
      double a = (double)acc;
      for (int off = 1; off < nparts; off <<= 1) a += __shfl_xor(a, off, 64);
      if (o < nout && pt_ == 0) l.v()[o] = a;
    }
  } else {
    // lam may be in global memory here: 16 loads in flight per thread
    for (int o = threadIdx.x; o < nout; o += NT) {
      int c = o / wf.nop, p = o - c * wf.nop;
      const T* ch = chi + c * wf.Mpad;
      T acc = T(0);
#pragma unroll 16
      for (int mu = 0; mu < wf.Mpad; ++mu) acc += ch[mu] * (T)lam[(size_t)mu * wf.nop + p];
      l.v()[o] = (double)acc;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Single-electron move of electron i to (px,py,pz): ratio of determinant sums
// S''/S (written to SC_RATIO) and Jastrow change dU (SC_TMP0); fills y (value
// channel), bcol (old B column), rho (SC_TMP1) and Qu.  v holds the orbital
// values at the trial position.
// ---------------------------------------------------------------------------
template <int NT>
__device__ void move_ratio(const DevWF& wf, const Ld& l, int i, double px, double py, double pz,
                           const double* v) {
  int s = spin_of(wf, i);
  const SpinTab& st = wf.sp[s];
  const int n = st.n, nP = st.nP;
  int il = i - st.e0;
  const double* B = l.B(s);
  const double* T = l.T(s);
  const int* ref = l.ref(s);
  const int* porb = l.porb(s);
  double* y = l.y();
  double* bc = l.bcol();
  double* vr = l.z() + n;  // gathered v[ref[j]] (z holds n more entries used on accept)
  // phase 1: gather v[ref], old B column, rho = sum_j v[ref_j] B[j][i]
  double prod = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) {
    double a = v[ref[j]], b = B[j * n + il];
    vr[j] = a;
    bc[j] = b;
    prod += a * b;
  }
  double rr[1] = {prod};
  block_sum<NT, 1>(rr, l.red());
  const double rho = rr[0];
  __syncthreads();
  // phase 2: y[q] = v[P_q] - sum_k v[ref_k] T[k][q]; Jastrow change in parallel
  for (int q = threadIdx.x; q < nP; q += NT) {
    double a = v[porb[q]];
#pragma unroll 4
    for (int k = 0; k < n; ++k) a -= vr[k] * T[k * nP + q];
    y[q] = a;
  }
  double part[2] = {0.0, 0.0};
  const double* R = l.R();
  const double* nuc = l.nuc();
  double xo = R[3 * i], yo = R[3 * i + 1], zo = R[3 * i + 2];
  const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
  const double kappa = wf.kappa;
  for (int j = threadIdx.x; j < wf.N + wf.nnuc; j += NT) {
    if (j == i) continue;
    double xj, yj, zj;
    PairCoef c;
    if (j < wf.N) {
      xj = R[3 * j]; yj = R[3 * j + 1]; zj = R[3 * j + 2];
      c = s != spin_of(wf, j) ? c_anti : c_par;
    } else {
      int nn = j - wf.N;
      xj = nuc[4 * nn]; yj = nuc[4 * nn + 1]; zj = nuc[4 * nn + 2];
      c = en_coef(l.en() + 6 * nn);
    }
    double rn = sqrt((px - xj) * (px - xj) + (py - yj) * (py - yj) + (pz - zj) * (pz - zj));
    double ro = sqrt((xo - xj) * (xo - xj) + (yo - yj) * (yo - yj) + (zo - zj) * (zo - zj));
    part[1] += pair_val(rn, kappa, c) - pair_val(ro, kappa, c);
  }
  __syncthreads();
  // phase 3: Q_u = rho R_u + y^T adj(T_JQ) B_J,i and S'' = sum_u Q_u W_u
  const int* uit = l.ui(s);
  for (int u = threadIdx.x; u < st.nU; u += NT) {
    const int* ui = uit + 8 * u;
    double m[9], yy[3], bb[3];
    int e = gather_u(ui, T, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < e) {
        yy[r] = y[ui[4 + r]];
        bb[r] = bc[ui[1 + r]];
      }
    double q = rho * l.Ru(s)[u] + adj_e(e, m, yy, bb);
    l.Qu()[u] = q;
    part[0] += q * l.Wu(s)[u];
  }
  block_sum<NT, 2>(part, l.red());
  if (threadIdx.x == 0) {
    l.sc()[SC_RATIO] = part[0] / l.sc()[SC_S];
    l.sc()[SC_TMP0] = part[1];
    l.sc()[SC_TMP1] = rho;
  }
  __syncthreads();
}

// Commit an accepted move of electron i (after move_ratio).
template <int NT>
__device__ void accept_move(const DevWF& wf, const Ld& l, int i, double px, double py, double pz) {
  int s = spin_of(wf, i);
  const SpinTab& st = wf.sp[s];
  int il = i - st.e0;
  double* B = l.B(s);
  double* T = l.T(s);
  double rho = l.sc()[SC_TMP1];
  double* z = l.z();
  const double* vr = l.z() + st.n;  // v[ref[k]], gathered by move_ratio
  for (int m = threadIdx.x; m < st.n; m += NT) {
    double a = 0.0;
#pragma unroll 4
    for (int k = 0; k < st.n; ++k) a += vr[k] * B[k * st.n + m];
    z[m] = (m == il ? a - 1.0 : a);
  }
  __syncthreads();
  double ir = 1.0 / rho;
  const double* bc = l.bcol();
  const double* y = l.y();
  if (st.n <= NT) {
    // lane m owns column m of B; rows j in sequence (no integer division)
    const int m = threadIdx.x;
    if (m < st.n) {
      double zm = z[m] * ir;
      for (int j = 0; j < st.n; ++j) B[j * st.n + m] -= bc[j] * zm;
    }
    if (m < st.nP) {
      double yq = y[m] * ir;
      for (int j = 0; j < st.n; ++j) T[j * st.nP + m] += bc[j] * yq;
    }
  } else {
    for (int idx = threadIdx.x; idx < st.n * st.n; idx += NT) {
      int j = idx / st.n, m = idx - j * st.n;
      B[idx] -= bc[j] * z[m] * ir;
    }
    for (int idx = threadIdx.x; idx < st.n * st.nP; idx += NT) {
      int j = idx / st.nP, q = idx - j * st.nP;
      T[idx] += bc[j] * y[q] * ir;
    }
  }
  if (threadIdx.x == 0) {
    double* sc = l.sc();
    sc[SC_LOGDET0 + s] += log(fabs(rho));
    if (rho < 0) sc[SC_SGN0 + s] = -sc[SC_SGN0 + s];
    sc[SC_NUPD0 + s] += 1.0;
    double* R = l.R();
    R[3 * i] = px; R[3 * i + 1] = py; R[3 * i + 2] = pz;
  }
  __syncthreads();
  // R_u of this spin, and S = sum_u R_u W_u (W of this spin does not depend
  // on this spin's R), then the other spin's W
  double vS[1] = {0.0};
  for (int u = threadIdx.x; u < st.nU; u += NT) {
    double m[9];
    int e = gather_u(l.ui(s) + 8 * u, T, st.nP, m, nullptr, nullptr, 0.0);
    double r = det_e(e, m);
    l.Ru(s)[u] = r;
    vS[0] += r * l.Wu(s)[u];
  }
  block_sum<NT, 1>(vS, l.red());
  if (threadIdx.x == 0) l.sc()[SC_S] = vS[0];
  __syncthreads();
  update_W<NT>(wf, l, 1 - s);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// DMC branching inputs of walker w (Sec. 2.3.2, birth/death; a walker that
// is flagged or whose new E_L is not finite gets no copies): the weight
// exp(-tau ((E_L + E_L') / 2 - E_T)) with both energies clipped to
// E_T +- sqrt(N / tau), its products with E_L' and with the clipped E_L', and
// the branching draw (purpose 2, electron index N).  The copy count
// floor(f w + u) waits for the step's population-control factor f.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dmc_branch_inputs(const DmcBranch& br, int64_t w, bool bad, double E_old, double En,
                                                  double ET, double tau, int N, uint64_t seed, uint32_t step) {
  const double cap = sqrt((double)N / tau);
  const double eo = fmin(fmax(E_old, ET - cap), ET + cap);
  const double en = fmin(fmax(En, ET - cap), ET + cap);
  const double wt = exp(-tau * (0.5 * (eo + en) - ET));
  // a non-finite local energy drops the walker like a singular one
  bad = bad || !isfinite(En);
  double ub, dummy;
  philox_pair(seed, (uint32_t)w, step, 4u * (uint32_t)N + 2u, 0u, ub, dummy);
  br.w[w] = bad ? NAN : wt;
  br.we[w] = bad ? NAN : wt * En;
  br.wc[w] = bad ? NAN : wt * en;
  br.ub[w] = ub;
  br.nc[w] = bad ? -1 : 0;
}

}  // namespace vbqmc
