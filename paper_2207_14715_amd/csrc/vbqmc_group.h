// Lane-group building blocks of the wavefront kernels that hold several
// walkers per 64-lane wavefront (gfx950): wavefront-scope LDS ordering, DPP
// group reductions and broadcasts, the per-walker LDS view, and the group
// versions of the determinant-ratio set-up and the reference inverse.
#pragma once

#include "vbqmc_device.h"

namespace vbqmc {

extern __shared__ double lds_dyn[];

// wavefront-scope ordering point: LDS accesses of one wavefront are performed
// in order, so a fence that stops the compiler from moving them across this
// point is all a group needs between its writes and another lane's reads
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// floor(idx / d) for 0 <= idx < 2^20, given rd = 1.0f / d: (idx + 0.5) / d lies
// at least 0.5 / d from an integer, far beyond the float rounding of the product
__device__ __forceinline__ int div_small(int idx, float rd) { return (int)(((float)idx + 0.5f) * rd); }

// DPP move of a double within 16-lane rows (ctrl: a GFX9 DPP control word)
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Lane k (0..15, the same in every lane) of each 16-lane row, to every lane
// of that row, through the LDS crossbar (ds_bpermute; a DPP row broadcast
// would need k as an immediate, and a switch over k costs more than the
// crossbar and splits the code around it into basic blocks).
__device__ __forceinline__ double row_bcast(double v, int k) {
  const int src = (((int)(threadIdx.x & 63) & ~15) | k) << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Sum over the 4 lanes of a quad (DPP quad permutations), the same bits in
// every lane of the quad.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_mov<0xB1>(v);  // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);  // quad_perm [2,3,0,1]
  return v;
}

// Sum over the G lanes of a group, the same bits in every lane: a butterfly
// whose in-row steps are DPP row rotations by 8 and 4 (equal to xor 8 and
// xor 4 once the previous steps have made the values symmetric) and quad
// permutations for xor 2 and xor 1; the step across 16-lane rows (G = 32)
// is a lane permute.
template <int G>
__device__ __forceinline__ double gsum(double v) {
  static_assert(G == 16 || G == 32, "group of 16 or 32 lanes");
  if constexpr (G == 32) v += __shfl_xor(v, 16, 32);
  v += dpp_mov<0x128>(v);  // row_ror:8
  v += dpp_mov<0x124>(v);  // row_ror:4
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  return v;
}

// One walker's view: tables and shared scratch at L, its state at S (state
// offsets of this layout are relative to the walker's state base).
struct Lg {
  double* L;
  double* S;
  const DevWF& wf;
  int q;  // lane within the group
  __device__ Lg(double* l, int g, const DevWF& w, int lane)
      : L(l), S(l + w.gw_base + g * w.gw_stride), wf(w), q(lane) {}
  __device__ const double* nuc() const { return L + wf.l_nuc; }
  __device__ const double* en() const { return L + wf.l_en; }
  __device__ const int* ref(int s) const { return (const int*)(L + wf.l_ref[s]); }
  __device__ const int* porb(int s) const { return (const int*)(L + wf.l_porb[s]); }
  __device__ const int* ui(int s) const { return (const int*)(L + wf.l_ui[s]); }
  __device__ const int* wrow(int s) const { return (const int*)(L + wf.l_wrow[s]); }
  __device__ const int* woth(int s) const { return (const int*)(L + wf.l_woth[s]); }
  __device__ const double* wcoef(int s) const { return L + wf.l_wcoef[s]; }
  __device__ double* R() const { return S + wf.l_R; }
  __device__ double* B(int s) const { return S + wf.l_B[s]; }
  __device__ double* T(int s) const { return S + wf.l_T[s]; }
  __device__ double* PP(int s) const { return S + wf.l_PP[s]; }
  __device__ double* Ru(int s) const { return S + wf.l_Ru[s]; }
  __device__ double* Wu(int s) const { return S + wf.l_Wu[s]; }
  __device__ double* Qu() const { return S + wf.l_Qu; }
  __device__ double* sc() const { return S + wf.l_sc; }
  __device__ int* ipiv() const { return (int*)(S + wf.l_ipiv); }
  __device__ double* f() const { return S + wf.l_f; }
  __device__ double* y() const { return S + wf.l_y; }
  __device__ double* bcol() const { return S + wf.l_bcol; }
  __device__ double* z() const { return S + wf.l_z; }
};

// R_u, W_u and S of one walker
template <int G>
__device__ void compute_RWS_g(const DevWF& wf, const Lg& l) {
  for (int s = 0; s < 2; ++s) {
    const SpinTab& st = wf.sp[s];
    for (int u = l.q; u < st.nU; u += G) {
      double m[9];
      int e = gather_u(l.ui(s) + 8 * u, l.T(s), st.nP, m, nullptr, nullptr, 0.0);
      l.Ru(s)[u] = det_e(e, m);
    }
  }
  wave_sync();
  for (int s = 0; s < 2; ++s) {
    const SpinTab& st = wf.sp[s];
    const double* Ro = l.Ru(1 - s);
    const int* wr = l.wrow(s);
    const int* wo = l.woth(s);
    const double* wc = l.wcoef(s);
    for (int u = l.q; u < st.nU; u += G) {
      double w = 0.0;
      for (int k = wr[u]; k < wr[u + 1]; ++k) w += wc[k] * Ro[wo[k]];
      l.Wu(s)[u] = w;
    }
  }
  wave_sync();
  double v = 0.0;
  for (int u = l.q; u < wf.sp[0].nU; u += G) v += l.Ru(0)[u] * l.Wu(0)[u];
  v = gsum<G>(v);
  if (l.q == 0) l.sc()[SC_S] = v;
  wave_sync();
}

// In-place Gauss-Jordan inverse with partial pivoting of an n x n matrix A
// (rows electrons, columns reference slots) -> A^{-1} by the H lanes qh of a
// half group.  log|det A| is accumulated as a mantissa product and an
// exponent sum (one log at the end).  Returns false if a pivot is exactly
// zero.  The pivot of column k is the largest |A[i][k]|, i >= k, the lowest
// row on ties: found by a butterfly over the lanes' partial maxima, or
// (SCAN) by every lane scanning the column itself (broadcast reads, no
// cross-lane steps; the same pivot).
template <int H, bool SCAN = false>
__device__ bool gj_invert_h(double* A, int n, int qh, int* piv, double* f, double& logdet, double& sgn) {
  const float rn = 1.0f / (float)n;
  double mant = 1.0;
  int ex = 0;
  sgn = 1.0;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = n;
    if constexpr (SCAN) {
      for (int i = k; i < n; ++i) {
        const double v = fabs(A[i * n + k]);
        if (v > best) { best = v; bi = i; }
      }
    } else {
      for (int i = k + qh; i < n; i += H) {
        double v = fabs(A[i * n + k]);
        if (v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int off = H / 2; off > 0; off >>= 1) {
        double ob = __shfl_xor(best, off, H);
        int oi = __shfl_xor(bi, off, H);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
    }
    if (!(best > 0.0)) return false;
    const int p = bi;
    if (qh == 0) piv[k] = p;
    if (p != k)
      for (int j = qh; j < n; j += H) {
        double t = A[k * n + j];
        A[k * n + j] = A[p * n + j];
        A[p * n + j] = t;
      }
    wave_sync();
    const double pv = A[k * n + k];
    int e2;
    mant = frexp(mant * fabs(pv), &e2);
    ex += e2;
    if (pv < 0) sgn = -sgn;
    if (p != k) sgn = -sgn;
    for (int i = qh; i < n; i += H) f[i] = A[i * n + k];
    wave_sync();
    const double ip = 1.0 / pv;
    for (int j = qh; j < n; j += H) A[k * n + j] = (j == k ? 1.0 : A[k * n + j]) * ip;
    wave_sync();
    for (int idx = qh; idx < n * n; idx += H) {
      int i = div_small(idx, rn), j = idx - i * n;
      if (i != k) A[idx] = (j == k ? 0.0 : A[idx]) - f[i] * A[k * n + j];
    }
    wave_sync();
  }
  for (int k = n - 1; k >= 0; --k) {
    int p = piv[k];
    if (p != k)
      for (int i = qh; i < n; i += H) {
        double t = A[i * n + k];
        A[i * n + k] = A[i * n + p];
        A[i * n + p] = t;
      }
    wave_sync();
  }
  logdet = log(mant) + (double)ex * 0.69314718055994530942;
  return true;
}

// Invert the staged reference matrices (in B) and form T = B PP.  The two
// halves of the group take one spin each.
template <int G>
__device__ bool finish_state_g(const DevWF& wf, const Lg& l) {
  constexpr int H = G / 2;
  const int s = l.q / H, qh = l.q - s * H;
  const int nmax = max(wf.sp[0].n, wf.sp[1].n);
  const SpinTab& st = wf.sp[s];
  double ld = 0.0, sg = 1.0;
  bool ok = true;
  if (st.n > 0) ok = gj_invert_h<H>(l.B(s), st.n, qh, l.ipiv() + s * nmax, l.f() + s * nmax, ld, sg);
  if (qh == 0) {
    l.sc()[SC_LOGDET0 + s] = ld;
    l.sc()[SC_SGN0 + s] = sg;
    l.sc()[SC_NUPD0 + s] = 0.0;
  }
  // both halves must have succeeded
  const bool ok_other = __shfl_xor((int)ok, H, G) != 0;
  ok = ok && ok_other;
  wave_sync();
  for (int s2 = 0; s2 < 2; ++s2) {
    const SpinTab& t2 = wf.sp[s2];
    const float rp = 1.0f / (float)max(t2.nP, 1);
    for (int idx = l.q; idx < t2.n * t2.nP; idx += G) {
      int j = div_small(idx, rp), c = idx - j * t2.nP;
      double a = 0.0;
      for (int i = 0; i < t2.n; ++i) a += l.B(s2)[j * t2.n + i] * l.PP(s2)[i * t2.nP + c];
      l.T(s2)[idx] = a;
    }
  }
  wave_sync();
  return ok;
}


}  // namespace vbqmc
