// Parameter derivatives of ln|Psi| and E_L (the adjoint form) for gfx950.
//
// For fixed configurations this computes, per walker, d ln|Psi| / dp and
// d E_L / dp for p = [c (structure coefficients) | lambda (orbital
// coefficients) | Jastrow pair parameters]: the per-sample quantities that
// the linear optimisation method consumes (Radenkovic, Domin, Toulouse,
// Braida 2022, Sec. 2.2, Eq. (PsiJVBp) and the gradient estimators of
// Eqs. (Hi0), (H0j) with E_{L,j} = d E_L / d p_j).
//
// Reverse-mode derivation (no stored per-electron intermediates; every spin
// determinant inverse is recomputed in each of the two passes):
//   E_L = -1/2 sum_i [lap_i U + |grad_i U|^2] + V + sum_k W_k e_k,
//   W_k = w_k Delta_k / D,  e_k = sum_spins tr(A_u^{-1} K_u),
// with A_u[i][j] = phi_{o_j}(r_i) the spin-determinant matrix in the slot
// order of its table entry and K_u[i][j] = -grad_i U . grad phi_{o_j}(r_i)
// - 1/2 lap phi_{o_j}(r_i) the "kinetic row" matrix.  With
// omega_u = sum_{k holding u} W_k and lbar_u = sum_{k holding u} W_k (e_k - ebar):
//   dE_L/dA_u = lbar_u A_u^{-T} - omega_u (A_u^{-1} K_u A_u^{-1})^T,
//   dE_L/dK_u = omega_u A_u^{-T},   d ln|D| / dA_u = omega_u A_u^{-T}.
// Scattering these onto orbital rows gives Gamma0[i][p] (value rows) and
// G[i][p] (gradient/Laplacian rows enter through K), and then
//   d E_L / d lambda[p][mu] = sum_i Gamma0[i][p] chi_mu(r_i) + G[i][p] kappa_mu(r_i),
//   d ln|Psi| / d lambda[p][mu] = sum_i G[i][p] chi_mu(r_i),
// kappa_mu = -grad U . grad chi_mu - 1/2 lap chi_mu: two contractions over
// electrons done on MFMA.  Structure coefficients and Jastrow parameters use
// their closed forms (Euler form in c; pair-function derivatives).

#include "vbqmc_device.h"
#include "vbqmc_group.h"

namespace vbqmc {

extern __shared__ double lds_adj[];

// all five basis channels of function mu at electron e of the current tile,
// from one load of the function's operands
template <typename T>
__device__ __forceinline__ void chan_all(const DevWF& wf, const Ld& l, int e, int mu, T* out) {
  const FnInfo fi = fn_info(l, mu);
  if (fi.sh < 0) {
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = T(0);
    return;
  }
  const ChanIn<T> in = chan_load<T, 3>(wf, l, e, fi);
  out[0] = chan_eval<T>(fi, in, 0);
  T o4[4];
  chan_eval4<T>(fi, in, o4);
#pragma unroll
  for (int c = 0; c < 4; ++c) out[1 + c] = o4[c];
}

// The five orbital-row channels of a group of ne electrons (rows e < ne of
// channel c to out + c * cstride + e * nop), FP64 on MFMA: a wavefront takes
// one 16-orbital column tile and a share of the basis functions, forming
// all five channels of each function from one load; when the column tiles
// leave wavefronts over, the functions are split among them and the shares
// are added into the rows in a fixed order (one block barrier per share).
template <int NT>
__device__ void adj_rows5(const DevWF& wf, const Ld& l, int ne, double* out, int cstride) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  const int nct = wf.nop / 16;
  const int KQ = max(1, NW / nct);
  const int nch = wf.Mpad / 16;  // chunks of 16 functions (four k-steps)
  const double* lam = l.lam<double>();
  const int e = lane & 15;
  const bool live = e < ne;
  // work items: (column tile, share of the functions); with KQ > 1 there is
  // one item per wavefront (nct * KQ <= NW) and the shares are added in
  // order
  const int nitem = nct * KQ;
  for (int item0 = 0; item0 < nitem; item0 += NW) {
    const int item = item0 + wave;
    const bool has = item < nitem;
    const int ct = has ? item % nct : 0, kq = has ? item / nct : 0;
    const int col = ct * 16 + (lane & 15);
    v4d acc0 = {0, 0, 0, 0}, acc1 = acc0, acc2 = acc0, acc3 = acc0, acc4 = acc0;
    if (has) {
      const int k_lo = 16 * (kq * nch / KQ), k_hi = 16 * ((kq + 1) * nch / KQ);
      for (int k0 = k_lo; k0 < k_hi; k0 += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * u + (lane >> 4);
          double ch[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
          if (live) chan_all<double>(wf, l, e, k, ch);
          const double b = lam[(size_t)k * wf.nop + col];
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ch[0], b, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ch[1], b, acc1, 0, 0, 0);
          acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ch[2], b, acc2, 0, 0, 0);
          acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ch[3], b, acc3, 0, 0, 0);
          acc4 = __builtin_amdgcn_mfma_f64_16x16x4f64(ch[4], b, acc4, 0, 0, 0);
        }
      }
    }
    // f64 16x16x4 output: register r of lane l holds row 4r + l/16
    for (int r = 0; r < KQ; ++r) {
      if (has && kq == r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 4 * q + (lane >> 4);
          if (row < ne) {
            double* o = out + row * wf.nop + col;
            const double v[5] = {acc0[q], acc1[q], acc2[q], acc3[q], acc4[q]};
#pragma unroll
            for (int c = 0; c < 5; ++c) o[(size_t)c * cstride] = r > 0 ? o[(size_t)c * cstride] + v[c] : v[c];
          }
        }
      __syncthreads();
    }
  }
}

// The Jastrow factor's gradient and Laplacian per electron, U and the
// potential (as jastrow_full without f_een), with each electron's partners
// spread over a segment of SEG lanes (SEG a power of two, N * SEG <= NT)
// and summed within the segment
template <int NT>
__device__ void adj_jastrow(const DevWF& wf, const Ld& l, const double* Rsrc) {
  const int N = wf.N, nn = wf.nnuc;
  int SEG = 64;
  while (SEG > 1 && N * SEG > NT) SEG >>= 1;
  const double* nuc = l.nuc();
  double part[2] = {0.0, 0.0};  // U, V
  for (int t0 = 0; t0 < N * SEG; t0 += NT) {
    const int t = t0 + (int)threadIdx.x;
    const int i = t / SEG, sub = t - i * SEG;
    const bool el = i < N;
    const int ii = el ? i : 0;
    const double xi = Rsrc[3 * ii], yi = Rsrc[3 * ii + 1], zi = Rsrc[3 * ii + 2];
    const int si = spin_of(wf, ii);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // gx, gy, gz, lap, U, V
    if (el)
      for (int pidx = sub; pidx < nn + N; pidx += SEG) {
        double dx, dy, dz, wu, wv;
        PairCoef cf;
        if (pidx < nn) {
          dx = xi - nuc[4 * pidx]; dy = yi - nuc[4 * pidx + 1]; dz = zi - nuc[4 * pidx + 2];
          cf = en_coef(l.en() + 6 * pidx);
          wu = 1.0;
          wv = -nuc[4 * pidx + 3];
        } else {
          const int j = pidx - nn;
          if (j == i) continue;
          dx = xi - Rsrc[3 * j]; dy = yi - Rsrc[3 * j + 1]; dz = zi - Rsrc[3 * j + 2];
          cf = ee_coef(wf, si != spin_of(wf, j));
          wu = 0.5;
          wv = 0.5;
        }
        const double r = sqrt(dx * dx + dy * dy + dz * dz), ir = 1.0 / r;
        double u, u1, u2;
        pair_fn(r, wf.kappa, cf, u, u1, u2);
        const double f = u1 * ir;
        v[0] += f * dx;
        v[1] += f * dy;
        v[2] += f * dz;
        v[3] += u2 + 2.0 * f;
        v[4] += wu * u;
        v[5] += wv * ir;
      }
    // (every lane of the wavefront takes part; xor offsets below SEG stay
    // inside the segment)
#pragma unroll
    for (int k = 0; k < 6; ++k)
      for (int off = SEG / 2; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if (el && sub == 0) {
      l.gU()[3 * i] = v[0];
      l.gU()[3 * i + 1] = v[1];
      l.gU()[3 * i + 2] = v[2];
      l.lU()[i] = v[3];
      part[0] += v[4];
      part[1] += v[5];
    }
  }
  block_sum<NT, 2>(part, l.red());
  if (threadIdx.x == 0) {
    l.sc()[SC_U] = part[0];
    l.sc()[SC_V] = part[1] + wf.vnn;
  }
  __syncthreads();
}

// derivatives (du, du', du'') of a pair function with respect to one of its
// parameters: kind 0 numerator a, 1 denominator b, 2..5 coefficient of R^kind
__device__ __forceinline__ void pair_param(double r, double kappa, double a, double b, int kind, double& du,
                                           double& du1, double& du2) {
  double den = 1.0 + kappa * r, iden = 1.0 / den;
  double R = r * iden, R1 = iden * iden, R2 = -2.0 * kappa * R1 * iden;
  double f, fR, fRR;
  if (kind == 0) {
    double ib = 1.0 / (1.0 + b * R);
    f = R * ib; fR = ib * ib; fRR = -2.0 * b * ib * ib * ib;
  } else if (kind == 1) {
    double ib = 1.0 / (1.0 + b * R);
    double ib3 = ib * ib * ib;
    f = -a * R * R * ib * ib; fR = -2.0 * a * R * ib3; fRR = -2.0 * a * ib3 + 6.0 * a * b * R * ib3 * ib;
  } else {
    int p = kind;
    double Rp2 = 1.0;
    for (int k = 0; k < p - 2; ++k) Rp2 *= R;
    f = Rp2 * R * R; fR = p * Rp2 * R; fRR = p * (p - 1) * Rp2;
  }
  du = f;
  du1 = fR * R1;
  du2 = fRR * R1 * R1 + fR * R2;
}

// orbital of slot j of unique determinant u (slots in reference order with the
// replaced slots J taking the table orbitals Q)
__device__ __forceinline__ int slot_orbital(const Ld& l, int s, const int* ui, int j) {
  int e = ui[0];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    if (r < e && ui[1 + r] == j) return l.porb(s)[ui[4 + r]];
  return l.ref(s)[j];
}

// ---------------------------------------------------------------------------
// Both passes through each spin's reference determinant.  A spin
// determinant u differs from the reference A_0 (electron x slot) in the e <= 3
// slots J_u, which hold the table orbitals Q_u; with B = A_0^-1 and
// T = B Phi_P (Phi_P: the table orbitals' values),
//   A_u^-1 = B - (T[:, Q] - E_J) V_u,   V_u = m_u^-1 B[J, :],  m_u = T[J, Q],
// det A_u = det A_0 det m_u, and with the kinetic rows K (K_0 and K_P as A_0
// and Phi_P), S = K_0 B and Xi = K_P - K_0 T:
//   K_u A_u^-1 = S + Xi[:, Q] V_u,   e_u = tr(A_u^-1 K_u) = tr S + tr(V_u Xi[:, Q]).
// The scatters of the second pass then collapse onto sums per table orbital q:
//   W_q = sum omega_u V_u[d, :], Wbar_q = sum lbar_u V_u[d, :],
//   X_q = sum omega_u (V_u K_u A_u^-1)[d, :]   (over u, d with Q_ud = q)
// (the terms a scatter would skip, the slots J_u of a reference row, vanish
// identically, since m_u V_u = B[J, :]), so the work per determinant is on
// e x e and e x n blocks and one inversion per spin replaces one per
// determinant.
// ---------------------------------------------------------------------------

// the kinetic-row entry -(grad U . grad phi_o) - Lap phi_o / 2 at electron e
__device__ __forceinline__ double adj_kin(const DevWF& wf, const Ld& l, const double* aPhi, int e, int o) {
  const int N = wf.N, nop = wf.nop;
  const double* gu = l.gU() + 3 * e;
  return -(gu[0] * aPhi[(1 * N + e) * nop + o] + gu[1] * aPhi[(2 * N + e) * nop + o] +
           gu[2] * aPhi[(3 * N + e) * nop + o]) - 0.5 * aPhi[(4 * N + e) * nop + o];
}

// spin s's reference quantities: B (in A, [slot][electron]), K_0, S = K_0 B,
// T, Xi, B S, B Xi; false if the reference is singular (block-uniform)
template <int NT>
__device__ bool adj_ref_spin(const DevWF& wf, const Ld& l, const double* aPhi, int s, double* B, double* K0,
                             double* S, double& ld0, double& sg0, double& trS, bool pre = false, int tid = -1,
                             int nth = NT, double* T = nullptr, double* Xi = nullptr, double* BS = nullptr,
                             double* BXi = nullptr) {
  // (tid, nth: the threads that take part, all of the block by default; T,
  // Xi, B S, B Xi: the outputs, the shared regions by default)
  if (tid < 0) tid = (int)threadIdx.x;
  if (!T) T = l.L + wf.l_aT;
  if (!Xi) Xi = l.L + wf.l_aXi;
  if (!BS) BS = l.L + wf.l_aBS;
  if (!BXi) BXi = l.L + wf.l_aBXi;
  const SpinTab& st = wf.sp[s];
  const int n = st.n, nP = st.nP, e0 = st.e0, N = wf.N, nop = wf.nop;
  const int* ref = l.ref(s);
  const int* porb = l.porb(s);
  // (pre: B already holds the inverse, ld0 and sg0 are given)
  for (int idx = tid; idx < n * n; idx += nth) {
    const int i = idx / n, j = idx - i * n;
    if (!pre) B[idx] = aPhi[(0 * N + e0 + i) * nop + ref[j]];
    K0[idx] = adj_kin(wf, l, aPhi, e0 + i, ref[j]);
  }
  __syncthreads();
  if (pre) {
  } else if (n <= 64) {
    // one wavefront inverts (no block barrier per pivot); its outcome
    // reaches the block through the scalar slots
    double* sc = l.sc();
    if (threadIdx.x < 64) {
      double ld, sg;
      const bool ok = gj_invert_h<64, true>(B, n, threadIdx.x, l.ipiv(), l.f(), ld, sg);
      if (threadIdx.x == 0) {
        sc[SC_GJ_OK] = ok ? 1.0 : 0.0;
        sc[SC_GJ_LD] = ok ? ld : 0.0;
        sc[SC_GJ_SG] = ok ? sg : 0.0;
      }
    }
    __syncthreads();
    if (sc[SC_GJ_OK] == 0.0) return false;
    ld0 = sc[SC_GJ_LD];
    sg0 = sc[SC_GJ_SG];
  } else if (!gj_invert<NT>(l, B, n, ld0, sg0)) {
    return false;
  }
  for (int idx = tid; idx < n * nP; idx += nth) {
    const int j = idx / nP, q = idx - j * nP;
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += B[j * n + i] * aPhi[(0 * N + e0 + i) * nop + porb[q]];
    T[idx] = t;
  }
  for (int idx = tid; idx < n * n; idx += nth) {
    const int i = idx / n, a = idx - i * n;
    double t = 0.0;
    for (int j = 0; j < n; ++j) t += K0[i * n + j] * B[j * n + a];
    S[idx] = t;
  }
  __syncthreads();
  for (int idx = tid; idx < n * nP; idx += nth) {
    const int i = idx / nP, q = idx - i * nP;
    double t = adj_kin(wf, l, aPhi, e0 + i, porb[q]);
    for (int k = 0; k < n; ++k) t -= K0[i * n + k] * T[k * nP + q];
    Xi[idx] = t;
  }
  for (int idx = tid; idx < n * n; idx += nth) {
    const int b = idx / n, a = idx - b * n;
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += B[b * n + i] * S[i * n + a];
    BS[idx] = t;
  }
  __syncthreads();
  for (int idx = tid; idx < n * nP; idx += nth) {
    const int b = idx / nP, q = idx - b * nP;
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += B[b * n + i] * Xi[i * nP + q];
    BXi[idx] = t;
  }
  trS = 0.0;
  for (int i = 0; i < n; ++i) trS += S[i * n + i];
  __syncthreads();
  return true;
}

// first pass: ln|Delta_u|, sign and e_u of every distinct spin determinant,
// and per determinant m_u^-1 and V_u Xi[:, Q] ([nU][18]); false if a
// reference is singular
template <int NT>
__device__ bool adj_ref_pass1(const DevWF& wf, const Ld& l, const double* aPhi, double* B, double* K0, double* S) {
  // with the first-pass copies kept, both spins' references are staged in
  // their keep areas and inverted at once, wavefront s taking spin s
  bool pre = false;
  if constexpr (NT >= 128) {
    pre = wf.adj_save && wf.sp[0].n <= 64 && wf.sp[1].n <= 64;
    if (pre) {
      double* sc = l.sc();
      for (int s = 0; s < 2; ++s) {
        const int n = wf.sp[s].n, e0 = wf.sp[s].e0;
        const int* ref = l.ref(s);
        double* sv = l.L + wf.l_aSave[s];
        for (int idx = threadIdx.x; idx < n * n; idx += NT) {
          const int i = idx / n, j = idx - i * n;
          sv[idx] = aPhi[(e0 + i) * wf.nop + ref[j]];
        }
      }
      __syncthreads();
      const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
      if (wave < 2 && wf.sp[wave].n > 0) {
        const int n = wf.sp[wave].n, nP = wf.sp[wave].nP;
        double* sv = l.L + wf.l_aSave[wave];
        double* f = sv + 2 * n * n + 2 * n * nP;
        int* piv = (int*)(f + n);
        double ld, sg;
        const bool ok = gj_invert_h<64, true>(sv, n, lane, piv, f, ld, sg);
        if (lane == 0) {
          sc[SC_GJ_OK + 3 * wave] = ok ? 1.0 : 0.0;
          sc[SC_GJ_LD + 3 * wave] = ok ? ld : 0.0;
          sc[SC_GJ_SG + 3 * wave] = ok ? sg : 0.0;
        }
      }
      __syncthreads();
    }
  }
  // with both inverses formed at once, the two spins' products and
  // determinants also run at once on the two halves of the block: spin s's
  // B S, T, B Xi straight into its keep area, its K_0, S, Xi in regions this
  // pass leaves free (spin 1: those of A, B S and T)
  const bool par = pre;
  if (par)
    for (int s = 0; s < 2; ++s)
      if (wf.sp[s].n > 0 && l.sc()[SC_GJ_OK + 3 * s] == 0.0) return false;
  const int nth = par ? NT / 2 : NT;
  const int grp = par ? (int)threadIdx.x / (NT / 2) : 0;
  const int tid = par ? (int)threadIdx.x - grp * (NT / 2) : (int)threadIdx.x;
  for (int it = 0; it < (par ? 1 : 2); ++it) {
    const int s = par ? grp : it;
    const SpinTab& st = wf.sp[s];
    const int nP = st.nP;
    double* uinf = l.L + wf.l_aU[s];
    double* V = l.L + wf.l_aV[s];
    double ld0 = 0.0, sg0 = 1.0, trS = 0.0;
    double* Bs = B;
    double *K0s = K0, *Ss = S, *Ts = l.L + wf.l_aT, *Xis = l.L + wf.l_aXi, *BSs = l.L + wf.l_aBS,
           *BXis = l.L + wf.l_aBXi;
    if (par) {
      const int n = st.n;
      double* sv = l.L + wf.l_aSave[s];
      BSs = sv + n * n;
      Ts = sv + 2 * n * n;
      BXis = Ts + n * nP;
      if (s == 1) {
        K0s = l.L + wf.l_aA;
        Ss = l.L + wf.l_aBS;
        Xis = l.L + wf.l_aT;
      }
    }
    if (pre && st.n > 0) {
      const double* sc = l.sc();
      if (sc[SC_GJ_OK + 3 * s] == 0.0) return false;
      ld0 = sc[SC_GJ_LD + 3 * s];
      sg0 = sc[SC_GJ_SG + 3 * s];
      Bs = l.L + wf.l_aSave[s];
    }
    // (in the parallel form both halves pass the same barriers, a spin
    // without electrons with empty loops)
    if ((st.n > 0 || par) &&
        !adj_ref_spin<NT>(wf, l, aPhi, s, Bs, K0s, Ss, ld0, sg0, trS, pre, tid, nth, Ts, Xis, BSs, BXis))
      return false;
    const double* T = Ts;
    const double* BXi = BXis;
    for (int u = tid; u < st.nU; u += nth) {
      const int* ui = l.ui(s) + 8 * u;
      const int e = st.n > 0 ? ui[0] : 0;
      double m[9], mi[9], vx[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int r = k / 3, c = k - 3 * r;
        m[k] = (r < e && c < e) ? T[ui[1 + r] * nP + ui[4 + c]] : (r == c ? 1.0 : 0.0);
      }
      // det and inverse of the leading e x e block (identity past e)
      const double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8], c02 = m[3] * m[7] - m[4] * m[6];
      const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
      const double id = det != 0.0 ? 1.0 / det : 0.0;
      mi[0] = c00 * id;
      mi[1] = (m[2] * m[7] - m[1] * m[8]) * id;
      mi[2] = (m[1] * m[5] - m[2] * m[4]) * id;
      mi[3] = c01 * id;
      mi[4] = (m[0] * m[8] - m[2] * m[6]) * id;
      mi[5] = (m[2] * m[3] - m[0] * m[5]) * id;
      mi[6] = c02 * id;
      mi[7] = (m[1] * m[6] - m[0] * m[7]) * id;
      mi[8] = (m[0] * m[4] - m[1] * m[3]) * id;
      double tr = trS;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int d = k / 3, c = k - 3 * d;
        double t = 0.0;
#pragma unroll
        for (int c2 = 0; c2 < 3; ++c2)
          if (c2 < e && c < e) t += mi[3 * d + c2] * BXi[ui[1 + c2] * nP + ui[4 + c]];
        vx[k] = (d < e && c < e) ? t : 0.0;
        if (d == c && d < e) tr += t;
      }
      const bool ok = det != 0.0;
      uinf[5 * u + 0] = ok ? ld0 + log(fabs(det)) : -INFINITY;
      uinf[5 * u + 1] = ok ? (det < 0.0 ? -sg0 : sg0) : 0.0;
      uinf[5 * u + 2] = ok ? tr : 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        V[18 * u + k] = mi[k];
        V[18 * u + 9 + k] = vx[k];
      }
    }
    if (wf.adj_save && st.n > 0 && !par) {
      // B, B S, T, B Xi of this spin for the second pass
      const int n = st.n, nn = n * n, np = n * nP;
      double* sv = l.L + wf.l_aSave[s];
      const double* BS = l.L + wf.l_aBS;
      for (int k = threadIdx.x + (pre ? nn : 0); k < 2 * nn + 2 * np; k += NT)
        sv[k] = k < nn ? B[k] : (k < 2 * nn ? BS[k - nn] : (k < 2 * nn + np ? T[k - 2 * nn] : BXi[k - 2 * nn - np]));
    }
    __syncthreads();
  }
  return true;
}

// second pass: the references again (recomputed, not stored), the sums
// W, Wbar, X per table orbital, their scatter onto the orbital rows G0
// (d E_L / d phi) and G (d ln|D| / d phi) of each spin's electrons, and the
// drift and Laplacian ratios of D from G
template <int NT>
__device__ void adj_ref_pass2(const DevWF& wf, const Ld& l, const double* aPhi, double* B, double* K0, double* S,
                              double* G0, double* G) {
  const int N = wf.N, nop = wf.nop;
  // with the first-pass copies kept, the two spins run at once on the two
  // halves of the block (their rows of G, G0 are disjoint), spin 1's sums
  // in the space of the reference matrices, which this pass then leaves
  // unused
  const bool par = NT >= 128 && wf.adj_save && 3 * wf.sp[1].n * wf.sp[1].nP <= wf.l_aU[0] - wf.l_aA;
  const int nth = par ? NT / 2 : NT;
  // masks of determinants per table orbital: at most 64 determinants per
  // spin, the masks of the spins that run at once fit the space of Xi
  const bool masks = wf.adj_save && wf.sp[0].nU <= 64 && wf.sp[1].nU <= 64 &&
                     wf.sp[0].nP + wf.sp[1].nP <= wf.l_aBXi - wf.l_aXi;
  const int grp = par ? (int)threadIdx.x / (NT / 2) : 0;
  const int tid = par ? (int)threadIdx.x - grp * (NT / 2) : (int)threadIdx.x;
  for (int it = 0; it < (par ? 1 : 2); ++it) {
    const int s = par ? grp : it;
    const SpinTab& st = wf.sp[s];
    const int n = st.n, nP = st.nP, e0 = st.e0;
    if (!par && n == 0) continue;  // (uniform)
    const double* Bp = B;
    const double* BS = l.L + wf.l_aBS;
    const double* T = l.L + wf.l_aT;
    const double* BXi = l.L + wf.l_aBXi;
    if (wf.adj_save) {
      const double* sv = l.L + wf.l_aSave[s];
      Bp = sv;
      BS = sv + n * n;
      T = sv + 2 * n * n;
      BXi = T + n * nP;
    } else {
      double ld0, sg0, trS;
      adj_ref_spin<NT>(wf, l, aPhi, s, B, K0, S, ld0, sg0, trS);
    }
    const double* uinf = l.L + wf.l_aU[s];
    const double* V = l.L + wf.l_aV[s];
    double* Wq = l.L + (par && s == 1 ? wf.l_aA : wf.l_aW);
    double* Wb = Wq + nP * n;
    double* Xq = Wq + 2 * nP * n;
    const int* ref = l.ref(s);
    const int* porb = l.porb(s);
    // per table orbital q, the mask of the (nonsingular) determinants that
    // put it in one of their replaced columns, so that a (q, a) sum visits
    // only those (in the space of Xi, which this pass leaves unused when the
    // first pass's copies are kept)
    unsigned long long* qmask = (unsigned long long*)(l.L + wf.l_aXi) + (par && s == 1 ? wf.sp[0].nP : 0);
    if (masks) {
      for (int q = tid; q < nP; q += nth) {
        unsigned long long m = 0;
        for (int u = 0; u < st.nU; ++u) {
          if (uinf[5 * u + 1] == 0.0) continue;
          const int* ui = l.ui(s) + 8 * u;
          for (int d = 0; d < ui[0]; ++d)
            if (ui[4 + d] == q) m |= 1ull << u;
        }
        qmask[q] = m;
      }
      __syncthreads();
    }
    for (int idx = tid; idx < nP * n; idx += nth) {
      const int q = idx / n, a = idx - q * n;
      double w = 0.0, wb = 0.0, x = 0.0;
      unsigned long long m = masks ? qmask[q] : 0ull;
      for (int u0 = 0; masks ? m != 0ull : u0 < st.nU; ++u0) {
        int u = u0;
        if (masks) {
          u = __builtin_ctzll(m);
          m &= m - 1;
        }
        const int* ui = l.ui(s) + 8 * u;
        const int e = ui[0];
        if (!masks) {
          if (uinf[5 * u + 1] == 0.0) continue;  // singular: no contribution
          bool has = false;
          for (int d = 0; d < e; ++d) has = has || ui[4 + d] == q;
          if (!has) continue;
        }
        const double om = uinf[5 * u + 3], lb = uinf[5 * u + 4];
        const double* mi = V + 18 * u;
        const double* vx = mi + 9;
        double va[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < e; ++c)
          for (int c2 = 0; c2 < e; ++c2) va[c] += mi[3 * c + c2] * Bp[ui[1 + c2] * n + a];
        for (int d = 0; d < e; ++d) {
          if (ui[4 + d] != q) continue;
          double U = 0.0;
          for (int c = 0; c < e; ++c) U += mi[3 * d + c] * BS[ui[1 + c] * n + a] + vx[3 * d + c] * va[c];
          w += om * va[d];
          wb += lb * va[d];
          x += om * U;
        }
      }
      Wq[idx] = w;
      Wb[idx] = wb;
      Xq[idx] = x;
    }
    double Om = 0.0, Lb = 0.0;
    for (int u = 0; u < st.nU; ++u)
      if (uinf[5 * u + 1] != 0.0) {
        Om += uinf[5 * u + 3];
        Lb += uinf[5 * u + 4];
      }
    __syncthreads();
    const int nc = n + nP;
    for (int idx = tid; idx < n * nc; idx += nth) {
      const int a = idx / nc, col = idx - a * nc, e = e0 + a;
      double g, g0;
      int o;
      if (col < n) {
        const int b = col;
        o = ref[b];
        double sT = 0.0, sTb = 0.0, sTX = 0.0, sBX = 0.0;
        for (int q = 0; q < nP; ++q) {
          const double t = T[b * nP + q];
          sT += t * Wq[q * n + a];
          sTb += t * Wb[q * n + a];
          sTX += t * Xq[q * n + a];
          sBX += BXi[b * nP + q] * Wq[q * n + a];
        }
        g = Om * Bp[b * n + a] - sT;
        g0 = Lb * Bp[b * n + a] - sTb - Om * BS[b * n + a] - sBX + sTX;
      } else {
        const int q = col - n;
        o = porb[q];
        g = Wq[q * n + a];
        g0 = Wb[q * n + a] - Xq[q * n + a];
      }
      G[e * nop + o] += g;
      G0[e * nop + o] += g0;
    }
    __syncthreads();
  }
  // drift and Laplacian ratios of D: sum over orbitals of the channel rows times G
  for (int idx = threadIdx.x; idx < 4 * N; idx += NT) {
    const int e = idx >> 2, c = 1 + (idx & 3);
    double t = 0.0;
    for (int o = 0; o < nop; ++o) t += aPhi[(c * N + e) * nop + o] * G[e * nop + o];
    if (c < 4) l.gD()[3 * e + c - 1] = t;
    else l.lD()[e] = t;
  }
  __syncthreads();
}

template <int NT, int PREC, bool EEN>
__global__ __launch_bounds__(NT) void k_param_grad(const DevWF* __restrict__ pwf, int64_t W,
                                                   const double* __restrict__ Rin, double* dlog, double* del) {
  const DevWF& wf = *pwf;
  const int64_t w = blockIdx.x;
  if (w >= W) return;
  Ld l(lds_adj, wf);
  stage_tables<NT, PREC>(wf, l);
  const int N = wf.N, nop = wf.nop, M = wf.M;
  const int np = wf.nstruct + wf.norb * M + 6 + 6 * wf.nnuc + wf.neen * wf.nnuc;
  double* oL = dlog + w * np;
  double* oE = del + w * np;
  for (int k = threadIdx.x; k < 3 * N; k += NT) l.R()[k] = Rin[w * 3 * N + k];
  __syncthreads();
  double* aPhi = l.L + wf.l_aPhi;  // [5][N][nop]
  double* G0 = l.L + wf.l_aG0;     // [N][nop]
  double* G = l.L + wf.l_aG;       // [N][nop]
  double* A = l.L + wf.l_aA;
  double* K = l.L + wf.l_aP;
  double* M1 = l.L + wf.l_aM;
  double* sc = l.sc();

  // A. orbital rows and their derivatives at every electron
  for (int g0 = 0; g0 < N; g0 += kGroup) {
    int ne = min(kGroup, N - g0);
    group_radial<NT, PREC>(wf, l, l.R(), g0, ne);
    if constexpr (PREC == 0) {
      adj_rows5<NT>(wf, l, ne, aPhi + g0 * nop, N * nop);
    } else {
      for (int c = 0; c < 5; ++c) {
        group_channel<NT, PREC>(wf, l, ne, c);
        for (int idx = threadIdx.x; idx < ne * nop; idx += NT) aPhi[(c * N + g0) * nop + idx] = l.Phi()[idx];
        __syncthreads();
      }
    }
  }
  for (int idx = threadIdx.x; idx < N * nop; idx += NT) {
    G0[idx] = 0.0;
    G[idx] = 0.0;
  }
  // B. Jastrow factor, its gradients and Laplacians, potential
  if constexpr (EEN) {
    jastrow_full<NT, EEN>(wf, l, l.R());
  } else {
    adj_jastrow<NT>(wf, l, l.R());
  }

  // C. first pass over the spin determinants: ln|Delta_u|, sign, e_u,
  // through each spin's reference (one inversion per spin); if a reference
  // is singular, one inversion per determinant instead
  const bool lowrank = adj_ref_pass1<NT>(wf, l, aPhi, A, K, M1);
  for (int s = 0; s < 2 && !lowrank; ++s) {
    const SpinTab& st = wf.sp[s];
    const int n = st.n;
    double* uinf = l.L + wf.l_aU[s];  // [nU][5]: L, sign, e, omega, lbar
    for (int u = 0; u < st.nU; ++u) {
      const int* ui = l.ui(s) + 8 * u;
      for (int idx = threadIdx.x; idx < n * n; idx += NT) {
        int i = idx / n, j = idx - i * n;
        int o = slot_orbital(l, s, ui, j), e = st.e0 + i;
        A[idx] = aPhi[(0 * N + e) * nop + o];
        const double* gu = l.gU() + 3 * e;
        K[idx] = -(gu[0] * aPhi[(1 * N + e) * nop + o] + gu[1] * aPhi[(2 * N + e) * nop + o] +
                   gu[2] * aPhi[(3 * N + e) * nop + o]) - 0.5 * aPhi[(4 * N + e) * nop + o];
      }
      __syncthreads();
      double ld = 0.0, sg = 1.0;
      bool ok = n == 0 || gj_invert<NT>(l, A, n, ld, sg);
      // e_u = tr(A^{-1} K) = sum_{i,j} K[i][j] Ainv[j][i]
      double tr[1] = {0.0};
      if (ok)
        for (int idx = threadIdx.x; idx < n * n; idx += NT) {
          int i = idx / n, j = idx - i * n;
          tr[0] += K[idx] * A[j * n + i];
        }
      block_sum<NT, 1>(tr, l.red());
      if (threadIdx.x == 0) {
        uinf[5 * u + 0] = ok ? ld : -INFINITY;
        uinf[5 * u + 1] = ok ? sg : 0.0;
        uinf[5 * u + 2] = ok ? tr[0] : 0.0;
      }
      __syncthreads();
    }
  }
  // D. combine over determinant pairs (spin-up CSR lists every pair once)
  {
    const double* U0 = l.L + wf.l_aU[0];
    const double* U1 = l.L + wf.l_aU[1];
    // the scale of the exponentials: the largest ln|Delta| of each spin
    // summed (a bound on every pair's, the same in both uses below)
    double m0 = -INFINITY, m1 = -INFINITY;
    for (int u = 0; u < wf.sp[0].nU; ++u) m0 = fmax(m0, U0[5 * u]);
    for (int u = 0; u < wf.sp[1].nU; ++u) m1 = fmax(m1, U1[5 * u]);
    const double lmax = m0 + m1;
    double acc[2] = {0.0, 0.0};  // D~, sum t_k e_k
    for (int u = threadIdx.x; u < wf.sp[0].nU; u += NT)
      for (int k = l.wrow(0)[u]; k < l.wrow(0)[u + 1]; ++k) {
        int ub = l.woth(0)[k];
        double t = l.wcoef(0)[k] * U0[5 * u + 1] * U1[5 * ub + 1] * exp(U0[5 * u] + U1[5 * ub] - lmax);
        acc[0] += t;
        acc[1] += t * (U0[5 * u + 2] + U1[5 * ub + 2]);
      }
    if (wf.sp[0].nU <= 64) {
      // (every contribution is in wavefront 0)
      if (threadIdx.x < 64)
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
    } else {
      block_sum<NT, 2>(acc, l.red());
    }
    if (threadIdx.x == 0) {
      sc[SC_TMP0] = lmax;
      sc[SC_S] = acc[0];
      sc[SC_TMP1] = acc[1] / acc[0];  // ebar
    }
    __syncthreads();
  }
  const double lmax = sc[SC_TMP0], Dt = sc[SC_S], ebar = sc[SC_TMP1];
  for (int s = 0; s < 2; ++s) {
    const SpinTab& st = wf.sp[s];
    double* us = l.L + wf.l_aU[s];
    const double* uo = l.L + wf.l_aU[1 - s];
    for (int u = threadIdx.x; u < st.nU; u += NT) {
      double om = 0.0, lb = 0.0;
      for (int k = l.wrow(s)[u]; k < l.wrow(s)[u + 1]; ++k) {
        int ub = l.woth(s)[k];
        double Wk = l.wcoef(s)[k] * us[5 * u + 1] * uo[5 * ub + 1] * exp(us[5 * u] + uo[5 * ub] - lmax) / Dt;
        om += Wk;
        lb += Wk * (us[5 * u + 2] + uo[5 * ub + 2] - ebar);
      }
      us[5 * u + 3] = om;
      us[5 * u + 4] = lb;
    }
  }
  for (int k = threadIdx.x; k < 4 * N; k += NT) {
    if (k < 3 * N) l.gD()[k] = 0.0; else l.lD()[k - 3 * N] = 0.0;
  }
  __syncthreads();

  // E. second pass: recompute the inverses, accumulate the drift and
  // Laplacian ratios and scatter the adjoint onto orbital rows
  if (lowrank) adj_ref_pass2<NT>(wf, l, aPhi, A, K, M1, G0, G);
  for (int s = 0; s < 2 && !lowrank; ++s) {
    const SpinTab& st = wf.sp[s];
    const int n = st.n;
    const double* uinf = l.L + wf.l_aU[s];
    for (int u = 0; u < st.nU; ++u) {
      const double om = uinf[5 * u + 3], lb = uinf[5 * u + 4];
      if (uinf[5 * u + 1] == 0.0 || n == 0) continue;  // singular: no contribution
      const int* ui = l.ui(s) + 8 * u;
      for (int idx = threadIdx.x; idx < n * n; idx += NT) {
        int i = idx / n, j = idx - i * n;
        int o = slot_orbital(l, s, ui, j), e = st.e0 + i;
        A[idx] = aPhi[(0 * N + e) * nop + o];
        const double* gu = l.gU() + 3 * e;
        K[idx] = -(gu[0] * aPhi[(1 * N + e) * nop + o] + gu[1] * aPhi[(2 * N + e) * nop + o] +
                   gu[2] * aPhi[(3 * N + e) * nop + o]) - 0.5 * aPhi[(4 * N + e) * nop + o];
      }
      __syncthreads();
      double ld, sg;
      gj_invert<NT>(l, A, n, ld, sg);
      // drift and Laplacian ratios of this determinant, weighted by omega
      for (int idx = threadIdx.x; idx < 4 * n; idx += NT) {
        int i = idx >> 2, c = 1 + (idx & 3), e = st.e0 + i;
        double g = 0.0;
        for (int j = 0; j < n; ++j) g += aPhi[(c * N + e) * nop + slot_orbital(l, s, ui, j)] * A[j * n + i];
        if (c < 4) l.gD()[3 * e + c - 1] += om * g; else l.lD()[e] += om * g;
      }
      // M1 = K A^{-1}
      for (int idx = threadIdx.x; idx < n * n; idx += NT) {
        int i = idx / n, a = idx - i * n;
        double t = 0.0;
        for (int j = 0; j < n; ++j) t += K[i * n + j] * A[j * n + a];
        M1[idx] = t;
      }
      __syncthreads();
      // Abar[a][b] = lbar Ainv[b][a] - omega sum_i Ainv[b][i] M1[i][a]; scatter
      for (int idx = threadIdx.x; idx < n * n; idx += NT) {
        int a = idx / n, b = idx - a * n;
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += A[b * n + i] * M1[i * n + a];
        int o = slot_orbital(l, s, ui, b), e = st.e0 + a;
        G0[e * nop + o] += lb * A[b * n + a] - om * t;
        G[e * nop + o] += om * A[b * n + a];
      }
      __syncthreads();
    }
  }

  // F. local energy (as a by-product), structure and Jastrow derivatives
  {
    double part[1] = {0.0};
    for (int i = threadIdx.x; i < N; i += NT) {
      double t = l.lU()[i] + l.lD()[i];
      for (int x = 0; x < 3; ++x) {
        double gu = l.gU()[3 * i + x];
        t += gu * gu + 2.0 * gu * l.gD()[3 * i + x];
      }
      part[0] += -0.5 * t;
    }
    block_sum<NT, 1>(part, l.red());
    if (threadIdx.x == 0) sc[SC_ELOC] = part[0] + sc[SC_V];
  }
  {
    const double* U0 = l.L + wf.l_aU[0];
    const double* U1 = l.L + wf.l_aU[1];
    for (int I = threadIdx.x; I < wf.nstruct; I += NT) {
      double r = 0.0, re = 0.0;
      for (int k = l.srow()[I]; k < l.srow()[I + 1]; ++k) {
        int u0 = l.slu()[2 * k], u1 = l.slu()[2 * k + 1];
        double t = l.slc()[k] * U0[5 * u0 + 1] * U1[5 * u1 + 1] * exp(U0[5 * u0] + U1[5 * u1] - lmax) / Dt;
        r += t;
        re += t * (U0[5 * u0 + 2] + U1[5 * u1 + 2]);
      }
      oL[I] = r;
      oE[I] = re - r * ebar;
    }
  }
  // Jastrow: electron-electron parameters [b_anti, b_par, b3..b6], one
  // electron pair per thread
  const int jb = wf.nstruct + wf.norb * M;
  {
    double acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    const double* R = l.R();
    for (int pidx = threadIdx.x; pidx < N * N; pidx += NT) {
      const int i = pidx / N, j = pidx - i * N;
      if (j <= i) continue;
      double dx = R[3 * i] - R[3 * j], dy = R[3 * i + 1] - R[3 * j + 1], dz = R[3 * i + 2] - R[3 * j + 2];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      bool anti = spin_of(wf, i) != spin_of(wf, j);
      double a = anti ? wf.ee[0] : wf.ee[1], b = anti ? wf.ee[2] : wf.ee[3];
      double proj = 0.0;
      {
        const double* gi = l.gU() + 3 * i;
        const double* gj = l.gU() + 3 * j;
        const double* di = l.gD() + 3 * i;
        const double* dj = l.gD() + 3 * j;
        proj = (dx * (gi[0] + di[0] - gj[0] - dj[0]) + dy * (gi[1] + di[1] - gj[1] - dj[1]) +
                dz * (gi[2] + di[2] - gj[2] - dj[2])) / r;
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        if (q == 0 && !anti) continue;
        if (q == 1 && anti) continue;
        double du, du1, du2;
        pair_param(r, wf.kappa, a, b, q < 2 ? 1 : q, du, du1, du2);
        acc[q] += du;
        acc[6 + q] += -0.5 * (2.0 * (du2 + 2.0 * du1 / r) + 2.0 * du1 * proj);
      }
    }
    block_sum<NT, 12>(acc, l.red());
    if (threadIdx.x == 0)
      for (int q = 0; q < 6; ++q) {
        oL[jb + q] = acc[q];
        oE[jb + q] = acc[6 + q];
      }
  }
  // electron-nucleus parameters [a1..a6] per nucleus: nucleus al on a
  // segment of SEG lanes (lane i of the segment takes electron i), summed
  // within the segment; more than 64 electrons: one nucleus at a time over
  // the block
  const int SEG = N <= 16 ? 16 : (N <= 32 ? 32 : 64);
  if (N <= 64) {
    const int per = NT / SEG;  // nuclei per pass over the block
    const int i = threadIdx.x % SEG;
    for (int base = 0; base < wf.nnuc; base += per) {
      const int al = base + threadIdx.x / SEG;
      double acc[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = 0.0;
      if (al < wf.nnuc && i < N) {
        const double* ja = l.en() + 6 * al;
        const double* nu = l.nuc() + 4 * al;
        const double* R = l.R() + 3 * i;
        double dx = R[0] - nu[0], dy = R[1] - nu[1], dz = R[2] - nu[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double* gi = l.gU() + 3 * i;
        const double* di = l.gD() + 3 * i;
        double proj = (dx * (gi[0] + di[0]) + dy * (gi[1] + di[1]) + dz * (gi[2] + di[2])) / r;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          double du, du1, du2;
          pair_param(r, wf.kappa, ja[0], ja[1], q, du, du1, du2);
          acc[q] = du;
          acc[6 + q] = -0.5 * ((du2 + 2.0 * du1 / r) + 2.0 * du1 * proj);
        }
      }
      // (every lane of the wavefront takes part; xor offsets below SEG stay
      // inside the segment)
#pragma unroll
      for (int k = 0; k < 12; ++k)
        for (int off = SEG / 2; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
      if (i == 0 && al < wf.nnuc)
        for (int q = 0; q < 6; ++q) {
          oL[jb + 6 + 6 * al + q] = acc[q];
          oE[jb + 6 + 6 * al + q] = acc[6 + q];
        }
    }
  } else {
    for (int al = 0; al < wf.nnuc; ++al) {
      double acc[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[k] = 0.0;
      const double* ja = l.en() + 6 * al;
      const double* nu = l.nuc() + 4 * al;
      for (int i = threadIdx.x; i < N; i += NT) {
        const double* R = l.R() + 3 * i;
        double dx = R[0] - nu[0], dy = R[1] - nu[1], dz = R[2] - nu[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double* gi = l.gU() + 3 * i;
        const double* di = l.gD() + 3 * i;
        double proj = (dx * (gi[0] + di[0]) + dy * (gi[1] + di[1]) + dz * (gi[2] + di[2])) / r;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          double du, du1, du2;
          pair_param(r, wf.kappa, ja[0], ja[1], q, du, du1, du2);
          acc[q] += du;
          acc[6 + q] += -0.5 * ((du2 + 2.0 * du1 / r) + 2.0 * du1 * proj);
        }
      }
      block_sum<NT, 12>(acc, l.red());
      if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q) {
          oL[jb + 6 + 6 * al + q] = acc[q];
          oE[jb + 6 + 6 * al + q] = acc[6 + q];
        }
      __syncthreads();
    }
  }
  // f_een coefficients [c_1..c_23] per nucleus: d ln|Psi|/dc_t is the sum
  // over pairs of term t, T_t = a^k B_t (a = Rbar_ij, B_t = b^(l+m) c^m +
  // b^m c^(l+m), b = Rbar_ia, c = Rbar_ja); d E_L/dc_t =
  // -1/2 sum_i (lap_i T_t + 2 grad_i T_t . grad_i ln|Psi|), each ordered
  // pair (i, j) giving electron i's derivatives (and half the value)
  if constexpr (EEN) {
    const int je = jb + 6 + 6 * wf.nnuc;
    const double kap = wf.kappa;
    for (int al = 0; al < wf.nnuc; ++al) {
      double acc[2 * kEenTerms];
#pragma unroll
      for (int k = 0; k < 2 * kEenTerms; ++k) acc[k] = 0.0;
      const double* nu = l.nuc() + 4 * al;
      for (int i = threadIdx.x; i < N; i += NT) {
        const double* Ri = l.R() + 3 * i;
        const double ex = Ri[0] - nu[0], ey = Ri[1] - nu[1], ez = Ri[2] - nu[2];
        const double ria = sqrt(ex * ex + ey * ey + ez * ez), iria = 1.0 / ria;
        const double b = 1.0 / (1.0 + kap * ria), b1 = -kap * b * b, b2 = 2.0 * kap * kap * b * b * b;
        const double* gi = l.gU() + 3 * i;
        const double* di = l.gD() + 3 * i;
        const double G0 = gi[0] + di[0], G1 = gi[1] + di[1], G2 = gi[2] + di[2];
        const double eG = (ex * G0 + ey * G1 + ez * G2) * iria;
        for (int j = 0; j < N; ++j) {
          if (j == i) continue;
          const double* Rj = l.R() + 3 * j;
          const double dx = Ri[0] - Rj[0], dy = Ri[1] - Rj[1], dz = Ri[2] - Rj[2];
          const double rij = sqrt(dx * dx + dy * dy + dz * dz), irij = 1.0 / rij;
          const double a = 1.0 / (1.0 + kap * rij), a1 = -kap * a * a, a2 = 2.0 * kap * kap * a * a * a;
          const double fx = Rj[0] - nu[0], fy = Rj[1] - nu[1], fz = Rj[2] - nu[2];
          const double c = 1.0 / (1.0 + kap * sqrt(fx * fx + fy * fy + fz * fz));
          const double dG = (dx * G0 + dy * G1 + dz * G2) * irij;
          const double cosde = (dx * ex + dy * ey + dz * ez) * irij * iria;
          double pa[5], pb[6], pc[6];
          pa[0] = pb[0] = pc[0] = 1.0;
#pragma unroll
          for (int q = 1; q < 6; ++q) {
            if (q < 5) pa[q] = pa[q - 1] * a;
            pb[q] = pb[q - 1] * b;
            pc[q] = pc[q - 1] * c;
          }
#pragma unroll
          for (int t = 0; t < kEenTerms; ++t) {
            const int k = kEenK[t], m = kEenM[t], n = kEenL[t] + m;
            const double B = pb[n] * pc[m] + pb[m] * pc[n];
            const double B1 = (n > 0 ? n * pb[n > 0 ? n - 1 : 0] * pc[m] : 0.0) +
                              (m > 0 ? m * pb[m > 0 ? m - 1 : 0] * pc[n] : 0.0);
            const double B2 = (n > 1 ? n * (n - 1) * pb[n > 1 ? n - 2 : 0] * pc[m] : 0.0) +
                              (m > 1 ? m * (m - 1) * pb[m > 1 ? m - 2 : 0] * pc[n] : 0.0);
            const double A1 = k > 0 ? k * pa[k > 0 ? k - 1 : 0] : 0.0;
            const double A2 = k > 1 ? k * (k - 1) * pa[k > 1 ? k - 2 : 0] : 0.0;
            const double gT = A1 * B * a1 * dG + pa[k] * B1 * b1 * eG;
            const double lT = A2 * B * a1 * a1 + A1 * B * (a2 + 2.0 * a1 * irij) + pa[k] * B2 * b1 * b1 +
                              pa[k] * B1 * (b2 + 2.0 * b1 * iria) + 2.0 * A1 * B1 * a1 * b1 * cosde;
            acc[t] += 0.5 * pa[k] * B;
            acc[kEenTerms + t] += -0.5 * (lT + 2.0 * gT);
          }
        }
      }
      // (reduced 16 at a time: the reduction scratch holds 64 doubles)
      for (int q0 = 0; q0 < 2 * kEenTerms; q0 += 16) {
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = q0 + k < 2 * kEenTerms ? acc[min(q0 + k, 2 * kEenTerms - 1)] : 0.0;
        block_sum<NT, 16>(v, l.red());
        if (threadIdx.x == 0)
          for (int k = 0; k < 16 && q0 + k < 2 * kEenTerms; ++k) {
            const int q = q0 + k;
            if (q < kEenTerms) oL[je + kEenTerms * al + q] = v[k];
            else oE[je + kEenTerms * al + q - kEenTerms] = v[k];
          }
      }
      __syncthreads();
    }
  }

  // G. orbital-coefficient derivatives: contractions over electrons on MFMA,
  // 16 (basis function) columns x up to two 16-orbital row tiles per wave at
  // a time, so that each basis function's channels at an electron are formed
  // once for both row tiles
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  const int npt = nop / 16, nmt = wf.Mpad / 16, npc = (npt + 1) / 2;
  double* oLl = oL + wf.nstruct;
  double* oEl = oE + wf.nstruct;
  for (int g0 = 0; g0 < N; g0 += kGroup) {
    int ne = min(kGroup, N - g0);
    group_radial<NT, 0>(wf, l, l.R(), g0, ne);  // FP64 basis rows for the contraction
    for (int tile = wave; tile < npc * nmt; tile += NW) {
      const int pc = tile / nmt, mt = tile - pc * nmt;
      const int pt0 = 2 * pc;
      const bool two = pt0 + 1 < npt;  // (the same in the whole wave)
      const int pcol = pt0 * 16 + (lane & 15), mcol = mt * 16 + (lane & 15);
      v4d accE[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, accL[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
      for (int k0 = 0; k0 < kGroup; k0 += 4) {
        int e = k0 + (lane >> 4);
        double a0[2] = {0.0, 0.0}, aG[2] = {0.0, 0.0}, bv = 0.0, bk = 0.0;
        if (e < ne) {
          a0[0] = G0[(g0 + e) * nop + pcol];
          aG[0] = G[(g0 + e) * nop + pcol];
          if (two) {
            a0[1] = G0[(g0 + e) * nop + pcol + 16];
            aG[1] = G[(g0 + e) * nop + pcol + 16];
          }
          double ch[5];
          chan_all<double>(wf, l, e, mcol, ch);
          const double* gu = l.gU() + 3 * (g0 + e);
          bv = ch[0];
          bk = -(gu[0] * ch[1] + gu[1] * ch[2] + gu[2] * ch[3]) - 0.5 * ch[4];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h == 1 && !two) break;
          accE[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[h], bv, accE[h], 0, 0, 0);
          accE[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(aG[h], bk, accE[h], 0, 0, 0);
          accL[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(aG[h], bv, accL[h], 0, 0, 0);
        }
      }
      // f64 output layout: register r of lane l holds row 4r + l/16
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h == 1 && !two) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int p = (pt0 + h) * 16 + 4 * r + (lane >> 4), mu = mt * 16 + (lane & 15);
          if (p < wf.norb && mu < M) {
            size_t o = (size_t)p * M + mu;
            if (g0 == 0) {
              oEl[o] = accE[h][r];
              oLl[o] = accL[h][r];
            } else {
              oEl[o] += accE[h][r];
              oLl[o] += accL[h][r];
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

size_t param_grad_ws_doubles(const DevWF& wf, int64_t W) {
  (void)wf;
  (void)W;
  return 0;
}

template <int NT, int PREC, bool EEN = false>
static hipError_t launch_pg(const DevWF& wf, const DevWF* dwf, int64_t W, const double* R, double* dl, double* de,
                            hipStream_t s) {
  size_t lds = (size_t)wf.lds_adj_doubles * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_param_grad<NT, PREC, EEN>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_param_grad<NT, PREC, EEN>), dim3((unsigned)W), dim3(NT), lds, s, dwf, W, R, dl, de);
  return hipGetLastError();
}

hipError_t launch_param_grad(const DevWF& wf, const DevWF* dwf, int nt, int64_t W, const double* R, double* dlogpsi,
                             double* deloc, double* ws, size_t ws_doubles, hipStream_t s) {
  (void)ws;
  (void)ws_doubles;
  // the adjoint runs its determinant algebra and contractions in FP64 for
  // every precision form; the orbital rows follow the context's precision
  // (f_een systems are FP64 only)
  if (wf.neen) {
    if (nt == 64) return launch_pg<64, 0, true>(wf, dwf, W, R, dlogpsi, deloc, s);
    if (nt == 128) return launch_pg<128, 0, true>(wf, dwf, W, R, dlogpsi, deloc, s);
    return launch_pg<256, 0, true>(wf, dwf, W, R, dlogpsi, deloc, s);
  }
  if (nt == 64) {
    if (wf.precision == 0) return launch_pg<64, 0>(wf, dwf, W, R, dlogpsi, deloc, s);
    return launch_pg<64, 1>(wf, dwf, W, R, dlogpsi, deloc, s);
  }
  if (nt == 128) {
    if (wf.precision == 0) return launch_pg<128, 0>(wf, dwf, W, R, dlogpsi, deloc, s);
    return launch_pg<128, 1>(wf, dwf, W, R, dlogpsi, deloc, s);
  }
  if (nt == 512 && wf.precision == 0) return launch_pg<512, 0>(wf, dwf, W, R, dlogpsi, deloc, s);
  if (wf.precision == 0) return launch_pg<256, 0>(wf, dwf, W, R, dlogpsi, deloc, s);
  return launch_pg<256, 1>(wf, dwf, W, R, dlogpsi, deloc, s);
}

}  // namespace vbqmc
