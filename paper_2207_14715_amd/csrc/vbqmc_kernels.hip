// gfx950 kernels for the Jastrow-Valence-Bond (JVB) QMC hot path.
//
// Design: one workgroup owns one walker.  Its hot state (positions, the
// reference inverse and determinant table of each spin) is held in LDS for the
// whole call, so a VMC call runs every step of every walker without touching
// HBM except at entry and exit, and a DMC step reads and writes each record
// once.  Per move the basis values at the trial position are formed by one
// lane per shell, contracted to orbital values on the VALU, and turned into
// determinant ratios with the reference + replaced-column table.  The local
// energy pass forms basis values/gradients/Laplacians for tiles of 16
// electrons in LDS and contracts them with the orbital coefficients on MFMA
// (FP64 16x16x4, FP32 16x16x4 or BF16 16x16x16 by precision form).
//
// Method (Radenkovic, Domin, Toulouse, Braida 2022):
//   Sec. 2.1 Eq. (PsiJVBSCF), Eq. (PhiI): Psi = J sum_I c_I Phi_I with HLSP
//     structures expanded into spin-determinant products.
//   Sec. 2.1: orbitals as basis expansions; Jastrow pair terms in
//     R = r / (1 + kappa r).
//   Sec. 2.3.1 Eq. (Elav): E_L = H Psi / Psi, Metropolis sampling.
//   Sec. 2.3.2 Eq. (E0DMCweights): weighted walkers with birth/death.
//
// Determinant algebra (exact identities, no approximation): for one spin with
// reference matrix A0[i][j] = phi_{ref_j}(r_i), B = A0^{-1} and the table
// T = B Phi[:, P] over the orbitals P that replace reference columns, a
// determinant replacing slots J by orbitals Q has ratio det(T[J, Q]) to the
// reference (matrix determinant lemma).  A row operator O on electron i
// (gradient or Laplacian) or a move of electron i with new row w gives
//   O_i Delta_u / Delta_0 = rho R_u + y_Q^T adj(T_JQ) B[J, i],
//   rho = sum_j w[ref_j] B[j][i],  y[q] = w[P_q] - sum_l w[ref_l] T[l][q],
// and an accepted move updates B and T by Sherman-Morrison rank-1 steps.

#include "vbqmc_device.h"
#include "vbqmc_ecp.h"

namespace vbqmc {

// ---------------------------------------------------------------------------
// record I/O
// ---------------------------------------------------------------------------
template <int NT>
__device__ void load_record(const DevWF& wf, const Ld& l, const double* rec) {
  for (int k = threadIdx.x; k < 3 * wf.N; k += NT) l.R()[k] = rec[wf.r_R + k];
  for (int s = 0; s < 2; ++s) {
    const SpinTab& st = wf.sp[s];
    for (int k = threadIdx.x; k < st.n * st.n; k += NT) l.B(s)[k] = rec[wf.r_B[s] + k];
    for (int k = threadIdx.x; k < st.n * st.nP; k += NT) l.T(s)[k] = rec[wf.r_T[s] + k];
  }
  for (int k = threadIdx.x; k < 8; k += NT) l.sc()[k] = rec[wf.r_sc + k];
  __syncthreads();
}

template <int NT>
__device__ void store_record(const DevWF& wf, const Ld& l, double* rec) {
  for (int k = threadIdx.x; k < 3 * wf.N; k += NT) rec[wf.r_R + k] = l.R()[k];
  for (int s = 0; s < 2; ++s) {
    const SpinTab& st = wf.sp[s];
    for (int k = threadIdx.x; k < st.n * st.n; k += NT) rec[wf.r_B[s] + k] = l.B(s)[k];
    for (int k = threadIdx.x; k < st.n * st.nP; k += NT) rec[wf.r_T[s] + k] = l.T(s)[k];
  }
  for (int k = threadIdx.x; k < 8; k += NT) rec[wf.r_sc + k] = l.sc()[k];
  // determinant ratios, their partner sums and S for the batched local energy
  const int n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
  for (int k = threadIdx.x; k < n0; k += NT) rec[wf.r_RW + k] = l.Ru(0)[k];
  for (int k = threadIdx.x; k < n1; k += NT) rec[wf.r_RW + n0 + k] = l.Ru(1)[k];
  for (int k = threadIdx.x; k < n0; k += NT) rec[wf.r_RW + n0 + n1 + k] = l.Wu(0)[k];
  for (int k = threadIdx.x; k < n1; k += NT) rec[wf.r_RW + 2 * n0 + n1 + k] = l.Wu(1)[k];
  if (threadIdx.x == 0) rec[wf.r_RW + 2 * (n0 + n1)] = l.sc()[SC_S];
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
extern __shared__ double lds_dyn[];

// ---------------------------------------------------------------------------
// Pseudopotential part of the local energy (Sec. 2.1: valence calculations
// with energy-consistent pseudopotentials; the semilocal form).  Per
// pseudo-nucleus a and electron i at distance r: the local radial part, and
// for r < r_cut each nonlocal channel l as (2l + 1) times the mean over the
// 12 icosahedron directions u_q of P_l(u_q . (r_i - a) / r) Psi(r_i -> a +
// r u_q) / Psi, the ratio formed like a single-electron move (orbital row at
// the point, determinant-table ratio, Jastrow change).  The whole workgroup
// runs every point; thread 0 sums.  Returns the energy in every thread.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ecp_radial(const double* t, int k0, int k1, double r) {
  double v = 0.0;
  for (int k = k0; k < k1; ++k) {
    const int n = (int)t[3 * k + 1];
    double p = 1.0;
    for (int e = 2; e < n; ++e) p *= r;
    for (int e = n; e < 2; ++e) p /= r;
    v += t[3 * k] * p * exp(-t[3 * k + 2] * r * r);
  }
  return v;
}

// direction q of the rule: the cyclic form q >> 2 of (0, +-1, +-g) / |.|,
// signs from the low bits
__device__ __forceinline__ void ecp_dir(int q, double& ux, double& uy, double& uz) {
  const double g = 1.6180339887498949, un = 1.0 / sqrt(1.0 + g * g);
  const double s1 = (q & 1) ? un : -un, s2 = (q & 2) ? g * un : -g * un;
  const int k = q >> 2;
  ux = k == 0 ? 0.0 : (k == 1 ? s1 : s2);
  uy = k == 0 ? s1 : (k == 1 ? s2 : 0.0);
  uz = k == 0 ? s2 : (k == 1 ? 0.0 : s1);
}

// The 12 ratios of electron i moved onto the sphere about a, all at once in
// the scratch: basis values of the points (one thread per point and
// function), their orbital rows, per point rho = sum_j v[ref_j] B[j][i],
// the table residuals y, the Jastrow change and S'' = sum_u Q_u W_u, the
// per-point sums split over C thread groups and added in a fixed order.
// Returns sum_q w_q Psi_q / Psi in thread 0.
template <int NT>
__device__ double ecp_pair_batched(const DevWF& wf, const Ld& l, const DevEcp& ep, int i, double ax, double ay,
                                   double az, double dx, double dy, double dz, double r, const double* vl, int L) {
  constexpr int K = kEcpPts;
  constexpr int C = NT / K > 0 ? NT / K : 1;
  const int s = spin_of(wf, i);
  const SpinTab& st = wf.sp[s];
  const int n = st.n, nP = st.nP, il = i - st.e0, nPm = ep.nPmax > 0 ? ep.nPmax : 1;
  const double* B = l.B(s);
  const double* T = l.T(s);
  const int* ref = l.ref(s);
  const int* porb = l.porb(s);
  const double* nuc = l.nuc();
  double* Pq = l.L + ep.l_scr;          // [K][4]
  double* chi = Pq + 4 * K;             // [K][Mpad]
  double* v = chi + K * wf.Mpad;        // [K][nop]
  double* y = v + K * wf.nop;           // [K][nPm]
  double* part = y + K * nPm;           // [3][C][K]
  double* res = part + 3 * C * K;       // [K][3]
  if (threadIdx.x < K) {
    double ux, uy, uz;
    ecp_dir(threadIdx.x, ux, uy, uz);
    Pq[4 * threadIdx.x] = ax + r * ux;
    Pq[4 * threadIdx.x + 1] = ay + r * uy;
    Pq[4 * threadIdx.x + 2] = az + r * uz;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < K * wf.Mpad; idx += NT) {
    const int q = idx / wf.Mpad, mu = idx - q * wf.Mpad;
    const int sh = l.fn()[2 * mu];
    double o = 0.0;
    if (sh >= 0) {
      const int* si = l.sh() + 8 * sh;
      const int a = si[0], kind = si[1], lq = si[2], p0 = si[4], np = si[5];
      const double x = Pq[4 * q] - nuc[4 * a], yy = Pq[4 * q + 1] - nuc[4 * a + 1], z = Pq[4 * q + 2] - nuc[4 * a + 2];
      const double r2 = x * x + yy * yy + z * z, rr = sqrt(r2);
      double g = 0.0;
      for (int k = 0; k < np; ++k) {
        const double t = kind == 0 ? l.pe()[p0 + k] * r2 : l.pe()[p0 + k] * rr;
        if (t < 50.0) g += l.pc()[p0 + k] * exp_neg<double>(t, l.L + wf.l_etab);
      }
      channels<double>(kind, lq, l.fn()[2 * mu + 1] & 15, x, yy, z, r2, rr, g, 0.0, 0.0, 1, &o);
    }
    chi[idx] = o;
  }
  __syncthreads();
  const double* lam = l.lam<double>();
  for (int idx = threadIdx.x; idx < K * wf.nop; idx += NT) {
    const int q = idx / wf.nop, o = idx - q * wf.nop;
    const double* ch = chi + q * wf.Mpad;
    double acc = 0.0;
#pragma unroll 4
    for (int mu = 0; mu < wf.Mpad; ++mu) acc += ch[mu] * lam[(size_t)mu * wf.nop + o];
    v[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < K * nP; idx += NT) {
    const int q = idx / nP, p = idx - q * nP;
    const double* vq = v + q * wf.nop;
    double a = vq[porb[p]];
    for (int k = 0; k < n; ++k) a -= vq[ref[k]] * T[k * nP + p];
    y[q * nPm + p] = a;
  }
  const double* R = l.R();
  const double xo = R[3 * i], yo = R[3 * i + 1], zo = R[3 * i + 2];
  const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
  for (int t = threadIdx.x; t < C * K; t += NT) {
    const int q = t % K, c = t / K;
    const double* vq = v + q * wf.nop;
    double rho = 0.0, du = 0.0;
    for (int j = c; j < n; j += C) rho += vq[ref[j]] * B[j * n + il];
    const double px = Pq[4 * q], py = Pq[4 * q + 1], pz = Pq[4 * q + 2];
    for (int j = c; j < wf.N + wf.nnuc; j += C) {
      if (j == i) continue;
      double xj, yj, zj;
      PairCoef cf;
      if (j < wf.N) {
        xj = R[3 * j]; yj = R[3 * j + 1]; zj = R[3 * j + 2];
        cf = s != spin_of(wf, j) ? c_anti : c_par;
      } else {
        const int nn = j - wf.N;
        xj = nuc[4 * nn]; yj = nuc[4 * nn + 1]; zj = nuc[4 * nn + 2];
        cf = en_coef(l.en() + 6 * nn);
      }
      const double rn = sqrt((px - xj) * (px - xj) + (py - yj) * (py - yj) + (pz - zj) * (pz - zj));
      const double ro = sqrt((xo - xj) * (xo - xj) + (yo - yj) * (yo - yj) + (zo - zj) * (zo - zj));
      du += pair_val(rn, wf.kappa, cf) - pair_val(ro, wf.kappa, cf);
    }
    part[c * K + q] = rho;
    part[(C + c) * K + q] = du;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    const int q = threadIdx.x;
    double rho = 0.0, du = 0.0;
    for (int c = 0; c < C; ++c) {
      rho += part[c * K + q];
      du += part[(C + c) * K + q];
    }
    res[3 * q] = rho;
    res[3 * q + 1] = du;
  }
  __syncthreads();
  const int* uit = l.ui(s);
  for (int t = threadIdx.x; t < C * K; t += NT) {
    const int q = t % K, c = t / K;
    const double rho = res[3 * q];
    double acc = 0.0;
    for (int u = c; u < st.nU; u += C) {
      const int* ui = uit + 8 * u;
      double m[9], yy[3], bb[3];
      const int e = gather_u(ui, T, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k < e) {
          yy[k] = y[q * nPm + ui[4 + k]];
          bb[k] = B[ui[1 + k] * n + il];
        }
      acc += (rho * l.Ru(s)[u] + adj_e(e, m, yy, bb)) * l.Wu(s)[u];
    }
    part[(2 * C + c) * K + q] = acc;
  }
  __syncthreads();
  double e = 0.0;
  if (threadIdx.x == 0) {
    const double S = l.sc()[SC_S];
    for (int q = 0; q < K; ++q) {
      double ux, uy, uz;
      ecp_dir(q, ux, uy, uz);
      const double x = (ux * dx + uy * dy + uz * dz) / r;
      const double P[kEcpMaxL] = {1.0, x, 0.5 * (3.0 * x * x - 1.0), 0.5 * (5.0 * x * x * x - 3.0 * x)};
      double wq = 0.0;
      for (int k = 0; k < L; ++k) wq += vl[k] * P[k];
      double Sq = 0.0;
      for (int c = 0; c < C; ++c) Sq += part[(2 * C + c) * K + q];
      e += wq * (Sq / S) * exp(res[3 * q + 1]);
    }
  }
  __syncthreads();  // the scratch is reused by the next pair
  return e;
}

template <int NT, int PREC>
__device__ double ecp_energy(const DevWF& wf, const Ld& l, const DevEcp& ep) {
  const double* nuc = l.nuc();
  double* sc = l.sc();
  double part[1] = {0.0};  // local parts (all threads) + nonlocal points (thread 0)
  for (int c = 0; c < ep.ncen; ++c) {
    const int* inf = ep.info + 8 * c;
    const int a = inf[0], L = inf[1];
    const double ax = nuc[4 * a], ay = nuc[4 * a + 1], az = nuc[4 * a + 2];
    for (int i = threadIdx.x; i < wf.N; i += NT) {
      const double dx = l.R()[3 * i] - ax, dy = l.R()[3 * i + 1] - ay, dz = l.R()[3 * i + 2] - az;
      part[0] += ecp_radial(ep.terms, inf[2], inf[3], sqrt(dx * dx + dy * dy + dz * dz));
    }
    if (L == 0) continue;
    const double rc = ep.rcut[c];
    for (int i = 0; i < wf.N; ++i) {
      const double dx = l.R()[3 * i] - ax, dy = l.R()[3 * i + 1] - ay, dz = l.R()[3 * i + 2] - az;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (!(r < rc)) continue;  // (the same decision in every thread)
      double vl[kEcpMaxL];
      for (int q = 0; q < L; ++q) vl[q] = (2 * q + 1) * ecp_radial(ep.terms, inf[3 + q], inf[4 + q], r) / kEcpPts;
      if (PREC == 0 && ep.l_scr >= 0) {
        part[0] += ecp_pair_batched<NT>(wf, l, ep, i, ax, ay, az, dx, dy, dz, r, vl, L);
        continue;
      }
      for (int q = 0; q < kEcpPts; ++q) {
        double ux, uy, uz;
        ecp_dir(q, ux, uy, uz);
        const double px = ax + r * ux, py = ay + r * uy, pz = az + r * uz;
        point_orbitals<NT, PREC>(wf, l, px, py, pz, 1);
        move_ratio<NT>(wf, l, i, px, py, pz, l.v());
        if (threadIdx.x == 0) {
          const double x = (ux * dx + uy * dy + uz * dz) / r;
          const double P[kEcpMaxL] = {1.0, x, 0.5 * (3.0 * x * x - 1.0), 0.5 * (5.0 * x * x * x - 3.0 * x)};
          double wq = 0.0;
          for (int m = 0; m < L; ++m) wq += vl[m] * P[m];
          part[0] += wq * sc[SC_RATIO] * exp(sc[SC_TMP0]);
        }
      }
    }
  }
  block_sum<NT, 1>(part, l.red());
  return part[0];
}

// E_L (SC_ELOC) += the pseudopotential energy
template <int NT, int PREC>
__device__ void ecp_add(const DevWF& wf, const Ld& l, const DevEcp& ep) {
  const double e = ecp_energy<NT, PREC>(wf, l, ep);
  if (threadIdx.x == 0) l.sc()[SC_ELOC] += e;
  __syncthreads();
}

template <int NT, int PREC, bool EEN = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_evaluate(const DevWF* __restrict__ pwf, int64_t W, const double* __restrict__ Rin,
                                                 int64_t rstride, double* logabs, int32_t* sign, double* grad,
                                                 double* eloc, double* ratio, double* state, DevEcp ecp) {
  const DevWF& wf = *pwf;
  int64_t w = blockIdx.x;
  if (w >= W) return;
  Ld l(lds_dyn, wf);
  stage_tables<NT, PREC>(wf, l);
  bool nonfinite = false;
  for (int k = threadIdx.x; k < 3 * wf.N; k += NT) {
    const double x = Rin[w * rstride + k];
    nonfinite |= !isfinite(x);
    l.R()[k] = x;
  }
  // a configuration with a non-finite coordinate is reported like Psi = 0
  // (and its record flagged) without being evaluated
  bool ok = !__syncthreads_or(nonfinite) && build_state<NT, PREC>(wf, l, l.R());
  if (ok) {
    compute_RWS<NT>(wf, l);
    ok = l.sc()[SC_S] != 0.0;
  }
  if (!ok) {
    if (threadIdx.x == 0) {
      if (logabs) logabs[w] = -INFINITY;
      if (sign) sign[w] = 0;
      if (eloc) eloc[w] = NAN;
    }
    if (grad)
      for (int k = threadIdx.x; k < 3 * wf.N; k += NT) grad[w * 3 * wf.N + k] = NAN;
    if (ratio)
      for (int k = threadIdx.x; k < wf.nstruct; k += NT) ratio[w * wf.nstruct + k] = NAN;
    if (state) {
      if (threadIdx.x == 0) {
        l.sc()[SC_ELOC] = NAN;
        l.sc()[SC_FLAGS] = 1.0;
      }
      __syncthreads();
      store_record<NT>(wf, l, state + w * wf.rec_len);
    }
    return;
  }
  local_energy<NT, PREC, EEN>(wf, l, state ? state + w * wf.rec_len + wf.r_gc : nullptr);
  if (ecp.ncen) ecp_add<NT, PREC>(wf, l, ecp);
  if (ratio) structure_ratios<NT>(wf, l);
  double* sc = l.sc();
  if (threadIdx.x == 0) {
    sc[SC_FLAGS] = 0.0;  // a freshly built record is valid
    if (logabs) logabs[w] = sc[SC_LOGPSI];
    if (sign) sign[w] = (int32_t)sc[SC_SIGN];
    if (eloc) eloc[w] = sc[SC_ELOC];
  }
  if (grad)
    for (int k = threadIdx.x; k < 3 * wf.N; k += NT) grad[w * 3 * wf.N + k] = l.gU()[k] + l.gD()[k];
  if (ratio)
    for (int k = threadIdx.x; k < wf.nstruct; k += NT) ratio[w * wf.nstruct + k] = l.ratio()[k];
  if (state) store_record<NT>(wf, l, state + w * wf.rec_len);
}

// all-electron Metropolis move (one per step)
template <int NT, int PREC, bool EEN>
__device__ bool all_electron_move(const DevWF& wf, const Ld& l, int64_t w, uint64_t seed, uint32_t step,
                                  double step_size) {
  double* sc = l.sc();
  // back up the current state in the record's backup area
  double* bk = l.bk;
  for (int k = threadIdx.x; k < 3 * wf.N; k += NT) bk[wf.r_R + k] = l.R()[k];
  for (int s = 0; s < 2; ++s) {
    const SpinTab& st = wf.sp[s];
    for (int k = threadIdx.x; k < st.n * st.n; k += NT) bk[wf.r_B[s] + k] = l.B(s)[k];
    for (int k = threadIdx.x; k < st.n * st.nP; k += NT) bk[wf.r_T[s] + k] = l.T(s)[k];
  }
  double old_log = sc[SC_U] + sc[SC_LOGDET0] + sc[SC_LOGDET1] + log(fabs(sc[SC_S]));
  double bks[4] = {sc[SC_LOGDET0], sc[SC_LOGDET1], sc[SC_SGN0], sc[SC_SGN1]};
  double bkS = sc[SC_S], bkU = sc[SC_U];
  __syncthreads();
  for (int e = threadIdx.x; e < wf.N; e += NT) {
    double a0, a1, b0, b1;
    philox_pair(seed, (uint32_t)w, step, 4u * e, 0u, a0, a1);
    philox_pair(seed, (uint32_t)w, step, 4u * e, 1u, b0, b1);
    l.R()[3 * e] += step_size * (2.0 * a0 - 1.0);
    l.R()[3 * e + 1] += step_size * (2.0 * a1 - 1.0);
    l.R()[3 * e + 2] += step_size * (2.0 * b0 - 1.0);
  }
  __syncthreads();
  bool ok = build_state<NT, PREC>(wf, l, l.R());
  double ua, dummy;
  philox_pair(seed, (uint32_t)w, step, 4u * wf.N + 1u, 0u, ua, dummy);
  bool accept = false;
  if (ok) {
    compute_RWS<NT>(wf, l);
    jastrow_full<NT, EEN>(wf, l, l.R());
    if (sc[SC_S] != 0.0) {
      double new_log = sc[SC_U] + sc[SC_LOGDET0] + sc[SC_LOGDET1] + log(fabs(sc[SC_S]));
      accept = ua < exp(2.0 * (new_log - old_log));
    }
  }
  __syncthreads();
  if (!accept) {
    __threadfence_block();
    for (int k = threadIdx.x; k < 3 * wf.N; k += NT) l.R()[k] = bk[wf.r_R + k];
    for (int s = 0; s < 2; ++s) {
      const SpinTab& st = wf.sp[s];
      for (int k = threadIdx.x; k < st.n * st.n; k += NT) l.B(s)[k] = bk[wf.r_B[s] + k];
      for (int k = threadIdx.x; k < st.n * st.nP; k += NT) l.T(s)[k] = bk[wf.r_T[s] + k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      sc[SC_LOGDET0] = bks[0]; sc[SC_LOGDET1] = bks[1]; sc[SC_SGN0] = bks[2]; sc[SC_SGN1] = bks[3];
      sc[SC_S] = bkS; sc[SC_U] = bkU;
    }
    __syncthreads();
    compute_RWS<NT>(wf, l);
  }
  return accept;
}

template <int NT, int PREC, bool EEN = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_vmc(const DevWF* __restrict__ pwf, double* state, int64_t W, int nsteps, uint64_t seed,
                                            uint64_t step0, double step_size, int all_electron, double* e_sum,
                                            double* e2_sum, double* n_acc, double* e_last, double* sij_sum,
                                            DevEcp ecp) {
  const DevWF& wf = *pwf;
  int64_t w = blockIdx.x;
  if (w >= W) return;
  Ld l(lds_dyn, wf);
  stage_tables<NT, PREC>(wf, l);
  double* rec = state + w * wf.rec_len;
  l.bk = rec + wf.r_bk;
  load_record<NT>(wf, l, rec);
  compute_RWS<NT>(wf, l);
  double* sc = l.sc();
  if (all_electron) jastrow_full<NT, EEN>(wf, l, l.R());
  const int nv = wf.nstruct;
  if (sij_sum)
    for (int k = threadIdx.x; k < nv * nv; k += NT) l.sij()[k] = 0.0;
  double es = 0.0, e2s = 0.0, na = 0.0;
  bool bad = !(sc[SC_S] != 0.0);
  for (int st = 0; st < nsteps && !bad; ++st) {
    uint32_t step = (uint32_t)(step0 + st);
    if (all_electron) {
      if (all_electron_move<NT, PREC, EEN>(wf, l, w, seed, step, step_size)) na += 1.0;
    } else {
      for (int i = 0; i < wf.N; ++i) {
        double a0, a1, b0, b1;
        philox_pair(seed, (uint32_t)w, step, 4u * i, 0u, a0, a1);
        philox_pair(seed, (uint32_t)w, step, 4u * i, 1u, b0, b1);
        const double* R = l.R();
        double px = R[3 * i] + step_size * (2.0 * a0 - 1.0);
        double py = R[3 * i + 1] + step_size * (2.0 * a1 - 1.0);
        double pz = R[3 * i + 2] + step_size * (2.0 * b0 - 1.0);
        point_orbitals<NT, PREC>(wf, l, px, py, pz, 1);
        move_ratio<NT>(wf, l, i, px, py, pz, l.v());
        double ratio = sc[SC_RATIO] * exp(sc[SC_TMP0]);
        double ua, dummy;
        philox_pair(seed, (uint32_t)w, step, 4u * i + 1u, 0u, ua, dummy);
        if (ua < ratio * ratio) {
          accept_move<NT>(wf, l, i, px, py, pz);
          na += 1.0;
        }
      }
      if (sc[SC_NUPD0] >= wf.refresh_every || sc[SC_NUPD1] >= wf.refresh_every) {
        bool ok = build_state<NT, PREC>(wf, l, l.R());
        if (!ok) { bad = true; break; }
        compute_RWS<NT>(wf, l);
      }
    }
    if (!(sc[SC_S] != 0.0)) { bad = true; break; }
    local_energy<NT, PREC, EEN>(wf, l, nullptr);
    if (ecp.ncen) ecp_add<NT, PREC>(wf, l, ecp);
    double el = sc[SC_ELOC];
    es += el;
    e2s += el * el;
    if (sij_sum) {
      structure_ratios<NT>(wf, l);
      for (int k = threadIdx.x; k < nv * nv; k += NT) {
        int I = k / nv, J = k - I * nv;
        l.sij()[k] += l.ratio()[I] * l.ratio()[J];
      }
    }
  }
  __syncthreads();
  if (bad && threadIdx.x == 0) sc[SC_FLAGS] = 1.0;
  __syncthreads();
  store_record<NT>(wf, l, rec);
  if (threadIdx.x == 0) {
    e_sum[w] += es;
    e2_sum[w] += e2s;
    n_acc[w] += na;
    e_last[w] = bad ? NAN : sc[SC_ELOC];
  }
  if (sij_sum)
    for (int k = threadIdx.x; k < nv * nv; k += NT) sij_sum[w * nv * nv + k] += l.sij()[k];
}


// ---------------------------------------------------------------------------
// Split VMC step: a walker-resident sweep kernel (moves only), a batched
// local-energy kernel over 16-electron tiles of all walkers, and a per-walker
// finish kernel.
// ---------------------------------------------------------------------------

// Sweep of single-electron moves.  A trial position depends only on the
// electron's own current position and its draws, so every trial position of
// the sweep, and its orbital row, is formed up front: one MFMA pass over tiles
// of 16 trial points.  The moves themselves then only run the determinant
// ratio, the Jastrow change and, when accepted, the rank-1 updates.
template <int NT, int PREC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep(const DevWF* __restrict__ pwf, double* state, int64_t W,
                                              uint64_t seed, uint32_t step, double step_size, double* n_acc) {
  const DevWF& wf = *pwf;
  int64_t w = blockIdx.x;
  if (w >= W) return;
  Ld l(lds_dyn, wf);
  stage_tables<NT, PREC>(wf, l);
  double* rec = state + w * wf.rec_len;
  load_record<NT>(wf, l, rec);
  compute_RWS<NT>(wf, l);
  double* sc = l.sc();
  double na = 0.0;
  bool bad = !(sc[SC_S] != 0.0) || sc[SC_FLAGS] != 0.0;
  if (!bad) {
    double* Rp = l.Rp();
    double* ua = l.ua();
    const double* R = l.R();
    for (int i = threadIdx.x; i < wf.N; i += NT) {
      double a0, a1, b0, b1, u, dummy;
      philox_pair(seed, (uint32_t)w, step, 4u * i, 0u, a0, a1);
      philox_pair(seed, (uint32_t)w, step, 4u * i, 1u, b0, b1);
      philox_pair(seed, (uint32_t)w, step, 4u * i + 1u, 0u, u, dummy);
      Rp[3 * i] = R[3 * i] + step_size * (2.0 * a0 - 1.0);
      Rp[3 * i + 1] = R[3 * i + 1] + step_size * (2.0 * a1 - 1.0);
      Rp[3 * i + 2] = R[3 * i + 2] + step_size * (2.0 * b0 - 1.0);
      ua[i] = u;
    }
    __syncthreads();
    for (int g0 = 0; g0 < wf.N; g0 += kGroup) {
      int ne = min(kGroup, wf.N - g0);
      group_radial<NT, PREC, 1>(wf, l, Rp, g0, ne);
      group_channel<NT, PREC, 1>(wf, l, ne, 0, l.Vn() + g0 * wf.nop, ne);
    }
    for (int i = 0; i < wf.N; ++i) {
      const double px = Rp[3 * i], py = Rp[3 * i + 1], pz = Rp[3 * i + 2];
      move_ratio<NT>(wf, l, i, px, py, pz, l.Vn() + i * wf.nop);
      double ratio = sc[SC_RATIO] * exp(sc[SC_TMP0]);
      if (ua[i] < ratio * ratio) {
        accept_move<NT>(wf, l, i, px, py, pz);
        na += 1.0;
      }
    }
    if (sc[SC_NUPD0] >= wf.refresh_every || sc[SC_NUPD1] >= wf.refresh_every) {
      // the trial rows are dead here: they serve as the tile scratch
      if (build_state<NT, PREC, 1>(wf, l, l.R(), l.Vn())) compute_RWS<NT>(wf, l);
      else bad = true;
    }
    if (!(sc[SC_S] != 0.0)) bad = true;
  }
  __syncthreads();
  if (bad && threadIdx.x == 0) sc[SC_FLAGS] = 1.0;
  __syncthreads();
  store_record<NT>(wf, l, rec);
  if (threadIdx.x == 0) n_acc[w] += na;
}

// Local-energy rows of one electron across 16 walkers.  One wave per block;
// each block walks `per_block` tiles.  A tile stages, per walker, the
// electron's position, column il of the spin's inverse, the table T, the
// determinant ratios, their partner sums, S and the valid flag; then forms
// the radial tables and the four MFMA channels (gradient, Laplacian) of the
// 16 positions, and 64 lanes = 16 walkers x 4 channels form the row-operator
// ratios grad_e D / D, lap_e D / D and store them in the walkers' scratch
// rows.
template <int PREC>
__global__ __launch_bounds__(64) void k_eloc_tiles(const DevWF* __restrict__ pwf, double* state, int64_t W,
                                                   int per_block) {
  const DevWF& wf = *pwf;
  Ld l(lds_dyn, wf);
  stage_tables<64, PREC>(wf, l);
  const int N = wf.N, nop = wf.nop;
  const int nPm = max(wf.sp[0].nP, wf.sp[1].nP);
  const int n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
  const int64_t nwb = (W + kGroup - 1) / kGroup;
  const int64_t ntiles = nwb * N;
  double* Rt = l.R();
  double* Phi4 = l.L + wf.l_Phi4;
  double* yb = l.L + wf.l_yb64;
  double* stg = l.L + wf.l_tstage;
  const int rowsz = wf.tstage_row;
  // Workgroups go to the 8 XCDs round-robin (block b -> XCD b mod 8), each XCD
  // with its own L2.  Block b works on the walker blocks wb = x (mod 8) of
  // its XCD x, so all N tiles of a walker block read its records through
  // one L2.
  const int x = blockIdx.x & (kXcds - 1);
  const int64_t jb = blockIdx.x / kXcds;
  const int64_t nwb_x = nwb > x ? (nwb - x + kXcds - 1) / kXcds : 0;
  const int64_t ntiles_x = nwb_x * N;
  (void)ntiles;
  for (int64_t tl = jb * per_block; tl < min(ntiles_x, (jb + 1) * per_block); ++tl) {
    const int64_t wb = (tl / N) * kXcds + x;
    const int e = (int)(tl - (tl / N) * N);
    const int64_t w0 = wb * kGroup;
    const int rows = (int)min((int64_t)kGroup, W - w0);
    const int s = spin_of(wf, e);
    const SpinTab& st = wf.sp[s];
    const int il = e - st.e0, n = st.n, nP = st.nP, nU = st.nU;
    const int oT = n, oRu = n + n * nP, oWu = oRu + nU, oS = oWu + nU;
    const int per_row = 3 + oS + 2;
    const int ru0 = wf.r_RW + (s ? n0 : 0), wu0 = wf.r_RW + n0 + n1 + (s ? n0 : 0);
    // gather: 8 independent loads per lane in flight, then the LDS stores
    const int total = rows * per_row;
    for (int base = threadIdx.x; base < total; base += 64 * 8) {
      double v[8];
      int dst[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + 64 * u;
        dst[u] = -1;
        if (idx < total) {
          const int t = idx / per_row, k = idx - t * per_row;
          const double* rec = state + (w0 + t) * wf.rec_len;
          int off;
          if (k < 3) {
            off = wf.r_R + 3 * e + k;
            dst[u] = wf.l_R + 3 * t + k;
          } else {
            const int q = k - 3;
            if (q < oT) off = wf.r_B[s] + q * n + il;
            else if (q < oRu) off = wf.r_T[s] + (q - oT);
            else if (q < oWu) off = ru0 + (q - oRu);
            else if (q < oS) off = wu0 + (q - oWu);
            else if (q == oS) off = wf.r_RW + 2 * (n0 + n1);
            else off = wf.r_sc + SC_FLAGS;
            dst[u] = wf.l_tstage + t * rowsz + q;
          }
          v[u] = rec[off];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (dst[u] >= 0) l.L[dst[u]] = v[u];
    }
    __syncthreads();
    group_radial<64, PREC>(wf, l, Rt, 0, rows);
    group_channels4<64, PREC>(wf, l, rows, Phi4);
    {
      const int t = threadIdx.x >> 2, c = threadIdx.x & 3;
      if (t < rows) {
        const double* sr = stg + t * rowsz;
        double tot = 0.0;
        if (sr[oS + 1] == 0.0)
          tot = row_op_sum_p(wf, l, s, Phi4 + (c * kGroup + t) * nop, yb + threadIdx.x * (nPm + 1), sr, 1, 0,
                             sr + oT, sr + oRu, sr + oWu);
        state[(w0 + t) * wf.rec_len + wf.r_gc + 4 * e + c] = tot / sr[oS];
      }
    }
    __syncthreads();
  }
}

// Per walker: Jastrow gradients and Laplacians and the potential, E_L from
// the tile results (Eq. Elav with Psi = e^U D), accumulators, and the
// structure-ratio products r_I r_J (Sec. 2.4) when requested.  Lanes are
// (electron i, part p) with the partners of i split P ways; every global
// read is issued at the start.
__global__ __launch_bounds__(64) void k_eloc_finish(const DevWF* __restrict__ pwf, double* state, int64_t W,
                                                    double* e_sum, double* e2_sum, double* e_last,
                                                    double* sij_sum) {
  __shared__ double sR[3 * kMaxFinishN];
  __shared__ double sred[4];
  const DevWF& wf = *pwf;
  const int64_t w = blockIdx.x;
  if (w >= W) return;
  const int N = wf.N, nn = wf.nnuc;
  const double* rec = state + w * wf.rec_len;
  // per lane: positions, then its electrons' gD / lD
  const int P = N <= 16 ? 4 : (N <= 32 ? 2 : 1);
  const int lanes_e = 64 / P;
  const int p = threadIdx.x % P;
  for (int k = threadIdx.x; k < 3 * N; k += 64) sR[k] = rec[wf.r_R + k];
  const bool bad = rec[wf.r_sc + SC_FLAGS] != 0.0;
  const double es0 = threadIdx.x == 0 ? e_sum[w] : 0.0, e2s0 = threadIdx.x == 0 ? e2_sum[w] : 0.0;
  __syncthreads();
  const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
  double tsum = 0.0, vsum = 0.0;
  for (int i0 = 0; i0 < N; i0 += lanes_e) {
    const int i = i0 + threadIdx.x / P;
    double gx = 0.0, gy = 0.0, gz = 0.0, lap = 0.0, V = 0.0;
    double gD[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < N) {
      if (p == 0)
        for (int c = 0; c < 4; ++c) gD[c] = rec[wf.r_gc + 4 * i + c];
      const double xi = sR[3 * i], yi = sR[3 * i + 1], zi = sR[3 * i + 2];
      const int si = spin_of(wf, i);
      for (int j = p; j < N + nn; j += P) {
        if (j == i) continue;
        double xj, yj, zj, wv;
        PairCoef cf;
        if (j < N) {
          xj = sR[3 * j]; yj = sR[3 * j + 1]; zj = sR[3 * j + 2];
          cf = si != spin_of(wf, j) ? c_anti : c_par;
          wv = 0.5;
        } else {
          const int a = j - N;
          xj = wf.nuc[4 * a]; yj = wf.nuc[4 * a + 1]; zj = wf.nuc[4 * a + 2];
          cf = en_coef(wf.en + 6 * a);
          wv = -wf.nuc[4 * a + 3];
        }
        const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
        const double r = sqrt(dx * dx + dy * dy + dz * dz), ir = 1.0 / r;
        double u, u1, u2;
        pair_fn(r, wf.kappa, cf, u, u1, u2);
        const double f = u1 * ir;
        gx += f * dx; gy += f * dy; gz += f * dz;
        lap += u2 + 2.0 * f;
        V += wv * ir;
      }
    }
    for (int off = 1; off < P; off <<= 1) {
      gx += __shfl_xor(gx, off, 64);
      gy += __shfl_xor(gy, off, 64);
      gz += __shfl_xor(gz, off, 64);
      lap += __shfl_xor(lap, off, 64);
      V += __shfl_xor(V, off, 64);
    }
    if (i < N && p == 0) {
      tsum += lap + gD[3] + gx * gx + gy * gy + gz * gz + 2.0 * (gx * gD[0] + gy * gD[1] + gz * gD[2]);
      vsum += V;
    }
  }
  double part[2] = {tsum, vsum};
  block_sum<64, 2>(part, sred);
  if (threadIdx.x == 0) {
    double* r = state + w * wf.rec_len;
    const double el = -0.5 * part[0] + part[1] + wf.vnn;
    r[wf.r_sc + SC_ELOC] = bad ? NAN : el;
    if (!bad) {
      e_sum[w] = es0 + el;
      e2_sum[w] = e2s0 + el * el;
    }
    e_last[w] = bad ? NAN : el;
  }
  if (sij_sum && !bad) {
    const int nv = wf.nstruct, n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
    const double* RW = rec + wf.r_RW;
    const double iS = 1.0 / RW[2 * (n0 + n1)];
    double* rt = state + w * wf.rec_len + wf.r_gc + 4 * N;  // r_I, after the tile results
    for (int I = threadIdx.x; I < nv; I += 64) {
      double a = 0.0;
      for (int k = wf.srow[I]; k < wf.srow[I + 1]; ++k) a += wf.slc[k] * RW[wf.slu[2 * k]] * RW[n0 + wf.slu[2 * k + 1]];
      rt[I] = a * iS;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nv * nv; k += 64) {
      const int I = k / nv, J = k - I * nv;
      sij_sum[w * nv * nv + k] += rt[I] * rt[J];
    }
  }
}

// ---------------------------------------------------------------------------
// DMC
// ---------------------------------------------------------------------------
// gradient of ln|Psi| for electron i: det part from row operators on rows
// w_c (3 rows of nop in `rows`, stride rstride) with the table of the current
// (or, with bc != null, rank-1-updated) state, Jastrow part at (px,py,pz).
// Results in SC_TMP0..2 is avoided: returned in g[3] (all lanes).
template <int NT>
__device__ void drift(const DevWF& wf, const Ld& l, int i, const double* rows, int rstride, double px,
                      double py, double pz, const double* bc, double irho, const double* Qnew,
                      double Snew, double* g) {
  int s = spin_of(wf, i);
  const SpinTab& st = wf.sp[s];
  int il = i - st.e0;
  const double* B = l.B(s);
  const double* T = l.T(s);
  const double* y0 = l.y();
  const int* ref = l.ref(s);
  const int* porb = l.porb(s);
  const int* uit = l.ui(s);
  const double* nuc = l.nuc();
  double* yb = l.yb();  // [3][nP + 1]: y'^c and rho'^c
  int ld = st.nP + 1;
  // y^c[q] = w_c[P_q] - sum_l w_c[ref_l] T'[l][q],  T' = T + bc y0^T irho
  for (int idx = threadIdx.x; idx < 3 * ld; idx += NT) {
    int c = idx / ld, q = idx - c * ld;
    const double* w = rows + c * rstride;
    if (q < st.nP) {
      double a = w[porb[q]], corr = 0.0;
      for (int k = 0; k < st.n; ++k) {
        a -= w[ref[k]] * T[k * st.nP + q];
        if (bc) corr += w[ref[k]] * bc[k];
      }
      if (bc) a -= corr * y0[q] * irho;
      yb[c * ld + q] = a;
    } else {
      double a = 0.0;
      for (int j = 0; j < st.n; ++j) a += w[ref[j]] * (bc ? bc[j] * irho : B[j * st.n + il]);
      yb[c * ld + q] = a;  // rho'^c
    }
  }
  __syncthreads();
  double part[6] = {0, 0, 0, 0, 0, 0};
  for (int idx = threadIdx.x; idx < 3 * st.nU; idx += NT) {
    int c = idx / st.nU, u = idx - c * st.nU;
    const int* ui = uit + 8 * u;
    double m[9], yy[3], bb[3];
    int e = gather_u(ui, T, st.nP, m, bc, y0, irho);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < e) {
        yy[r] = yb[c * ld + ui[4 + r]];
        bb[r] = bc ? bc[ui[1 + r]] * irho : B[ui[1 + r] * st.n + il];
      }
    double Rn = bc ? Qnew[u] * irho : l.Ru(s)[u];
    double t = (yb[c * ld + st.nP] * Rn + adj_e(e, m, yy, bb)) * l.Wu(s)[u];
    if (c == 0) part[0] += t; else if (c == 1) part[1] += t; else part[2] += t;
  }
  // Jastrow gradient at (px,py,pz)
  const double* R = l.R();
  const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
  for (int j = threadIdx.x; j < wf.N + wf.nnuc; j += NT) {
    if (j == i) continue;
    double xj, yj, zj;
    PairCoef c;
    if (j < wf.N) {
      xj = R[3 * j]; yj = R[3 * j + 1]; zj = R[3 * j + 2];
      c = s != spin_of(wf, j) ? c_anti : c_par;
    } else {
      int n = j - wf.N;
      xj = nuc[4 * n]; yj = nuc[4 * n + 1]; zj = nuc[4 * n + 2];
      c = en_coef(l.en() + 6 * n);
    }
    double dx = px - xj, dy = py - yj, dz = pz - zj;
    double r = sqrt(dx * dx + dy * dy + dz * dz), u, u1, u2;
    pair_fn(r, wf.kappa, c, u, u1, u2);
    double f = u1 / r;
    part[3] += f * dx; part[4] += f * dy; part[5] += f * dz;
  }
  block_sum<NT, 6>(part, l.red());
  double S = bc ? Snew : l.sc()[SC_S];
  for (int c = 0; c < 3; ++c) g[c] = part[3 + c] + part[c] / S;
  __syncthreads();
}

template <int NT, int PREC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_dmc_step(const DevWF* __restrict__ pwf, double* state, const double* ctrl, int nsteps_done,
                                                 uint64_t seed, uint32_t step, double tau, DmcBranch br,
                                                 double* nacc, DevEcp ecp) {
  const DevWF& wf = *pwf;
  int64_t w = blockIdx.x;
  int64_t W = (int64_t)ctrl[DC_W];
  if (ctrl[DC_ERR] != 0.0 || w >= W) return;
  Ld l(lds_dyn, wf);
  stage_tables<NT, PREC>(wf, l);
  double* rec = state + w * wf.rec_len;
  double* gc = rec + wf.r_gc;
  load_record<NT>(wf, l, rec);
  compute_RWS<NT>(wf, l);
  double* sc = l.sc();
  const double ET = ctrl[DC_ET];
  const double E_old = sc[SC_ELOC];
  const double sqt = sqrt(tau);
  double na = 0.0, d2p = 0.0, d2a = 0.0;
  bool bad = !(sc[SC_S] != 0.0);
  for (int i = 0; i < wf.N && !bad; ++i) {
    const double* R = l.R();
    double rx = R[3 * i], ry = R[3 * i + 1], rz = R[3 * i + 2];
    double v[3];
    // the cached gradient rows of electron i, staged into LDS in one copy
    double* grow = l.part();
    for (int k = threadIdx.x; k < 3 * wf.nop; k += NT) grow[k] = gc[(size_t)i * 3 * wf.nop + k];
    __syncthreads();
    drift<NT>(wf, l, i, grow, wf.nop, rx, ry, rz, nullptr, 0.0, nullptr, 0.0, v);
    double a0, a1, b0, b1;
    philox_pair(seed, (uint32_t)w, step, 4u * i, 0u, a0, a1);
    philox_pair(seed, (uint32_t)w, step, 4u * i, 1u, b0, b1);
    const double two_pi = 6.283185307179586476925286766559;
    double r0 = sqrt(-2.0 * log(1.0 - a0)), r1 = sqrt(-2.0 * log(1.0 - b0));
    double zx = r0 * cos(two_pi * a1), zy = r0 * sin(two_pi * a1), zz = r1 * cos(two_pi * b1);
    double px = rx + tau * v[0] + sqt * zx, py = ry + tau * v[1] + sqt * zy, pz = rz + tau * v[2] + sqt * zz;
    point_orbitals<NT, PREC>(wf, l, px, py, pz, 4);
    move_ratio<NT>(wf, l, i, px, py, pz, l.v());
    double rdet = sc[SC_RATIO];
    double dU = sc[SC_TMP0];
    double rho = sc[SC_TMP1];
    bool accept = false;
    const double d2 = (px - rx) * (px - rx) + (py - ry) * (py - ry) + (pz - rz) * (pz - rz);
    d2p += d2;
    if (rdet > 0.0 && rho != 0.0) {
      double vn[3];
      double Snew = sc[SC_S] * rdet / rho;  // S' relative to the updated reference
      drift<NT>(wf, l, i, l.v() + wf.nop, wf.nop, px, py, pz, l.bcol(), 1.0 / rho, l.Qu(), Snew, vn);
      double fwd = 0.0, bwd = 0.0;
      double d[3] = {px - rx, py - ry, pz - rz};
      for (int x = 0; x < 3; ++x) {
        double fa = d[x] - tau * v[x];
        double ba = -d[x] - tau * vn[x];
        fwd += fa * fa;
        bwd += ba * ba;
      }
      double p = rdet * rdet * exp(2.0 * dU + (fwd - bwd) / (2.0 * tau));
      double ua, dummy;
      philox_pair(seed, (uint32_t)w, step, 4u * i + 1u, 0u, ua, dummy);
      accept = ua < p;
    }
    if (accept) {
      accept_move<NT>(wf, l, i, px, py, pz);
      for (int k = threadIdx.x; k < 3 * wf.nop; k += NT) gc[(size_t)i * 3 * wf.nop + k] = l.v()[wf.nop + k];
      na += 1.0;
      d2a += d2;
      __syncthreads();
    }
    if (!(sc[SC_S] != 0.0)) bad = true;
  }
  if (!bad && (sc[SC_NUPD0] >= wf.refresh_every || sc[SC_NUPD1] >= wf.refresh_every)) {
    if (!build_state<NT, PREC>(wf, l, l.R())) bad = true;
    else compute_RWS<NT>(wf, l);
  }
  if (!bad) local_energy<NT, PREC>(wf, l, gc);
  // pseudopotentials: the projected term with the trial function (locality approximation)
  if (!bad && ecp.ncen) ecp_add<NT, PREC>(wf, l, ecp);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double En = bad ? NAN : sc[SC_ELOC];
    dmc_branch_inputs(br, w, bad, E_old, En, ET, tau, wf.N, seed, step);
    nacc[3 * w] = na;
    nacc[3 * w + 1] = d2p;
    nacc[3 * w + 2] = d2a;
    if (bad) sc[SC_FLAGS] = 1.0;
  }
  __syncthreads();
  store_record<NT>(wf, l, rec);
}

// Single-workgroup population control, scan, reduction and trial-energy
// update of one DMC step (Sec. 2.3.2).  Pass 1 sums the weights; if the
// expected next population sum_w w lies outside [0.95, 1.05] W_target, every
// weight is scaled by the one factor f that brings the sum to the nearer
// bound (the step then ran at E_T + ln(f) / tau, which is what the log
// records).  Pass 2 forms the copy counts min(3, floor(f w + u)), their
// exclusive scan and the sums of the log.  Each thread sums a contiguous
// chunk and the chunks are combined by a fixed tree, so the results do not
// depend on timing.
__global__ __launch_bounds__(1024) void k_dmc_scan(double* ctrl, DmcBranch br, const double* nacc, int* offs,
                                                   int64_t capacity, int N, int st, double tau,
                                                   double W_target, double* pop, double* wsum,
                                                   double* wesum, double* wcsum, double* etrial, double* lacc,
                                                   double* lprop, double* ld2a, double* ld2p) {
  __shared__ double sw[1024], swe[1024], swc[1024], sa[1024], sdp[1024], sda[1024];
  __shared__ int sc_[1024];
  __shared__ int bad;
  __shared__ double fsh;
  const int t = threadIdx.x;
  if (ctrl[DC_ERR] != 0.0) return;
  const int64_t W = (int64_t)ctrl[DC_W];
  const int64_t per = (W + 1023) / 1024;
  const int64_t b = t * per, e = min(W, b + per);
  double a = 0;
  int nbad = 0;
  for (int64_t k = b; k < e; ++k) {
    if (br.nc[k] < 0) { ++nbad; continue; }
    a += br.w[k];
  }
  if (t == 0) bad = 0;
  sw[t] = a;
  __syncthreads();
  if (nbad) atomicAdd(&bad, nbad);
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) sw[t] += sw[t + off];
    __syncthreads();
  }
  if (t == 0) {
    double f = 1.0;
    if (sw[0] > 1.05 * W_target) f = 1.05 * W_target / sw[0];
    else if (sw[0] < 0.95 * W_target) f = 0.95 * W_target / sw[0];
    fsh = f;
  }
  __syncthreads();
  const double f = fsh;
  double aw = 0, ae = 0, ac = 0, aa = 0, adp = 0, ada = 0;
  int cnt = 0;
  for (int64_t k = b; k < e; ++k) {
    if (br.nc[k] < 0) continue;
    const double wk = f * br.w[k];
    const int nc = min(3, (int)floor(wk + br.ub[k]));
    br.nc[k] = nc;
    aw += wk;
    ae += f * br.we[k];
    ac += f * br.wc[k];
    aa += nacc[3 * k];
    adp += nacc[3 * k + 1];
    ada += nacc[3 * k + 2];
    cnt += nc;
  }
  __syncthreads();
  sw[t] = aw; swe[t] = ae; swc[t] = ac; sa[t] = aa; sdp[t] = adp; sda[t] = ada; sc_[t] = cnt;
  __syncthreads();
  // inclusive scan of copy counts (Hillis-Steele) and tree sums
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? sc_[t - off] : 0;
    __syncthreads();
    sc_[t] += v;
    __syncthreads();
  }
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) {
      sw[t] += sw[t + off];
      swe[t] += swe[t + off];
      swc[t] += swc[t + off];
      sa[t] += sa[t + off];
      sdp[t] += sdp[t + off];
      sda[t] += sda[t + off];
    }
    __syncthreads();
  }
  int base = t > 0 ? sc_[t - 1] : 0;
  for (int64_t k = b; k < e; ++k) {
    offs[k] = base;
    base += br.nc[k] > 0 ? br.nc[k] : 0;
  }
  if (t == 0) {
    int64_t Wn = sc_[1023];
    offs[W] = (int)Wn;
    pop[st] = (double)W;
    wsum[st] = sw[0];
    wesum[st] = swe[0];
    if (wcsum) wcsum[st] = swc[0];
    etrial[st] = ctrl[DC_ET] + log(f) / tau;
    lacc[st] = sa[0];
    lprop[st] = (double)W * N;
    if (ld2a) ld2a[st] = sda[0];
    if (ld2p) ld2p[st] = sdp[0];
    if (bad || Wn <= 0 || Wn > capacity) {
      ctrl[DC_ERR] = bad ? 1.0 : 2.0;
      ctrl[DC_ERRSTEP] = (double)st;
      ctrl[DC_WNEW] = (double)Wn;
    } else {
      ctrl[DC_RUN_NUM] += swc[0];
      ctrl[DC_RUN_DEN] += sw[0];
      ctrl[DC_WNEW] = (double)Wn;
      ctrl[DC_ET] = ctrl[DC_RUN_NUM] / ctrl[DC_RUN_DEN] - (0.1 / tau) * log((double)Wn / W_target);
    }
  }
}

// copy record of each destination slot from its parent (binary search in offs)
__global__ void k_dmc_copy(const double* ctrl, const double* src, double* dst, const int* offs, int rec_len) {
  if (ctrl[DC_ERR] != 0.0) return;
  int64_t W = (int64_t)ctrl[DC_W];
  int64_t Wn = (int64_t)ctrl[DC_WNEW];
  int64_t d = blockIdx.x;
  if (d >= Wn) return;
  int64_t lo = 0, hi = W - 1;  // largest parent p with offs[p] <= d
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if (offs[mid] <= d) lo = mid; else hi = mid - 1;
  }
  // records are 256-byte multiples at 256-byte aligned bases: 16-byte copies
  const double2* s = (const double2*)(src + lo * rec_len);
  double2* o = (double2*)(dst + d * rec_len);
  const int n2 = rec_len >> 1;
#pragma unroll 4
  for (int k = threadIdx.x; k < n2; k += blockDim.x) o[k] = s[k];
}

__global__ void k_dmc_commit(double* ctrl) {
  if (ctrl[DC_ERR] != 0.0) return;
  ctrl[DC_W] = ctrl[DC_WNEW];
}

__global__ void k_copy_records(const double* src, double* dst, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_positions(const DevWF* __restrict__ pwf, int64_t W, const double* state, double* R) {
  const DevWF& wf = *pwf;
  int64_t w = blockIdx.x;
  if (w >= W) return;
  for (int k = threadIdx.x; k < 3 * wf.N; k += blockDim.x) R[w * 3 * wf.N + k] = state[w * wf.rec_len + wf.r_R + k];
}

__global__ void k_record_eloc(const DevWF* __restrict__ pwf, int64_t W, const double* state, double* e) {
  const DevWF& wf = *pwf;
  int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (w < W) e[w] = state[w * wf.rec_len + wf.r_sc + SC_ELOC];
}

// out[k] = sum_w wts[w] in[w][k] (wts may be null: weight 1), fixed order:
// each block owns one column, each lane a strided slice of walkers, then a
// lane tree.
__global__ __launch_bounds__(256) void k_reduce(int64_t W, int K, const double* wts, const double* in,
                                                double* out) {
  __shared__ double s[256];
  int k = blockIdx.x;
  double a = 0.0;
  for (int64_t w = threadIdx.x; w < W; w += 256) a += (wts ? wts[w] : 1.0) * in[w * K + k];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = s[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int NT, int PREC>
static hipError_t set_lds(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int NT, int PREC, bool EEN = false>
static hipError_t launch_evaluate_t(const DevWF& wf, const DevWF* dwf, int64_t W, const double* R, int64_t rstride,
                                    double* logabs, int32_t* sign, double* grad, double* eloc, double* ratio,
                                    double* state, const DevEcp& ecp, hipStream_t s) {
  size_t lds = (size_t)(wf.lds_doubles + (ecp.ncen && ecp.l_scr >= 0 ? ecp.scr_doubles : 0)) * sizeof(double);
  hipError_t e = set_lds<NT, PREC>((const void*)k_evaluate<NT, PREC, EEN>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_evaluate<NT, PREC, EEN>), dim3((unsigned)W), dim3(NT), lds, s, dwf, W, R, rstride, logabs, sign, grad,
                     eloc, ratio, state, ecp);
  return hipGetLastError();
}

template <int NT, int PREC, bool EEN = false>
static hipError_t launch_vmc_t(const DevWF& wf, const DevWF* dwf, double* state, int64_t W, int nsteps, uint64_t seed,
                               uint64_t step0, double step_size, int all_e, double* es, double* e2s,
                               double* na, double* el, double* sij, const DevEcp& ecp, hipStream_t s) {
  size_t lds = (size_t)(wf.lds_doubles + (ecp.ncen && ecp.l_scr >= 0 ? ecp.scr_doubles : 0)) * sizeof(double);
  hipError_t e = set_lds<NT, PREC>((const void*)k_vmc<NT, PREC, EEN>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_vmc<NT, PREC, EEN>), dim3((unsigned)W), dim3(NT), lds, s, dwf, state, W, nsteps, seed, step0,
                     step_size, all_e, es, e2s, na, el, sij, ecp);
  return hipGetLastError();
}

template <int NT, int PREC>
static hipError_t launch_dmc_step_t(const DevWF& wf, const DevWF* dwf, double* state, const double* ctrl, int64_t cap, uint64_t seed,
                                    uint32_t step, double tau, const DmcBranch& br, double* nacc,
                                    const DevEcp& ecp, hipStream_t s) {
  size_t lds = (size_t)(wf.lds_doubles + (ecp.ncen && ecp.l_scr >= 0 ? ecp.scr_doubles : 0)) * sizeof(double);
  hipError_t e = set_lds<NT, PREC>((const void*)k_dmc_step<NT, PREC>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dmc_step<NT, PREC>), dim3((unsigned)cap), dim3(NT), lds, s, dwf, state, ctrl, 0, seed, step,
                     tau, br, nacc, ecp);
  return hipGetLastError();
}

#define VB_DISPATCH(NTV, FN, ...)                                              \
  switch (wf.precision) {                                                      \
    case 0: return FN<NTV, 0>(__VA_ARGS__);                                    \
    case 1: return FN<NTV, 1>(__VA_ARGS__);                                    \
    default: return FN<NTV, 2>(__VA_ARGS__);                                   \
  }

#define VB_DISPATCH_NT(NT, FN, ...)                                            \
  switch (NT) {                                                                \
    case 64: VB_DISPATCH(64, FN, __VA_ARGS__)                                  \
    case 128: VB_DISPATCH(128, FN, __VA_ARGS__)                                \
    default: VB_DISPATCH(256, FN, __VA_ARGS__)                                 \
  }

// (f_een: FP64 only, its own instantiations)
#define VB_DISPATCH_EEN(NT, FN, ...)                                           \
  switch (NT) {                                                                \
    case 64: return FN<64, 0, true>(__VA_ARGS__);                              \
    case 128: return FN<128, 0, true>(__VA_ARGS__);                            \
    default: return FN<256, 0, true>(__VA_ARGS__);                             \
  }

hipError_t launch_evaluate(const DevWF& wf, const DevWF* dwf, int nt, int64_t W, const double* R, int64_t rstride,
                           double* logabs, int32_t* sign, double* grad, double* eloc, double* ratio, double* state,
                           const DevEcp& ecp, hipStream_t s) {
  if (wf.neen)
    VB_DISPATCH_EEN(nt, launch_evaluate_t, wf, dwf, W, R, rstride, logabs, sign, grad, eloc, ratio, state, ecp, s)
  VB_DISPATCH_NT(nt, launch_evaluate_t, wf, dwf, W, R, rstride, logabs, sign, grad, eloc, ratio, state, ecp, s)
}

hipError_t launch_vmc(const DevWF& wf, const DevWF* dwf, int nt, double* state, int64_t W, int nsteps, uint64_t seed, uint64_t step0,
                      double step_size, int all_e, double* es, double* e2s, double* na, double* el, double* sij,
                      const DevEcp& ecp, hipStream_t s) {
  if (wf.neen)
    VB_DISPATCH_EEN(nt, launch_vmc_t, wf, dwf, state, W, nsteps, seed, step0, step_size, all_e, es, e2s, na, el, sij,
                    ecp, s)
  VB_DISPATCH_NT(nt, launch_vmc_t, wf, dwf, state, W, nsteps, seed, step0, step_size, all_e, es, e2s, na, el, sij, ecp,
                 s)
}


hipError_t launch_sweep_g(const DevWF& wf, const DevWF* dwf, int G, double* state, int64_t W, uint64_t seed,
                          uint32_t step, double step_size, double* n_acc, hipStream_t s);

template <int NT, int PREC>
static hipError_t launch_vmc_split_t(const DevWF& wf, const DevWF* dwf, const DevWF* dwf_g, int G,
                                     const DevWF* dwf_aux, int phases, double* state, int64_t W, int nsteps,
                                     uint64_t seed, uint64_t step0, double step_size, double* es, double* e2s,
                                     double* na, double* el, double* sij, hipStream_t s) {
  size_t lds_sw = (size_t)wf.lds_sweep_doubles * sizeof(double);
  size_t lds_ti = (size_t)wf.lds_tile_doubles * sizeof(double);
  hipError_t e = set_lds<NT, PREC>((const void*)k_sweep<NT, PREC>, lds_sw);
  if (e == hipSuccess) e = set_lds<64, PREC>((const void*)k_eloc_tiles<PREC>, lds_ti);
  if (e != hipSuccess) return e;
  // tiles per XCD (walker blocks wb = x mod 8), rounded up to whole blocks
  const int64_t nwb = (W + kGroup - 1) / kGroup;
  // tiles per block: just enough for every block to be resident at once
  // (workgroups per CU from the LDS footprint, at most 8 one-wave blocks)
  const int64_t tiles_xcd = (nwb + kXcds - 1) / kXcds * wf.N;
  const int64_t slots_xcd = (int64_t)(kCus / kXcds) * std::max(1, std::min(8, (int)(163840 / std::max<size_t>(lds_ti, 1))));
  const int per_block = (int)std::max<int64_t>(1, (tiles_xcd + slots_xcd - 1) / slots_xcd);
  const int64_t per_xcd = (tiles_xcd + per_block - 1) / per_block;
  const unsigned tblocks = (unsigned)(per_xcd * kXcds);
  for (int st = 0; st < nsteps; ++st) {
    uint32_t step = (uint32_t)(step0 + st);
    if ((phases & 1) && G < 64) {
      hipError_t e2 = launch_sweep_g(wf, dwf_g, G, state, W, seed, step, step_size, na, s);
      if (e2 != hipSuccess) return e2;
    } else if (phases & 1) {
      hipLaunchKernelGGL((k_sweep<NT, PREC>), dim3((unsigned)W), dim3(NT), lds_sw, s, dwf, state, W, seed, step,
                         step_size, na);
    }
    if (phases & 2) {
      hipLaunchKernelGGL((k_eloc_tiles<PREC>), dim3(tblocks), dim3(64), lds_ti, s, dwf_aux, state, W, per_block);
      hipLaunchKernelGGL(k_eloc_finish, dim3((unsigned)W), dim3(64), 0, s, dwf_aux, state, W, es, e2s, el, sij);
    }
  }
  return hipGetLastError();
}

// phases: 1 = sweep (moves), 2 = measure (local energy), 3 = both, per step
hipError_t launch_vmc_split(const DevWF& wf, const DevWF* dwf, const DevWF* dwf_g, int G, const DevWF* dwf_aux,
                            int nt, int phases, double* state, int64_t W, int nsteps, uint64_t seed, uint64_t step0,
                            double step_size, double* es, double* e2s, double* na, double* el, double* sij,
                            hipStream_t s) {
  VB_DISPATCH_NT(nt, launch_vmc_split_t, wf, dwf, dwf_g, G, dwf_aux, phases, state, W, nsteps, seed, step0, step_size, es, e2s, na, el, sij, s)
}

hipError_t launch_dmc_step(const DevWF& wf, const DevWF* dwf, int nt, double* state, const double* ctrl, int64_t cap, uint64_t seed,
                           uint32_t step, double tau, const DmcBranch& br, double* nacc, const DevEcp& ecp,
                           hipStream_t s) {
  VB_DISPATCH_NT(nt, launch_dmc_step_t, wf, dwf, state, ctrl, cap, seed, step, tau, br, nacc, ecp, s)
}

hipError_t launch_dmc_tail(double* ctrl, const DmcBranch& br, const double* nacc, int* offs, int64_t cap, int N,
                           int st, double tau, double W_target, double* pop, double* wsum, double* wesum,
                           double* wcsum, double* etrial, double* lacc, double* lprop, double* ld2a, double* ld2p,
                           const double* src, double* dst, int rec_len, hipStream_t s) {
  hipLaunchKernelGGL(k_dmc_scan, dim3(1), dim3(1024), 0, s, ctrl, br, nacc, offs, cap, N, st, tau, W_target, pop,
                     wsum, wesum, wcsum, etrial, lacc, lprop, ld2a, ld2p);
  hipLaunchKernelGGL(k_dmc_copy, dim3((unsigned)cap), dim3(256), 0, s, ctrl, src, dst, offs, rec_len);
  hipLaunchKernelGGL(k_dmc_commit, dim3(1), dim3(1), 0, s, ctrl);
  return hipGetLastError();
}

hipError_t launch_copy_records(const double* src, double* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_records, dim3(1024), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_positions(const DevWF& wf, const DevWF* dwf, int64_t W, const double* state, double* R, hipStream_t s) {
  hipLaunchKernelGGL(k_positions, dim3((unsigned)W), dim3(64), 0, s, dwf, W, state, R);
  return hipGetLastError();
}

hipError_t launch_record_eloc(const DevWF& wf, const DevWF* dwf, int64_t W, const double* state, double* e, hipStream_t s) {
  hipLaunchKernelGGL(k_record_eloc, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, s, dwf, W, state, e);
  return hipGetLastError();
}

hipError_t launch_reduce(int64_t W, int K, const double* wts, const double* in, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)K), dim3(256), 0, s, W, K, wts, in, out);
  return hipGetLastError();
}

}  // namespace vbqmc
