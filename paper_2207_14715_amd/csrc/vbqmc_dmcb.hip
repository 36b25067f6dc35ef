// gfx950 DMC moves, electron-major: every walker moves electron i together.
//
// A fixed-node DMC step (Sec. 2.3.2) moves the electrons one after the
// other; within one electron's move the walkers are independent.  For
// systems whose walker state is too large to keep several walkers per CU, the
// step is cut into launches per electron over all walkers:
//   propose  one wavefront per walker: drift v = grad_i ln|Psi| at the current
//            point (gradient rows of electron i cached in the record) and the
//            drift-diffusion proposal r' = r + tau v + sqrt(tau) chi;
//   rows     16 walkers per wavefront: value and gradient orbital rows at the
//            16 proposals on MFMA;
//   accept   one wavefront per walker: determinant ratio (reference inverse +
//            replaced-column table, as in the VMC kernels), node check, drift
//            at r' from the rank-1-updated state, Green's-function ratio,
//            Metropolis decision and, when accepted, the Sherman-Morrison
//            update with lane k owning column k of [B | T] in registers.
// The walker records stay in HBM between launches and each launch streams
// what it needs, so occupancy no longer depends on how much state a walker
// has.  Inverse refresh, the local energy and the branching weight follow in
// a per-walker kernel after the last electron.

#include "vbqmc_device.h"

namespace vbqmc {

extern __shared__ double lds_dyn[];

// sum over the 64 lanes of a wavefront, the same bits in every lane
template <int K>
__device__ __forceinline__ void wave_sum(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
}

// determinant ratios R_u, partner sums W_u and S of a record
struct RecRW {
  const double* Ru;
  const double* Wu;
  double S;
};
__device__ __forceinline__ RecRW rec_rw(const DevWF& wf, const double* rec, int s) {
  const int n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
  const double* RW = rec + wf.r_RW;
  return {RW + (s ? n0 : 0), RW + n0 + n1 + (s ? n0 : 0), RW[2 * (n0 + n1)]};
}

// Jastrow gradient of electron i at point x (the other electrons at their
// record positions): sum over partners of u'(r)/r (x - x_j), lanes over
// partners, not reduced
__device__ __forceinline__ void jastrow_grad_part(const DevWF& wf, const double* R, int i, const double* x,
                                                  double (&g)[3]) {
  const int s = spin_of(wf, i);
  const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
  for (int j = threadIdx.x; j < wf.N + wf.nnuc; j += 64) {
    if (j == i) continue;
    double xj, yj, zj;
    PairCoef c;
    if (j < wf.N) {
      xj = R[3 * j]; yj = R[3 * j + 1]; zj = R[3 * j + 2];
      c = s != spin_of(wf, j) ? c_anti : c_par;
    } else {
      const int a = j - wf.N;
      xj = wf.nuc[4 * a]; yj = wf.nuc[4 * a + 1]; zj = wf.nuc[4 * a + 2];
      c = en_coef(wf.en + 6 * a);
    }
    const double dx = x[0] - xj, dy = x[1] - yj, dz = x[2] - zj;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double u, u1, u2;
    pair_fn(r, wf.kappa, c, u, u1, u2);
    const double f = u1 / r;
    g[0] += f * dx;
    g[1] += f * dy;
    g[2] += f * dz;
  }
}

// ---------------------------------------------------------------------------
// propose: drift at the current point and the drift-diffusion proposal
// ---------------------------------------------------------------------------
// LDS (doubles): bcol [64] | yc [3][64]
__global__ __launch_bounds__(64) void k_dmcb_propose(const DevWF* __restrict__ pwf, double* state,
                                                     double* ctrl, int i, uint64_t seed, uint32_t step,
                                                     double tau, double* P, double* V, double* nacc) {
  __shared__ double bcol[64], yc[3 * 64];
  const DevWF& wf = *pwf;
  const int64_t w = blockIdx.x;
  const int64_t W = (int64_t)ctrl[DC_W];
  if (ctrl[DC_ERR] != 0.0 || w >= W) return;
  const int lane = threadIdx.x;
  double* rec = state + w * wf.rec_len;
  const int s = spin_of(wf, i);
  const SpinTab& sp = wf.sp[s];
  const int n = sp.n, nP = sp.nP, il = i - sp.e0;
  const RecRW rw = rec_rw(wf, rec, s);
  if (i == 0) {
    // a step starts: clear the acceptance count; a walker whose
    // determinant sum vanishes is dropped at branching
    if (lane == 0) {
      nacc[w] = 0.0;
      if (!(rw.S != 0.0)) rec[wf.r_sc + SC_FLAGS] = 1.0;
    }
    __syncthreads();
  }
  if (rec[wf.r_sc + SC_FLAGS] != 0.0) return;
  const double* B = rec + wf.r_B[s];
  const double* T = rec + wf.r_T[s];
  const double* gr = rec + wf.r_gc + (size_t)i * 3 * wf.nop;  // gradient rows of electron i
  const int* ref = sp.ref;
  const int* porb = sp.porb;
  // column il of B and the three table-row corrections y^c
  double rp[3] = {0.0, 0.0, 0.0};
  if (lane < n) {
    const double b = B[lane * n + il];
    bcol[lane] = b;
    const int rj = ref[lane];
#pragma unroll
    for (int c = 0; c < 3; ++c) rp[c] = gr[c * wf.nop + rj] * b;
  }
  if (lane < nP) {
    const int pq = porb[lane];
    double a[3] = {gr[pq], gr[wf.nop + pq], gr[2 * wf.nop + pq]};
    for (int l = 0; l < n; ++l) {
      const double t = T[l * nP + lane];
      const int rl = ref[l];
#pragma unroll
      for (int c = 0; c < 3; ++c) a[c] -= gr[c * wf.nop + rl] * t;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) yc[c * 64 + lane] = a[c];
  }
  wave_sum<3>(rp);
  __syncthreads();
  double part[6] = {0, 0, 0, 0, 0, 0};
  for (int u = lane; u < sp.nU; u += 64) {
    const int* ui = sp.uinfo + 8 * u;
    double m[9], bb[3] = {0, 0, 0};
    const int e = gather_u(ui, T, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < e) bb[r] = bcol[ui[1 + r]];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double yy[3] = {0, 0, 0};
#pragma unroll
      for (int r = 0; r < 3; ++r)
        if (r < e) yy[r] = yc[c * 64 + ui[4 + r]];
      part[c] += (rp[c] * rw.Ru[u] + adj_e(e, m, yy, bb)) * rw.Wu[u];
    }
  }
  const double* R = rec + wf.r_R;
  const double x[3] = {R[3 * i], R[3 * i + 1], R[3 * i + 2]};
  double g[3] = {0, 0, 0};
  jastrow_grad_part(wf, R, i, x, g);
  part[3] = g[0];
  part[4] = g[1];
  part[5] = g[2];
  wave_sum<6>(part);
  if (lane == 0) {
    double v[3];
    for (int c = 0; c < 3; ++c) v[c] = part[3 + c] + part[c] / rw.S;
    double a0, a1, b0, b1;
    philox_pair(seed, (uint32_t)w, step, 4u * i, 0u, a0, a1);
    philox_pair(seed, (uint32_t)w, step, 4u * i, 1u, b0, b1);
    const double two_pi = 6.283185307179586476925286766559;
    const double r0 = sqrt(-2.0 * log(1.0 - a0)), r1 = sqrt(-2.0 * log(1.0 - b0));
    const double zx = r0 * cos(two_pi * a1), zy = r0 * sin(two_pi * a1), zz = r1 * cos(two_pi * b1);
    const double sqt = sqrt(tau);
    P[3 * w] = x[0] + tau * v[0] + sqt * zx;
    P[3 * w + 1] = x[1] + tau * v[1] + sqt * zy;
    P[3 * w + 2] = x[2] + tau * v[2] + sqt * zz;
    V[3 * w] = v[0];
    V[3 * w + 1] = v[1];
    V[3 * w + 2] = v[2];
  }
}

// ---------------------------------------------------------------------------
// rows: value and gradient orbital rows at the proposals of 16 walkers
// ---------------------------------------------------------------------------
// value, x, y, z channels of function mu at electron e of the tile (GS = 3 tables)
template <typename T>
__device__ __forceinline__ void chan_vg(const DevWF& wf, const Ld& l, int e, int mu, T (&o)[4]) {
  const int* fn = l.fn();
  const int sh = fn[2 * mu];
  if (sh < 0) {
    o[0] = o[1] = o[2] = o[3] = T(0);
    return;
  }
  const int m = fn[2 * mu + 1];
  const int* si = l.sh() + 8 * sh;
  const int kind = si[1], lq = si[2];
  const T* d = (const T*)l.disp() + e * disp_stride(wf) + 4 * si[0];
  const T* gg = (const T*)l.gtab() + e * gtab_stride<3>(wf) + 3 * sh;
  const T x = d[0], y = d[1], z = d[2], r2 = d[3];
  const T g = gg[0], g1 = gg[1];
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
  const T fr = kind == 0 ? T(2) * g1 : g1 / sqrt(r2);
  o[0] = P * g;
  o[1] = Px * g + P * fr * x;
  o[2] = Py * g + P * fr * y;
  o[3] = Pz * g + P * fr * z;
}

// Tile of 16 walkers (rows e < ne): out[(w0 + e) * 4 * nop + c * nop + p].
template <int PREC>
__global__ __launch_bounds__(64) void k_dmcb_rows(const DevWF* __restrict__ pwf, const double* ctrl,
                                                  const double* P, double* out) {
  const DevWF& wf = *pwf;
  const int64_t W = (int64_t)ctrl[DC_W];
  const int64_t w0 = (int64_t)blockIdx.x * kGroup;
  if (ctrl[DC_ERR] != 0.0 || w0 >= W) return;
  const int ne = (int)min((int64_t)kGroup, W - w0);
  Ld l(lds_dyn, wf);
  stage_tables<64, PREC>(wf, l);
  group_radial<64, PREC, 3>(wf, l, P + 3 * w0, 0, ne);
  const int lane = threadIdx.x;
  const int nct = wf.nop / 16;
  const size_t ost = (size_t)4 * wf.nop;
  double* o = out + (size_t)w0 * ost;
  for (int ct = 0; ct < nct; ++ct) {
    const int col = ct * 16 + (lane & 15);
    const int e = lane & 15;
    const bool live = e < ne;
    if constexpr (PREC == 0) {
      const double* lam = wf.lamT;
      v4d acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = v4d{0, 0, 0, 0};
      for (int k0 = 0; k0 < wf.Mpad; k0 += 4) {
        const int k = k0 + (lane >> 4);
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        if (live) chan_vg<double>(wf, l, e, k, a);
        const double b = lam[(size_t)k * wf.nop + col];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c], b, acc[c], 0, 0, 0);
      }
      // f64 16x16x4 output: register r of lane l holds row 4r + l/16
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * r + (lane >> 4) < ne) o[(4 * r + (lane >> 4)) * ost + c * wf.nop + col] = acc[c][r];
    } else if constexpr (PREC == 1) {
      const float* lam = wf.lamT32;
      v4f acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = v4f{0, 0, 0, 0};
      for (int k0 = 0; k0 < wf.Mpad; k0 += 4) {
        const int k = k0 + (lane >> 4);
        float a[4] = {0.f, 0.f, 0.f, 0.f};
        if (live) chan_vg<float>(wf, l, e, k, a);
        const float b = lam[(size_t)k * wf.nop + col];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], b, acc[c], 0, 0, 0);
      }
      // f32 output: register r of lane l holds row 4(l/16) + r
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * (lane >> 4) + r < ne) o[(4 * (lane >> 4) + r) * ost + c * wf.nop + col] = (double)acc[c][r];
    } else {
      const uint16_t* lam = wf.lamT16;
      v4f acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = v4f{0, 0, 0, 0};
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        const int kb = k0 + 4 * (lane >> 4);
        v4s a[4], b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float v[4] = {0.f, 0.f, 0.f, 0.f};
          if (live) chan_vg<float>(wf, l, e, kb + j, v);
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
          if (4 * (lane >> 4) + r < ne) o[(4 * (lane >> 4) + r) * ost + c * wf.nop + col] = (double)acc[c][r];
    }
  }
}

// ---------------------------------------------------------------------------
// accept: ratio, node check, drift at r', Green's function, Metropolis,
// Sherman-Morrison update
// ---------------------------------------------------------------------------
// LDS (doubles): bcol [64] | y0 [64] | yc [3][64] | Qn [nUmax] | Rn [nUmax]
template <int NB>
__global__ __launch_bounds__(64) void k_dmcb_accept(const DevWF* __restrict__ pwf, double* state,
                                                    const double* ctrl, int i, uint64_t seed, uint32_t step,
                                                    double tau, const double* P, const double* V,
                                                    const double* Vp, double* nacc) {
  const DevWF& wf = *pwf;
  const int64_t w = blockIdx.x;
  const int64_t W = (int64_t)ctrl[DC_W];
  if (ctrl[DC_ERR] != 0.0 || w >= W) return;
  double* rec = state + w * wf.rec_len;
  if (rec[wf.r_sc + SC_FLAGS] != 0.0) return;
  const int lane = threadIdx.x;
  const int s = spin_of(wf, i);
  const SpinTab& sp = wf.sp[s];
  const int n = sp.n, nP = sp.nP, nU = sp.nU, il = i - sp.e0;
  const int nUm = max(wf.sp[0].nU, wf.sp[1].nU);
  double* bcol = lds_dyn;
  double* y0 = lds_dyn + 64;
  double* yc = lds_dyn + 128;
  double* Qn = lds_dyn + 320;
  double* Rn = Qn + nUm;
  const int n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
  double* RW = rec + wf.r_RW;
  double* Ru = RW + (s ? n0 : 0);
  const double* Wu = RW + n0 + n1 + (s ? n0 : 0);
  const double S = RW[2 * (n0 + n1)];
  double* Bg = rec + wf.r_B[s];
  double* Tg = rec + wf.r_T[s];
  const int* ref = sp.ref;
  const int* porb = sp.porb;
  const double* vp = Vp + (size_t)w * 4 * wf.nop;
  const bool bl = lane < n, tl = lane >= n && lane < n + nP;
  // column lane of [B | T]
  double C[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double v = 0.0;
    if (j < n) {
      if (bl) v = Bg[j * n + lane];
      else if (tl) v = Tg[j * nP + (lane - n)];
    }
    C[j] = v;
  }
  // t_k = sum_j v[ref_j] C[j][k]: u = v_ref^T B on B lanes, v_ref^T T on table lanes
  double t = 0.0;
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < n) t += vp[ref[j]] * C[j];
  const double rho = __shfl(t, il, 64);
  const double y = tl ? vp[porb[lane - n]] - t : 0.0;
  if (lane == il) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (j < n) bcol[j] = C[j];
  }
  if (tl) y0[lane - n] = y;
  __syncthreads();
  // Q_u = rho R_u + y_Q^T adj(T_JQ) B_J,il ; S'' = sum_u Q_u W_u ; Jastrow change
  double part[2] = {0.0, 0.0};
  for (int u = lane; u < nU; u += 64) {
    const int* ui = sp.uinfo + 8 * u;
    double m[9], yy[3] = {0, 0, 0}, bb[3] = {0, 0, 0};
    const int e = gather_u(ui, Tg, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < e) {
        yy[r] = y0[ui[4 + r]];
        bb[r] = bcol[ui[1 + r]];
      }
    const double q = rho * Ru[u] + adj_e(e, m, yy, bb);
    Qn[u] = q;
    part[0] += q * Wu[u];
  }
  const double* R = rec + wf.r_R;
  const double p[3] = {P[3 * w], P[3 * w + 1], P[3 * w + 2]};
  const double x[3] = {R[3 * i], R[3 * i + 1], R[3 * i + 2]};
  {
    const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
    for (int j = lane; j < wf.N + wf.nnuc; j += 64) {
      if (j == i) continue;
      double xj[3];
      PairCoef c;
      if (j < wf.N) {
        xj[0] = R[3 * j]; xj[1] = R[3 * j + 1]; xj[2] = R[3 * j + 2];
        c = s != spin_of(wf, j) ? c_anti : c_par;
      } else {
        const int a = j - wf.N;
        xj[0] = wf.nuc[4 * a]; xj[1] = wf.nuc[4 * a + 1]; xj[2] = wf.nuc[4 * a + 2];
        c = en_coef(wf.en + 6 * a);
      }
      const double rn = sqrt((p[0] - xj[0]) * (p[0] - xj[0]) + (p[1] - xj[1]) * (p[1] - xj[1]) +
                             (p[2] - xj[2]) * (p[2] - xj[2]));
      const double ro = sqrt((x[0] - xj[0]) * (x[0] - xj[0]) + (x[1] - xj[1]) * (x[1] - xj[1]) +
                             (x[2] - xj[2]) * (x[2] - xj[2]));
      part[1] += pair_val(rn, wf.kappa, c) - pair_val(ro, wf.kappa, c);
    }
  }
  wave_sum<2>(part);
  const double rdet = part[0] / S, dU = part[1];
  bool accept = false;
  const double ir = 1.0 / rho;
  if (rdet > 0.0 && rho != 0.0) {
    // drift at r' with the state after the move: B'[:, il] = bcol / rho,
    // T' = T + bcol y^T / rho, R'_u = Q_u / rho, S' = S rdet / rho
    const double Snew = S * rdet / rho;
    double a[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* wc = vp + (1 + c) * wf.nop;
      double tc = 0.0;
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < n) tc += wc[ref[j]] * C[j];
      a[c] = __shfl(tc, il, 64);  // sum_j w_c[ref_j] bcol_j
      if (tl) yc[c * 64 + (lane - n)] = wc[porb[lane - n]] - tc - a[c] * y * ir;
    }
    __syncthreads();
    double dp[6] = {0, 0, 0, 0, 0, 0};
    for (int u = lane; u < nU; u += 64) {
      const int* ui = sp.uinfo + 8 * u;
      double m[9], bb[3] = {0, 0, 0};
      const int e = gather_u(ui, Tg, nP, m, bcol, y0, ir);
#pragma unroll
      for (int r = 0; r < 3; ++r)
        if (r < e) bb[r] = bcol[ui[1 + r]] * ir;
      const double Rnew = Qn[u] * ir;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double yy[3] = {0, 0, 0};
#pragma unroll
        for (int r = 0; r < 3; ++r)
          if (r < e) yy[r] = yc[c * 64 + ui[4 + r]];
        dp[c] += (a[c] * ir * Rnew + adj_e(e, m, yy, bb)) * Wu[u];
      }
    }
    double g[3] = {0, 0, 0};
    jastrow_grad_part(wf, R, i, p, g);
    dp[3] = g[0];
    dp[4] = g[1];
    dp[5] = g[2];
    wave_sum<6>(dp);
    double fwd = 0.0, bwd = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double vn = dp[3 + c] + dp[c] / Snew;
      const double d = p[c] - x[c];
      const double fa = d - tau * V[3 * w + c];
      const double ba = -d - tau * vn;
      fwd += fa * fa;
      bwd += ba * ba;
    }
    const double prob = rdet * rdet * exp(2.0 * dU + (fwd - bwd) / (2.0 * tau));
    double ua, dummy;
    philox_pair(seed, (uint32_t)w, step, 4u * i + 1u, 0u, ua, dummy);
    accept = ua < prob;
  }
  if (!accept) return;
  // R_u from the updated minors (old table + bcol y^T / rho, as the column
  // update below forms it) and S, read before any table entry is rewritten
  double vs[1] = {0.0};
  for (int u = lane; u < nU; u += 64) {
    const int* ui = sp.uinfo + 8 * u;
    double m[9];
    const int e = gather_u(ui, Tg, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (r < e && c < e) m[r * 3 + c] = m[r * 3 + c] + bcol[ui[1 + r]] * (y0[ui[4 + c]] * ir);
    const double r = det_e(e, m);
    Rn[u] = r;
    vs[0] += r * Wu[u];
  }
  wave_sum<1>(vs);
  __syncthreads();
  // Sherman-Morrison: B'[j][k] = B[j][k] - bcol_j (u_k - delta_k,il) / rho,
  // T' = T + bcol y^T / rho
  double f = 0.0;
  if (bl) f = -(t - (lane == il ? 1.0 : 0.0)) * ir;
  else if (tl) f = y * ir;
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < n) {
      const double v = C[j] + bcol[j] * f;
      if (bl) Bg[j * n + lane] = v;
      else if (tl) Tg[j * nP + (lane - n)] = v;
    }
  for (int u = lane; u < nU; u += 64) Ru[u] = Rn[u];
  {
    const int o = 1 - s;
    const SpinTab& so = wf.sp[o];
    double* Wo = RW + n0 + n1 + (o ? n0 : 0);
    for (int u = lane; u < so.nU; u += 64) {
      double a = 0.0;
      for (int k = so.wrow[u]; k < so.wrow[u + 1]; ++k) a += so.wcoef[k] * Rn[so.wother[k]];
      Wo[u] = a;
    }
  }
  // gradient rows of electron i at its new point
  double* gr = rec + wf.r_gc + (size_t)i * 3 * wf.nop;
  for (int k = lane; k < 3 * wf.nop; k += 64) gr[k] = vp[wf.nop + k];
  if (lane == 0) {
    RW[2 * (n0 + n1)] = vs[0];
    double* sc = rec + wf.r_sc;
    sc[SC_LOGDET0 + s] += log(fabs(rho));
    if (rho < 0) sc[SC_SGN0 + s] = -sc[SC_SGN0 + s];
    sc[SC_NUPD0 + s] += 1.0;
    if (!(vs[0] != 0.0)) sc[SC_FLAGS] = 1.0;
    double* Rw = rec + wf.r_R;
    Rw[3 * i] = p[0];
    Rw[3 * i + 1] = p[1];
    Rw[3 * i + 2] = p[2];
    nacc[w] += 1.0;
  }
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
template <int PREC>
static hipError_t launch_rows_t(size_t lds, const DevWF* dwf_rows, const double* ctrl, int64_t cap,
                                const double* P, double* Vp, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dmcb_rows<PREC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       163840);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_dmcb_rows<PREC>), dim3((unsigned)((cap + kGroup - 1) / kGroup)), dim3(64), lds, s, dwf_rows,
                     ctrl, P, Vp);
  return hipSuccess;
}

template <int NB>
static hipError_t launch_accept_t(const DevWF& wf, const DevWF* dwf, double* state, const double* ctrl, int64_t cap,
                                  int i, uint64_t seed, uint32_t step, double tau, const double* P, const double* V,
                                  const double* Vp, double* nacc, hipStream_t s) {
  const int nUm = std::max(wf.sp[0].nU, wf.sp[1].nU);
  const size_t lds = (size_t)(320 + 2 * nUm) * sizeof(double);
  hipLaunchKernelGGL((k_dmcb_accept<NB>), dim3((unsigned)cap), dim3(64), lds, s, dwf, state, ctrl, i, seed, step,
                     tau, P, V, Vp, nacc);
  return hipSuccess;
}

// One electron's move for every walker: propose, rows, accept.  P, V [cap][3]
// and Vp [cap][4][nop] are workspace; rows_lds is the LDS of the row tiles'
// layout (dwf_rows).
hipError_t launch_dmcb_move(const DevWF& wf, const DevWF* dwf, const DevWF* dwf_rows, size_t rows_lds, double* state,
                            double* ctrl, int64_t cap, int i, uint64_t seed, uint32_t step, double tau, double* P,
                            double* V, double* Vp, double* nacc, hipStream_t s) {
  hipLaunchKernelGGL(k_dmcb_propose, dim3((unsigned)cap), dim3(64), 0, s, dwf, state, ctrl, i, seed, step, tau, P,
                     V, nacc);
  hipError_t e;
  switch (wf.precision) {
    case 0: e = launch_rows_t<0>(rows_lds, dwf_rows, ctrl, cap, P, Vp, s); break;
    case 1: e = launch_rows_t<1>(rows_lds, dwf_rows, ctrl, cap, P, Vp, s); break;
    default: e = launch_rows_t<2>(rows_lds, dwf_rows, ctrl, cap, P, Vp, s); break;
  }
  if (e != hipSuccess) return e;
  const int nmax = std::max(wf.sp[0].n, wf.sp[1].n);
  if (nmax <= 16) e = launch_accept_t<16>(wf, dwf, state, ctrl, cap, i, seed, step, tau, P, V, Vp, nacc, s);
  else if (nmax <= 32) e = launch_accept_t<32>(wf, dwf, state, ctrl, cap, i, seed, step, tau, P, V, Vp, nacc, s);
  else e = launch_accept_t<64>(wf, dwf, state, ctrl, cap, i, seed, step, tau, P, V, Vp, nacc, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace vbqmc
