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
//            update, lane k owning column k of [B | T] (streamed from the
//            record, the table also kept in LDS for the minors).
// The walker records stay in HBM between launches and each launch streams
// what it needs, so occupancy no longer depends on how much state a walker
// has.  Inverse refresh, the local energy and the branching weight follow in
// a per-walker kernel after the last electron.

#include "vbqmc_group.h"

namespace vbqmc {

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

// Distinct determinants u = lane and u = lane + 64 of a wavefront: replaced
// slots J, table indices Q, R_u and W_u held in registers for the whole
// kernel (at most 128 distinct determinants per spin).
struct DetLanes {
  int e[2], J[2][3], Q[2][3];
  double R[2], W[2];
};

__device__ __forceinline__ void load_det_lanes(const SpinTab& sp, const double* Ru, const double* Wu, int lane,
                                               DetLanes& d) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int u = lane + 64 * h;
    d.e[h] = 0;
    d.R[h] = 0.0;
    d.W[h] = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) d.J[h][r] = d.Q[h][r] = 0;
    if (u < sp.nU) {
      const int* ui = sp.uinfo + 8 * u;
      d.e[h] = ui[0];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        d.J[h][r] = ui[1 + r];
        d.Q[h][r] = ui[4 + r];
      }
      d.R[h] = Ru[u];
      d.W[h] = Wu[u];
    }
  }
}

// the e x e minor T[J, Q] (+ bc_J y_Q^T * irho when bc is set) from a table in LDS
__device__ __forceinline__ void minor_of(const DetLanes& d, int h, const double* T, int nP, double* m,
                                         const double* bc, const double* y, double irho) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (r < d.e[h] && c < d.e[h]) {
        double v = T[d.J[h][r] * nP + d.Q[h][c]];
        if (bc) v += bc[d.J[h][r]] * y[d.Q[h][c]] * irho;
        m[r * 3 + c] = v;
      }
}

// ---------------------------------------------------------------------------
// propose: drift at the current point and the drift-diffusion proposal
// ---------------------------------------------------------------------------
// LDS (doubles): bcol [64] | yc [4][64] | T [n nP]
__global__ __launch_bounds__(64) void k_dmcb_propose(const DevWF* __restrict__ pwf, double* state,
                                                     double* ctrl, int i, uint64_t seed, uint32_t step,
                                                     double tau, double* P, double* V, double* nacc) {
  double* bcol = lds_dyn;
  double* yc = lds_dyn + 64;
  double* Tl = lds_dyn + 320;
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
      nacc[3 * w] = 0.0;
      nacc[3 * w + 1] = 0.0;
      nacc[3 * w + 2] = 0.0;
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
  DetLanes d;
  load_det_lanes(sp, rw.Ru, rw.Wu, lane, d);
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
      Tl[l * nP + lane] = t;
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
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (lane + 64 * h >= sp.nU) continue;
    double m[9], bb[3] = {0, 0, 0};
    minor_of(d, h, Tl, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < d.e[h]) bb[r] = bcol[d.J[h][r]];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double yy[3] = {0, 0, 0};
#pragma unroll
      for (int r = 0; r < 3; ++r)
        if (r < d.e[h]) yy[r] = yc[c * 64 + d.Q[h][r]];
      part[c] += (rp[c] * d.R[h] + adj_e(d.e[h], m, yy, bb)) * d.W[h];
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
  const FnInfo fi = fn_info(l, mu);
  const int sh = fi.sh;
  if (sh < 0) {
    o[0] = o[1] = o[2] = o[3] = T(0);
    return;
  }
  const int m = fi.m, kind = fi.kind, lq = fi.lq;
  const T* d = (const T*)l.disp() + e * disp_stride(wf) + 4 * fi.nuc;
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

// Row tiles of 16 walkers (rows e < ne), three uses:
//   MODE 0  value and gradient rows at the proposals P:
//           out[(w0 + e) * 4 * nop + c * nop + p], c = value, x, y, z;
//   MODE 1  value rows at electron i of walkers whose spin-s reference inverse
//           is due for a refresh, scattered into the record: reference
//           columns into the matrix A (the B area, inverted in place later),
//           table columns into PP (the backup area's T slot);
//   MODE 2  gradient and Laplacian rows at electron i:
//           out[(w0 + e) * 4 * nop + c * nop + p], c = x, y, z, Laplacian;
//           with write_gc also the gradient rows into the record's cache.
// A tile is one workgroup of NT threads (NT / 64 wavefronts): the wavefronts
// share the staged basis tables and split the radial sums, then take the
// 16-column output tiles in turn.
template <int PREC, int MODE, int NT>
__global__ __launch_bounds__(NT) void k_dmcb_rows(const DevWF* __restrict__ pwf, const double* ctrl,
                                                  const double* P, double* out, double* state, int i,
                                                  int write_gc) {
  typedef typename std::conditional<PREC == 0, double, float>::type T;
  constexpr int NW = NT / 64;
  const DevWF& wf = *pwf;
  const int64_t W = (int64_t)ctrl[DC_W];
  const int64_t w0 = (int64_t)blockIdx.x * kGroup;
  if (ctrl[DC_ERR] != 0.0 || w0 >= W) return;
  const int ne = (int)min((int64_t)kGroup, W - w0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s = spin_of(wf, i);
  const SpinTab& sp = wf.sp[s];
  const int il = i - sp.e0;
  if constexpr (MODE == 1) {
    bool need = false;  // walker threadIdx.x (< ne) refreshes spin s
    if (threadIdx.x < ne) {
      const double* sc = state + (w0 + threadIdx.x) * wf.rec_len + wf.r_sc;
      need = sc[SC_FLAGS] == 0.0 && (wf.refresh_each_step || sc[SC_NUPD0 + s] >= wf.refresh_every);
    }
    if (!__syncthreads_or(need)) return;
  }
  Ld l(lds_dyn, wf);
  stage_tables<NT, PREC>(wf, l);
  const double* Rsrc = P + 3 * w0;
  if constexpr (MODE != 0) {
    double* Rt = l.R();
    if (threadIdx.x < 3 * ne)
      Rt[threadIdx.x] = state[(w0 + threadIdx.x / 3) * wf.rec_len + wf.r_R + 3 * i + threadIdx.x % 3];
    Rsrc = Rt;
    __syncthreads();
  }
  group_radial<NT, PREC, 3>(wf, l, Rsrc, 0, ne);
  const int nct = wf.nop / 16;
  const size_t ost = (size_t)4 * wf.nop;
  double* o = out + (size_t)w0 * ost;
  const int e = lane & 15;
  const bool live = e < ne;
  constexpr int NC = MODE == 1 ? 1 : 4;
  typedef typename std::conditional<PREC == 0, v4d, v4f>::type acc_t;
  for (int ct = wave; ct < nct; ct += NW) {
    const int col = ct * 16 + (lane & 15);
    acc_t acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[c][r] = 0;
    if constexpr (PREC != 2) {
      const T* lam = PREC == 0 ? (const T*)wf.lamT : (const T*)wf.lamT32;
      // Mpad is a multiple of 16: four k-steps of 4 functions per pass, their
      // coefficient loads and A operands formed before the MFMAs
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        T a[4][4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * u + (lane >> 4);
          b[u] = lam[(size_t)k * wf.nop + col];
          a[u][0] = a[u][1] = a[u][2] = a[u][3] = T(0);
          if (live) {
            if constexpr (MODE == 0) chan_vg<T>(wf, l, e, k, a[u]);
            else if constexpr (MODE == 1) a[u][0] = chan_value<T, 3>(wf, l, e, k, 0);
            else chan_value4<T>(wf, l, e, k, a[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            if constexpr (PREC == 0) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][c], b[u], acc[c], 0, 0, 0);
            else acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][c], b[u], acc[c], 0, 0, 0);
          }
      }
    } else {
      const uint16_t* lam = wf.lamT16;
      for (int k0 = 0; k0 < wf.Mpad; k0 += 16) {
        const int kb = k0 + 4 * (lane >> 4);
        v4s a[NC], b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float v[4] = {0.f, 0.f, 0.f, 0.f};
          if (live) {
            if constexpr (MODE == 0) chan_vg<float>(wf, l, e, kb + j, v);
            else if constexpr (MODE == 1) v[0] = chan_value<float, 3>(wf, l, e, kb + j, 0);
            else chan_value4<float>(wf, l, e, kb + j, v);
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) a[c][j] = (short)f2bf(v[c]);
          b[j] = (short)lam[(size_t)(kb + j) * wf.nop + col];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[c], b, acc[c], 0, 0, 0);
      }
    }
    // output rows of register r: f64 16x16x4 holds row 4r + lane/16, the
    // f32 and bf16 forms row 4(lane/16) + r
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = PREC == 0 ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r;
      if (row >= ne) continue;
      if constexpr (MODE == 1) {
        const int m = sp.omap[col];
        if (m < 0) continue;
        double* rec = state + (w0 + row) * wf.rec_len;
        const double* sc = rec + wf.r_sc;
        if (!(sc[SC_FLAGS] == 0.0 && (wf.refresh_each_step || sc[SC_NUPD0 + s] >= wf.refresh_every))) continue;
        if (m < sp.n) rec[wf.r_B[s] + il * sp.n + m] = (double)acc[0][r];
        else rec[wf.r_bk + wf.r_T[s] - wf.r_R + il * sp.nP + (m - sp.n)] = (double)acc[0][r];
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) o[row * ost + c * wf.nop + col] = (double)acc[c][r];
        if (MODE == 2 && write_gc) {
          double* gr = state + (w0 + row) * wf.rec_len + wf.r_gc + (size_t)i * 3 * wf.nop;
#pragma unroll
          for (int c = 0; c < 3; ++c) gr[c * wf.nop + col] = (double)acc[c][r];
        }
      }
    }
  }
}

constexpr int kRowsNT = 256;  // threads of a row tile

// ---------------------------------------------------------------------------
// accept: ratio, node check, drift at r', Green's function, Metropolis,
// Sherman-Morrison update
// ---------------------------------------------------------------------------
// LDS (doubles): bcol [64] | y0 [64] | yc [3][64] | Qn [128] | Rn [128] | T [n nP]
__global__ __launch_bounds__(64) void k_dmcb_accept(const DevWF* __restrict__ pwf, double* state,
                                                    const double* __restrict__ ctrl, int i, uint64_t seed,
                                                    uint32_t step, double tau, const double* __restrict__ P,
                                                    const double* __restrict__ V,
                                                    const double* __restrict__ Vp, double* nacc) {
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
  double* bcol = lds_dyn;
  double* y0 = lds_dyn + 64;
  double* yc = lds_dyn + 128;
  double* Qn = lds_dyn + 320;
  double* Rn = Qn + 128;
  double* Tl = Rn + 128;  // the table T, for the minors of the distinct determinants
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
  DetLanes d;
  load_det_lanes(sp, Ru, Wu, lane, d);
  // t^c_k = sum_j w_c[ref_j] C[j][k] for the value (c = 0) and gradient rows,
  // C = [B | T] streamed column by column: u = v_ref^T B on B lanes,
  // v_ref^T T on table lanes
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < n; ++j) {
    double cj = 0.0;
    if (bl) cj = Bg[j * n + lane];
    else if (tl) cj = Tg[j * nP + (lane - n)];
    const int rj = ref[j];
#pragma unroll
    for (int c = 0; c < 4; ++c) t[c] += vp[c * wf.nop + rj] * cj;
    if (lane == il) bcol[j] = cj;
    if (tl) Tl[j * nP + (lane - n)] = cj;
  }
  const double rho = __shfl(t[0], il, 64);
  const double y = tl ? vp[porb[lane - n]] - t[0] : 0.0;
  if (tl) y0[lane - n] = y;
  __syncthreads();
  // Q_u = rho R_u + y_Q^T adj(T_JQ) B_J,il ; S'' = sum_u Q_u W_u ; Jastrow change
  double part[2] = {0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int u = lane + 64 * h;
    if (u >= nU) continue;
    double m[9], yy[3] = {0, 0, 0}, bb[3] = {0, 0, 0};
    minor_of(d, h, Tl, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < d.e[h]) {
        yy[r] = y0[d.Q[h][r]];
        bb[r] = bcol[d.J[h][r]];
      }
    const double q = rho * d.R[h] + adj_e(d.e[h], m, yy, bb);
    Qn[u] = q;
    part[0] += q * d.W[h];
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
      a[c] = __shfl(t[1 + c], il, 64);  // sum_j w_c[ref_j] bcol_j
      if (tl) yc[c * 64 + (lane - n)] = vp[(1 + c) * wf.nop + porb[lane - n]] - t[1 + c] - a[c] * y * ir;
    }
    __syncthreads();
    double dp[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int u = lane + 64 * h;
      if (u >= nU) continue;
      double m[9], bb[3] = {0, 0, 0};
      minor_of(d, h, Tl, nP, m, bcol, y0, ir);
#pragma unroll
      for (int r = 0; r < 3; ++r)
        if (r < d.e[h]) bb[r] = bcol[d.J[h][r]] * ir;
      const double Rnew = Qn[u] * ir;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double yy[3] = {0, 0, 0};
#pragma unroll
        for (int r = 0; r < 3; ++r)
          if (r < d.e[h]) yy[r] = yc[c * 64 + d.Q[h][r]];
        dp[c] += (a[c] * ir * Rnew + adj_e(d.e[h], m, yy, bb)) * d.W[h];
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
      const double dd = p[c] - x[c];
      const double fa = dd - tau * V[3 * w + c];
      const double ba = -dd - tau * vn;
      fwd += fa * fa;
      bwd += ba * ba;
    }
    const double prob = rdet * rdet * exp(2.0 * dU + (fwd - bwd) / (2.0 * tau));
    double ua, dummy;
    philox_pair(seed, (uint32_t)w, step, 4u * i + 1u, 0u, ua, dummy);
    accept = ua < prob;
  }
  if (lane == 0) {
    // squared displacement of the proposal (effective time step)
    const double d2 = (p[0] - x[0]) * (p[0] - x[0]) + (p[1] - x[1]) * (p[1] - x[1]) + (p[2] - x[2]) * (p[2] - x[2]);
    nacc[3 * w + 1] += d2;
    if (accept) nacc[3 * w + 2] += d2;
  }
  if (!accept) return;
  // R_u from the updated minors (old table + bcol y^T / rho, as the column
  // update below forms it) and S
  double vs[1] = {0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int u = lane + 64 * h;
    if (u >= nU) continue;
    double m[9];
    minor_of(d, h, Tl, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (r < d.e[h] && c < d.e[h]) m[r * 3 + c] = m[r * 3 + c] + bcol[d.J[h][r]] * (y0[d.Q[h][c]] * ir);
    const double r = det_e(d.e[h], m);
    Rn[u] = r;
    vs[0] += r * d.W[h];
  }
  wave_sum<1>(vs);
  __syncthreads();
  // Sherman-Morrison: B'[j][k] = B[j][k] - bcol_j (u_k - delta_k,il) / rho,
  // T' = T + bcol y^T / rho, column by column
  double f = 0.0;
  if (bl) f = -(t[0] - (lane == il ? 1.0 : 0.0)) * ir;
  else if (tl) f = y * ir;
  if (bl) {
    for (int j = 0; j < n; ++j) Bg[j * n + lane] += bcol[j] * f;
  } else if (tl) {
    for (int j = 0; j < n; ++j) Tg[j * nP + (lane - n)] = Tl[j * nP + (lane - n)] + bcol[j] * f;
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
    nacc[3 * w] += 1.0;
  }
}

// ---------------------------------------------------------------------------
// end of a step: inverse refresh, local energy, branching weight
// ---------------------------------------------------------------------------
// Refresh of the walkers whose spin reached refresh_every updates: the value
// rows were scattered into the record as A (B area) and PP (backup T slot);
// the two half-waves invert the two spins' A in LDS at the same time, then
// T = B PP, and R_u, W_u and S of both spins are rebuilt.
// LDS (doubles): per spin A [n^2], PP [n nP], T [n nP]; pivots and columns.
__global__ __launch_bounds__(64) void k_dmcb_refresh(const DevWF* __restrict__ pwf, double* state,
                                                     const double* ctrl) {
  const DevWF& wf = *pwf;
  const int64_t w = blockIdx.x;
  const int64_t W = (int64_t)ctrl[DC_W];
  if (ctrl[DC_ERR] != 0.0 || w >= W) return;
  double* rec = state + w * wf.rec_len;
  double* sc = rec + wf.r_sc;
  if (sc[SC_FLAGS] != 0.0) return;
  bool need[2];
  for (int s = 0; s < 2; ++s)
    need[s] = wf.sp[s].n > 0 && (wf.refresh_each_step || sc[SC_NUPD0 + s] >= wf.refresh_every);
  if (!need[0] && !need[1]) return;
  const int lane = threadIdx.x;
  const int nmax = max(wf.sp[0].n, wf.sp[1].n);
  double* A[2];
  double* PP[2];
  double* Tl[2];
  {
    double* p = lds_dyn;
    for (int s = 0; s < 2; ++s) {
      const int n = wf.sp[s].n, nP = wf.sp[s].nP;
      A[s] = p; p += n * n;
      PP[s] = p; p += n * nP;
      Tl[s] = p; p += n * nP;
    }
    // pivots (2 nmax ints in nmax doubles) and the pivot columns of both spins
    int* piv = (int*)p;
    double* f = p + nmax;
    for (int s = 0; s < 2; ++s) {
      const SpinTab& sp = wf.sp[s];
      const int n = sp.n, nP = sp.nP;
      if (need[s]) {
        for (int k = lane; k < n * n; k += 64) A[s][k] = rec[wf.r_B[s] + k];
        for (int k = lane; k < n * nP; k += 64) PP[s][k] = rec[wf.r_bk + wf.r_T[s] - wf.r_R + k];
      } else {
        for (int k = lane; k < n * nP; k += 64) Tl[s][k] = rec[wf.r_T[s] + k];
      }
    }
    __syncthreads();
    // half-wave h inverts spin h
    const int h = lane >> 5, qh = lane & 31;
    bool ok = true;
    double ld = 0.0, sg = 1.0;
    if (need[h]) ok = gj_invert_h<32>(A[h], wf.sp[h].n, qh, piv + h * nmax, f + h * nmax, ld, sg);
    const bool ok_other = __shfl_xor((int)ok, 32, 64) != 0;
    ok = ok && ok_other;
    if (qh == 0 && need[h]) {
      sc[SC_LOGDET0 + h] = ld;
      sc[SC_SGN0 + h] = sg;
      sc[SC_NUPD0 + h] = 0.0;
    }
    __syncthreads();
    if (!ok) {
      if (lane == 0) sc[SC_FLAGS] = 1.0;
      return;
    }
  }
  // T = B PP of the refreshed spins; B and T back to the record
  for (int s = 0; s < 2; ++s) {
    if (!need[s]) continue;
    const int n = wf.sp[s].n, nP = wf.sp[s].nP;
    for (int idx = lane; idx < n * nP; idx += 64) {
      const int j = idx / max(nP, 1), c = idx - j * nP;
      double a = 0.0;
      for (int k = 0; k < n; ++k) a += A[s][j * n + k] * PP[s][k * nP + c];
      Tl[s][idx] = a;
      rec[wf.r_T[s] + idx] = a;
    }
    for (int k = lane; k < n * n; k += 64) rec[wf.r_B[s] + k] = A[s][k];
  }
  __syncthreads();
  // R_u of both spins, W_u from the other spin's R, S
  const int n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
  double* RW = rec + wf.r_RW;
  double* Rl = lds_dyn + (A[1] - lds_dyn) + wf.sp[1].n * (wf.sp[1].n + 2 * wf.sp[1].nP) + 3 * nmax;  // R_u, both spins
  for (int s = 0; s < 2; ++s) {
    const SpinTab& sp = wf.sp[s];
    for (int u = lane; u < sp.nU; u += 64) {
      double m[9];
      const int e = gather_u(sp.uinfo + 8 * u, Tl[s], sp.nP, m, nullptr, nullptr, 0.0);
      Rl[(s ? n0 : 0) + u] = det_e(e, m);
    }
  }
  __syncthreads();
  double vs[1] = {0.0};
  for (int s = 0; s < 2; ++s) {
    const SpinTab& sp = wf.sp[s];
    const double* Ro = Rl + (s ? 0 : n0);
    for (int u = lane; u < sp.nU; u += 64) {
      double a = 0.0;
      for (int k = sp.wrow[u]; k < sp.wrow[u + 1]; ++k) a += sp.wcoef[k] * Ro[sp.wother[k]];
      const double r = Rl[(s ? n0 : 0) + u];
      RW[(s ? n0 : 0) + u] = r;
      RW[n0 + n1 + (s ? n0 : 0) + u] = a;
      if (s == 0) vs[0] += r * a;
    }
  }
  wave_sum<1>(vs);
  if (lane == 0) {
    RW[2 * (n0 + n1)] = vs[0];
    if (!(vs[0] != 0.0)) sc[SC_FLAGS] = 1.0;
  }
}

// Local-energy terms of electron i (Eq. Elav with Psi = e^U D) from its
// gradient and Laplacian rows (MODE 2 tiles): grad_i D / D and lap_i D / D by
// the row-operator formula of the moves, the Jastrow gradient and Laplacian
// and the potential of electron i (e-e terms halved); kinetic and potential
// sums per walker in ek, ep (overwritten for i = 0).
__global__ __launch_bounds__(64) void k_dmcb_eterm(const DevWF* __restrict__ pwf, const double* state,
                                                   const double* ctrl, int i, const double* __restrict__ Vp,
                                                   double* ek, double* ep) {
  double* bcol = lds_dyn;
  double* yc = lds_dyn + 64;
  double* Tl = lds_dyn + 320;
  const DevWF& wf = *pwf;
  const int64_t w = blockIdx.x;
  const int64_t W = (int64_t)ctrl[DC_W];
  if (ctrl[DC_ERR] != 0.0 || w >= W) return;
  const double* rec = state + w * wf.rec_len;
  if (rec[wf.r_sc + SC_FLAGS] != 0.0) return;
  const int lane = threadIdx.x;
  const int s = spin_of(wf, i);
  const SpinTab& sp = wf.sp[s];
  const int n = sp.n, nP = sp.nP, il = i - sp.e0;
  const RecRW rw = rec_rw(wf, rec, s);
  const double* B = rec + wf.r_B[s];
  const double* T = rec + wf.r_T[s];
  const double* vr = Vp + (size_t)w * 4 * wf.nop;
  const int* ref = sp.ref;
  const int* porb = sp.porb;
  DetLanes d;
  load_det_lanes(sp, rw.Ru, rw.Wu, lane, d);
  double rp[4] = {0.0, 0.0, 0.0, 0.0};
  if (lane < n) {
    const double b = B[lane * n + il];
    bcol[lane] = b;
    const int rj = ref[lane];
#pragma unroll
    for (int c = 0; c < 4; ++c) rp[c] = vr[c * wf.nop + rj] * b;
  }
  if (lane < nP) {
    const int pq = porb[lane];
    double a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = vr[c * wf.nop + pq];
    for (int l = 0; l < n; ++l) {
      const double t = T[l * nP + lane];
      Tl[l * nP + lane] = t;
      const int rl = ref[l];
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] -= vr[c * wf.nop + rl] * t;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) yc[c * 64 + lane] = a[c];
  }
  wave_sum<4>(rp);
  __syncthreads();
  double part[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (lane + 64 * h >= sp.nU) continue;
    double m[9], bb[3] = {0, 0, 0};
    minor_of(d, h, Tl, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < d.e[h]) bb[r] = bcol[d.J[h][r]];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double yy[3] = {0, 0, 0};
#pragma unroll
      for (int r = 0; r < 3; ++r)
        if (r < d.e[h]) yy[r] = yc[c * 64 + d.Q[h][r]];
      part[c] += (rp[c] * d.R[h] + adj_e(d.e[h], m, yy, bb)) * d.W[h];
    }
  }
  // Jastrow gradient, Laplacian and potential of electron i
  {
    const double* R = rec + wf.r_R;
    const double xi = R[3 * i], yi = R[3 * i + 1], zi = R[3 * i + 2];
    const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
    for (int j = lane; j < wf.N + wf.nnuc; j += 64) {
      if (j == i) continue;
      double xj, yj, zj, wv;
      PairCoef cf;
      if (j < wf.N) {
        xj = R[3 * j]; yj = R[3 * j + 1]; zj = R[3 * j + 2];
        cf = s != spin_of(wf, j) ? c_anti : c_par;
        wv = 0.5;
      } else {
        const int a = j - wf.N;
        xj = wf.nuc[4 * a]; yj = wf.nuc[4 * a + 1]; zj = wf.nuc[4 * a + 2];
        cf = en_coef(wf.en + 6 * a);
        wv = -wf.nuc[4 * a + 3];
      }
      const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
      const double r = sqrt(dx * dx + dy * dy + dz * dz), ir = 1.0 / r;
      double u, u1, u2;
      pair_fn(r, wf.kappa, cf, u, u1, u2);
      const double f = u1 * ir;
      part[4] += f * dx;
      part[5] += f * dy;
      part[6] += f * dz;
      part[7] += u2 + 2.0 * f;
      part[8] += wv * ir;
    }
  }
  wave_sum<9>(part);
  if (lane == 0) {
    const double iS = 1.0 / rw.S;
    const double gx = part[4], gy = part[5], gz = part[6];
    const double t = part[7] + part[3] * iS + gx * gx + gy * gy + gz * gz +
                     2.0 * (gx * part[0] + gy * part[1] + gz * part[2]) * iS;
    ek[w] = i == 0 ? t : ek[w] + t;
    ep[w] = i == 0 ? part[8] : ep[w] + part[8];
  }
}

// E_L = -1/2 sum_i T_i + V + V_nn and the branching inputs of the walker, as
// at the end of k_dmc_step.
__global__ __launch_bounds__(256) void k_dmcb_weight(const DevWF* __restrict__ pwf, double* state,
                                                     const double* ctrl, uint64_t seed, uint32_t step, double tau,
                                                     const double* ek, const double* ep, DmcBranch br,
                                                     int only_eloc) {
  const DevWF& wf = *pwf;
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t W = (int64_t)ctrl[DC_W];
  if (ctrl[DC_ERR] != 0.0 || w >= W) return;
  double* sc = state + w * wf.rec_len + wf.r_sc;
  const bool bad = sc[SC_FLAGS] != 0.0;
  const double ET = ctrl[DC_ET];
  const double E_old = sc[SC_ELOC];
  const double En = bad ? NAN : -0.5 * ek[w] + ep[w] + wf.vnn;
  if (only_eloc) {
    sc[SC_ELOC] = En;
    return;
  }
  dmc_branch_inputs(br, w, bad, E_old, En, ET, tau, wf.N, seed, step);
  sc[SC_ELOC] = En;
}

// Rebuild of every record from its positions before a DMC call: clears the
// invalid flag and marks both spins due for a refresh, so that the refresh
// launches rebuild the inverses, tables and ratios from fresh rows.
__global__ __launch_bounds__(256) void k_dmcb_prep(const DevWF* __restrict__ pwf, double* state,
                                                   const double* ctrl) {
  const DevWF& wf = *pwf;
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= (int64_t)ctrl[DC_W]) return;
  double* sc = state + w * wf.rec_len + wf.r_sc;
  sc[SC_FLAGS] = 0.0;
  sc[SC_NUPD0] = wf.refresh_every;
  sc[SC_NUPD1] = wf.refresh_every;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
// the dynamic LDS limit of a row-tile kernel, raised to what this launch needs
// (the kernels' static LDS counts against the device maximum)
static hipError_t rows_lds_attr(const void* fn, size_t lds, size_t& cur) {
  if (lds <= cur) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) cur = lds;
  return e;
}

template <int PREC>
static hipError_t launch_rows_t(size_t lds, const DevWF* dwf_rows, const double* ctrl, int64_t cap,
                                const double* P, double* Vp, hipStream_t s) {
  static size_t cur = 0;
  hipError_t e = rows_lds_attr((const void*)k_dmcb_rows<PREC, 0, kRowsNT>, lds, cur);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dmcb_rows<PREC, 0, kRowsNT>), dim3((unsigned)((cap + kGroup - 1) / kGroup)), dim3(kRowsNT),
                     lds, s, dwf_rows, ctrl, P, Vp, nullptr, 0, 0);
  return hipSuccess;
}

static hipError_t launch_accept(const DevWF& wf, const DevWF* dwf, double* state, const double* ctrl, int64_t cap,
                                int i, uint64_t seed, uint32_t step, double tau, const double* P, const double* V,
                                const double* Vp, double* nacc, hipStream_t s) {
  const int nT = std::max(wf.sp[0].n * wf.sp[0].nP, wf.sp[1].n * wf.sp[1].nP);
  const size_t lds = (size_t)(320 + 256 + nT) * sizeof(double);
  hipLaunchKernelGGL(k_dmcb_accept, dim3((unsigned)cap), dim3(64), lds, s, dwf, state, ctrl, i, seed, step, tau, P,
                     V, Vp, nacc);
  return hipSuccess;
}

// One electron's move for every walker: propose, rows, accept.  P, V [cap][3]
// and Vp [cap][4][nop] are workspace; rows_lds is the LDS of the row tiles'
// layout (dwf_rows).
hipError_t launch_dmcb_move(const DevWF& wf, const DevWF* dwf, const DevWF* dwf_rows, size_t rows_lds, double* state,
                            double* ctrl, int64_t cap, int i, uint64_t seed, uint32_t step, double tau, double* P,
                            double* V, double* Vp, double* nacc, hipStream_t s) {
  const size_t lds_pe = (size_t)(320 + std::max(wf.sp[0].n * wf.sp[0].nP, wf.sp[1].n * wf.sp[1].nP)) * 8;
  hipLaunchKernelGGL(k_dmcb_propose, dim3((unsigned)cap), dim3(64), lds_pe, s, dwf, state, ctrl, i, seed, step, tau,
                     P, V, nacc);
  hipError_t e;
  switch (wf.trial_prec) {  // proposal rows: the mixed form takes them in FP32
    case 0: e = launch_rows_t<0>(rows_lds, dwf_rows, ctrl, cap, P, Vp, s); break;
    case 1: e = launch_rows_t<1>(rows_lds, dwf_rows, ctrl, cap, P, Vp, s); break;
    default: e = launch_rows_t<2>(rows_lds, dwf_rows, ctrl, cap, P, Vp, s); break;
  }
  if (e != hipSuccess) return e;
  e = launch_accept(wf, dwf, state, ctrl, cap, i, seed, step, tau, P, V, Vp, nacc, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// End of an electron-major step: refresh rows and inversions, E_L rows and
// terms per electron, weights.  ek, ep [cap] are workspace.
// With rebuild set (before the first step of a call), every record is
// rebuilt from its positions: inverses, tables, ratios, the gradient-row cache
// and E_L, and no weight is formed.
hipError_t launch_dmcb_finish(const DevWF& wf, const DevWF* dwf, const DevWF* dwf_rows, size_t rows_lds,
                              double* state, double* ctrl, int64_t cap, uint64_t seed, uint32_t step, double tau,
                              double* Vp, double* ek, double* ep, const DmcBranch& br, int rebuild,
                              hipStream_t s) {
  const unsigned tiles = (unsigned)((cap + kGroup - 1) / kGroup);
  static size_t cur[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  auto rows = [&](auto kern, int prec, int mi, int i) -> hipError_t {
    hipError_t e = rows_lds_attr((const void*)kern, rows_lds, cur[prec][mi]);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(tiles), dim3(kRowsNT), rows_lds, s, dwf_rows, ctrl, nullptr, Vp, state, i,
                       rebuild);
    return hipSuccess;
  };
  hipError_t e = hipSuccess;
  const size_t lds_pe = (size_t)(320 + std::max(wf.sp[0].n * wf.sp[0].nP, wf.sp[1].n * wf.sp[1].nP)) * 8;
  if (rebuild)
    hipLaunchKernelGGL(k_dmcb_prep, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, dwf, state, ctrl);
  for (int i = 0; i < wf.N && e == hipSuccess; ++i) {
    switch (wf.precision) {
      case 0: e = rows(k_dmcb_rows<0, 1, kRowsNT>, 0, 0, i); break;
      case 1: e = rows(k_dmcb_rows<1, 1, kRowsNT>, 1, 0, i); break;
      default: e = rows(k_dmcb_rows<2, 1, kRowsNT>, 2, 0, i); break;
    }
  }
  if (e != hipSuccess) return e;
  size_t rl = 0;
  const int nmax = std::max(wf.sp[0].n, wf.sp[1].n);
  for (int sp = 0; sp < 2; ++sp) rl += (size_t)wf.sp[sp].n * (wf.sp[sp].n + 2 * wf.sp[sp].nP);
  rl += 3 * (size_t)nmax + (size_t)(wf.sp[0].nU + wf.sp[1].nU);
  static size_t cur_ref = 0;
  e = rows_lds_attr((const void*)k_dmcb_refresh, rl * sizeof(double), cur_ref);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmcb_refresh, dim3((unsigned)cap), dim3(64), rl * sizeof(double), s, dwf, state, ctrl);
  for (int i = 0; i < wf.N && e == hipSuccess; ++i) {
    switch (wf.precision) {
      case 0: e = rows(k_dmcb_rows<0, 2, kRowsNT>, 0, 1, i); break;
      case 1: e = rows(k_dmcb_rows<1, 2, kRowsNT>, 1, 1, i); break;
      default: e = rows(k_dmcb_rows<2, 2, kRowsNT>, 2, 1, i); break;
    }
    if (e == hipSuccess)
      hipLaunchKernelGGL(k_dmcb_eterm, dim3((unsigned)cap), dim3(64), lds_pe, s, dwf, state, ctrl, i, Vp, ek, ep);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dmcb_weight, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, dwf, state, ctrl, seed,
                     step, tau, ek, ep, br, rebuild);
  return hipGetLastError();
}

}  // namespace vbqmc
