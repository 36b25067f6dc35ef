// gfx950 sweep kernel with several walkers per wavefront.
//
// One single-electron sweep (Sec. 2.3.1: Metropolis moves of one electron at
// a time) touches only small per-walker objects: an n x n reference inverse,
// an n x nP table and a few determinant ratios.  With one walker per 64-lane
// wavefront most lanes idle in loops of length n.  Here a wavefront holds
// 64 / G walkers, each owning G lanes (a "group"); a group's loops run over
// its G lanes, its reductions are butterfly shuffles inside the group, and
// its lanes synchronise through wavefront-ordered LDS accesses, so groups may
// take different branches (accept or reject) without a workgroup barrier.
// The trial orbital rows of all walkers of the wavefront are formed in one
// MFMA pass over 16-row tiles of (walker, electron) rows, and so are the
// reference rows of a refresh.
//
// The algebra is that of the block-per-walker kernels: for spin s with
// reference inverse B and table T = B Phi[:, P], a move of electron i to a
// point with orbital row v has
//   rho = sum_j v[ref_j] B[j][i],  y[q] = v[P_q] - sum_k v[ref_k] T[k][q],
//   Q_u = rho R_u + y_Q^T adj(T_JQ) B_J,i,  S'' = sum_u Q_u W_u,
// acceptance probability min(1, (S''/S)^2 exp(2 dU)) with dU the Jastrow
// change, and accepted moves update B and T by Sherman-Morrison rank-1 steps.

#include "vbqmc_group.h"

namespace vbqmc {

// Determinant-sum ratio numerator S'' and Jastrow change dU of moving
// electron i to p, whose orbital row is v.  Leaves the gathered v[ref] (z + n),
// the old inverse column (bcol), y and Q_u for accept_move_g.
template <int G>
__device__ void move_ratio_g(const DevWF& wf, const Lg& l, int i, double px, double py, double pz,
                             const double* v, double& Snew, double& dU, double& rho) {
  const int s = spin_of(wf, i);
  const SpinTab& st = wf.sp[s];
  const int n = st.n, nP = st.nP, il = i - st.e0, q = l.q;
  const double* B = l.B(s);
  const double* T = l.T(s);
  const int* ref = l.ref(s);
  const int* porb = l.porb(s);
  double* y = l.y();
  double* bc = l.bcol();
  double* vr = l.z() + n;
  double prod = 0.0;
  for (int j = q; j < n; j += G) {
    double a = v[ref[j]], b = B[j * n + il];
    vr[j] = a;
    bc[j] = b;
    prod += a * b;
  }
  rho = gsum<G>(prod);
  wave_sync();
  for (int c = q; c < nP; c += G) {
    double a = v[porb[c]];
#pragma unroll 4
    for (int k = 0; k < n; ++k) a -= vr[k] * T[k * nP + c];
    y[c] = a;
  }
  const double* R = l.R();
  const double* nuc = l.nuc();
  const double xo = R[3 * i], yo = R[3 * i + 1], zo = R[3 * i + 2];
  const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
  const double kappa = wf.kappa;
  double du = 0.0;
  for (int j = q; j < wf.N + wf.nnuc; j += G) {
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
    du += pair_val(rn, kappa, c) - pair_val(ro, kappa, c);
  }
  wave_sync();
  const int* uit = l.ui(s);
  double acc = 0.0;
  for (int u = q; u < st.nU; u += G) {
    const int* ui = uit + 8 * u;
    double m[9], yy[3], bb[3];
    int e = gather_u(ui, T, nP, m, nullptr, nullptr, 0.0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (r < e) {
        yy[r] = y[ui[4 + r]];
        bb[r] = bc[ui[1 + r]];
      }
    double qv = rho * l.Ru(s)[u] + adj_e(e, m, yy, bb);
    l.Qu()[u] = qv;
    acc += qv * l.Wu(s)[u];
  }
  Snew = gsum<G>(acc);
  dU = gsum<G>(du);
  wave_sync();
}

// commit an accepted move of electron i (after move_ratio_g)
template <int G>
__device__ void accept_move_g(const DevWF& wf, const Lg& l, int i, double px, double py, double pz,
                              double rho) {
  const int s = spin_of(wf, i);
  const SpinTab& st = wf.sp[s];
  const int n = st.n, nP = st.nP, il = i - st.e0, q = l.q;
  double* B = l.B(s);
  double* T = l.T(s);
  double* z = l.z();
  const double* vr = l.z() + n;
  for (int m = q; m < n; m += G) {
    double a = 0.0;
#pragma unroll 4
    for (int k = 0; k < n; ++k) a += vr[k] * B[k * n + m];
    z[m] = (m == il ? a - 1.0 : a);
  }
  wave_sync();
  const double ir = 1.0 / rho;
  const double* bc = l.bcol();
  const double* y = l.y();
  const float rn = 1.0f / (float)n, rp = 1.0f / (float)max(nP, 1);
  for (int idx = q; idx < n * n; idx += G) {
    int j = div_small(idx, rn), m = idx - j * n;
    B[idx] -= bc[j] * (z[m] * ir);
  }
  for (int idx = q; idx < n * nP; idx += G) {
    int j = div_small(idx, rp), c = idx - j * nP;
    T[idx] += bc[j] * (y[c] * ir);
  }
  if (q == 0) {
    double* sc = l.sc();
    sc[SC_LOGDET0 + s] += log(fabs(rho));
    if (rho < 0) sc[SC_SGN0 + s] = -sc[SC_SGN0 + s];
    sc[SC_NUPD0 + s] += 1.0;
    double* R = l.R();
    R[3 * i] = px; R[3 * i + 1] = py; R[3 * i + 2] = pz;
  }
  wave_sync();
  // R_u of this spin and S (W of this spin does not depend on this spin's
  // R), then the other spin's W
  double vS = 0.0;
  for (int u = q; u < st.nU; u += G) {
    double m[9];
    int e = gather_u(l.ui(s) + 8 * u, T, nP, m, nullptr, nullptr, 0.0);
    double r = det_e(e, m);
    l.Ru(s)[u] = r;
    vS += r * l.Wu(s)[u];
  }
  vS = gsum<G>(vS);
  if (q == 0) l.sc()[SC_S] = vS;
  wave_sync();
  const int o = 1 - s;
  const double* Ro = l.Ru(s);
  const int* wr = l.wrow(o);
  const int* wo = l.woth(o);
  const double* wc = l.wcoef(o);
  for (int u = q; u < wf.sp[o].nU; u += G) {
    double w = 0.0;
    for (int k = wr[u]; k < wr[u + 1]; ++k) w += wc[k] * Ro[wo[k]];
    l.Wu(o)[u] = w;
  }
  wave_sync();
}

// one wavefront, NG = 64 / G walkers
// PT: precision of the trial rows; PE: of the refresh rows
template <int G, int PT, int PE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_g(
    const DevWF* __restrict__ pwf, double* state, int64_t W, uint64_t seed, uint32_t step, double step_size,
    double* n_acc) {
  constexpr int NG = 64 / G;
  const DevWF& wf = *pwf;
  const int g = threadIdx.x / G, q = threadIdx.x & (G - 1);
  const int64_t w = (int64_t)blockIdx.x * NG + g;
  const bool live = w < W;
  const int N = wf.N;
  Ld l(lds_dyn, wf);
  stage_tables<64, PE>(wf, l);
  Lg lg(lds_dyn, g, wf, q);
  // records of the wavefront's walkers, read by all 64 lanes
  for (int gg = 0; gg < NG; ++gg) {
    const int64_t ww = (int64_t)blockIdx.x * NG + gg;
    if (ww >= W) break;
    const double* rec = state + ww * wf.rec_len;
    double* S = lds_dyn + wf.gw_base + gg * wf.gw_stride;
    for (int k = threadIdx.x; k < 3 * N; k += 64) S[wf.l_R + k] = rec[wf.r_R + k];
    for (int s = 0; s < 2; ++s) {
      const SpinTab& st = wf.sp[s];
      for (int k = threadIdx.x; k < st.n * st.n; k += 64) S[wf.l_B[s] + k] = rec[wf.r_B[s] + k];
      for (int k = threadIdx.x; k < st.n * st.nP; k += 64) S[wf.l_T[s] + k] = rec[wf.r_T[s] + k];
    }
    if (threadIdx.x < 8) S[wf.l_sc + threadIdx.x] = rec[wf.r_sc + threadIdx.x];
  }
  __syncthreads();
  double* sc = lg.sc();
  const double na0 = live && q == 0 ? n_acc[w] : 0.0;  // read early: the tail then only stores
  bool bad = true;
  if (live) {
    compute_RWS_g<G>(wf, lg);
    bad = !(sc[SC_S] != 0.0) || sc[SC_FLAGS] != 0.0;
  }
  // trial positions and acceptance draws of every electron of every walker
  double* Rp = lds_dyn + wf.l_Rp;  // [NG][N][3]
  double* ua = lds_dyn + wf.l_ua;  // [NG][N]
  double* Vn = lds_dyn + wf.l_Vn;  // [NG][N][nop]
  {
    const double* R = lg.R();
    for (int i = q; i < N; i += G) {
      double px = 0.0, py = 0.0, pz = 0.0, u = 1.0;
      if (live && !bad) {
        double a0, a1, b0, b1, dummy;
        philox_pair(seed, (uint32_t)w, step, 4u * i, 0u, a0, a1);
        philox_pair(seed, (uint32_t)w, step, 4u * i, 1u, b0, b1);
        philox_pair(seed, (uint32_t)w, step, 4u * i + 1u, 0u, u, dummy);
        px = R[3 * i] + step_size * (2.0 * a0 - 1.0);
        py = R[3 * i + 1] + step_size * (2.0 * a1 - 1.0);
        pz = R[3 * i + 2] + step_size * (2.0 * b0 - 1.0);
      }
      const int r = g * N + i;
      Rp[3 * r] = px; Rp[3 * r + 1] = py; Rp[3 * r + 2] = pz;
      ua[r] = u;
    }
  }
  __syncthreads();
  for (int g0 = 0; g0 < NG * N; g0 += kGroup) {
    const int ne = min(kGroup, NG * N - g0);
    group_radial<64, PT, 1>(wf, l, Rp, g0, ne);
    group_channel<64, PT, 1>(wf, l, ne, 0, Vn + g0 * wf.nop, ne);
  }
  double na = 0.0;
  if (live && !bad) {
    for (int i = 0; i < N; ++i) {
      const int r = g * N + i;
      const double px = Rp[3 * r], py = Rp[3 * r + 1], pz = Rp[3 * r + 2];
      double Snew, dU, rho;
      move_ratio_g<G>(wf, lg, i, px, py, pz, Vn + r * wf.nop, Snew, dU, rho);
      const double ratio = Snew / sc[SC_S] * exp(dU);
      if (ua[r] < ratio * ratio) {
        accept_move_g<G>(wf, lg, i, px, py, pz, rho);
        na += 1.0;
      }
    }
  }
  // refresh the walkers that reached the update limit: reference and table
  // rows at the current positions on MFMA (trial rows are dead here)
  const bool need = live && !bad && (wf.refresh_each_step || sc[SC_NUPD0] >= wf.refresh_every ||
                                       sc[SC_NUPD1] >= wf.refresh_every);
  const unsigned long long lead = __ballot(need && q == 0);  // one bit per group that refreshes
  if (lead) {
    // rows of the refreshing walkers only, packed in group order
    const int slot = __popcll(lead & ((1ull << (g * G)) - 1ull));
    const int nrows = __popcll(lead) * N;
    if (need) {
      const double* R = lg.R();
      for (int k = q; k < 3 * N; k += G) Rp[3 * slot * N + k] = R[k];
    }
    __syncthreads();
    for (int g0 = 0; g0 < nrows; g0 += kGroup) {
      const int ne = min(kGroup, nrows - g0);
      group_radial<64, PE, 1>(wf, l, Rp, g0, ne);
      group_channel<64, PE, 1>(wf, l, ne, 0, Vn + g0 * wf.nop, ne);
    }
    if (need) {
      for (int s = 0; s < 2; ++s) {
        const SpinTab& st = wf.sp[s];
        const int wdt = st.n + st.nP;
        const int* ref = lg.ref(s);
        const int* porb = lg.porb(s);
        const float rw = 1.0f / (float)wdt;
        for (int idx = q; idx < st.n * wdt; idx += G) {
          const int il = div_small(idx, rw), j = idx - il * wdt;
          const double* row = Vn + (size_t)(slot * N + st.e0 + il) * wf.nop;
          if (j < st.n) lg.B(s)[il * st.n + j] = row[ref[j]];
          else lg.PP(s)[il * st.nP + (j - st.n)] = row[porb[j - st.n]];
        }
      }
      wave_sync();
      if (finish_state_g<G>(wf, lg)) compute_RWS_g<G>(wf, lg);
      else bad = true;
    }
  }
  if (live && !bad && !(sc[SC_S] != 0.0)) bad = true;
  if (live && bad && q == 0) sc[SC_FLAGS] = 1.0;
  __syncthreads();
  for (int gg = 0; gg < NG; ++gg) {
    const int64_t ww = (int64_t)blockIdx.x * NG + gg;
    if (ww >= W) break;
    double* rec = state + ww * wf.rec_len;
    const double* S = lds_dyn + wf.gw_base + gg * wf.gw_stride;
    for (int k = threadIdx.x; k < 3 * N; k += 64) rec[wf.r_R + k] = S[wf.l_R + k];
    for (int s = 0; s < 2; ++s) {
      const SpinTab& st = wf.sp[s];
      for (int k = threadIdx.x; k < st.n * st.n; k += 64) rec[wf.r_B[s] + k] = S[wf.l_B[s] + k];
      for (int k = threadIdx.x; k < st.n * st.nP; k += 64) rec[wf.r_T[s] + k] = S[wf.l_T[s] + k];
    }
    if (threadIdx.x < 8) rec[wf.r_sc + threadIdx.x] = S[wf.l_sc + threadIdx.x];
    // determinant ratios, partner sums and S for the batched local energy
    const int n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
    for (int k = threadIdx.x; k < 2 * (n0 + n1) + 1; k += 64) {
      double v;
      if (k < n0) v = S[wf.l_Ru[0] + k];
      else if (k < n0 + n1) v = S[wf.l_Ru[1] + k - n0];
      else if (k < 2 * n0 + n1) v = S[wf.l_Wu[0] + k - n0 - n1];
      else if (k < 2 * (n0 + n1)) v = S[wf.l_Wu[1] + k - 2 * n0 - n1];
      else v = S[wf.l_sc + SC_S];
      rec[wf.r_RW + k] = v;
    }
  }
  if (live && q == 0) n_acc[w] = na0 + na;
}

template <int G, int PT, int PE>
static hipError_t launch_sweep_g_t(const DevWF& wf, const DevWF* dwf, double* state, int64_t W, uint64_t seed,
                                   uint32_t step, double step_size, double* n_acc, hipStream_t s) {
  constexpr int NG = 64 / G;
  size_t lds = (size_t)wf.lds_sweepg_doubles * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_sweep_g<G, PT, PE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_sweep_g<G, PT, PE>), dim3((unsigned)((W + NG - 1) / NG)), dim3(64), lds, s, dwf, state, W,
                     seed, step, step_size, n_acc);
  return hipSuccess;
}

// wavefront sweep with G lanes per walker (G = 16 or 32); the mixed form takes
// the trial rows in FP32 and the refresh rows in FP64
template <int G>
static hipError_t launch_sweep_g_p(const DevWF& wf, const DevWF* dwf, double* state, int64_t W, uint64_t seed,
                                   uint32_t step, double step_size, double* n_acc, hipStream_t s) {
  if (wf.trial_prec != wf.precision)
    return launch_sweep_g_t<G, 1, 0>(wf, dwf, state, W, seed, step, step_size, n_acc, s);
  switch (wf.precision) {
    case 0: return launch_sweep_g_t<G, 0, 0>(wf, dwf, state, W, seed, step, step_size, n_acc, s);
    case 1: return launch_sweep_g_t<G, 1, 1>(wf, dwf, state, W, seed, step, step_size, n_acc, s);
    default: return launch_sweep_g_t<G, 2, 2>(wf, dwf, state, W, seed, step, step_size, n_acc, s);
  }
}

hipError_t launch_sweep_g(const DevWF& wf, const DevWF* dwf, int G, double* state, int64_t W, uint64_t seed,
                          uint32_t step, double step_size, double* n_acc, hipStream_t s) {
  if (G == 16) return launch_sweep_g_p<16>(wf, dwf, state, W, seed, step, step_size, n_acc, s);
  return launch_sweep_g_p<32>(wf, dwf, state, W, seed, step, step_size, n_acc, s);
}

}  // namespace vbqmc
