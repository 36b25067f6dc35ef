// gfx950 VMC step kernel with one walker per 16-lane DPP row.
//
// For spin determinants of at most 16 columns (reference slots plus table
// orbitals) a walker's single-electron moves (Sec. 2.3.1) fit one 16-lane row
// of a wavefront: lane k keeps column k of [B | T] (the reference inverse and
// the replaced-column table of the spin being moved) in registers, so that
// with the trial orbital row of a move, kept compact as v_j = orbital ref_j at
// the trial point (j < n) followed by the table orbitals v_P,
//   t_k = sum_{j<n} v_j C[j][k]
// is at once the Sherman-Morrison vector u = v_ref^T B (lanes k < n), the
// determinant ratio rho = u_il of the reference, and y = v_P - v_ref^T T
// (table lanes).  An accepted move is one register FMA per column entry with
// the old column il of B broadcast to the row.  Lane u also keeps the minor
// T[J_u, Q_u] of distinct determinant u and its ratio R_u, so that
//   Q_u = rho R_u + y_Q^T adj(T_JQ) B_J,il,  S'' = sum_u Q_u W_u
// is one row reduction.  The Jastrow change of every move is prepared before
// the sweep: with x_ij (electron i moves while j sits at its old point) and
// y_ij (j already moved) for every pair, the change for electron i is the
// running sum of x_ij over the later electrons and x_ij or y_ij over the
// earlier ones, so a move only adds one table entry per lane when it is
// accepted.  Four walkers share a wavefront; the trial rows of all their
// electrons (formed once per step, both spins together), the reference rows
// of an inverse refresh and the local-energy rows of the four walkers are
// formed on MFMA in tiles of 16 (walker, electron) rows, and the local energy
// (Eq. Elav) is evaluated in the same launch, so that a walker's record
// crosses HBM once per launch however many steps it makes.

#include "vbqmc_group.h"

namespace vbqmc {

constexpr int kRowMaxRounds = 18;  // pair tasks per lane: 4 walkers x N (N - 1) / 2 pairs over 64 lanes

// row of (walker g, electron i) in the trial tables: spins are blocked, then
// walkers, then the spin's electrons (spin 0 holds electrons 0..nup-1)
__device__ __forceinline__ int trial_row(int nup, int ndn, int g, int i) {
  return i < nup ? g * nup + i : kRowWalkers * nup + g * ndn + (i - nup);
}

__device__ __forceinline__ double dist3(const double* a, const double* b) {
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return sqrt(dx * dx + dy * dy + dz * dz);
}

// pair p = i (i - 1) / 2 + j of electrons i > j >= 0
__device__ __forceinline__ void unrank_pair(int p, int& i, int& j) {
  int a = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)p)) * 0.5f);
  if (a * (a - 1) / 2 > p) --a;
  if ((a + 1) * a / 2 <= p) ++a;
  i = a;
  j = p - a * (a - 1) / 2;
}

// PT: precision of the trial rows; PE: of the refresh and local-energy rows
template <int PT, int PE, int NE>
__global__ __launch_bounds__(64) void k_vmc_rows(const DevWF* __restrict__ pwf, double* state, int64_t W,
                                                 int nsteps, uint64_t seed, uint64_t step0, double step_size,
                                                 double* e_sum, double* e2_sum, double* n_acc, double* e_last,
                                                 double* sij_sum) {
  const DevWF& wf = *pwf;
  const int lane = threadIdx.x, g = lane >> 4, q = lane & 15;
  const int64_t wbase = (int64_t)blockIdx.x * kRowWalkers;
  const int64_t w = wbase + g;
  const bool live = w < W;
  const int nlive = (int)min((int64_t)kRowWalkers, W - wbase);
  const int N = wf.N, nn = wf.nnuc, Nup = wf.nup, Ndn = wf.ndn;
  Ld l(lds_dyn, wf);
  stage_tables<64, PE>(wf, l);
  Lg lg(lds_dyn, g, wf, q);
  double* sc = lg.sc();
  // records of the wavefront's walkers
  for (int gg = 0; gg < nlive; ++gg) {
    const double* rec = state + (wbase + gg) * wf.rec_len;
    double* S = lds_dyn + wf.gw_base + gg * wf.gw_stride;
    for (int k = lane; k < 3 * N; k += 64) S[wf.l_R + k] = rec[wf.r_R + k];
    for (int s = 0; s < 2; ++s) {
      const SpinTab& st = wf.sp[s];
      for (int k = lane; k < st.n * st.n; k += 64) S[wf.l_B[s] + k] = rec[wf.r_B[s] + k];
      for (int k = lane; k < st.n * st.nP; k += 64) S[wf.l_T[s] + k] = rec[wf.r_T[s] + k];
    }
    if (lane < 8) S[wf.l_sc + lane] = rec[wf.r_sc + lane];
  }
  __syncthreads();
  // accumulators continue the caller's sums step by step (the same rounding
  // as one launch per step)
  const double na0 = live && q == 0 ? n_acc[w] : 0.0;
  double na = 0.0, elast = 0.0;
  double es = live && q == 0 ? e_sum[w] : 0.0, e2s = live && q == 0 ? e2_sum[w] : 0.0;
  double* Rp = l.L + wf.l_Rp;  // trial positions [spin][walker][electron of spin][3]
  double* ua = l.L + wf.l_ua;  // acceptance draws, same rows
  double* Vn = l.L + wf.l_Vn;  // trial orbital rows [spin][walker][electron of spin][VW]
  const int VW = wf.rows_vw;
  // column map of the trial rows: orbital ref_j of a spin to position j,
  // table orbital p to n + p, every other orbital to -1
  int* cmap = (int*)(l.L + wf.l_cmap);
  for (int k = lane; k < 2 * wf.nop; k += 64) cmap[k] = -1;
  __syncthreads();
  for (int s = 0; s < 2; ++s) {
    const int n = wf.sp[s].n, w2 = n + wf.sp[s].nP;
    for (int j = lane; j < w2; j += 64) cmap[s * wf.nop + (j < n ? l.ref(s)[j] : l.porb(s)[j - n])] = j;
  }
  __syncthreads();
  double* Xj = l.L + wf.l_jx;  // Jastrow move tables [walker][N][N]
  const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
  const double kappa = wf.kappa;
  const int npair = N * (N - 1) / 2;
  const float rnp = 1.0f / (float)max(npair, 1);

  for (int stp = 0; stp < nsteps; ++stp) {
    const uint32_t step = (uint32_t)(step0 + stp);
    bool bad = true;
    if (live) {
      compute_RWS_g<16>(wf, lg);
      bad = !(sc[SC_S] != 0.0) || sc[SC_FLAGS] != 0.0;
    }
    // ---- trial positions and acceptance draws ----
    {
      const double* R = lg.R();
      for (int i = q; i < N; i += 16) {
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
        const int r = trial_row(Nup, Ndn, g, i);
        Rp[3 * r] = px; Rp[3 * r + 1] = py; Rp[3 * r + 2] = pz;
        ua[r] = u;
      }
    }
    __syncthreads();
    // ---- Jastrow move tables ----
    // pair task (walker g2, i > j): x_ij = u(r_i' - r_j) - u(r_i - r_j) in X[i][j],
    // x_ji = u(r_j' - r_i) - u(r_j - r_i) in X[j][i], and the correction
    // y_ij - x_ij = [u(r_i' - r_j') - u(r_i - r_j')] - x_ij kept in a register
    double dreg[kRowMaxRounds];
#pragma unroll
    for (int rd = 0; rd < kRowMaxRounds; ++rd) {
      const int t = rd * 64 + lane;
      dreg[rd] = 0.0;
      if (t < nlive * npair) {
        const int g2 = div_small(t, rnp), p = t - g2 * npair;
        int i, j;
        unrank_pair(p, i, j);
        const double* R2 = lds_dyn + wf.gw_base + g2 * wf.gw_stride + wf.l_R;
        const double* ri = R2 + 3 * i;
        const double* rj = R2 + 3 * j;
        const double* pi = Rp + 3 * trial_row(Nup, Ndn, g2, i);
        const double* pj = Rp + 3 * trial_row(Nup, Ndn, g2, j);
        const PairCoef c = (i < Nup ? 0 : 1) != (j < Nup ? 0 : 1) ? c_anti : c_par;
        // (kappa = 0, the plain Pade form, skips a division per pair function)
        double o, aij, aji, nw;
        if (kappa == 0.0) {
          o = pair_val<true>(dist3(ri, rj), kappa, c);
          aij = pair_val<true>(dist3(pi, rj), kappa, c);
          aji = pair_val<true>(dist3(pj, ri), kappa, c);
          nw = pair_val<true>(dist3(pi, pj), kappa, c);
        } else {
          o = pair_val(dist3(ri, rj), kappa, c);
          aij = pair_val(dist3(pi, rj), kappa, c);
          aji = pair_val(dist3(pj, ri), kappa, c);
          nw = pair_val(dist3(pi, pj), kappa, c);
        }
        double* X = Xj + g2 * N * N;
        X[i * N + j] = aij - o;
        X[j * N + i] = aji - o;
        dreg[rd] = (nw - aji) - (aij - o);
      }
    }
    __syncthreads();
    // run0 / run1: Jastrow change of electrons q / q + 16 given the moves made
    // so far; starts with every earlier electron at its old point
    double run0 = 0.0, run1 = 0.0;
    {
      const double* R = lg.R();
      const double* X = Xj + g * N * N;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int i = q + 16 * k;
        if (i < N && live) {
          const double* pi = Rp + 3 * trial_row(Nup, Ndn, g, i);
          double a = 0.0;
          for (int b = 0; b < nn; ++b) {
            const PairCoef c = en_coef(l.en() + 6 * b);
            a += pair_val(dist3(pi, l.nuc() + 4 * b), kappa, c) - pair_val(dist3(R + 3 * i, l.nuc() + 4 * b), kappa, c);
          }
          // (every entry loaded, the diagonal one dropped by a select: the
          // loads of the row are in flight together)
          for (int j = 0; j < N; ++j) {
            const double x = X[i * N + j];
            a += j != i ? x : 0.0;
          }
          if (k == 0) run0 = a;
          else run1 = a;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int rd = 0; rd < kRowMaxRounds; ++rd) {
      const int t = rd * 64 + lane;
      if (t < nlive * npair) {
        const int g2 = div_small(t, rnp), p = t - g2 * npair;
        int i, j;
        unrank_pair(p, i, j);
        Xj[g2 * N * N + i * N + j] = dreg[rd];
      }
    }
    __syncthreads();
    // ---- trial orbital rows of all electrons of the four walkers ----
    // (rows in the order of Rp; only the columns a move reads are kept)
    for (int g0 = 0; g0 < kRowWalkers * N; g0 += kGroup) {
      const int ne = min(kGroup, kRowWalkers * N - g0);
      group_radial<64, PT, 1>(wf, l, Rp, g0, ne);
      group_channel<64, PT, 1>(wf, l, ne, 0, Vn + g0 * VW, ne, cmap, VW, g0, kRowWalkers * Nup);
    }
    // a move of spin s reads the first NE columns of its row against zero
    // coefficients past n: the columns past the spin's own n + nP get zeros
    for (int s = 0; s < 2; ++s) {
      const int w0 = wf.sp[s].n + wf.sp[s].nP, nz = NE - w0;
      if (wf.sp[s].n == 0 || nz <= 0) continue;
      const int r0 = kRowWalkers * wf.sp[s].e0, nr = kRowWalkers * wf.sp[s].n;
      for (int k = lane; k < nr * nz; k += 64) Vn[(r0 + k / nz) * VW + w0 + k % nz] = 0.0;
    }
    wave_sync();
    // ---- the moves, spin by spin ----
    for (int s = 0; s < 2; ++s) {
      const SpinTab& sp = wf.sp[s];
      const int n = sp.n, nP = sp.nP, nU = sp.nU, e0 = sp.e0;
      if (n == 0) continue;
      const bool own = q >= n && q < n + nP;  // lane of a table orbital
      double C[NE];
      {
        const double* B = lg.B(s);
        const double* T = lg.T(s);
#pragma unroll
        for (int j = 0; j < NE; ++j) {
          double v = 0.0;
          if (j < n) {
            if (q < n) v = B[j * n + q];
            else if (q < n + nP) v = T[j * nP + (q - n)];
          }
          C[j] = v;
        }
      }
      int eu = 0, Ju[3] = {0, 0, 0}, Qx[3] = {0, 0, 0};
      double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      double Ru = 0.0, Wu = 0.0;
      if (q < nU) {
        const int* ui = l.ui(s) + 8 * q;
        eu = gather_u(ui, lg.T(s), nP, m, nullptr, nullptr, 0.0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          Ju[a] = ui[1 + a];
          Qx[a] = ui[4 + a];
        }
        Ru = lg.Ru(s)[q];
        Wu = lg.Wu(s)[q];
      }
      double S = sc[SC_S];
      double mant = 1.0, sgn = sc[SC_SGN0 + s], nupd = sc[SC_NUPD0 + s];
      int ex = 0;
      double* xch = lg.S + wf.l_xch;  // [0, 16): old column il of B; [16, 32): y
      const double* X = Xj + g * N * N;
      // Every load of a move is issued unconditionally (padding slots read
      // zeros or meet zero coefficients), so that the loads of a step are
      // in flight together; the exponential of the Jastrow change, the
      // acceptance draw and the Jastrow table entries do not depend on the
      // determinant ratio and are started first.
      for (int il = 0; il < n; ++il) {
        const int i = e0 + il;
        const double* Vrow = Vn + (kRowWalkers * e0 + g * n + il) * VW;
        const int r = kRowWalkers * e0 + g * n + il;  // trial row of (walker g, electron i)
        const double u_r = ua[r];
        const double xr0 = X[min(q, N - 1) * N + i];
        const double xr1 = X[min(q + 16, N - 1) * N + i];
        double vr[NE];
#pragma unroll
        for (int j = 0; j < NE; ++j) vr[j] = Vrow[j];
        const double vo = Vrow[own ? q : 0];
        const double eU = exp(row_bcast(i < 16 ? run0 : run1, i & 15));
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int j = 0; j < NE; j += 2) {
          t0 += vr[j] * C[j];
          t1 += vr[j + 1] * C[j + 1];
        }
        const double t = t0 + t1;
        const double y = (own ? vo : 0.0) - t;
        const double rho = row_bcast(t, il);
        if (q == il) {
          // (columns past n hold zeros: no test needed)
#pragma unroll
          for (int j = 0; j < NE; ++j) xch[j] = C[j];
        }
        if (own) xch[16 + (q - n)] = y;
        wave_sync();
        double bc[NE];
#pragma unroll
        for (int j = 0; j < NE; ++j) bc[j] = xch[j];
        double yy[3], bb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          yy[a] = xch[16 + Qx[a]];
          bb[a] = xch[Ju[a]];
        }
        const double ir = 1.0 / rho;
        double part = 0.0;
        if (q < nU) {
#pragma unroll
          for (int a = 0; a < 3; ++a)
            if (a >= eu) yy[a] = bb[a] = 0.0;
          part = (rho * Ru + adj_e(eu, m, yy, bb)) * Wu;
        }
        const double Snew = gsum<16>(part);
        const double ratio = Snew / S * eU;
        const bool accept = live && !bad && u_r < ratio * ratio;
        if (accept) {
          // later electrons see electron i at its new point
          if (q > i && q < N) run0 += xr0;
          if (q + 16 > i && q + 16 < N) run1 += xr1;
          double f = 0.0;
          if (q < n) f = -(t - (q == il ? 1.0 : 0.0)) * ir;
          else if (own) f = y * ir;
#pragma unroll
          for (int j = 0; j < NE; ++j)
            if (j < n) C[j] += bc[j] * f;
          double pr = 0.0;
          if (q < nU) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int b = 0; b < 3; ++b)
                if (a < eu && b < eu) m[a * 3 + b] += bb[a] * yy[b] * ir;
            Ru = det_e(eu, m);
            pr = Ru * Wu;
          }
          S = gsum<16>(pr);
          int e2;
          mant = frexp(mant * fabs(rho), &e2);
          ex += e2;
          if (rho < 0) sgn = -sgn;
          nupd += 1.0;
          na += 1.0;
          if (q < 3) lg.R()[3 * i + q] = Rp[3 * r + q];
        }
        wave_sync();
      }
      // this spin's state back to LDS
      {
        double* B = lg.B(s);
        double* T = lg.T(s);
#pragma unroll
        for (int j = 0; j < NE; ++j)
          if (j < n) {
            if (q < n) B[j * n + q] = C[j];
            else if (own) T[j * nP + (q - n)] = C[j];
          }
        if (q < nU) lg.Ru(s)[q] = Ru;
        if (q == 0) {
          sc[SC_LOGDET0 + s] += log(mant) + (double)ex * 0.69314718055994530942;
          sc[SC_SGN0 + s] = sgn;
          sc[SC_NUPD0 + s] = nupd;
          sc[SC_S] = S;
        }
      }
      wave_sync();
      // the other spin's partner sums W from this spin's R
      {
        const int o = 1 - s;
        const double* Ro = lg.Ru(s);
        const int* wr = l.wrow(o);
        const int* wo = l.woth(o);
        const double* wc = l.wcoef(o);
        for (int u = q; u < wf.sp[o].nU; u += 16) {
          double a = 0.0;
          for (int k = wr[u]; k < wr[u + 1]; ++k) a += wc[k] * Ro[wo[k]];
          lg.Wu(o)[u] = a;
        }
      }
      wave_sync();
    }
    // ---- inverse refresh ----
    // Once one walker of the wavefront has reached the update limit, every
    // walker of the wavefront is rebuilt: the row tiles of the refresh are then
    // full (4N rows instead of N), and an earlier rebuild only makes an inverse
    // fresher.
    const bool due = live && !bad && (wf.refresh_each_step || sc[SC_NUPD0] >= wf.refresh_every ||
                                      sc[SC_NUPD1] >= wf.refresh_every);
    const bool need = live && !bad && __ballot(due) != 0;
    const unsigned long long lead = __ballot(need && q == 0);
    if (lead) {
      const int slot = __popcll(lead & ((1ull << (g * 16)) - 1ull));
      const int nrows = __popcll(lead) * N;
      double* Rr = Rp;
      double* Vr = l.L + wf.l_Vr;
      __syncthreads();
      if (need) {
        const double* R = lg.R();
        for (int k = q; k < 3 * N; k += 16) Rr[3 * slot * N + k] = R[k];
      }
      __syncthreads();
      for (int g0 = 0; g0 < nrows; g0 += kGroup) {
        const int ne = min(kGroup, nrows - g0);
        group_radial<64, PE, 1>(wf, l, Rr, g0, ne);
        group_channel<64, PE, 1>(wf, l, ne, 0, Vr + g0 * wf.nop, ne);
      }
      if (need) {
        for (int s = 0; s < 2; ++s) {
          const SpinTab& st = wf.sp[s];
          const int wdt = st.n + st.nP;
          const int* ref = lg.ref(s);
          const int* porb = lg.porb(s);
          const float rw = 1.0f / (float)max(wdt, 1);
          for (int idx = q; idx < st.n * wdt; idx += 16) {
            const int il = div_small(idx, rw), j = idx - il * wdt;
            const double* row = Vr + (size_t)(slot * N + st.e0 + il) * wf.nop;
            if (j < st.n) lg.B(s)[il * st.n + j] = row[ref[j]];
            else lg.PP(s)[il * st.nP + (j - st.n)] = row[porb[j - st.n]];
          }
        }
        wave_sync();
        if (finish_state_g<16>(wf, lg)) compute_RWS_g<16>(wf, lg);
        else bad = true;
      }
    }
    if (live && !bad && !(sc[SC_S] != 0.0)) bad = true;
    if (live && bad && q == 0) sc[SC_FLAGS] = 1.0;
    __syncthreads();
    // ---- local energy (Eq. Elav with Psi = e^U D) ----
    double* Rall = l.L + wf.l_Rall;  // [walker][N][3]
    double* Phi4 = l.L + wf.l_Phi4;
    double* yb = l.L + wf.l_yb64;
    double* gc4 = l.L + wf.l_gc4;    // [walker][N][4]: grad_i D / D, lap_i D / D
    {
      const double* R = lg.R();
      for (int k = q; k < 3 * N; k += 16) Rall[3 * N * g + k] = R[k];
    }
    __syncthreads();
    {
      const int nPm = max(wf.sp[0].nP, wf.sp[1].nP);
      const float rN = 1.0f / (float)N;
      const int nrows = nlive * N;
      for (int g0 = 0; g0 < nrows; g0 += kGroup) {
        const int ne = min(kGroup, nrows - g0);
        group_radial<64, PE, 3>(wf, l, Rall, g0, ne);
        group_channels4<64, PE>(wf, l, ne, Phi4);
        const int t = lane >> 2, c = lane & 3;
        if (t < ne) {
          const int rr = g0 + t, g2 = div_small(rr, rN), i = rr - g2 * N;
          const double* S2 = lds_dyn + wf.gw_base + g2 * wf.gw_stride;
          const int s = (i < Nup ? 0 : 1);
          double tot = 0.0;
          if (S2[wf.l_sc + SC_FLAGS] == 0.0)
            tot = row_op_sum_r<NE>(wf, l, s, Phi4 + (c * kGroup + t) * wf.nop, yb + lane * (nPm + 1), S2 + wf.l_B[s],
                               wf.sp[s].n, i - wf.sp[s].e0, S2 + wf.l_T[s], S2 + wf.l_Ru[s], S2 + wf.l_Wu[s]);
          gc4[4 * rr + c] = tot / S2[wf.l_sc + SC_S];
        }
        __syncthreads();
      }
    }
    // Jastrow gradients and Laplacians and the potential: lanes of a row are
    // 4 electrons x 4 parts of each electron's partners
    double tsum = 0.0, vsum = 0.0;
    {
      const double* R = Rall + 3 * N * g;
      const int p = q & 3, e4 = q >> 2;
      for (int i0 = 0; i0 < N; i0 += 4) {
        const int i = i0 + e4;
        double gx = 0.0, gy = 0.0, gz = 0.0, lap = 0.0, V = 0.0;
        if (i < N && live) {
          const double xi = R[3 * i], yi = R[3 * i + 1], zi = R[3 * i + 2];
          const int si = (i < Nup ? 0 : 1);
          for (int j = p; j < N + nn; j += 4) {
            if (j == i) continue;
            double xj, yj, zj, wv;
            PairCoef cf;
            if (j < N) {
              xj = R[3 * j]; yj = R[3 * j + 1]; zj = R[3 * j + 2];
              cf = si != (j < Nup ? 0 : 1) ? c_anti : c_par;
              wv = 0.5;
            } else {
              const int a = j - N;
              const double* nu = l.nuc() + 4 * a;
              xj = nu[0]; yj = nu[1]; zj = nu[2];
              cf = en_coef(l.en() + 6 * a);
              wv = -nu[3];
            }
            const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
            const double rij = sqrt(dx * dx + dy * dy + dz * dz), ir = 1.0 / rij;
            double u, u1, u2;
            if (kappa == 0.0) pair_fn<true>(rij, kappa, cf, u, u1, u2);
            else pair_fn<false>(rij, kappa, cf, u, u1, u2);
            const double f = u1 * ir;
            gx += f * dx; gy += f * dy; gz += f * dz;
            lap += u2 + 2.0 * f;
            V += wv * ir;
          }
        }
        gx = quad_sum(gx);
        gy = quad_sum(gy);
        gz = quad_sum(gz);
        lap = quad_sum(lap);
        V = quad_sum(V);
        if (i < N && p == 0 && live) {
          const double* gd = gc4 + 4 * (g * N + i);
          tsum += lap + gd[3] + gx * gx + gy * gy + gz * gz + 2.0 * (gx * gd[0] + gy * gd[1] + gz * gd[2]);
          vsum += V;
        }
      }
    }
    tsum = gsum<16>(tsum);
    vsum = gsum<16>(vsum);
    if (live) {
      const bool badw = sc[SC_FLAGS] != 0.0;
      const double el = -0.5 * tsum + vsum + wf.vnn;
      if (!badw) {
        es += el;
        e2s += el * el;
      }
      elast = badw ? NAN : el;
      wave_sync();
      if (q == 0) sc[SC_ELOC] = elast;
      // structure-ratio products r_I r_J (Sec. 2.4)
      if (sij_sum && !badw) {
        const int nv = wf.nstruct, n0 = wf.sp[0].nU;
        double* rI = l.L + wf.l_rI + g * nv;
        const double iS = 1.0 / sc[SC_S];
        const int* srow = l.srow();
        const int* slu = l.slu();
        const double* slc = l.slc();
        for (int I = q; I < nv; I += 16) {
          double a = 0.0;
          for (int k = srow[I]; k < srow[I + 1]; ++k) a += slc[k] * lg.Ru(0)[slu[2 * k]] * lg.Ru(1)[slu[2 * k + 1]];
          rI[I] = a * iS;
        }
        (void)n0;
        wave_sync();
        double* sj = sij_sum + w * nv * nv;
        for (int k = q; k < nv * nv; k += 16) {
          const int I = k / nv, J = k - I * nv;
          sj[k] += rI[I] * rI[J];
        }
      }
    }
    __syncthreads();
  }
  // ---- records back to HBM ----
  for (int gg = 0; gg < nlive; ++gg) {
    double* rec = state + (wbase + gg) * wf.rec_len;
    const double* S = lds_dyn + wf.gw_base + gg * wf.gw_stride;
    for (int k = lane; k < 3 * N; k += 64) rec[wf.r_R + k] = S[wf.l_R + k];
    for (int s = 0; s < 2; ++s) {
      const SpinTab& st = wf.sp[s];
      for (int k = lane; k < st.n * st.n; k += 64) rec[wf.r_B[s] + k] = S[wf.l_B[s] + k];
      for (int k = lane; k < st.n * st.nP; k += 64) rec[wf.r_T[s] + k] = S[wf.l_T[s] + k];
    }
    if (lane < 8) rec[wf.r_sc + lane] = S[wf.l_sc + lane];
    // determinant ratios, partner sums and S, as the sweep kernels leave them
    const int n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
    for (int k = lane; k < 2 * (n0 + n1) + 1; k += 64) {
      double v;
      if (k < n0) v = S[wf.l_Ru[0] + k];
      else if (k < n0 + n1) v = S[wf.l_Ru[1] + k - n0];
      else if (k < 2 * n0 + n1) v = S[wf.l_Wu[0] + k - n0 - n1];
      else if (k < 2 * (n0 + n1)) v = S[wf.l_Wu[1] + k - 2 * n0 - n1];
      else v = S[wf.l_sc + SC_S];
      rec[wf.r_RW + k] = v;
    }
  }
  if (live && q == 0) {
    n_acc[w] = na0 + na;
    e_sum[w] = es;
    e2_sum[w] = e2s;
    e_last[w] = elast;
  }
}

template <int PT, int PE, int NE>
static hipError_t launch_vmc_rows_t(const DevWF& wf, const DevWF* dwf, double* state, int64_t W, int nsteps,
                                    uint64_t seed, uint64_t step0, double step_size, double* es, double* e2s,
                                    double* na, double* el, double* sij, hipStream_t s) {
  const size_t lds = (size_t)wf.lds_rows_doubles * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_vmc_rows<PT, PE, NE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       163840);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const unsigned blocks = (unsigned)((W + kRowWalkers - 1) / kRowWalkers);
  hipLaunchKernelGGL((k_vmc_rows<PT, PE, NE>), dim3(blocks), dim3(64), lds, s, dwf, state, W, nsteps, seed, step0,
                     step_size, es, e2s, na, el, sij);
  return hipGetLastError();
}

// single-electron VMC steps with the row kernel (one launch for all steps);
// NE: register columns per lane, 10 when no spin has more than 10 electrons
template <int NE>
static hipError_t launch_vmc_rows_n(const DevWF& wf, const DevWF* dwf, double* state, int64_t W, int nsteps,
                                    uint64_t seed, uint64_t step0, double step_size, double* es, double* e2s,
                                    double* na, double* el, double* sij, hipStream_t s) {
  if (wf.trial_prec != wf.precision)  // the mixed form
    return launch_vmc_rows_t<1, 0, NE>(wf, dwf, state, W, nsteps, seed, step0, step_size, es, e2s, na, el, sij, s);
  switch (wf.precision) {
    case 0: return launch_vmc_rows_t<0, 0, NE>(wf, dwf, state, W, nsteps, seed, step0, step_size, es, e2s, na, el, sij, s);
    case 1: return launch_vmc_rows_t<1, 1, NE>(wf, dwf, state, W, nsteps, seed, step0, step_size, es, e2s, na, el, sij, s);
    default: return launch_vmc_rows_t<2, 2, NE>(wf, dwf, state, W, nsteps, seed, step0, step_size, es, e2s, na, el, sij, s);
  }
}

hipError_t launch_vmc_rows(const DevWF& wf, const DevWF* dwf, double* state, int64_t W, int nsteps, uint64_t seed,
                           uint64_t step0, double step_size, double* es, double* e2s, double* na, double* el,
                           double* sij, hipStream_t s) {
  if (wf.nup <= 10 && wf.ndn <= 10)
    return launch_vmc_rows_n<10>(wf, dwf, state, W, nsteps, seed, step0, step_size, es, e2s, na, el, sij, s);
  return launch_vmc_rows_n<16>(wf, dwf, state, W, nsteps, seed, step0, step_size, es, e2s, na, el, sij, s);
}

}  // namespace vbqmc
