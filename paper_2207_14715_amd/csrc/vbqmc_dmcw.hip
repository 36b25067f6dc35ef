// gfx950 fixed-node DMC step with the walkers resident in a workgroup.
//
// A DMC step (Sec. 2.3.2) moves every electron of a walker once with a
// drift-diffusion proposal, then weighs the walker for birth/death.  Here a
// workgroup of four wavefronts owns four walkers for the whole step, one
// walker per wavefront:
//   * lane k keeps column k of [B | T] of the spin being moved in registers
//     (B the reference inverse, T the replaced-column table), and lanes
//     u, u + 64 keep the minor T[J_u, Q_u], R_u and W_u of distinct spin
//     determinant u, so that a move's determinant ratio, its drift at the
//     proposal and an accepted Sherman-Morrison update touch no memory but
//     a few broadcast rows in LDS;
//   * the four walkers move the same electron together: the value and
//     gradient orbital rows at their four proposals are one 16-row MFMA tile
//     (row = walker x channel), contracted with lambda^T on FP64 MFMA;
//   * the value and gradient rows of an accepted proposal are the rows of
//     the electron's new position: they are kept in the walker's record
//     (compact, reference slots then table orbitals), so the drift of the
//     next step reads them instead of re-evaluating the orbitals, the
//     inverse refresh after refresh_every updates needs no orbital
//     evaluation, and the local energy evaluates only the Laplacian rows
//     (16-row MFMA tiles of four walkers x four electrons).
// A walker's record then crosses HBM a few times per step instead of once
// per electron.  The branching weight closes the step; the population
// control, scan and compaction are the shared kernels of the other DMC paths.
//
// Limits (checked by the host): FP64, Gaussian shells, at most 32 electrons,
// 64 reference slots plus table orbitals and 128 distinct determinants per
// spin, at most 64 (padded) orbitals.

#include "vbqmc_group.h"

namespace vbqmc {

constexpr int kDwW = 4;            // walkers (wavefronts) of a workgroup
constexpr int kDwNT = 64 * kDwW;   // threads of a workgroup

// one lane's value of a double from lane src (src the same in every lane)
__device__ __forceinline__ double dw_readlane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, the same bits in every lane: DPP sums within each
// 16-lane row (gsum), then the four row sums read from lanes 0, 16, 32 and
// 48 and added in that order.
template <int K>
__device__ __forceinline__ void dw_wsum(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = gsum<16>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k)
    v[k] = ((dw_readlane(v[k], 0) + dw_readlane(v[k], 16)) + dw_readlane(v[k], 32)) + dw_readlane(v[k], 48);
}

// Distinct determinants u = lane + 64 h (h = 0, 1) of the spin being moved:
// replaced slots J, table indices Q, the minor T[J, Q] (XE x XE, XE the
// largest number of columns a determinant replaces), R_u and W_u.  Lanes
// past the spin's determinants hold e = 0 and W = 0 (they add nothing).
template <int XE>
struct DwDets {
  int e[2], J[2][XE], Q[2][XE];
  double m[2][XE * XE];
  double R[2], W[2];
};

// determinant of the leading e x e block of an XE x XE matrix (e <= XE)
template <int XE>
__device__ __forceinline__ double dw_det(int e, const double* m) {
  if constexpr (XE == 2) {
    return e == 0 ? 1.0 : (e == 1 ? m[0] : m[0] * m[3] - m[1] * m[2]);
  } else {
    return det_e(e, m);
  }
}

// y^T adj(m) b for the leading e x e block
template <int XE>
__device__ __forceinline__ double dw_adj(int e, const double* m, const double* y, const double* b) {
  if constexpr (XE == 2) {
    if (e == 0) return 0.0;
    if (e == 1) return y[0] * b[0];
    return y[0] * (m[3] * b[0] - m[1] * b[1]) + y[1] * (-m[2] * b[0] + m[0] * b[1]);
  } else {
    return adj_e(e, m, y, b);
  }
}

// from the table T (row-major n x nP, any memory) and R_u, W_u
template <int XE>
__device__ __forceinline__ void dw_load_dets(const SpinTab& sp, const double* T, const double* Ru, const double* Wu,
                                             int lane, DwDets<XE>& d) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int u = lane + 64 * h;
    const bool ok = u < sp.nU;
    const int* ui = sp.uinfo + 8 * (ok ? u : 0);
    d.e[h] = ok ? ui[0] : 0;
#pragma unroll
    for (int r = 0; r < XE; ++r) {
      d.J[h][r] = ok ? ui[1 + r] : 0;
      d.Q[h][r] = ok ? ui[4 + r] : 0;
    }
#pragma unroll
    for (int r = 0; r < XE; ++r)
#pragma unroll
      for (int c = 0; c < XE; ++c) {
        const double v = T[d.J[h][r] * sp.nP + d.Q[h][c]];
        d.m[h][r * XE + c] = (r < d.e[h] && c < d.e[h]) ? v : 0.0;
      }
    d.R[h] = ok ? Ru[u] : 0.0;
    d.W[h] = ok ? Wu[u] : 0.0;
  }
}

// y (indexed by table orbital) and b (indexed by slot) of determinant h,
// zero past its e replaced columns
template <int XE>
__device__ __forceinline__ void dw_gather(const DwDets<XE>& d, int h, const double* y, const double* b,
                                          double (&yy)[XE], double (&bb)[XE]) {
  // (the loads are unconditional: J and Q are valid indices in every lane)
#pragma unroll
  for (int r = 0; r < XE; ++r) {
    const bool in = r < d.e[h];
    const double yv = y[d.Q[h][r]], bv = b[d.J[h][r]];
    yy[r] = in ? yv : 0.0;
    bb[r] = in ? bv : 0.0;
  }
}

// sum over this lane's determinants of (rp R_u + y_Q^T adj(T_JQ) b_J) W_u:
// the numerator of O_i D / D for a row operator O whose row-operator products
// with the reference columns are rp (at slot il) and y (table residuals)
template <int XE>
__device__ __forceinline__ double dw_detsum(const DwDets<XE>& d, double rp, const double* y, const double* b) {
  double s = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double yy[XE], bb[XE];
    dw_gather<XE>(d, h, y, b, yy, bb);
    s += (rp * d.R[h] + dw_adj<XE>(d.e[h], d.m[h], yy, bb)) * d.W[h];
  }
  return s;
}

// t_k = sum_{j < n} row[j] C[j], summed over all NC entries: C[j] is zero
// for j >= n and every row entry is finite (the broadcast rows are cleared
// when the kernel starts and after each refresh), so the entries past n add
// exact zeros
// The scheduling barrier after each half keeps the compiler from loading the
// rows of several dot products ahead at once (that would hold 2 NC registers
// per row beside the columns).
template <int NC>
__device__ __forceinline__ double dw_dot(const double* row, const double (&C)[NC]) {
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int j = 0; j < NC / 2; j += 2) {
    a0 += row[j] * C[j];
    a1 += row[j + 1] * C[j + 1];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = NC / 2; j < NC; j += 2) {
    a0 += row[j] * C[j];
    a1 += row[j + 1] * C[j + 1];
  }
  __builtin_amdgcn_sched_barrier(0);
  return a0 + a1;
}

// The same sum with the row held across the lanes (lane j holds row[j]):
// each entry reaches every lane through readlane, so the dot product needs
// no LDS round trip.  Same summation order as dw_dot.
template <int NC>
__device__ __forceinline__ double dw_dotl(double r, const double (&C)[NC]) {
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int j = 0; j < NC; j += 2) {
    a0 += dw_readlane(r, j) * C[j];
    a1 += dw_readlane(r, j + 1) * C[j + 1];
  }
  return a0 + a1;
}

// column lane of [B | T] from the record: lane k < n takes column k of B,
// lane n + q column q of T; other lanes and rows past n hold zero.  Every
// load is in the record (row index clamped), the mask zeroes what is unused.
template <int NC>
__device__ __forceinline__ void dw_load_columns(const double* Bg, const double* Tg, int n, int nP, int lane,
                                                double (&C)[NC]) {
  const bool bl = lane < n, tl = lane >= n && lane < n + nP;
  const double* src = tl ? Tg + (lane - n) : Bg + (bl ? lane : 0);
  const int str = tl ? nP : n;
  const double own = (bl || tl) ? 1.0 : 0.0;
#pragma unroll
  for (int j = 0; j < NC; ++j) C[j] = src[min(j, n - 1) * str] * (j < n ? own : 0.0);
}

// ---------------------------------------------------------------------------
// row tiles
// ---------------------------------------------------------------------------
// Radial sums of NPT points for every shell, from the displacement table:
// MODE 0 stores g = sum c e^{-a r^2} and g1 = dg/d(r^2) per shell (stride
// 2 nshell + 1 per point), MODE 1 the Laplacian factor
// sum c e^{-a r^2} a (4 a r^2 - 2 (2l + 3)), so that the Laplacian of a basis
// function is its angular polynomial times that factor (stride nshell | 1).
// A Slater shell (sum c e^{-a r}) stores g1 = sum -a c e^{-a r} / (2r) and the
// factor sum c e^{-a r} a (a - 2 (l + 1) / r) (the harmonic polynomial P of
// degree l has lap(P g) = P (g'' + 2 (l + 1) g' / r)).  Each shell's terms
// are added in the order of its primitives.
template <int NPT, int MODE>
__device__ __forceinline__ void dw_radial_plain(const DevWF& wf, const Ld& l) {
#pragma clang fp contract(off)
  const double* disp = l.L + wf.dw_disp;
  double* gt = l.L + wf.dw_gtab;
  const int ds = 4 * wf.nnuc + 1;
  const int gs = MODE == 0 ? 2 * wf.nshell + 1 : (wf.nshell | 1);
  const double* etab = l.L + wf.l_etab;
  const float rn = 1.0f / (float)wf.nshell;
  for (int idx = threadIdx.x; idx < NPT * wf.nshell; idx += kDwNT) {
    const int p = div_small(idx, rn), sh = idx - p * wf.nshell;
    const int* si = l.sh() + 8 * sh;
    const double r2 = disp[p * ds + 4 * si[0] + 3];
    const int k0 = si[4], nk = si[5];
    const bool sto = si[1] == 1;
    const double r = sto ? sqrt(r2) : 0.0, ir = sto ? 1.0 / r : 0.0;
    const double c2l = (double)(2 * (2 * si[2] + 3));
    double g = 0.0, g1 = 0.0;
    for (int k = 0; k < nk; ++k) {
      const double a = l.pe()[k0 + k];
      const double t = sto ? a * r : a * r2;
      if (t < 50.0) {
        const double ex = l.pc()[k0 + k] * exp_neg<double>(t, etab);
        if constexpr (MODE == 0) {
          g += ex;
          if (sto) g1 -= a * ex * (0.5 * ir);
          else g1 -= a * ex;
        } else {
          if (sto) g += ex * a * (a - (double)(2 * (si[2] + 1)) * ir);
          else g += ex * a * (4.0 * t - c2l);
        }
      }
    }
    if constexpr (MODE == 0) {
      gt[p * gs + 2 * sh] = g;
      gt[p * gs + 2 * sh + 1] = g1;
    } else {
      gt[p * gs + sh] = g;
    }
  }
}

// The same sums from a radial schedule of kDwNT / NPT bins (the shells dealt
// to bins by the host, longest first, each to the bin with the fewest
// primitives): thread t takes point t % NPT and bin t / NPT and walks the
// bin's primitives two at a time in a loop of fixed length, the schedule
// entries and operands of the next step already loaded.  A shell's running
// sum restarts at its first primitive and is stored at every entry, so the
// last store holds the whole sum (padding entries repeat the bin's last shell
// and add nothing); each shell is still summed in one thread in the order of
// its primitives, so the sums equal those of dw_radial_plain bit for bit.
template <int NPT, int MODE, bool STO>
__device__ __forceinline__ void dw_radial_bins(const DevWF& wf, const Ld& l) {
#pragma clang fp contract(off)
  constexpr int NB = kDwNT / NPT;
  const int e = threadIdx.x & (NPT - 1);
  const double* de = l.L + wf.dw_disp + e * (4 * wf.nnuc + 1);
  double* o = l.L + wf.dw_gtab + e * (MODE == 0 ? 2 * wf.nshell + 1 : (wf.nshell | 1));
  const unsigned* sc = (const unsigned*)(l.L + wf.dw_rs) + (NPT == 4 ? wf.dw_rs4_off : wf.dw_rs16_off) +
                       threadIdx.x / NPT;
  const int len = NPT == 4 ? wf.dw_rs4_len : wf.dw_rs16_len;
  const double* pe = l.pe();
  const double* pc = l.pc();
  const double* etab = l.L + wf.l_etab;
  const int* sht = l.sh();
  auto nuc = [](unsigned f) { return (int)((f >> kRsNucShift) & kRsNucMask); };
  auto shl = [](unsigned f) { return (int)((f >> kRsShift) & kRsShMask); };
  unsigned n0 = sc[0], n1 = sc[NB], m0 = sc[2 * NB], m1 = sc[3 * NB];
  double a0 = pe[n0 & kRsPrim], c0 = pc[n0 & kRsPrim], a1 = pe[n1 & kRsPrim], c1 = pc[n1 & kRsPrim];
  double d0 = de[4 * nuc(n0) + 3], d1 = de[4 * nuc(n1) + 3];
  int l0 = MODE == 1 ? sht[8 * shl(n0) + 2] : 0, l1 = MODE == 1 ? sht[8 * shl(n1) + 2] : 0;
  double g = 0.0, g1 = 0.0;
  // ir: 1/r of a Slater entry (STO only)
  auto add = [&](double ex, double a, double r2, double ir, int lq, unsigned f) {
    const bool first = f & kRsFirst;
    if constexpr (MODE == 0) {
      g = (first ? 0.0 : g) + ex;
      if (STO && (f & kRsSto)) g1 = (first ? 0.0 : g1) - a * ex * (0.5 * ir);
      else g1 = (first ? 0.0 : g1) - a * ex;
      double* q = o + 2 * shl(f);
      q[0] = g;
      q[1] = g1;
    } else {
      if (STO && (f & kRsSto)) g = (first ? 0.0 : g) + ex * a * (a - (double)(2 * (lq + 1)) * ir);
      else g = (first ? 0.0 : g) + ex * a * (4.0 * (a * r2) - (double)(2 * (2 * lq + 3)));
      o[shl(f)] = g;
    }
  };
  for (int j = 0; j < len; j += 2) {
    const unsigned f0 = n0, f1 = n1;
    const double A0 = a0, C0 = c0, R0 = d0, A1 = a1, C1 = c1, R1 = d1;
    const int L0 = l0, L1 = l1;
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
    if constexpr (MODE == 1) {
      l0 = sht[8 * shl(n0) + 2];
      l1 = sht[8 * shl(n1) + 2];
    }
    double t0 = A0 * R0, t1 = A1 * R1, ir0 = 0.0, ir1 = 0.0;
    if constexpr (STO) {
      if (f0 & kRsSto) {
        const double r = sqrt(R0);
        t0 = A0 * r;
        ir0 = 1.0 / r;
      }
      if (f1 & kRsSto) {
        const double r = sqrt(R1);
        t1 = A1 * r;
        ir1 = 1.0 / r;
      }
    }
    double ex0, ex1;
    exp_neg2<double>(fmin(t0, 64.0), fmin(t1, 64.0), etab, ex0, ex1);
    const double x0 = C0 * ex0, x1 = C1 * ex1;
    add(((f0 & kRsLive) && t0 < 50.0) ? x0 : 0.0, A0, R0, ir0, L0, f0);
    add(((f1 & kRsLive) && t1 < 50.0) ? x1 : 0.0, A1, R1, ir1, L1, f1);
  }
}

template <int NPT, int MODE>
__device__ __forceinline__ void dw_radial(const DevWF& wf, const Ld& l) {
  if ((NPT == 4 ? wf.dw_rs4_len : wf.dw_rs16_len) > 0) {
    if (wf.rsched_sto) dw_radial_bins<NPT, MODE, true>(wf, l);
    else dw_radial_bins<NPT, MODE, false>(wf, l);
  } else {
    dw_radial_plain<NPT, MODE>(wf, l);
  }
}

// The contraction with lambda^T is split over the basis functions: wavefront
// g takes k-steps g kper .. (g + 1) kper - 1 (kper = Mpad / 16; a k-step is
// four functions) for every 16-column tile.  Its slice of lambda^T in the
// MFMA B-operand layout is loaded into registers once per launch and serves
// every row tile of the step (lambda is constant).  LK (4, 8 or 16) is the
// smallest of those that holds kper: k-steps past kper carry zeros.
constexpr int kDwLK = 16;  // most k-steps per wavefront: Mpad <= 4 kDwW kDwLK = 256
constexpr int kDwLC = 3;   // column tiles: nop <= 48

template <int LK>
struct DwLam {
  double b[LK][kDwLC];
};

template <int LK>
__device__ __forceinline__ void dw_load_lam(const DevWF& wf, DwLam<LK>& L) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kper = wf.Mpad / (4 * kDwW), nct = wf.nop / 16;
#pragma unroll
  for (int t = 0; t < LK; ++t)
#pragma unroll
    for (int c = 0; c < kDwLC; ++c) {
      const bool in = t < kper && c < nct;
      const int k = in ? 4 * (wave * kper + t) + (lane >> 4) : 0;
      const int col = in ? 16 * c + (lane & 15) : 0;
      const double v = wf.lamT[(size_t)k * wf.nop + col];
      L.b[t][c] = in ? v : 0.0;
    }
}

// a choice between two values already formed, kept as a select (marked
// unpredictable so that the compiler does not turn it into a branch)
__device__ __forceinline__ double dw_sel(bool c, double a, double b) { return __builtin_unpredictable(c) ? a : b; }

// Tables of a row tile of NPT points (point p at pts + ps p): the
// displacement from each nucleus a with its square, and the harmonic table,
// for harmonic h = m + l^2 of the unnormalised set (1; x, y, z; xy, yz, zx,
// x^2 - y^2, 2z^2 - x^2 - y^2) the polynomial at the displacement and, for
// MODE 0, its x, y, z derivatives.  With the harmonic table an element of
// the contraction is a lookup, not a branch over harmonics.  MODE 0: wave
// ch forms channel ch (value, d/dx, d/dy, d/dz) of every (p, a), so that the
// channel's formulas are the same across the wave.
template <int NPT, int MODE>
__device__ __forceinline__ void dw_tile_tables(const DevWF& wf, const Ld& l, const double* pts, int ps) {
  const int nn = wf.nnuc;
  double* H = l.L + wf.dw_harm;
  const int ch = MODE == 0 ? (int)(threadIdx.x >> 6) : 0;
  const int first = MODE == 0 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  const int stride = MODE == 0 ? 64 : kDwNT;
  for (int pa = first; pa < NPT * nn; pa += stride) {
    const int p = pa / nn, a = pa - p * nn;
    const double* nu = l.nuc() + 4 * a;
    const double x = pts[ps * p] - nu[0], y = pts[ps * p + 1] - nu[1], z = pts[ps * p + 2] - nu[2];
    if (ch == 0) {
      double* d = l.L + wf.dw_disp + p * (4 * nn + 1) + 4 * a;
      d[0] = x; d[1] = y; d[2] = z; d[3] = x * x + y * y + z * z;
    }
    double v[9];
    if (ch == 0) {
      v[0] = 1.0; v[1] = x; v[2] = y; v[3] = z;
      v[4] = x * y; v[5] = y * z; v[6] = z * x; v[7] = x * x - y * y; v[8] = 2.0 * z * z - x * x - y * y;
    } else if (ch == 1) {
      v[0] = 0.0; v[1] = 1.0; v[2] = 0.0; v[3] = 0.0;
      v[4] = y; v[5] = 0.0; v[6] = z; v[7] = 2.0 * x; v[8] = -2.0 * x;
    } else if (ch == 2) {
      v[0] = 0.0; v[1] = 0.0; v[2] = 1.0; v[3] = 0.0;
      v[4] = x; v[5] = z; v[6] = 0.0; v[7] = -2.0 * y; v[8] = -2.0 * y;
    } else {
      v[0] = 0.0; v[1] = 0.0; v[2] = 0.0; v[3] = 1.0;
      v[4] = 0.0; v[5] = y; v[6] = x; v[7] = 0.0; v[8] = 4.0 * z;
    }
#pragma unroll
    for (int h = 0; h < 9; ++h) {
      if constexpr (MODE == 0) H[(pa * 9 + h) * 4 + ch] = v[h];
      else H[pa * 9 + h] = v[h];
    }
  }
}

// One 16-row tile on MFMA: rows r = 4 p + c of the A operand are built on
// the fly from the radial and harmonic tables (MODE 0: channel c = value,
// d/dx, d/dy, d/dz of point p; MODE 1: the Laplacian of point r), contracted
// with lambda^T from registers.  The element of k-step t + 1 is formed while the products of
// k-step t run; the LK steps carry no branch (steps past kper add zeros).  The four wavefronts' partial sums meet in part ([4][kDwLC][4]
// [64] doubles) and are added in a fixed order; output row 4 q + lane / 16 of
// register q at orbital column p goes to out[row][slot], slot = cmap[p]
// (orbitals a spin does not use are dropped).  Ends with a barrier.
template <int MODE, int LK>
__device__ __forceinline__ void dw_mfma(const DevWF& wf, const Ld& l, const int* cmap, double* out, double* part,
                                       const DwLam<LK>& L) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int p = MODE == 0 ? row >> 2 : row, c = row & 3;
  const int ax = c == 0 ? 0 : c - 1;
  const double* disp = l.L + wf.dw_disp + p * (4 * wf.nnuc + 1);
  const double* gt = l.L + wf.dw_gtab + p * (MODE == 0 ? 2 * wf.nshell + 1 : (wf.nshell | 1));
  const int nct = wf.nop / 16, kper = wf.Mpad / (4 * kDwW), kb = wave * kper;
  // A element of k-step t (function 4 (kb + t) + kq; padding functions and
  // steps past kper read function 0 and give 0), in three stages so that
  // loads can be issued ahead of their use: the function word, the table
  // entries (harmonic, its derivative along this lane's axis, the
  // displacement along it, the radial entries), then the element
  struct Src {
    double P, D, dc, g0, g1;
    bool fn;
  };
  const double* harm = l.L + wf.dw_harm;
  const int nn = wf.nnuc;
  auto word = [&](int t) -> int2 {
    // (one 8-byte load, so that the second word is not loaded under a branch)
    const long long v = ((const long long*)l.fn())[t < kper ? 4 * (kb + t) + kq : 0];
    return make_int2((int)v, (int)(v >> 32));
  };
  auto fetch = [&](int t, int2 w) -> Src {
    Src q;
    q.fn = t < kper && w.x >= 0;
    const int sh = q.fn ? w.x : 0, nuc = q.fn ? (w.y >> 8) : 0;
    const int lq = (w.y >> 4) & 3, h = q.fn ? (w.y & 15) + lq * lq : 0;
    if constexpr (MODE == 0) {
      const double* hp = harm + ((p * nn + nuc) * 9 + h) * 4;
      q.P = hp[0];
      q.D = hp[c];
      q.dc = disp[4 * nuc + ax];
      q.g0 = gt[2 * sh];
      q.g1 = gt[2 * sh + 1];
    } else {
      q.P = harm[(p * nn + nuc) * 9 + h];
      q.D = q.dc = q.g1 = 0.0;
      q.g0 = gt[sh];
    }
    return q;
  };
  auto elem = [&](const Src& q) -> double {
    double v;
    if constexpr (MODE == 0) {
      const double v0 = q.P * q.g0, vd = q.D * q.g0 + 2.0 * q.g1 * q.P * q.dc;
      v = dw_sel(c == 0, v0, vd);
    } else {
      v = q.P * q.g0;
    }
    return dw_sel(q.fn, v, 0.0);
  };
  v4d acc[kDwLC];
#pragma unroll
  for (int ct = 0; ct < kDwLC; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[ct][r] = 0.0;
  // software pipeline: at step t the table entries of step t + 2 are
  // requested, the products of step t issued and the element of step t + 1
  // formed; the scheduling barriers keep the compiler from moving the loads
  // back next to their use
  int2 wn = word(0);
  Src q1 = fetch(0, wn);
  double a = elem(q1);
  if (LK > 1) q1 = fetch(1, word(1));
  if (LK > 2) wn = word(2);
#pragma unroll
  for (int t = 0; t < LK; ++t) {
    // (the word load first: the next step waits for it without waiting for
    // the table loads behind it, the LDS counter being in order)
    int2 w3 = wn;
    if (t + 3 < LK) w3 = word(t + 3);
    __builtin_amdgcn_sched_barrier(0);
    Src q2 = q1;
    if (t + 2 < LK) q2 = fetch(t + 2, wn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ct = 0; ct < kDwLC; ++ct) acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, L.b[t][ct], acc[ct], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < LK) a = elem(q1);
    __builtin_amdgcn_sched_barrier(0);
    q1 = q2;
    wn = w3;
  }
  double* pw = part + wave * (kDwLC * 4 * 64);
#pragma unroll
  for (int ct = 0; ct < kDwLC; ++ct)
#pragma unroll
    for (int q = 0; q < 4; ++q) pw[(ct * 4 + q) * 64 + lane] = acc[ct][q];
  __syncthreads();
  constexpr int PW = kDwLC * 4 * 64;
  for (int e = threadIdx.x; e < nct * 4 * 64; e += kDwNT) {
    const double v = ((part[e] + part[PW + e]) + part[2 * PW + e]) + part[3 * PW + e];
    const int ct = e >> 8, q = (e >> 6) & 3, ln = e & 63;
    const int slot = cmap[16 * ct + (ln & 15)];
    if (slot >= 0) out[(4 * q + (ln >> 4)) * 64 + slot] = v;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// inverse refresh on MFMA
// ---------------------------------------------------------------------------
// largest residual entry for which a refresh takes the Newton-Schulz step
// (the error after the step is of the order of its square plus rounding)
constexpr double kDwNsTol = 1e-8;

__device__ __forceinline__ double dw_wmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Refresh of a spin's reference inverse from the cached value rows: with A
// (electron x reference slot, rows at vrow with stride WD, n <= 32) and the
// current inverse B (column k in register array C of lane k < n),
// R = I - A B and B' = B + B R (one Newton-Schulz step, which squares the
// error of B); then T = B' PP with PP the table orbitals' cached values.  All
// three products are 32 x 32 (x nP) FP64 MFMA tiles.  The accumulator layout
// of the 16x16x4 FP64 MFMA (register r of lane l: row 4 r + l / 16, column
// l % 16) is the B-operand layout of k-step 4 mt + r (k = l / 16,
// n = l % 16), so R feeds the second product from registers.  B goes
// through the wavefront's LDS area Wm (n x n, then T as n x nP).  Returns
// false (and changes nothing but Wm) when max |R| > kDwNsTol, when it is not
// finite or when nP > 32: the caller then takes a Gauss-Jordan refresh.  On
// success lane k < n holds column k of B' in C, lane n + q column q of T,
// and Wm holds T row-major (stride nP).
template <int NC>
__device__ bool dw_refresh_ns(double* Wm, const double* vrow, int WD, int n, int nP, int lane, double (&C)[NC]) {
  if (nP > 32) return false;
  const int m = lane & 15, kq = lane >> 4;
  const bool bl = lane < n, tl = lane >= n && lane < n + nP;
  if (bl)
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < n) Wm[j * n + lane] = C[j];
  wave_sync();
  // operands with every index clamped into the matrices, zero outside
  auto aop = [&](int i, int k) -> double {
    const bool in = i < n && k < n;
    const double v = vrow[(size_t)(in ? i : 0) * WD + (in ? k : 0)];
    return in ? v : 0.0;
  };
  auto bop = [&](int j, int k) -> double {
    const bool in = j < n && k < n;
    const double v = Wm[(in ? j : 0) * n + (in ? k : 0)];
    return in ? v : 0.0;
  };
  auto pop = [&](int k, int q) -> double {
    const bool in = k < n && q < nP;
    const double v = vrow[(size_t)(in ? k : 0) * WD + (in ? n + q : 0)];
    return in ? v : 0.0;
  };
  v4d P[2][2], D[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[a][b][r] = D[a][b][r] = 0.0;
  // P = A B
#pragma unroll
  for (int kt = 0; kt < 8; ++kt) {
    const int k = 4 * kt + kq;
    const double a0 = aop(m, k), a1 = aop(16 + m, k), b0 = bop(k, m), b1 = bop(k, 16 + m);
    P[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, P[0][0], 0, 0, 0);
    P[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, P[0][1], 0, 0, 0);
    P[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, P[1][0], 0, 0, 0);
    P[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, P[1][1], 0, 0, 0);
  }
  // R = I - P (the padding block past n is the identity, which adds nothing below)
  double rmax = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * a + 4 * r + kq, col = 16 * b + m;
        P[a][b][r] = (row == col ? 1.0 : 0.0) - P[a][b][r];
        if (row < n && col < n) rmax = fmax(rmax, fabs(P[a][b][r]));
      }
  rmax = dw_wmax(rmax);
  if (!(rmax <= kDwNsTol)) return false;
  // D = B R, then B' = B + D in place
#pragma unroll
  for (int kt = 0; kt < 8; ++kt) {
    const int k = 4 * kt + kq;
    const double a0 = bop(m, k), a1 = bop(16 + m, k);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      D[0][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, P[kt >> 2][b][kt & 3], D[0][b], 0, 0, 0);
      D[1][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, P[kt >> 2][b][kt & 3], D[1][b], 0, 0, 0);
    }
  }
  wave_sync();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * a + 4 * r + kq, col = 16 * b + m;
        if (row < n && col < n) Wm[row * n + col] += D[a][b][r];
      }
  wave_sync();
  // T = B' PP (reuses D)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) D[a][b][r] = 0.0;
#pragma unroll
  for (int kt = 0; kt < 8; ++kt) {
    const int k = 4 * kt + kq;
    const double a0 = bop(m, k), a1 = bop(16 + m, k), p0 = pop(k, m), p1 = pop(k, 16 + m);
    D[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, p0, D[0][0], 0, 0, 0);
    D[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, p0, D[1][0], 0, 0, 0);
    D[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, p1, D[0][1], 0, 0, 0);
    D[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, p1, D[1][1], 0, 0, 0);
  }
  // columns of B' to the reference lanes, then T over Wm for the table lanes and the minors
  if (bl)
#pragma unroll
    for (int j = 0; j < NC; ++j) C[j] = j < n ? Wm[min(j, n - 1) * n + lane] : 0.0;
  wave_sync();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * a + 4 * r + kq, col = 16 * b + m;
        if (row < n && col < nP) Wm[row * nP + col] = D[a][b][r];
      }
  wave_sync();
  if (tl)
#pragma unroll
    for (int j = 0; j < NC; ++j) C[j] = j < n ? Wm[min(j, n - 1) * nP + (lane - n)] : 0.0;
  return true;
}

// ---------------------------------------------------------------------------
// the step kernel
// ---------------------------------------------------------------------------
// prep = 1: rebuild each record from its positions (orbital-row caches of
// every electron, fresh inverses, tables, ratios, E_L) with no move and no
// weight; prep = 0: one DMC step.
// VMC = true: one single-electron Metropolis step (Sec. 2.3.1) instead: a
// uniform-cube proposal r' = r + s (2u - 1) per component, accepted iff
// u' < |Psi'/Psi|^2 (no drift, no node rejection, no weight), E_L added to
// the walker's VMC accumulators (vm; ctrl, tau, br and nacc unused).
// EEN: the Jastrow factor has the three-body term f_een (its value, the
// gradient of the moving electron and, in E_L, every electron's gradient and
// Laplacian; coefficients read from global memory).
template <int NC, int XE, int LK, bool VMC, bool EEN>
__global__ __launch_bounds__(kDwNT) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_dmcw(const DevWF* __restrict__ pwf, double* state, const double* ctrl,
                                                uint64_t seed, uint32_t step, double tau, DmcBranch br, double* nacc,
                                                int prep, DwVmc vm) {
  const DevWF& wf = *pwf;
  const int64_t W = VMC ? vm.W : (int64_t)ctrl[DC_W];
  const int64_t wbase = (int64_t)blockIdx.x * kDwW;
  if ((!VMC && ctrl[DC_ERR] != 0.0) || wbase >= W) return;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t w = wbase + g;
  const bool live = w < W;
  const int N = wf.N, nn = wf.nnuc, WD = wf.dw_width;
  Ld l(lds_dyn, wf);
  stage_tables<kDwNT, 0>(wf, l);
  // column map of each spin: orbital -> slot (reference slot j, n + table
  // index q, or -1)
  int* cmap = (int*)(lds_dyn + wf.dw_cmap);
  for (int k = threadIdx.x; k < 2 * wf.nop; k += kDwNT) cmap[k] = -1;
  {
    unsigned* rs = (unsigned*)(lds_dyn + wf.dw_rs);
    for (int k = threadIdx.x; k < wf.dw_rs_words; k += kDwNT) rs[k] = wf.dw_rs_g[k];
  }
  __syncthreads();
  for (int s = 0; s < 2; ++s) {
    const SpinTab& sp = wf.sp[s];
    for (int j = threadIdx.x; j < sp.n + sp.nP; j += kDwNT)
      cmap[s * wf.nop + (j < sp.n ? sp.ref[j] : sp.porb[j - sp.n])] = j;
  }
  double* wa = lds_dyn + wf.dw_wave + g * wf.dw_wstride;  // this walker's area
  double* Rl = wa + wf.dwo_R;     // positions [N][3]
  double* bc = wa + wf.dwo_bc;    // column il of B (slot-indexed)
  double* xr = wa + wf.dwo_x;     // broadcast rows [4][64] (slot-indexed)
  double* yr = wa + wf.dwo_y;     // table residuals [4][64] (table-indexed)
  double* Pw = lds_dyn + wf.dw_P; // per walker: proposal x, y, z, drift x, y, z
  double* V4 = lds_dyn + wf.dw_V4;
  double* part = lds_dyn + wf.dw_part;  // partial sums of the row tiles
  DwLam<LK> lam;
  dw_load_lam<LK>(wf, lam);
  // records of dead wavefronts (past W) are never read or written
  double* rec = state + (live ? w : wbase) * wf.rec_len;
  for (int k = lane; k < 3 * N; k += 64) Rl[k] = rec[wf.r_R + k];
  // broadcast rows start finite (dw_dot reads all NC entries)
  for (int k = lane; k < 64; k += 64) bc[k] = 0.0;
  for (int k = lane; k < 4 * 64; k += 64) {
    xr[k] = 0.0;
    yr[k] = 0.0;
  }
  for (int k = threadIdx.x; k < 16 * 64; k += kDwNT) V4[k] = 0.0;
  const int n0 = wf.sp[0].nU, n1 = wf.sp[1].nU;
  double* RW = rec + wf.r_RW;
  double S = RW[2 * (n0 + n1)];
  const double E_old = rec[wf.r_sc + SC_ELOC];
  // (VMC keeps a walker flagged by an earlier call flagged through the rebuild)
  bool bad = !live || ((!prep || VMC) && rec[wf.r_sc + SC_FLAGS] != 0.0) || (!prep && !(S != 0.0));
  double na = 0.0;
  double d2p = 0.0, d2a = 0.0;  // squared displacements proposed / accepted (DMC)
  const double ET = VMC ? 0.0 : ctrl[DC_ET];
  const double sqt = VMC ? 0.0 : sqrt(tau);
  const PairCoef c_anti = ee_coef(wf, true), c_par = ee_coef(wf, false);
  const double kappa = wf.kappa;
  double* vc = rec + wf.r_vc;  // value rows [N][WD]
  double* gc = rec + wf.r_gc;  // gradient rows [N][3][WD]
  __syncthreads();

  // ---- prep: orbital-row caches at every electron's position ----
  if (prep) {
#pragma unroll 1
    for (int i = 0; i < N; ++i) {
      const int s = spin_of(wf, i);
      if (lane < 3) Pw[6 * g + lane] = live ? Rl[3 * i + lane] : 0.0;
      __syncthreads();
      dw_tile_tables<kDwW, 0>(wf, l, Pw, 6);
      __syncthreads();
      dw_radial<kDwW, 0>(wf, l);
      __syncthreads();
      dw_mfma<0>(wf, l, cmap + s * wf.nop, V4, part, lam);
      if (live)
        for (int k = lane; k < WD; k += 64) {
          vc[(size_t)i * WD + k] = V4[(4 * g) * 64 + k];
#pragma unroll
          for (int c = 0; c < 3; ++c) gc[((size_t)i * 3 + c) * WD + k] = V4[(4 * g + 1 + c) * 64 + k];
        }
      __syncthreads();
    }
  }

  // ---- moves, spin by spin ----
  double C[NC];
  DwDets<XE> d;
#pragma unroll 1
  for (int s = 0; s < 2; ++s) {
    const SpinTab& sp = wf.sp[s];
    const int n = sp.n, nP = sp.nP, e0 = sp.e0;
    if (n == 0) continue;
    const bool blane = lane < n, tlane = lane >= n && lane < n + nP;
    double* Bg = rec + wf.r_B[s];
    double* Tg = rec + wf.r_T[s];
    double* Ru = RW + (s ? n0 : 0);
    double* Wu = RW + n0 + n1 + (s ? n0 : 0);
    // this spin's log|reference determinant|, its sign and update count
    double ldS = rec[wf.r_sc + SC_LOGDET0 + s];
    double sgS = rec[wf.r_sc + SC_SGN0 + s];
    double nuS = prep ? (double)wf.refresh_every : rec[wf.r_sc + SC_NUPD0 + s];
    dw_load_columns<NC>(Bg, Tg, n, nP, lane, C);
    dw_load_dets(sp, Tg, Ru, Wu, lane, d);
    // the draws of this spin's moves, lane il for electron e0 + il: the
    // Box-Muller normals of the proposal and the acceptance uniform
    double* rnd = wa + wf.dw_rnd;
    if (!prep && lane < n) {
      const uint32_t ie = (uint32_t)(e0 + lane);
      double a0, a1, b0, b1, ua, dummy;
      philox_pair(seed, (uint32_t)w, step, 4u * ie, 0u, a0, a1);
      philox_pair(seed, (uint32_t)w, step, 4u * ie, 1u, b0, b1);
      philox_pair(seed, (uint32_t)w, step, 4u * ie + 1u, 0u, ua, dummy);
      if constexpr (VMC) {
        // (the displacement of the uniform cube)
        rnd[4 * lane] = vm.step * (2.0 * a0 - 1.0);
        rnd[4 * lane + 1] = vm.step * (2.0 * a1 - 1.0);
        rnd[4 * lane + 2] = vm.step * (2.0 * b0 - 1.0);
      } else {
        const double two_pi = 6.283185307179586476925286766559;
        const double r0 = sqrt(-2.0 * log(1.0 - a0)), r1 = sqrt(-2.0 * log(1.0 - b0));
        rnd[4 * lane] = r0 * cos(two_pi * a1);
        rnd[4 * lane + 1] = r0 * sin(two_pi * a1);
        rnd[4 * lane + 2] = r1 * cos(two_pi * b1);
      }
      rnd[4 * lane + 3] = ua;
    }
    // the cached gradient rows of the next electron to move, in flight
    // while the current move runs (electron e0 + il + 1 does not move in
    // move il, so its rows do not change)
    double gn[3] = {0.0, 0.0, 0.0};
    if (!VMC && !prep && lane < WD)
#pragma unroll
      for (int c = 0; c < 3; ++c) gn[c] = gc[((size_t)e0 * 3 + c) * WD + lane];
    wave_sync();
    for (int il = 0; il < n && !prep; ++il) {
      const int i = e0 + il;
      const bool act = !bad;
      double uo[2] = {0.0, 0.0};  // Jastrow pair values at the current point, per partner lane
      if constexpr (VMC) {
        // (A) the uniform-cube proposal and the Jastrow pair values at the
        // current point
        if (act) {
          if (lane == il)
#pragma unroll
            for (int j = 0; j < NC; ++j) bc[j] = C[j];
          const double xi = Rl[3 * i], yi = Rl[3 * i + 1], zi = Rl[3 * i + 2];
#pragma unroll
          for (int it = 0; it < 2; ++it) {
            const int j = lane + 64 * it;
            if (j >= N + nn || j == i) continue;
            double xj, yj, zj;
            PairCoef cf;
            if (j < N) {
              xj = Rl[3 * j]; yj = Rl[3 * j + 1]; zj = Rl[3 * j + 2];
              cf = s != spin_of(wf, j) ? c_anti : c_par;
            } else {
              const double* nu = l.nuc() + 4 * (j - N);
              xj = nu[0]; yj = nu[1]; zj = nu[2];
              cf = en_coef(l.en() + 6 * (j - N));
            }
            const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
            double u, u1, u2;
            pair_fn(sqrt(dx * dx + dy * dy + dz * dz), kappa, cf, u, u1, u2);
            if constexpr (EEN) {
              if (j < N) {
                double ge[3], le;
                een_partner<0>(wf, l.nuc(), xi, yi, zi, xj, yj, zj, u, ge, le);
              }
            }
            uo[it] = u;
          }
          if (lane < 3) Pw[6 * g + lane] = Rl[3 * i + lane] + rnd[4 * il + lane];
        } else if (lane < 3) {
          Pw[6 * g + lane] = 0.0;
        }
      } else {
      // (A) drift at the current point from the cached gradient rows
      if (act) {
        const double g3[3] = {gn[0], gn[1], gn[2]};
        if (il + 1 < n && lane < WD)
#pragma unroll
          for (int c = 0; c < 3; ++c) gn[c] = gc[((size_t)(i + 1) * 3 + c) * WD + lane];
        if (lane == il)
#pragma unroll
          for (int j = 0; j < NC; ++j) bc[j] = C[j];
        double t[3], rp[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          t[c] = dw_dotl<NC>(g3[c], C);
          rp[c] = dw_readlane(t[c], il);
          if (tlane) yr[c * 64 + (lane - n)] = g3[c] - t[c];
        }
        wave_sync();
        double part[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) part[c] = dw_detsum(d, rp[c], yr + c * 64, bc);
        part[3] = part[4] = part[5] = 0.0;
        const double xi = Rl[3 * i], yi = Rl[3 * i + 1], zi = Rl[3 * i + 2];
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          const int j = lane + 64 * it;
          if (j >= N + nn || j == i) continue;
          double xj, yj, zj;
          PairCoef cf;
          if (j < N) {
            xj = Rl[3 * j]; yj = Rl[3 * j + 1]; zj = Rl[3 * j + 2];
            cf = s != spin_of(wf, j) ? c_anti : c_par;
          } else {
            const double* nu = l.nuc() + 4 * (j - N);
            xj = nu[0]; yj = nu[1]; zj = nu[2];
            cf = en_coef(l.en() + 6 * (j - N));
          }
          const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          double u, u1, u2;
          pair_fn(r, kappa, cf, u, u1, u2);
          const double f = u1 / r;
          part[3] += f * dx;
          part[4] += f * dy;
          part[5] += f * dz;
          if constexpr (EEN) {
            if (j < N) {
              double le;
              een_partner<1>(wf, l.nuc(), xi, yi, zi, xj, yj, zj, u, part + 3, le);
            }
          }
          uo[it] = u;
        }
        dw_wsum<6>(part);
        if (lane == 0) {
          double v[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) v[c] = part[3 + c] + part[c] / S;
          const double zx = rnd[4 * il], zy = rnd[4 * il + 1], zz = rnd[4 * il + 2];
          Pw[6 * g] = xi + tau * v[0] + sqt * zx;
          Pw[6 * g + 1] = yi + tau * v[1] + sqt * zy;
          Pw[6 * g + 2] = zi + tau * v[2] + sqt * zz;
          Pw[6 * g + 3] = v[0];
          Pw[6 * g + 4] = v[1];
          Pw[6 * g + 5] = v[2];
        }
      } else if (lane < 3) {
        Pw[6 * g + lane] = 0.0;
      }
      }
      __syncthreads();
      // (B) value and gradient rows at the four proposals
      dw_tile_tables<kDwW, 0>(wf, l, Pw, 6);
      __syncthreads();
      dw_radial<kDwW, 0>(wf, l);
      __syncthreads();
      dw_mfma<0>(wf, l, cmap + s * wf.nop, V4, part, lam);
      // (C) ratio, node check, drift at the proposal, Green's function,
      // Metropolis decision and the Sherman-Morrison update
      if (act) {
        const double* vr = V4 + (4 * g) * 64;  // rows value, x, y, z
        // value channel first; the gradient channels only once the ratio
        // passes the node check
        const double v0 = vr[lane];
        const double t0 = dw_dotl<NC>(v0, C);
        const double rho = dw_readlane(t0, il);
        const double yv = tlane ? v0 - t0 : 0.0;
        if (tlane) yr[lane - n] = yv;
        wave_sync();
        double qh[2], part[2] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double yy[XE], bb[XE];
          dw_gather<XE>(d, h, yr, bc, yy, bb);
          qh[h] = rho * d.R[h] + dw_adj<XE>(d.e[h], d.m[h], yy, bb);
          part[0] += qh[h] * d.W[h];
        }
        const double px = Pw[6 * g], py = Pw[6 * g + 1], pz = Pw[6 * g + 2];
        const double xi = Rl[3 * i], yi = Rl[3 * i + 1], zi = Rl[3 * i + 2];
        double jg[3] = {0.0, 0.0, 0.0};
        (void)xi; (void)yi; (void)zi;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          const int j = lane + 64 * it;
          if (j >= N + nn || j == i) continue;
          double xj, yj, zj;
          PairCoef cf;
          if (j < N) {
            xj = Rl[3 * j]; yj = Rl[3 * j + 1]; zj = Rl[3 * j + 2];
            cf = s != spin_of(wf, j) ? c_anti : c_par;
          } else {
            const double* nu = l.nuc() + 4 * (j - N);
            xj = nu[0]; yj = nu[1]; zj = nu[2];
            cf = en_coef(l.en() + 6 * (j - N));
          }
          const double dx = px - xj, dy = py - yj, dz = pz - zj;
          const double rn = sqrt(dx * dx + dy * dy + dz * dz);
          double u, u1, u2;
          pair_fn(rn, kappa, cf, u, u1, u2);
          const double f = u1 / rn;
          jg[0] += f * dx;
          jg[1] += f * dy;
          jg[2] += f * dz;
          if constexpr (EEN) {
            if (j < N) {
              double le;
              een_partner<VMC ? 0 : 1>(wf, l.nuc(), px, py, pz, xj, yj, zj, u, jg, le);
            }
          }
          part[1] += u - uo[it];
        }
        dw_wsum<2>(part);
        const double rdet = part[0] / S, dU = part[1];
        bool accept = false;
        const double ir = 1.0 / rho;
        const double d2 = (px - xi) * (px - xi) + (py - yi) * (py - yi) + (pz - zi) * (pz - zi);
        if constexpr (VMC) {
          // |Psi'/Psi|^2 (either sign; a move that makes the reference
          // determinant exactly singular, a set of measure zero, is refused)
          accept = rho != 0.0 && rnd[4 * il + 3] < rdet * rdet * exp(2.0 * dU);
        } else if (rdet > 0.0 && rho != 0.0) {
          // drift at r' with the state after the move: B'[:, il] = bc / rho,
          // T' = T + bc y^T / rho, R'_u = Q_u / rho, S' = S rdet / rho
          const double Snew = S * rdet / rho;
          double a[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double vg = vr[(1 + c) * 64 + lane];
            const double tc = dw_dotl<NC>(vg, C);
            a[c] = dw_readlane(tc, il);
            if (tlane) yr[(1 + c) * 64 + (lane - n)] = vg - tc - a[c] * yv * ir;
          }
          wave_sync();
          double dp[6] = {0.0, 0.0, 0.0, jg[0], jg[1], jg[2]};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            double yy0[XE], bb[XE], mm[XE * XE];
            dw_gather<XE>(d, h, yr, bc, yy0, bb);
#pragma unroll
            for (int r = 0; r < XE; ++r) {
#pragma unroll
              for (int c2 = 0; c2 < XE; ++c2) mm[r * XE + c2] = d.m[h][r * XE + c2] + bb[r] * yy0[c2] * ir;
              bb[r] *= ir;
            }
            const double Rnew = qh[h] * ir;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              double yy[XE], bz[XE];
              dw_gather<XE>(d, h, yr + (1 + c) * 64, bc, yy, bz);
              dp[c] += (a[c] * ir * Rnew + dw_adj<XE>(d.e[h], mm, yy, bb)) * d.W[h];
            }
          }
          dw_wsum<6>(dp);
          double fwd = 0.0, bwd = 0.0;
          const double dd3[3] = {px - xi, py - yi, pz - zi};
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double vn = dp[3 + c] + dp[c] / Snew;
            const double fa = dd3[c] - tau * Pw[6 * g + 3 + c];
            const double ba = -dd3[c] - tau * vn;
            fwd += fa * fa;
            bwd += ba * ba;
          }
          const double prob = rdet * rdet * exp(2.0 * dU + (fwd - bwd) / (2.0 * tau));
          accept = rnd[4 * il + 3] < prob;
        }
        d2p += d2;
        if (accept) {
          d2a += d2;
          double f = 0.0;
          if (blane) f = -(t0 - (lane == il ? 1.0 : 0.0)) * ir;
          else if (tlane) f = yv * ir;
#pragma unroll
          for (int j = 0; j < NC; ++j) C[j] += bc[j] * f;
          double vs[1] = {0.0};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            double yy0[XE], bb[XE];
            dw_gather<XE>(d, h, yr, bc, yy0, bb);
            // (bb and yy0 are zero past e: the unused entries stay zero)
#pragma unroll
            for (int r = 0; r < XE; ++r)
#pragma unroll
              for (int c2 = 0; c2 < XE; ++c2) d.m[h][r * XE + c2] += bb[r] * (yy0[c2] * ir);
            d.R[h] = dw_det<XE>(d.e[h], d.m[h]);
            vs[0] += d.R[h] * d.W[h];
          }
          dw_wsum<1>(vs);
          S = vs[0];
          ldS += log(fabs(rho));
          if (rho < 0) sgS = -sgS;
          nuS += 1.0;
          na += 1.0;
          if (!(S != 0.0)) bad = true;
          for (int k = lane; k < WD; k += 64) {
            vc[(size_t)i * WD + k] = vr[k];
#pragma unroll
            for (int c = 0; c < 3; ++c) gc[((size_t)i * 3 + c) * WD + k] = vr[(1 + c) * 64 + k];
          }
          wave_sync();
          if (lane == 0) {
            Rl[3 * i] = px;
            Rl[3 * i + 1] = py;
            Rl[3 * i + 2] = pz;
          }
        }
        wave_sync();
      }
    }
    // ---- inverse refresh of this spin from the cached value rows ----
    __syncthreads();  // the refresh matrices overlay the row-tile tables
    const bool due = !bad && nuS >= (double)wf.refresh_every;
    if (due) {
      double* A = lds_dyn + wf.dw_A + g * wf.dw_Astride;
      // a Newton-Schulz step from the current inverse when it is close
      // (not when the records are being rebuilt); else Gauss-Jordan
      const bool ns = !prep && dw_refresh_ns<NC>(A, vc + (size_t)e0 * WD, WD, n, nP, lane, C);
      bool ok = true;
      double ld = ldS, sg = sgS;
      if (!ns) {
        int* piv = (int*)(wa + wf.dwo_piv);
        double* fz = wa + wf.dwo_f;
        for (int k = lane; k < n * n; k += 64) {
          const int ii = k / n, j = k - ii * n;
          A[k] = vc[(size_t)(e0 + ii) * WD + j];
        }
        // the row dot products below read up to NC entries from the last row
        // start: the 64 doubles past the matrix are part of this area, zeroed
        A[n * n + lane] = 0.0;
        wave_sync();
        ok = gj_invert_h<64>(A, n, lane, piv, fz, ld, sg);
        if (ok) {
          // B to the reference lanes; T = B PP on the table lanes (lane n + q
          // takes column q of PP from its cached values, one row at a time);
          // row indices clamped into the matrix, rows past n masked to zero
          const double bm = blane ? 1.0 : 0.0, tm = tlane ? 1.0 : 0.0;
          const int kl = blane ? lane : 0;
          double pp[NC];  // column q of PP on table lane n + q (zero elsewhere)
#pragma unroll
          for (int ii = 0; ii < NC; ++ii)
            pp[ii] = vc[(size_t)(e0 + min(ii, n - 1)) * WD + (tlane ? lane : 0)] * (ii < n ? tm : 0.0);
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            const double* Aj = A + min(j, n - 1) * n;
            double v = Aj[kl] * bm;
            if (tlane) v = dw_dot<NC>(Aj, pp);
            C[j] = j < n ? v : 0.0;
          }
          wave_sync();
          // the new table, for the minors (rows past n are not written)
          if (tlane)
#pragma unroll
            for (int j = 0; j < NC; ++j)
              if (j < n) A[j * nP + (lane - n)] = C[j];
          wave_sync();
        }
      }
      if (!ok) {
        bad = true;
      } else {
        // minors of the new table (row-major in A), R_u and S
        double vs[1] = {0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int u = lane + 64 * h;
#pragma unroll
          for (int r = 0; r < XE; ++r)
#pragma unroll
            for (int c2 = 0; c2 < XE; ++c2) {
              const double v = A[d.J[h][r] * nP + d.Q[h][c2]];
              d.m[h][r * XE + c2] = (r < d.e[h] && c2 < d.e[h]) ? v : 0.0;
            }
          d.R[h] = u < sp.nU ? dw_det<XE>(d.e[h], d.m[h]) : 0.0;
          vs[0] += d.R[h] * d.W[h];
        }
        dw_wsum<1>(vs);
        S = vs[0];
        // (a Newton-Schulz step keeps the running ln|det| and sign of the moves)
        ldS = ld;
        sgS = sg;
        nuS = 0.0;
      }
    }
    __syncthreads();
    // the refresh matrices overwrote the row tiles: clear the rows again
    if (__syncthreads_or(due))
      for (int k = threadIdx.x; k < 16 * 64; k += kDwNT) V4[k] = 0.0;
    // ---- this spin's state back to the record; the other spin's W ----
    if (live) {
      if (lane == 0) {
        rec[wf.r_sc + SC_LOGDET0 + s] = ldS;
        rec[wf.r_sc + SC_SGN0 + s] = sgS;
        rec[wf.r_sc + SC_NUPD0 + s] = nuS;
      }
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (j < n) {
          if (blane) Bg[j * n + lane] = C[j];
          else if (tlane) Tg[j * nP + (lane - n)] = C[j];
        }
      double* Rs = xr;  // R_u of this spin, for the partner sums
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int u = lane + 64 * h;
        if (u < sp.nU) {
          Ru[u] = d.R[h];
          Rs[u] = d.R[h];
        }
      }
      wave_sync();
      const int o = 1 - s;
      const SpinTab& so = wf.sp[o];
      double* Wo = RW + n0 + n1 + (o ? n0 : 0);
      for (int u = lane; u < so.nU; u += 64) {
        double a = 0.0;
        for (int k = so.wrow[u]; k < so.wrow[u + 1]; ++k) a += so.wcoef[k] * Rs[so.wother[k]];
        Wo[u] = a;
      }
      wave_sync();
    }
  }
  if (!(S != 0.0)) bad = true;

  // ---- local energy (Eq. Elav with Psi = e^U D) ----
  // Jastrow gradient and Laplacian and the potential of electron i = lane
  // (i < N), each lane summing over all its partners (the same partner in
  // every lane at a time, so nothing is reduced across lanes here)
  double jg[3] = {0.0, 0.0, 0.0}, jl = 0.0, jv = 0.0;
  if (!bad) {
    const bool el = lane < N;
    const int si = spin_of(wf, el ? lane : 0);
    const double xi = Rl[3 * (el ? lane : 0)], yi = Rl[3 * (el ? lane : 0) + 1], zi = Rl[3 * (el ? lane : 0) + 2];
#pragma unroll 2
    for (int j = 0; j < N + nn; ++j) {
      double xj, yj, zj, wv;
      PairCoef cf;
      if (j < N) {
        xj = Rl[3 * j]; yj = Rl[3 * j + 1]; zj = Rl[3 * j + 2];
        cf = si != spin_of(wf, j) ? c_anti : c_par;
        wv = 0.5;
      } else {
        const double* nu = l.nuc() + 4 * (j - N);
        xj = nu[0]; yj = nu[1]; zj = nu[2];
        cf = en_coef(l.en() + 6 * (j - N));
        wv = -nu[3];
      }
      const bool on = el && j != lane;
      const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
      const double r = sqrt(on ? dx * dx + dy * dy + dz * dz : 1.0), irr = 1.0 / r;
      double u, u1, u2;
      pair_fn(r, kappa, cf, u, u1, u2);
      const double m = on ? 1.0 : 0.0;
      const double f = m * (u1 * irr);
      jg[0] += f * dx;
      jg[1] += f * dy;
      jg[2] += f * dz;
      jl += m * (u2 + 2.0 * (u1 * irr));
      jv += m * (wv * irr);
      if constexpr (EEN) {
        if (on && j < N) {
          double ue = 0.0;
          een_partner<2>(wf, l.nuc(), xi, yi, zi, xj, yj, zj, ue, jg, jl);
        }
      }
    }
  }
  // spin 1's columns are in registers after the moves: its electrons first
  double tsum = 0.0, vsum = 0.0;
#pragma unroll 1
  for (int s2 = 1; s2 >= 0; --s2) {
    const SpinTab& sp = wf.sp[s2];
    const int n = sp.n, nP = sp.nP, e0 = sp.e0;
    if (n == 0) continue;
    const bool tlane = lane >= n && lane < n + nP;
    if (s2 == 0) {
      // spin 0's columns and determinants as its moves left them (its W from
      // spin 1's final ratios)
      const double* Tg = rec + wf.r_T[0];
      dw_load_columns<NC>(rec + wf.r_B[0], Tg, n, nP, lane, C);
      dw_load_dets(sp, Tg, RW, RW + n0 + n1, lane, d);
    }
    double ge[3] = {0.0, 0.0, 0.0};  // cached gradient rows of the next electron, in flight
#pragma unroll 1
    for (int i0 = 0; i0 < n; i0 += 4) {
      if (!bad && lane < WD)
#pragma unroll
        for (int c = 0; c < 3; ++c) ge[c] = gc[((size_t)(e0 + i0) * 3 + c) * WD + lane];
      // Laplacian rows of electrons e0 + i0 .. + 3 of the four walkers
      if (threadIdx.x < 3 * 16) {
        const int p = threadIdx.x / 3, c = threadIdx.x - 3 * p;
        const int gw = p >> 2, il = i0 + (p & 3);
        const double* Rg = lds_dyn + wf.dw_wave + gw * wf.dw_wstride + wf.dwo_R;
        Pw[24 + 3 * p + c] = il < n ? Rg[3 * (e0 + il) + c] : 0.0;
      }
      __syncthreads();
      dw_tile_tables<16, 1>(wf, l, Pw + 24, 3);
      __syncthreads();
      dw_radial<16, 1>(wf, l);
      __syncthreads();
      dw_mfma<1>(wf, l, cmap + s2 * wf.nop, V4, part, lam);
      if (!bad) {
#pragma unroll 1
        for (int e4 = 0; e4 < 4 && i0 + e4 < n; ++e4) {
          const int il = i0 + e4, i = e0 + il;
          const double rw[4] = {ge[0], ge[1], ge[2], V4[(4 * g + e4) * 64 + lane]};
          if (e4 + 1 < 4 && il + 1 < n && lane < WD)
#pragma unroll
            for (int c = 0; c < 3; ++c) ge[c] = gc[((size_t)(i + 1) * 3 + c) * WD + lane];
          if (lane == il)
#pragma unroll
            for (int j = 0; j < NC; ++j) bc[j] = C[j];
          double t[4], rp[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            t[c] = dw_dotl<NC>(rw[c], C);
            rp[c] = dw_readlane(t[c], il);
            if (tlane) yr[c * 64 + (lane - n)] = rw[c] - t[c];
          }
          wave_sync();
          double part[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) part[c] = dw_detsum(d, rp[c], yr + c * 64, bc);
          dw_wsum<4>(part);
          const double iS = 1.0 / S;
          const double gx = dw_readlane(jg[0], i), gy = dw_readlane(jg[1], i), gz = dw_readlane(jg[2], i);
          tsum += part[3] * iS + 2.0 * (gx * part[0] + gy * part[1] + gz * part[2]) * iS;
          wave_sync();
        }
      }
      __syncthreads();
    }
  }
  {
    // the Jastrow-only terms of every electron: sum of Lap U + |grad U|^2, and the potential
    const bool el = lane < N;
    double q[2] = {el ? jl + jg[0] * jg[0] + jg[1] * jg[1] + jg[2] * jg[2] : 0.0, el ? jv : 0.0};
    dw_wsum<2>(q);
    tsum += q[0];
    vsum += q[1];
  }
  // ---- E_L, weight, record scalars ----
  if (live && lane == 0) {
    const double En = bad ? NAN : -0.5 * tsum + vsum + wf.vnn;
    if constexpr (VMC) {
      if (!prep) {
        if (!bad) {
          vm.e_sum[w] += En;
          vm.e2_sum[w] += En * En;
        }
        vm.n_accept[w] += na;
        vm.e_last[w] = En;
      }
    } else if (!prep) {
      dmc_branch_inputs(br, w, bad, E_old, En, ET, tau, N, seed, step);
      nacc[3 * w] = na;
      nacc[3 * w + 1] = d2p;
      nacc[3 * w + 2] = d2a;
    }
    double* sc = rec + wf.r_sc;
    sc[SC_ELOC] = En;
    sc[SC_FLAGS] = bad ? 1.0 : 0.0;
    RW[2 * (n0 + n1)] = S;
  }
  if (live)
    for (int k = lane; k < 3 * N; k += 64) rec[wf.r_R + k] = Rl[k];
  if constexpr (VMC) {
    // S_IJ sums (Sec. 2.4): the structure ratios r_I = sum over the
    // structure's determinant pairs of d R_up R_dn / S from the ratios this
    // step left in the record, then r_I r_J into the walker's matrix (the
    // host sends at most 256 structures here: r_I sits in the broadcast rows)
    if (!prep && vm.sij && live && !bad) {
      const int nv = wf.nstruct;
      double* rI = xr;
      for (int I = lane; I < nv; I += 64) {
        double a = 0.0;
        for (int k = wf.srow[I]; k < wf.srow[I + 1]; ++k)
          a += wf.slc[k] * RW[wf.slu[2 * k]] * RW[n0 + wf.slu[2 * k + 1]];
        rI[I] = a / S;
      }
      wave_sync();
      double* sj = vm.sij + (size_t)w * nv * nv;
      for (int k = lane; k < nv * nv; k += 64) {
        const int I = k / nv, J = k - I * nv;
        sj[k] += rI[I] * rI[J];
      }
    }
  }
}

template <int NC, int XE, int LK, bool VMC, bool EEN>
static hipError_t launch_dmcw_t(const DevWF& wf, const DevWF* dwf, double* state, const double* ctrl, int64_t cap,
                                uint64_t seed, uint32_t step, double tau, const DmcBranch& br, double* nacc, int prep,
                                const DwVmc& vm, hipStream_t s) {
  const size_t lds = (size_t)wf.lds_dmcw_doubles * sizeof(double);
  static size_t cur = 0;
  if (lds > cur) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dmcw<NC, XE, LK, VMC, EEN>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    cur = lds;
  }
  const unsigned blocks = (unsigned)((cap + kDwW - 1) / kDwW);
  hipLaunchKernelGGL((k_dmcw<NC, XE, LK, VMC, EEN>), dim3(blocks), dim3(kDwNT), lds, s, dwf, state, ctrl, seed, step, tau,
                     br, nacc, prep, vm);
  return hipGetLastError();
}

template <bool VMC>
static hipError_t launch_dmcw_any(const DevWF& wf, const DevWF* dwf, double* state, const double* ctrl, int64_t cap,
                                  uint64_t seed, uint32_t step, double tau, const DmcBranch& br, double* nacc,
                                  int prep, const DwVmc& vm, hipStream_t s) {
  const int kper = wf.Mpad / (4 * kDwW);
#define VBQMC_DMCW(XE, LK, EEN) \
  return launch_dmcw_t<32, XE, LK, VMC, EEN>(wf, dwf, state, ctrl, cap, seed, step, tau, br, nacc, prep, vm, s)
  if (wf.neen) {
    // (f_een systems: the three-replaced-column form serves every dw_xe <= 3)
    if (kper <= 4) VBQMC_DMCW(3, 4, true);
    if (kper <= 8) VBQMC_DMCW(3, 8, true);
    VBQMC_DMCW(3, 16, true);
  }
  if (wf.dw_xe <= 2) {
    if (kper <= 4) VBQMC_DMCW(2, 4, false);
    if (kper <= 8) VBQMC_DMCW(2, 8, false);
    VBQMC_DMCW(2, 16, false);
  }
  if (kper <= 4) VBQMC_DMCW(3, 4, false);
  if (kper <= 8) VBQMC_DMCW(3, 8, false);
  VBQMC_DMCW(3, 16, false);
#undef VBQMC_DMCW
}

// one DMC step (prep = 0) or the rebuild of every record from its positions
// (prep = 1) for the walkers of ctrl[DC_W] in state; wf is the host copy of
// the layout in dwf (dw_xe: the most columns a determinant replaces)
hipError_t launch_dmcw(const DevWF& wf, const DevWF* dwf, double* state, const double* ctrl, int64_t cap,
                       uint64_t seed, uint32_t step, double tau, const DmcBranch& br, double* nacc, int prep,
                       hipStream_t s) {
  return launch_dmcw_any<false>(wf, dwf, state, ctrl, cap, seed, step, tau, br, nacc, prep, DwVmc{}, s);
}

// one single-electron VMC step (prep = 0) or the rebuild of every record
// (prep = 1) for the vm.W walkers of state, accumulating into vm
hipError_t launch_dmcw_vmc(const DevWF& wf, const DevWF* dwf, double* state, uint64_t seed, uint32_t step, int prep,
                           const DwVmc& vm, hipStream_t s) {
  return launch_dmcw_any<true>(wf, dwf, state, nullptr, vm.W, seed, step, 0.0, DmcBranch{}, nullptr, prep, vm, s);
}

}  // namespace vbqmc
