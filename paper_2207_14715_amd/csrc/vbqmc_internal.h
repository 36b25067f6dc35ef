// Internal layout shared by the host code and the gfx950 kernels of the JVB
// library.  Nothing here is part of the public C ABI (include/vbqmc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vbqmc {

constexpr int kGroup = 16;     // electrons per MFMA row tile
// radial schedule entry (one 32-bit word): primitive in bits 0-10, shell in
// bits 11-20, nucleus in bits 21-28, then the flags
constexpr unsigned kRsPrim = 0x7FFu, kRsShift = 11, kRsShMask = 0x3FFu, kRsNucShift = 21, kRsNucMask = 0xFFu;
constexpr unsigned kRsSto = 1u << 29, kRsFirst = 1u << 30, kRsLive = 1u << 31;
constexpr int kChunk = 16;     // basis functions are padded to a multiple of this
constexpr int kMaxExc = 3;     // columns a spin determinant may differ from its reference
constexpr int kMaxSpin = 64;   // electrons per spin
constexpr int kRedSlots = 64;  // doubles of block-reduction scratch
constexpr int kMaxFinishN = 128;  // electrons per walker (2 x kMaxSpin)
constexpr int kXcds = 8;          // accelerator dies (each with its own L2) on MI355X
constexpr int kCus = 256;         // compute units on MI355X
constexpr int kRowWalkers = 4;    // walkers per wavefront in the row step kernel (16 lanes each)
constexpr int kRowMaxN = 24;      // electrons per walker in the row step kernel

// One spin's determinant table (reference determinant + replaced columns).
struct SpinTab {
  int n;            // electrons of this spin
  int e0;           // index of its first electron
  int nP;           // table orbitals: orbitals that replace reference columns
  int nU;           // distinct spin determinants; u = 0 is the reference
  const int* ref;   // [n] reference orbitals, ascending
  const int* porb;  // [nP] table orbitals, ascending
  const int* uinfo; // [nU][8]: e, J0, J1, J2, Q0, Q1, Q2, 0  (J: slots, Q: table index)
  const int* wrow;  // [nU + 1] CSR over the determinant pairs holding u
  const int* wother;     // other spin's determinant of each pair
  const double* wcoef;   // w_k = sum_I c_I d'_{I,k} of each pair
  const int* omap;       // [nop] per orbital: its reference slot j, or n + its table index q, or -1
};

// terms per nucleus of the three-body Jastrow f_een (Sec. 2.1: the
// expansion up to p = 5)
constexpr int kEenTerms = 23;

// Constant description of the wave function plus layouts, passed by value to
// every kernel.
struct DevWF {
  int N, nup, ndn, nnuc, nshell, M, Mpad, norb, nop, nstruct, nprim, nlinks;
  int precision, refresh_every;
  // mixed form: trial / proposal rows in trial_prec (FP32), the reference
  // inverse rebuilt from rows in `precision` before every local energy
  int trial_prec, refresh_each_step;
  double kappa, vnn;
  double ee[8];
  const double* nuc;    // [nnuc][4]: x, y, z, Z
  const double* en;     // [nnuc][6]
  int neen;             // f_een terms per nucleus (kEenTerms), or 0 without f_een
  const double* een;    // [nnuc][neen] f_een coefficients (global memory)
  const int* shtab;     // [nshell][8]: center, kind, l, first function, first primitive, count, 0, 0
  const double* pexp;
  const double* pcoef;
  const int* pshell;    // [nprim] shell of each primitive
  const int* fnmap;     // [Mpad][2]: shell (or -1 for padding), m | l << 4 | kind << 6 | center << 8
  const double* lamT;   // [Mpad][nop] lambda transposed, zero padded
  const float* lamT32;
  const uint16_t* lamT16;  // bf16 bit patterns
  SpinTab sp[2];
  int nwl[2];           // CSR lengths of the per-spin pair lists
  const int* srow;      // [nstruct + 1] CSR of structure links
  const int* slu;       // [nlinks][2]: up, down spin determinant
  const double* slc;    // [nlinks] d'_{I,k}
  const double* timg;   // [timg_len] the LDS table region, laid out as in LDS (one contiguous copy)
  int timg_len;
  // walker record (doubles)
  int rec_len, hot_len;
  int r_R, r_B[2], r_T[2], r_sc, r_RW, r_gc, r_bk;  // r_RW: Ru0 | Ru1 | Wu0 | Wu1 | S
  // LDS layout (offsets in doubles): constant tables staged once per block
  int lam_in_lds;
  int l_fn, l_sh, l_pe, l_pc, l_psh, l_nuc, l_en, l_lam;
  int l_ref[2], l_porb[2], l_ui[2], l_wrow[2], l_woth[2], l_wcoef[2], l_srow, l_slu, l_slc;
  // radial schedules of a 64-lane block: the shells dealt to four bins (16
  // electrons per pass) and to eight bins (8 electrons per pass, for a tile of
  // at most 8 rows), entry j of bin b at [j][b] (one word, see kRsPrim);
  // rsched_len / rsched_len8 rows (even) plus four padding rows each, none
  // when the length is 0
  int l_rsched, rsched_len, rsched_sto, l_rsched8, rsched_len8;
  int l_etab;  // 2^(j/64), j = 0..63, for the exponentials of the radial sums
  // walker state and scratch
  int l_R, l_B[2], l_T[2], l_PP[2];
  int l_Ru[2], l_Wu[2], l_Qu, l_sc, l_red, l_ipiv, l_f;
  int l_gU, l_lU, l_gD, l_lD;
  int l_disp, l_gtab, l_Phi, l_part, l_chi, l_v, l_y, l_bcol, l_z, l_pt, l_yb, l_sij, l_ratio;
  int l_Phi4, l_yb64, l_tstage, tstage_row, l_Rall;
  int l_Rp, l_ua, l_Vn;  // sweep kernel: trial positions, acceptance draws, trial orbital rows
  // adjoint kernel
  int l_aPhi, l_aG0, l_aG, l_aA, l_aP, l_aM, l_aU[2];
  // adjoint through each spin's reference: B S [n][n], T, Xi = K_P - K_0 T,
  // B Xi [n][nP], the sums W, Wbar, X [3][nP][n], and per distinct spin
  // determinant the inverse of its minor and V Xi_Q ([nU][18])
  int l_aBS, l_aT, l_aXi, l_aBXi, l_aW, l_aV[2];
  int adj_save, l_aSave[2];  // the first pass's B, B S, T, B Xi per spin, kept for the second (if they fit)
  int lds_doubles, lds_sweep_doubles, lds_finish_doubles, lds_tile_doubles, lds_adj_doubles;
  // wavefront sweep (several walkers per wavefront): walker g's state starts
  // at gw_base + g * gw_stride, and the state offsets of that layout are
  // relative to it
  int gw_base, gw_stride, lds_sweepg_doubles;
  // row step kernel (one walker per 16-lane row): per walker the exchange
  // slots of a move (l_xch, walker-relative); per wavefront the Jastrow
  // move tables, refresh rows, local-energy row results and structure ratios
  int l_xch, l_jx, l_Vr, l_gc4, l_rI, lds_rows_doubles;
  // row kernel: trial rows of both spins keep only the columns a move reads
  // (reference slots, then table orbitals), rows_vw doubles per row, placed
  // by the column map l_cmap ([spin][orbital] -> position or -1)
  int l_cmap, rows_vw;
  // walker-resident DMC (four walkers per workgroup, one per wavefront):
  // record caches of the value rows r_vc [N][dw_width] and gradient rows
  // r_gc [N][3][dw_width] at the electrons' positions, in slot order
  // (reference slots, then table orbitals; dw_width = max over spins of
  // n + nP); per wavefront an area at dw_wave + g dw_wstride holding
  // positions (dwo_R), a column of B (dwo_bc), broadcast rows [4][64]
  // (dwo_x), table residuals [4][64] (dwo_y) and the pivots and column of a
  // refresh (dwo_piv, dwo_f); shared: proposals and drifts [4][6] then
  // local-energy points [16][3] (dw_P), the column maps [2][nop] (dw_cmap),
  // the row-tile tables (dw_disp [16][4 nnuc + 1], dw_gtab) and rows
  // (dw_V4 [16][64]), overlaid by the refresh matrices dw_A + g dw_Astride
  int dw_width, r_vc, dw_xe;  // dw_xe: the most columns a spin determinant replaces
  int dw_wave, dw_wstride, dwo_R, dwo_bc, dwo_x, dwo_y, dwo_piv, dwo_f;
  int dw_P, dw_cmap, dw_disp, dw_gtab, dw_V4, dw_A, dw_Astride, lds_dmcw_doubles;
  int dw_part;  // partial sums of the row-tile contraction [4][3][4][64]
  // harmonic table of a row tile (in the tile region): per point p and
  // nucleus a the nine angular polynomials h = m + l^2 at the displacement,
  // with (four points) their x, y, z derivatives: [p][a][9][4], else [p][a][9]
  int dw_harm;
  int dw_rnd;   // per wavefront, the draws of a spin's moves [64][4] (normals, acceptance uniform)
  // radial schedules of the row tiles (four points x 64 bins; sixteen
  // points x 16 bins; entry j of bin b at [j][b], words as kRsPrim), staged
  // from dw_rs_g to LDS offset dw_rs; a length of 0 means no schedule
  const unsigned* dw_rs_g;
  int dw_rs, dw_rs_words, dw_rs4_off, dw_rs4_len, dw_rs16_off, dw_rs16_len;
};

// scalar slots in the record's / LDS scalar block
enum {
  SC_LOGDET0 = 0, SC_LOGDET1, SC_SGN0, SC_SGN1, SC_NUPD0, SC_NUPD1, SC_ELOC, SC_FLAGS,
  SC_S, SC_U, SC_V, SC_LOGPSI, SC_SIGN, SC_RATIO, SC_ACC, SC_TMP0, SC_TMP1, SC_TMP2, SC_TMP3,
  SC_GJ_OK, SC_GJ_LD, SC_GJ_SG,  // a one-wavefront inversion's outcome, ln|det| and sign for the block
  SC_GJ_OK1, SC_GJ_LD1, SC_GJ_SG1,  // (the same for a second spin inverted at the same time)
  SC_COUNT = 32
};

// DMC device-side control block (doubles), in the caller's workspace.
enum {
  DC_W = 0, DC_ET, DC_RUN_NUM, DC_RUN_DEN, DC_ERR, DC_WNEW, DC_ERRSTEP, DC_COUNT = 8
};

// Per-walker branching inputs of one DMC step, in the caller's workspace:
// weight w (before population control), w E_L, w E_L clipped, the branching
// draw u, and the copy count (-1 for an invalid walker; set by the scan once
// the population-control factor of the step is known).
struct DmcBranch {
  double* w;
  double* we;
  double* wc;
  double* ub;
  int* nc;
};

// Walker-resident kernel in VMC mode (single-electron Metropolis steps):
// step size, walker count and the per-walker accumulators of vbqmc_vmc_acc
// (sij: [W][nstruct][nstruct] or null).
struct DwVmc {
  double step;
  int64_t W;
  double* e_sum;
  double* e2_sum;
  double* n_accept;
  double* e_last;
  double* sij;
};

}  // namespace vbqmc
