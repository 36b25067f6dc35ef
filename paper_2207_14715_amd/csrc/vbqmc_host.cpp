// Host side of the JVB library: the C ABI of include/vbqmc.h, the expansion of
// HLSP structures into a reference-determinant table, the walker-record and
// LDS layouts, and kernel launches.
//
// Method references (Radenkovic, Domin, Toulouse, Braida 2022): Sec. 2.1
// Eq. (PhiI) for the structures; Sec. 2.3 for the walks; Sec. 2.4 for the
// structure weights.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vbqmc.h"
#include "vbqmc_internal.h"
#include "vbqmc_ecp.h"

namespace vbqmc {
hipError_t launch_evaluate(const DevWF& wf, const DevWF* dwf, int nt, int64_t W, const double* R, int64_t rstride,
                           double* logabs, int32_t* sign, double* grad, double* eloc, double* ratio, double* state,
                           const DevEcp& ecp, hipStream_t s);
hipError_t launch_vmc(const DevWF& wf, const DevWF* dwf, int nt, double* state, int64_t W, int nsteps, uint64_t seed, uint64_t step0,
                      double step_size, int all_e, double* es, double* e2s, double* na, double* el, double* sij,
                      const DevEcp& ecp, hipStream_t s);
hipError_t launch_vmc_split(const DevWF& wf, const DevWF* dwf, const DevWF* dwf_g, int G, const DevWF* dwf_aux,
                            int nt, int phases, double* state, int64_t W, int nsteps, uint64_t seed, uint64_t step0,
                            double step_size, double* es, double* e2s, double* na, double* el, double* sij,
                            hipStream_t s);
hipError_t launch_dmc_step(const DevWF& wf, const DevWF* dwf, int nt, double* state, const double* ctrl, int64_t cap, uint64_t seed,
                           uint32_t step, double tau, const DmcBranch& br, double* nacc, const DevEcp& ecp,
                           hipStream_t s);
hipError_t launch_dmc_tail(double* ctrl, const DmcBranch& br, const double* nacc, int* offs, int64_t cap, int N,
                           int st, double tau, double W_target, double* pop, double* wsum, double* wesum,
                           double* wcsum, double* etrial, double* lacc, double* lprop, double* ld2a, double* ld2p,
                           const double* src, double* dst, int rec_len, hipStream_t s);
hipError_t launch_vmc_rows(const DevWF& wf, const DevWF* dwf, double* state, int64_t W, int nsteps, uint64_t seed,
                           uint64_t step0, double step_size, double* es, double* e2s, double* na, double* el,
                           double* sij, hipStream_t s);
hipError_t launch_dmcb_finish(const DevWF& wf, const DevWF* dwf, const DevWF* dwf_rows, size_t rows_lds,
                              double* state, double* ctrl, int64_t cap, uint64_t seed, uint32_t step, double tau,
                              double* Vp, double* ek, double* ep, const DmcBranch& br,
                              int rebuild, hipStream_t s);
hipError_t launch_dmcb_move(const DevWF& wf, const DevWF* dwf, const DevWF* dwf_rows, size_t rows_lds, double* state,
                            double* ctrl, int64_t cap, int i, uint64_t seed, uint32_t step, double tau, double* P,
                            double* V, double* Vp, double* nacc, hipStream_t s);
hipError_t launch_copy_records(const double* src, double* dst, int64_t n, hipStream_t s);
hipError_t launch_dmcw(const DevWF& wf, const DevWF* dwf, double* state, const double* ctrl, int64_t cap,
                       uint64_t seed, uint32_t step, double tau, const DmcBranch& br, double* nacc, int prep,
                       hipStream_t s);
hipError_t launch_dmcw_vmc(const DevWF& wf, const DevWF* dwf, double* state, uint64_t seed, uint32_t step, int prep,
                           const DwVmc& vm, hipStream_t s);
hipError_t launch_positions(const DevWF& wf, const DevWF* dwf, int64_t W, const double* state, double* R, hipStream_t s);
hipError_t launch_record_eloc(const DevWF& wf, const DevWF* dwf, int64_t W, const double* state, double* e, hipStream_t s);
hipError_t launch_reduce(int64_t W, int K, const double* wts, const double* in, double* out, hipStream_t s);
hipError_t launch_lm_accumulate(int P, int64_t W, const double* O, const double* D, const double* E,
                                const double* w, double* acc, hipStream_t s);
hipError_t launch_rotation_grad(int P, int lam_off, int M, int nop, int norb, int64_t W, int npair,
                                const int* pairs, const double* lamT, const double* dl, const double* de,
                                double* odl, double* ode, hipStream_t s);
hipError_t launch_param_grad(const DevWF& wf, const DevWF* dwf, int nt, int64_t W, const double* R, double* dlogpsi, double* deloc,
                             double* ws, size_t ws_doubles, hipStream_t s);
size_t param_grad_ws_doubles(const DevWF& wf, int64_t W);
}  // namespace vbqmc

using namespace vbqmc;

namespace {

int nfunc(int l) { return l == 0 ? 1 : (l == 1 ? 3 : 5); }

int parity_of(const std::vector<int>& v) {
  int inv = 0;
  for (size_t a = 0; a < v.size(); ++a)
    for (size_t b = a + 1; b < v.size(); ++b)
      if (v[a] > v[b]) ++inv;
  return inv & 1;
}

uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct Term {
  int I;
  std::vector<int> inact, pairs, unp;
};

// One spin determinant in the slot order of Eq. (PhiI): inactive orbitals,
// then one orbital per pair, then (spin up only) unpaired orbitals.
struct Product {
  int I;
  std::vector<int> up, dn;
};

void expand(const Term& t, std::vector<Product>& out) {
  std::vector<int> distinct;
  int np = (int)t.pairs.size() / 2;
  for (int k = 0; k < np; ++k)
    if (t.pairs[2 * k] != t.pairs[2 * k + 1]) distinct.push_back(k);
  for (int mask = 0; mask < (1 << distinct.size()); ++mask) {
    Product p;
    p.I = t.I;
    p.up = t.inact;
    p.dn = t.inact;
    for (int k = 0; k < np; ++k) {
      int a = t.pairs[2 * k], b = t.pairs[2 * k + 1];
      int pos = (int)(std::find(distinct.begin(), distinct.end(), k) - distinct.begin());
      bool flip = pos < (int)distinct.size() && ((mask >> pos) & 1);
      // a+_{a up} a+_{b dn} - a+_{a dn} a+_{b up} = a+_{a up} a+_{b dn} + a+_{b up} a+_{a dn}
      p.up.push_back(flip ? b : a);
      p.dn.push_back(flip ? a : b);
    }
    for (int q : t.unp) p.up.push_back(q);
    out.push_back(p);
  }
}

struct SpinHost {
  int n = 0, e0 = 0;
  std::vector<int> ref, porb, uinfo, wrow, wother;
  std::vector<double> wcoef;
  std::map<std::vector<int>, int> index;
  std::vector<std::vector<int>> sets;
  std::vector<int> sgn;  // parity of the aligned order of each unique set
};

}  // namespace

struct vbqmc_ctx {
  std::string err;
  DevWF wf{};
  int nt = 64;
  int lds_limit = 65536;
  // host copies
  int N = 0, nup = 0, ndn = 0, nnuc = 0, M = 0, Mpad = 0, norb = 0, nop = 0, nstruct = 0, nshell = 0;
  std::vector<double> nuc, en, een, pexp, pcoef, lam, c;
  std::vector<int> shtab, fnmap, pshell;
  std::vector<unsigned> rsched;  // radial schedules of 64-lane blocks: 4 bins, then 8 bins
  std::vector<unsigned> dw_rs;   // radial schedules of the walker-resident DMC row tiles: 64 bins, then 16
  int dw_rs4_len = 0, dw_rs16_len = 0, dw_rs16_off = 0;
  int rsched_len = 0, rsched_len8 = 0, rsched8_off = 0;
  double ee[8];
  double kappa = 0;
  SpinHost sp[2];
  // determinant pairs k: (u_up, u_dn) and structure links (I, k, d')
  std::vector<int> pair_up, pair_dn;
  std::vector<std::vector<std::pair<int, double>>> pair_links;  // per k: (I, d')
  std::vector<int> srow, slu;
  std::vector<double> slc;
  // device arena
  char* dmem = nullptr;
  size_t dbytes = 0;
  // offsets of mutable device tables
  double* d_lamT = nullptr;
  float* d_lamT32 = nullptr;
  uint16_t* d_lamT16 = nullptr;
  double* d_en = nullptr;
  double* d_een = nullptr;
  double* d_wcoef[2] = {nullptr, nullptr};
  double* d_slc = nullptr;
  DevWF* d_wf = nullptr;
  DevEcp ecp{};                 // pseudopotentials (vbqmc_set_ecp); ncen = 0 for none
  char* d_ecp = nullptr;        // their tables
  DevWF* d_wf_sweep = nullptr;  // same tables, compact LDS layout of the sweep kernel
  DevWF* d_wf_sweepg = nullptr; // same tables, layout of the wavefront sweep (several walkers per wavefront)
  int sweep_g = 64;             // lanes per walker in the single-electron sweep
  DevWF* d_wf_aux = nullptr;    // same tables, compact LDS layout of the batched local-energy kernels
  DevWF* d_wf_rows = nullptr;   // same tables, layout of the row step kernel (four walkers per wavefront)
  int step_kernel = 1;          // single-electron VMC steps: 1 sweep + local-energy kernels, 2 row kernel,
                                // 3 walker-resident kernel
  DevWF* d_wf_dmcb = nullptr;   // same tables, layout of the electron-major DMC row tiles
  int dmc_kernel = 1;           // DMC steps: 1 one workgroup per walker, 2 electron-major, 3 walker-resident
  DevWF* d_wf_dmcw = nullptr;   // same tables, layout of the walker-resident DMC kernel
  double* d_timg = nullptr;     // LDS table image
  int dev = 0;                  // device the context was created on
  void* scratch = nullptr;      // that device's copy of the no-alloc scratch array
};

// Scratch of vbqmc_dmc_advance_noalloc: a file-scope device array of
// kNoAllocScratchBytes, one copy per device, held until the process ends.
// Host code never uses the array's name as an address: each device's copy is
// reached through the pointer hipGetSymbolAddress returns with that device
// current (taken once per device at vbqmc_create).
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// the device address of the scratch array on device dev (current), looked up
// once per device
std::mutex g_scratch_mu;
void* g_scratch_ptr[256] = {};

hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int fail(vbqmc_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hipfail(vbqmc_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, VBQMC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// (re)compute w_k and structure-link coefficients from c
void build_coefficients(vbqmc_ctx* x, std::vector<double> (&wcoef)[2], std::vector<double>& slc) {
  int nk = (int)x->pair_up.size();
  std::vector<double> wk(nk, 0.0);
  for (int k = 0; k < nk; ++k)
    for (auto& pr : x->pair_links[k]) wk[k] += x->c[pr.first] * pr.second;
  for (int s = 0; s < 2; ++s) {
    SpinHost& h = x->sp[s];
    wcoef[s].clear();
    int nU = (int)h.sets.size();
    for (int u = 0; u < nU; ++u)
      for (int k = 0; k < nk; ++k)
        if ((s == 0 ? x->pair_up[k] : x->pair_dn[k]) == u) wcoef[s].push_back(wk[k]);
  }
  slc = x->slc;
}

template <class T> T* carve(char*& p, size_t n) {
  T* r = (T*)p;
  size_t b = (n * sizeof(T) + 255) & ~(size_t)255;
  p += b;
  return r;
}

size_t arena_bytes_for(size_t n, size_t sz) { return (n * sz + 255) & ~(size_t)255; }

int upload_lambda(vbqmc_ctx* x) {
  std::vector<double> lt((size_t)x->Mpad * x->nop, 0.0);
  std::vector<float> l32(lt.size(), 0.f);
  std::vector<uint16_t> l16(lt.size(), 0);
  for (int p = 0; p < x->norb; ++p)
    for (int mu = 0; mu < x->M; ++mu) {
      double v = x->lam[(size_t)p * x->M + mu];
      size_t k = (size_t)mu * x->nop + p;
      lt[k] = v;
      l32[k] = (float)v;
      l16[k] = to_bf16((float)v);
    }
  hipError_t e = hipMemcpy(x->d_lamT, lt.data(), lt.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->d_lamT32, l32.data(), l32.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->d_lamT16, l16.data(), l16.size() * 2, hipMemcpyHostToDevice);
  return e == hipSuccess ? 0 : hipfail(x, e, "upload lambda");
}

// LDS allocator: offsets in doubles, each region 16-byte aligned
struct LdsAlloc {
  int o;
  int operator()(int n) { int r = o; o += (std::max(n, 1) + 1) / 2 * 2; return r; }
  int ints(int n) { return (*this)((n + 1) / 2); }
};

// Radial schedules of the 64-lane blocks.  With NB bins, lane l takes
// electron l % (64 / NB) of a row tile and bin l / (64 / NB); the shells are
// dealt to the bins longest first, each to the bin with the fewest primitives
// so far, so every lane walks about 1/NB of the primitives in one
// fixed-length loop.  A bin lists its shells' primitives in shell order (the
// order of the contraction sums) and flags the first primitive of each shell.
// It is padded to the longest bin rounded up to even, plus four rows read
// ahead, with empty entries (no primitive term) of its last shell, which store
// that shell's sum again.  Returns the length (0: fewer than NB shells, no
// schedule).
static int deal_radial_bins(const vbqmc_ctx* x, int NB, std::vector<unsigned>& out) {
  out.clear();
  if (x->nshell < NB) return 0;
  std::vector<int> order(x->nshell);
  for (int s = 0; s < x->nshell; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return x->shtab[8 * a + 5] > x->shtab[8 * b + 5]; });
  std::vector<std::vector<int>> bins(NB);
  std::vector<int> load(NB, 0);
  for (int s : order) {
    int b = 0;
    for (int k = 1; k < NB; ++k)
      if (load[k] < load[b]) b = k;
    bins[b].push_back(s);
    load[b] += x->shtab[8 * s + 5];
  }
  int L = 0;
  for (int b = 0; b < NB; ++b) {
    std::sort(bins[b].begin(), bins[b].end());
    L = std::max(L, load[b]);
  }
  L += L & 1;  // walked two entries at a time, with two steps loaded ahead
  out.assign((size_t)NB * (L + 4), 0u);
  auto where = [&](int s) { return ((unsigned)s << kRsShift) | ((unsigned)x->shtab[8 * s] << kRsNucShift); };
  for (int b = 0; b < NB; ++b) {
    int j = 0;
    for (int s : bins[b]) {
      const int* si = &x->shtab[8 * s];
      for (int k = 0; k < si[5]; ++k, ++j) {
        unsigned f = (unsigned)(si[4] + k) | where(s) | kRsLive;
        if (si[1] == 1) f |= kRsSto;
        if (k == 0) f |= kRsFirst;
        out[(size_t)NB * j + b] = f;
      }
    }
    for (; j < L + 4; ++j) out[(size_t)NB * j + b] = where(bins[b].back());
  }
  return L;
}

// schedules of the walker-resident DMC kernel's row tiles (256 threads):
// four points x 64 bins and sixteen points x 16 bins
void build_dmcw_schedule(vbqmc_ctx* x) {
  x->dw_rs.clear();
  x->dw_rs4_len = x->dw_rs16_len = x->dw_rs16_off = 0;
  const int nprim = (int)x->pexp.size();
  if (nprim > (int)kRsPrim + 1 || x->nshell > (int)kRsShMask + 1 || x->nnuc > (int)kRsNucMask + 1) return;
  std::vector<unsigned> a, b;
  const int L64 = deal_radial_bins(x, 64, a);
  const int L16 = deal_radial_bins(x, 16, b);
  if (L64 > 0) {
    x->dw_rs = a;
    x->dw_rs4_len = L64;
  }
  if (L16 > 0) {
    x->dw_rs16_off = (int)x->dw_rs.size();
    x->dw_rs.insert(x->dw_rs.end(), b.begin(), b.end());
    x->dw_rs16_len = L16;
  }
  if (x->dw_rs.size() & 1) x->dw_rs.push_back(0u);  // whole doubles in LDS
}

void build_radial_schedule(vbqmc_ctx* x) {
  x->rsched.clear();
  x->rsched_len = x->rsched_len8 = 0;
  x->rsched8_off = 0;
  const int nprim = (int)x->pexp.size();
  if (nprim > (int)kRsPrim + 1 || x->nshell > (int)kRsShMask + 1 || x->nnuc > (int)kRsNucMask + 1) return;
  std::vector<unsigned> s4, s8;
  const int L4 = deal_radial_bins(x, 4, s4);
  if (L4 == 0) return;
  const int L8 = deal_radial_bins(x, 8, s8);
  x->rsched = s4;
  x->rsched_len = L4;
  if (L8 > 0) {
    x->rsched8_off = (int)s4.size();  // a multiple of 4 words: whole doubles
    x->rsched.insert(x->rsched.end(), s8.begin(), s8.end());
    x->rsched_len8 = L8;
  }
}

// Sweep kernel: the tables without the orbital coefficients (read from global
// memory there), the walker state, value-only tile tables and the trial
// positions, draws and orbital rows.
DevWF sweep_layout(const vbqmc_ctx* x) {
  DevWF a = x->wf;
  const int nmax = std::max(x->nup, x->ndn);
  int nUm = 1, nPm = 1;
  for (int s = 0; s < 2; ++s) {
    nUm = std::max(nUm, (int)x->sp[s].sets.size());
    nPm = std::max(nPm, (int)x->sp[s].porb.size());
  }
  LdsAlloc lds{a.l_rsched};
  a.timg_len = lds.o;
  a.lam_in_lds = 0;
  a.l_R = lds(3 * x->N);
  a.l_sc = lds(SC_COUNT);
  a.l_red = lds(x->nt > 64 ? kRedSlots : 1);
  a.l_ipiv = lds.ints(nmax);
  a.l_f = lds(nmax);
  for (int s = 0; s < 2; ++s) {
    int n = x->sp[s].n, nP = (int)x->sp[s].porb.size();
    a.l_B[s] = lds(n * n);
    a.l_T[s] = lds(n * nP);
    a.l_PP[s] = lds(n * nP);
    a.l_Ru[s] = lds((int)x->sp[s].sets.size());
    a.l_Wu[s] = lds((int)x->sp[s].sets.size());
  }
  a.l_Qu = lds(nUm);
  a.l_y = lds(nPm + 1);
  a.l_bcol = lds(nmax);
  a.l_z = lds(2 * nmax);
  a.l_disp = lds(kGroup * (4 * x->nnuc + 1));
  a.l_gtab = lds(kGroup * (x->nshell | 1));
  a.l_Rp = lds(3 * x->N);
  a.l_ua = lds(x->N);
  a.l_Vn = lds(x->N * x->nop);
  a.lds_sweep_doubles = lds.o;
  return a;
}

// Wavefront sweep with G lanes per walker: the tables without the orbital
// coefficients, value-only tile tables, the trial positions, draws and
// orbital rows of all 64 / G walkers, then one state block per walker.
DevWF sweepg_layout(const vbqmc_ctx* x, int G) {
  DevWF a = x->wf;
  const int NG = 64 / G;
  const int nmax = std::max(x->nup, x->ndn);
  int nUm = 1, nPm = 1;
  for (int s = 0; s < 2; ++s) {
    nUm = std::max(nUm, (int)x->sp[s].sets.size());
    nPm = std::max(nPm, (int)x->sp[s].porb.size());
  }
  LdsAlloc lds{a.l_rsched};
  a.timg_len = lds.o;
  a.lam_in_lds = 0;
  a.l_disp = lds(kGroup * (4 * x->nnuc + 1));
  a.l_gtab = lds(kGroup * (x->nshell | 1));
  a.l_Rp = lds(3 * NG * x->N);
  a.l_ua = lds(NG * x->N);
  a.l_Vn = lds(NG * x->N * x->nop);
  a.gw_base = lds.o;
  LdsAlloc w{0};
  a.l_R = w(3 * x->N);
  a.l_sc = w(SC_COUNT);
  a.l_ipiv = w.ints(2 * nmax);  // one pivot list and column per spin
  a.l_f = w(2 * nmax);
  for (int s = 0; s < 2; ++s) {
    int n = x->sp[s].n, nP = (int)x->sp[s].porb.size();
    a.l_B[s] = w(n * n);
    a.l_T[s] = w(n * nP);
    a.l_PP[s] = w(n * nP);
    a.l_Ru[s] = w((int)x->sp[s].sets.size());
    a.l_Wu[s] = w((int)x->sp[s].sets.size());
  }
  a.l_Qu = w(nUm);
  a.l_y = w(nPm + 1);
  a.l_bcol = w(nmax);
  a.l_z = w(2 * nmax);
  a.gw_stride = w.o;
  a.lds_sweepg_doubles = a.gw_base + NG * a.gw_stride;
  return a;
}

// Row step kernel (four walkers per wavefront, 16 lanes each): the tables
// without the orbital coefficients, the tile tables, one state block per
// walker (with the exchange slots of a move), then one region whose use
// changes over a step: trial positions, draws, trial rows of one spin and
// the Jastrow move tables during the moves; packed reference rows during an
// inverse refresh; positions, derivative rows and per-electron results
// during the local energy.
// register columns per lane of the row kernel (its NE template argument)
int rows_columns(const vbqmc_ctx* x) { return x->nup <= 10 && x->ndn <= 10 ? 10 : 16; }

DevWF rows_layout(const vbqmc_ctx* x) {
  DevWF a = x->wf;
  const int NG = kRowWalkers, N = x->N, nop = x->nop;
  const int nmax = std::max(x->nup, x->ndn);
  int nUm = 1, nPm = 1;
  for (int s = 0; s < 2; ++s) {
    nUm = std::max(nUm, (int)x->sp[s].sets.size());
    nPm = std::max(nPm, (int)x->sp[s].porb.size());
  }
  LdsAlloc lds{a.l_psh};
  a.timg_len = lds.o;
  a.lam_in_lds = 0;
  a.l_disp = lds(kGroup * (4 * x->nnuc + 1));
  a.l_gtab = lds(kGroup * ((3 * x->nshell) | 1));
  a.gw_base = lds.o;
  LdsAlloc w{0};
  a.l_R = w(3 * N);
  a.l_sc = w(SC_COUNT);
  a.l_ipiv = w.ints(2 * nmax);
  a.l_f = w(2 * nmax);
  for (int s = 0; s < 2; ++s) {
    int n = x->sp[s].n, nP = (int)x->sp[s].porb.size();
    a.l_B[s] = w(n * n);
    a.l_T[s] = w(n * nP);
    a.l_PP[s] = w(n * nP);
    a.l_Ru[s] = w((int)x->sp[s].sets.size());
    a.l_Wu[s] = w((int)x->sp[s].sets.size());
  }
  a.l_Qu = w(nUm);
  a.l_y = w(nPm + 1);
  a.l_bcol = w(nmax);
  a.l_z = w(2 * nmax);
  a.l_xch = w(32);
  a.gw_stride = w.o;
  lds.o += NG * a.gw_stride;
  a.l_cmap = lds.ints(2 * nop);
  int vw = 1;
  for (int s = 0; s < 2; ++s) vw = std::max(vw, x->sp[s].n + (int)x->sp[s].porb.size());
  a.rows_vw = std::max(vw, rows_columns(x));
  const int u0 = lds.o;
  a.l_Rp = lds(3 * NG * N);
  a.l_ua = lds(NG * N);
  const int v0 = lds.o;
  a.l_Vn = lds(NG * N * a.rows_vw);
  a.l_jx = lds(NG * N * N);
  const int end_moves = lds.o;
  lds.o = v0;
  a.l_Vr = lds(NG * N * nop);
  const int end_refresh = lds.o;
  lds.o = u0;
  a.l_Rall = lds(3 * NG * N);
  a.l_Phi4 = lds(4 * kGroup * nop);
  a.l_yb64 = lds(64 * (nPm + 1));
  a.l_gc4 = lds(4 * NG * N);
  a.l_rI = lds(NG * x->nstruct);
  a.lds_rows_doubles = std::max(std::max(end_moves, end_refresh), lds.o);
  return a;
}

// Electron-major DMC row tiles: only the basis tables (the first part of
// the table image, up to the Jastrow coefficients) and the tile tables
// (positions, radial sums with both derivatives).
DevWF dmcb_layout(const vbqmc_ctx* x) {
  DevWF a = x->wf;
  LdsAlloc lds{a.l_en};
  a.timg_len = lds.o;
  a.lam_in_lds = 0;
  a.l_R = lds(3 * kGroup);
  a.l_disp = lds(kGroup * (4 * x->nnuc + 1));
  a.l_gtab = lds(kGroup * ((3 * x->nshell) | 1));
  a.lds_tile_doubles = lds.o;
  return a;
}

// electron-major DMC handles the system: every spin's reference slots plus
// table orbitals fit the 64 lanes of a wavefront, and the row tiles fit LDS
bool dmcb_fit(const vbqmc_ctx* x) {
  size_t refresh = 3 * (size_t)std::max(x->nup, x->ndn);  // LDS of the refresh kernel (doubles)
  for (int s = 0; s < 2; ++s) {
    const int n = x->sp[s].n, nP = (int)x->sp[s].porb.size();
    if (n + nP > 64 || x->sp[s].sets.size() > 128) return false;
    refresh += (size_t)n * (n + 2 * nP) + x->sp[s].sets.size();
  }
  return (size_t)dmcb_layout(x).lds_tile_doubles * 8 <= (size_t)x->lds_limit &&
         refresh * 8 <= (size_t)x->lds_limit;
}

// Walker-resident DMC (four walkers per workgroup, one per wavefront): the
// tables up to the Jastrow coefficients, proposals, column maps, one area per
// wavefront, then the row-tile tables and rows, overlaid by the refresh
// matrices.
DevWF dmcw_layout(const vbqmc_ctx* x) {
  DevWF a = x->wf;
  LdsAlloc lds{a.l_ref[0]};
  a.timg_len = lds.o;
  a.lam_in_lds = 0;
  a.dw_P = lds(24 + 48);
  a.dw_rs = lds((int)x->dw_rs.size() / 2);
  a.dw_rs_words = (int)x->dw_rs.size();
  a.dw_rs4_off = 0;
  a.dw_rs4_len = x->dw_rs4_len;
  a.dw_rs16_off = x->dw_rs16_off;
  a.dw_rs16_len = x->dw_rs16_len;
  a.dw_cmap = lds.ints(2 * x->nop);
  a.dw_wave = lds.o;
  LdsAlloc w{0};
  a.dwo_R = w(3 * x->N);
  a.dwo_bc = w(64);
  a.dwo_x = w(4 * 64);
  a.dwo_y = w(4 * 64);
  a.dwo_piv = w.ints(64);
  a.dwo_f = w(64);
  a.dw_rnd = w(4 * 64);
  a.dw_wstride = w.o;
  lds.o += 4 * a.dw_wstride;
  a.dw_part = lds(4 * 3 * 4 * 64);
  const int t0 = lds.o;
  a.dw_disp = lds(16 * (4 * x->nnuc + 1));
  a.dw_gtab = lds(std::max(4 * (2 * x->nshell + 1), 16 * (x->nshell | 1)));
  a.dw_V4 = lds(16 * 64);
  a.dw_harm = lds(std::max(4 * 9 * 4, 16 * 9) * x->nnuc);
  const int tend = lds.o;
  lds.o = t0;
  int astr = 1;
  for (int sp = 0; sp < 2; ++sp)
    astr = std::max(astr, x->sp[sp].n * std::max(x->sp[sp].n, (int)x->sp[sp].porb.size()));
  a.dw_Astride = (astr + 64 + 1) / 2 * 2;  // the matrix and 64 zeroed doubles past it
  a.dw_A = lds(4 * a.dw_Astride);
  a.lds_dmcw_doubles = std::max(tend, lds.o);
  return a;
}

// the walker-resident DMC kernel handles the system: FP64 rows, at most 256
// (padded) basis functions and 48 (padded) orbitals, at most
// 32 electrons, 64 reference slots plus table orbitals and 128 distinct
// determinants per spin, at most 64 (padded) orbitals, spin-up electrons
// present, and its layout fits the device's LDS
bool dmcw_fit(const vbqmc_ctx* x) {
  if (x->wf.precision != VBQMC_FP64 || x->wf.trial_prec != VBQMC_FP64 || x->wf.refresh_each_step) return false;
  if (x->nop > 48 || x->Mpad > 256 || x->nup < 1 || x->nup > 32 || x->ndn > 32 || x->N + x->nnuc > 128) return false;
  for (int sp = 0; sp < 2; ++sp) {
    if (x->sp[sp].n + (int)x->sp[sp].porb.size() > 64 || x->sp[sp].sets.size() > 128) return false;
  }
  return (size_t)dmcw_layout(x).lds_dmcw_doubles * 8 <= (size_t)x->lds_limit;
}

// the row step kernel handles the system: at most 16 columns (reference
// slots + table orbitals) and 16 distinct determinants per spin, at most 24
// electrons, and its layout fits the device's LDS
bool rows_fit(const vbqmc_ctx* x) {
  if (x->N < 1 || x->N > kRowMaxN) return false;
  for (int s = 0; s < 2; ++s) {
    if (x->sp[s].n + (int)x->sp[s].porb.size() > 16) return false;
    if ((int)x->sp[s].sets.size() > 16) return false;
  }
  return (size_t)rows_layout(x).lds_rows_doubles * 8 <= (size_t)x->lds_limit;
}

// Batched local-energy kernels: the tables, then only what the finish and
// tile kernels touch.
DevWF aux_layout(const vbqmc_ctx* x) {
  DevWF a = x->wf;
  int nPm = 1;
  for (int s = 0; s < 2; ++s) nPm = std::max(nPm, (int)x->sp[s].porb.size());
  // the orbital coefficients are read from global memory here (more tiles
  // resident per CU); the rest of the table image is staged
  LdsAlloc lds{a.l_rsched};
  a.timg_len = lds.o;
  a.lam_in_lds = 0;
  a.l_R = lds(std::max(3 * x->N, 3 * kGroup));
  a.l_sc = lds(SC_COUNT);
  a.l_red = lds(kRedSlots);
  a.l_gU = lds(3 * x->N);
  a.l_lU = lds(x->N);
  a.l_ratio = lds(x->nstruct);
  a.lds_finish_doubles = lds.o;
  a.l_disp = lds(kGroup * (4 * x->nnuc + 1));
  a.l_gtab = lds(kGroup * ((3 * x->nshell) | 1));
  a.l_Phi4 = lds(4 * kGroup * x->nop);
  a.l_yb64 = lds(64 * (nPm + 1));
  // per walker of a tile: inverse column, table, R_u, W_u, S, valid flag
  int row = 0;
  for (int s = 0; s < 2; ++s) {
    int n = x->sp[s].n, nP = (int)x->sp[s].porb.size(), nU = (int)x->sp[s].sets.size();
    row = std::max(row, n + n * nP + 2 * nU + 2);
  }
  a.tstage_row = row;
  a.l_tstage = lds(kGroup * row);
  a.lds_tile_doubles = lds.o;
  return a;
}

// The constant tables exactly as they sit at the start of a block's LDS, so
// that a kernel stages them with one contiguous copy.
int upload_table_image(vbqmc_ctx* x) {
  const DevWF& wf = x->wf;
  if (!x->d_timg) return 0;
  std::vector<double> img((size_t)wf.timg_len, 0.0);
  auto put = [&](int off, const void* src, size_t bytes) {
    if (bytes) std::memcpy((char*)img.data() + (size_t)off * 8, src, bytes);
  };
  put(wf.l_fn, x->fnmap.data(), x->fnmap.size() * 4);
  put(wf.l_sh, x->shtab.data(), x->shtab.size() * 4);
  put(wf.l_pe, x->pexp.data(), x->pexp.size() * 8);
  put(wf.l_pc, x->pcoef.data(), x->pcoef.size() * 8);
  put(wf.l_psh, x->pshell.data(), x->pshell.size() * 4);
  put(wf.l_rsched, x->rsched.data(), x->rsched.size() * 4);
  double etab[64];
  for (int j = 0; j < 64; ++j) etab[j] = (double)exp2l((long double)j / 64.0L);
  put(wf.l_etab, etab, sizeof(etab));
  put(wf.l_nuc, x->nuc.data(), x->nuc.size() * 8);
  put(wf.l_en, x->en.data(), x->en.size() * 8);
  std::vector<double> wc[2], slc;
  build_coefficients(x, wc, slc);
  for (int s = 0; s < 2; ++s) {
    const SpinHost& h = x->sp[s];
    put(wf.l_ref[s], h.ref.data(), h.ref.size() * 4);
    put(wf.l_porb[s], h.porb.data(), h.porb.size() * 4);
    put(wf.l_ui[s], h.uinfo.data(), h.uinfo.size() * 4);
    put(wf.l_wrow[s], h.wrow.data(), h.wrow.size() * 4);
    put(wf.l_woth[s], h.wother.data(), h.wother.size() * 4);
    put(wf.l_wcoef[s], wc[s].data(), wc[s].size() * 8);
  }
  put(wf.l_srow, x->srow.data(), x->srow.size() * 4);
  put(wf.l_slu, x->slu.data(), x->slu.size() * 4);
  put(wf.l_slc, slc.data(), slc.size() * 8);
  if (wf.lam_in_lds) {
    size_t n = (size_t)x->Mpad * x->nop;
    std::vector<double> lt(n, 0.0);
    std::vector<float> l32(n, 0.f);
    std::vector<uint16_t> l16(n, 0);
    for (int p = 0; p < x->norb; ++p)
      for (int mu = 0; mu < x->M; ++mu) {
        double v = x->lam[(size_t)p * x->M + mu];
        size_t k = (size_t)mu * x->nop + p;
        lt[k] = v;
        l32[k] = (float)v;
        l16[k] = to_bf16((float)v);
      }
    if (wf.precision == 0) put(wf.l_lam, lt.data(), n * 8);
    else if (wf.precision == 1) put(wf.l_lam, l32.data(), n * 4);
    else put(wf.l_lam, l16.data(), n * 2);
  }
  hipError_t e = hipMemcpy(x->d_timg, img.data(), img.size() * 8, hipMemcpyHostToDevice);
  return e == hipSuccess ? 0 : hipfail(x, e, "upload table image");
}

int upload_coefficients(vbqmc_ctx* x) {
  std::vector<double> wc[2], slc;
  build_coefficients(x, wc, slc);
  hipError_t e = hipSuccess;
  for (int s = 0; s < 2 && e == hipSuccess; ++s)
    if (!wc[s].empty()) e = hipMemcpy(x->d_wcoef[s], wc[s].data(), wc[s].size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && !slc.empty()) e = hipMemcpy(x->d_slc, slc.data(), slc.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->d_en, x->en.data(), x->en.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && x->d_een) e = hipMemcpy(x->d_een, x->een.data(), x->een.size() * 8, hipMemcpyHostToDevice);
  for (int k = 0; k < 8; ++k) x->wf.ee[k] = x->ee[k];
  if (e == hipSuccess && x->d_wf) e = hipMemcpy(x->d_wf, &x->wf, sizeof(DevWF), hipMemcpyHostToDevice);
  if (e == hipSuccess && x->d_wf_sweep) {
    DevWF a = sweep_layout(x);
    e = hipMemcpy(x->d_wf_sweep, &a, sizeof(DevWF), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && x->d_wf_sweepg && x->sweep_g < 64) {
    DevWF a = sweepg_layout(x, x->sweep_g);
    e = hipMemcpy(x->d_wf_sweepg, &a, sizeof(DevWF), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && x->d_wf_aux) {
    DevWF a = aux_layout(x);
    e = hipMemcpy(x->d_wf_aux, &a, sizeof(DevWF), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && x->d_wf_dmcb && x->dmc_kernel == 2) {
    DevWF a = dmcb_layout(x);
    e = hipMemcpy(x->d_wf_dmcb, &a, sizeof(DevWF), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && x->d_wf_dmcw && (x->dmc_kernel == 3 || x->step_kernel == 3)) {
    DevWF a = dmcw_layout(x);
    e = hipMemcpy(x->d_wf_dmcw, &a, sizeof(DevWF), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && x->d_wf_rows && x->step_kernel == 2) {
    DevWF a = rows_layout(x);
    e = hipMemcpy(x->d_wf_rows, &a, sizeof(DevWF), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) return upload_table_image(x);
  return e == hipSuccess ? 0 : hipfail(x, e, "upload coefficients");
}

}  // namespace

extern "C" {

const char* vbqmc_last_error(const vbqmc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int vbqmc_create(const vbqmc_system* sys, const vbqmc_wavefunction* wfi, const vbqmc_options* opt,
                 vbqmc_ctx** out) {
  if (!sys || !wfi || !out) return VBQMC_EINVAL;
  *out = nullptr;
  vbqmc_ctx* x = new (std::nothrow) vbqmc_ctx();
  if (!x) return VBQMC_ENOMEM;
  auto bad = [&](const std::string& m) {
    std::fprintf(stderr, "vbqmc_create: %s\n", m.c_str());
    delete x;
    return VBQMC_EINVAL;
  };
  x->nnuc = sys->n_nuclei;
  x->nup = sys->n_up;
  x->ndn = sys->n_dn;
  x->N = x->nup + x->ndn;
  if (x->nnuc < 1 || x->nup < 0 || x->ndn < 0 || x->N < 1) return bad("bad electron or nucleus count");
  if (x->nup > kMaxSpin || x->ndn > kMaxSpin) return bad("more than 64 electrons of one spin");
  for (int a = 0; a < x->nnuc; ++a) {
    for (int k = 0; k < 3; ++k) x->nuc.push_back(sys->position[3 * a + k]);
    x->nuc.push_back(sys->charge[a]);
  }
  // basis
  x->nshell = wfi->n_shells;
  int off = 0, fn = 0;
  for (int s = 0; s < x->nshell; ++s) {
    int cen = wfi->shell_center[s], kind = wfi->shell_kind[s], l = wfi->shell_l[s], np = wfi->shell_nprim[s];
    if (cen < 0 || cen >= x->nnuc || (kind != 0 && kind != 1) || l < 0 || l > 2 || np < 1)
      return bad("bad shell description");
    x->shtab.insert(x->shtab.end(), {cen, kind, l, fn, off, np, 0, 0});
    for (int k = 0; k < np; ++k) {
      x->pexp.push_back(wfi->prim_exp[off + k]);
      x->pcoef.push_back(wfi->prim_coef[off + k]);
      x->pshell.push_back(s);
    }
    // per function: shell, and m | l << 4 | kind << 6 | center << 8 (one load
    // gives a tile pass everything it needs to find the radial tables)
    for (int m = 0; m < nfunc(l); ++m) x->fnmap.insert(x->fnmap.end(), {s, m | (l << 4) | (kind << 6) | (cen << 8)});
    off += np;
    fn += nfunc(l);
  }
  x->M = fn;
  if (x->M < 1 || x->M > 1024) return bad("basis size outside 1..1024");
  build_radial_schedule(x);
  build_dmcw_schedule(x);
  x->Mpad = (x->M + kChunk - 1) / kChunk * kChunk;
  for (int mu = x->M; mu < x->Mpad; ++mu) x->fnmap.insert(x->fnmap.end(), {-1, 0});
  x->norb = wfi->n_orbitals;
  if (x->norb < 1 || x->norb > 256) return bad("orbital count outside 1..256");
  x->nop = (x->norb + 15) / 16 * 16;
  x->lam.assign(wfi->lambda, wfi->lambda + (size_t)x->norb * x->M);
  // structures
  x->nstruct = wfi->n_structures;
  if (x->nstruct < 1) return bad("no structures");
  x->c.assign(wfi->coef, wfi->coef + x->nstruct);
  std::vector<Product> prods;
  int q = 0;
  for (int t = 0; t < wfi->n_terms; ++t) {
    Term term;
    term.I = wfi->term_structure[t];
    int ni = wfi->term_counts[3 * t], np = wfi->term_counts[3 * t + 1], nu = wfi->term_counts[3 * t + 2];
    if (term.I < 0 || term.I >= x->nstruct) return bad("term structure index out of range");
    term.inact.assign(wfi->term_orbitals + q, wfi->term_orbitals + q + ni);
    term.pairs.assign(wfi->term_orbitals + q + ni, wfi->term_orbitals + q + ni + 2 * np);
    term.unp.assign(wfi->term_orbitals + q + ni + 2 * np, wfi->term_orbitals + q + ni + 2 * np + nu);
    q += ni + 2 * np + nu;
    for (int o : term.inact) if (o < 0 || o >= x->norb) return bad("orbital index out of range");
    for (int o : term.pairs) if (o < 0 || o >= x->norb) return bad("orbital index out of range");
    for (int o : term.unp) if (o < 0 || o >= x->norb) return bad("orbital index out of range");
    if (ni + np + nu != x->nup || ni + np != x->ndn) return bad("term electron counts differ from n_up/n_dn");
    expand(term, prods);
  }
  // spin determinants: sort each slot list, drop identically zero ones,
  // dedupe by set, align to the reference
  struct Entry { int I, u0, u1; double d; };
  std::vector<Entry> entries;
  for (int s = 0; s < 2; ++s) {
    x->sp[s].n = s == 0 ? x->nup : x->ndn;
    x->sp[s].e0 = s == 0 ? 0 : x->nup;
  }
  for (auto& p : prods) {
    Entry en{p.I, 0, 0, 1.0};
    bool zero = false;
    for (int s = 0; s < 2 && !zero; ++s) {
      const std::vector<int>& L = s == 0 ? p.up : p.dn;
      std::vector<int> srt = L;
      std::sort(srt.begin(), srt.end());
      if (std::adjacent_find(srt.begin(), srt.end()) != srt.end()) { zero = true; break; }
      if (parity_of(L)) en.d = -en.d;
      SpinHost& h = x->sp[s];
      auto it = h.index.find(srt);
      int u;
      if (it == h.index.end()) {
        u = (int)h.sets.size();
        h.index[srt] = u;
        h.sets.push_back(srt);
      } else {
        u = it->second;
      }
      (s == 0 ? en.u0 : en.u1) = u;
    }
    if (!zero) entries.push_back(en);
  }
  if (entries.empty()) return bad("every determinant vanishes identically");
  for (int s = 0; s < 2; ++s) {
    SpinHost& h = x->sp[s];
    h.ref = h.sets[0];
    std::vector<int> allx;
    for (auto& st : h.sets)
      for (int o : st)
        if (!std::binary_search(h.ref.begin(), h.ref.end(), o)) allx.push_back(o);
    std::sort(allx.begin(), allx.end());
    allx.erase(std::unique(allx.begin(), allx.end()), allx.end());
    h.porb = allx;
    for (auto& st : h.sets) {
      std::vector<int> J, ext;
      for (int j = 0; j < h.n; ++j)
        if (!std::binary_search(st.begin(), st.end(), h.ref[j])) J.push_back(j);
      for (int o : st)
        if (!std::binary_search(h.ref.begin(), h.ref.end(), o)) ext.push_back(o);
      if (J.size() > (size_t)kMaxExc)
        return bad("a spin determinant differs from its reference in more than 3 orbitals");
      std::vector<int> aligned = h.ref;
      for (size_t r = 0; r < J.size(); ++r) aligned[J[r]] = ext[r];
      h.sgn.push_back(parity_of(aligned) ? -1 : 1);
      int ui[8] = {(int)J.size(), 0, 0, 0, 0, 0, 0, 0};
      for (size_t r = 0; r < J.size(); ++r) {
        ui[1 + r] = J[r];
        ui[4 + r] = (int)(std::lower_bound(h.porb.begin(), h.porb.end(), ext[r]) - h.porb.begin());
      }
      h.uinfo.insert(h.uinfo.end(), ui, ui + 8);
    }
  }
  // determinant pairs and links
  std::map<std::pair<int, int>, int> pairidx;
  for (auto& en : entries) {
    double d = en.d * x->sp[0].sgn[en.u0] * x->sp[1].sgn[en.u1];
    auto key = std::make_pair(en.u0, en.u1);
    auto it = pairidx.find(key);
    int k;
    if (it == pairidx.end()) {
      k = (int)x->pair_up.size();
      pairidx[key] = k;
      x->pair_up.push_back(en.u0);
      x->pair_dn.push_back(en.u1);
      x->pair_links.emplace_back();
    } else {
      k = it->second;
    }
    bool merged = false;
    for (auto& pr : x->pair_links[k])
      if (pr.first == en.I) { pr.second += d; merged = true; }
    if (!merged) x->pair_links[k].push_back({en.I, d});
  }
  // structure CSR
  x->srow.assign(x->nstruct + 1, 0);
  for (int I = 0; I < x->nstruct; ++I) {
    x->srow[I] = (int)x->slc.size();
    for (size_t k = 0; k < x->pair_up.size(); ++k)
      for (auto& pr : x->pair_links[k])
        if (pr.first == I) {
          x->slu.push_back(x->pair_up[k]);
          x->slu.push_back(x->pair_dn[k]);
          x->slc.push_back(pr.second);
        }
  }
  x->srow[x->nstruct] = (int)x->slc.size();
  // per-spin CSR of the pairs holding each unique determinant
  for (int s = 0; s < 2; ++s) {
    SpinHost& h = x->sp[s];
    int nU = (int)h.sets.size();
    h.wrow.assign(nU + 1, 0);
    for (int u = 0; u < nU; ++u) {
      h.wrow[u] = (int)h.wother.size();
      for (size_t k = 0; k < x->pair_up.size(); ++k)
        if ((s == 0 ? x->pair_up[k] : x->pair_dn[k]) == u) h.wother.push_back(s == 0 ? x->pair_dn[k] : x->pair_up[k]);
    }
    h.wrow[nU] = (int)h.wother.size();
  }
  // Jastrow
  x->kappa = wfi->kappa;
  for (int k = 0; k < 8; ++k) x->ee[k] = wfi->ee[k];
  x->en.assign(wfi->en, wfi->en + 6 * x->nnuc);
  if (wfi->een) x->een.assign(wfi->een, wfi->een + (size_t)kEenTerms * x->nnuc);

  // ---- layouts ----
  DevWF& wf = x->wf;
  wf.N = x->N; wf.nup = x->nup; wf.ndn = x->ndn; wf.nnuc = x->nnuc; wf.nshell = x->nshell;
  wf.M = x->M; wf.Mpad = x->Mpad; wf.norb = x->norb; wf.nop = x->nop; wf.nstruct = x->nstruct;
  wf.precision = opt ? opt->precision : VBQMC_FP64;
  if (wf.precision < 0 || wf.precision > 3) return bad("unknown precision");
  // the mixed form: FP32 trial rows, everything else (including the rows of
  // the local energy and of the per-step refresh) FP64
  wf.trial_prec = wf.precision == VBQMC_MIXED ? VBQMC_FP32 : wf.precision;
  wf.refresh_each_step = wf.precision == VBQMC_MIXED ? 1 : 0;
  if (wf.precision == VBQMC_MIXED) wf.precision = VBQMC_FP64;
  wf.refresh_every = opt && opt->refresh_every > 0 ? opt->refresh_every : 32;
  wf.kappa = x->kappa;
  double vnn = 0;
  for (int a = 0; a < x->nnuc; ++a)
    for (int b = a + 1; b < x->nnuc; ++b) {
      double dx = x->nuc[4 * a] - x->nuc[4 * b], dy = x->nuc[4 * a + 1] - x->nuc[4 * b + 1],
             dz = x->nuc[4 * a + 2] - x->nuc[4 * b + 2];
      vnn += x->nuc[4 * a + 3] * x->nuc[4 * b + 3] / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  wf.vnn = vnn;
  wf.nprim = (int)x->pexp.size();
  wf.nlinks = (int)x->slc.size();
  for (int s = 0; s < 2; ++s) wf.nwl[s] = (int)x->sp[s].wother.size();
  // threads per walker: one wave for small systems, more waves as the
  // electron count and orbital tiles grow
  x->nt = 64;
  if (x->nop > 16 || x->N > 24) x->nt = 128;
  if (x->nop > 32 || x->N > 48) x->nt = 256;

  int nPm = std::max(x->sp[0].porb.size(), x->sp[1].porb.size());
  int nUm = std::max(x->sp[0].sets.size(), x->sp[1].sets.size());
  // walker record
  int o = 0;
  auto rec = [&](int n) { int r = o; o += (n + 1) / 2 * 2; return r; };
  wf.r_R = rec(3 * x->N);
  for (int s = 0; s < 2; ++s) wf.r_B[s] = rec(x->sp[s].n * x->sp[s].n);
  for (int s = 0; s < 2; ++s) wf.r_T[s] = rec(x->sp[s].n * (int)x->sp[s].porb.size());
  wf.r_sc = rec(8);
  wf.r_RW = rec(2 * (int)(x->sp[0].sets.size() + x->sp[1].sets.size()) + 1);
  wf.hot_len = o;
  // gradient cache of the DMC kernel, or the per-electron local-energy terms
  // and structure ratios of the batched local energy
  wf.r_gc = rec(std::max(3 * x->N * x->nop, 4 * x->N + x->nstruct));
  // value rows of the walker-resident DMC kernel (its gradient rows use r_gc)
  wf.dw_width = 1;
  for (int s = 0; s < 2; ++s) wf.dw_width = std::max(wf.dw_width, x->sp[s].n + (int)x->sp[s].porb.size());
  wf.r_vc = rec(x->N * wf.dw_width);
  wf.dw_xe = 0;
  for (int s = 0; s < 2; ++s)
    for (size_t u = 0; u < x->sp[s].sets.size(); ++u) wf.dw_xe = std::max(wf.dw_xe, x->sp[s].uinfo[8 * u]);
  wf.r_bk = rec(wf.hot_len);
  wf.rec_len = (o + 31) / 32 * 32;
  // LDS: constant tables, walker state, scratch (offsets in doubles, each
  // region 16-byte aligned; int tables use half a double per entry)
  o = 0;
  auto lds = [&](int n) { int r = o; o += (std::max(n, 1) + 1) / 2 * 2; return r; };
  auto ilds = [&](int n) { return lds((n + 1) / 2); };
  wf.l_fn = ilds(2 * x->Mpad);
  wf.l_sh = ilds(8 * x->nshell);
  wf.l_pe = lds(wf.nprim);
  wf.l_pc = lds(wf.nprim);
  wf.l_etab = lds(64);
  wf.l_nuc = lds(4 * x->nnuc);
  wf.l_en = lds(6 * x->nnuc);
  for (int s = 0; s < 2; ++s) {
    SpinHost& h = x->sp[s];
    wf.l_ref[s] = ilds((int)h.ref.size());
    wf.l_porb[s] = ilds((int)h.porb.size());
    wf.l_ui[s] = ilds((int)h.uinfo.size());
    wf.l_wrow[s] = ilds((int)h.wrow.size());
    wf.l_woth[s] = ilds((int)h.wother.size());
    wf.l_wcoef[s] = lds((int)h.wother.size());
  }
  wf.l_srow = ilds((int)x->srow.size());
  wf.l_slu = ilds((int)x->slu.size());
  wf.l_slc = lds((int)x->slc.size());
  wf.rsched_len = x->rsched_len;
  wf.rsched_sto = 0;
  for (int s = 0; s < x->nshell; ++s) wf.rsched_sto |= x->shtab[8 * s + 1] == 1;
  // the radial schedule and the primitive-to-shell map close the table
  // image: a layout stages the prefix it needs (the row kernel up to the
  // schedule, the sweeps and the tile kernel only the tables before it)
  wf.l_rsched = ilds((int)x->rsched.size());
  wf.l_rsched8 = wf.l_rsched + x->rsched8_off / 2;
  wf.rsched_len8 = x->rsched_len8;
  wf.l_psh = ilds(wf.nprim);
  int lam_elems = x->Mpad * x->nop;
  int lam_doubles = wf.precision == 0 ? lam_elems : (wf.precision == 1 ? (lam_elems + 1) / 2 : (lam_elems + 3) / 4);
  // orbital coefficients go to LDS when they take at most 16 KiB
  wf.lam_in_lds = lam_doubles * 8 <= 16384 ? 1 : 0;
  wf.l_lam = wf.lam_in_lds ? lds(lam_doubles) : 0;
  const int tables_end = o;
  wf.timg_len = tables_end;
  // regions used by every walker kernel
  wf.l_R = lds(std::max(3 * x->N, 3 * kGroup));
  wf.l_sc = lds(SC_COUNT);
  wf.l_red = lds(2 * kRedSlots);  // (the adjoint's 512-thread reductions of 12 values)
  int nmax = std::max(x->nup, x->ndn);
  wf.l_ipiv = ilds(nmax);
  wf.l_f = lds(nmax);
  // walker state and move scratch (every walker kernel)
  for (int s = 0; s < 2; ++s) {
    int n = x->sp[s].n, nP = (int)x->sp[s].porb.size();
    wf.l_B[s] = lds(n * n);
    wf.l_T[s] = lds(n * nP);
    wf.l_PP[s] = lds(n * nP);
    wf.l_Ru[s] = lds((int)x->sp[s].sets.size());
    wf.l_Wu[s] = lds((int)x->sp[s].sets.size());
  }
  wf.l_Qu = lds(nUm);
  wf.l_y = lds(nPm + 1);
  wf.l_bcol = lds(nmax);
  wf.l_z = lds(2 * nmax);
  // electron-tile regions of the MFMA passes; the primitive terms of a point
  // evaluation share this space (the two are never live at the same time)
  const int tile0 = o;
  wf.l_disp = lds(kGroup * (4 * x->nnuc + 1));
  wf.l_gtab = lds(kGroup * ((3 * x->nshell) | 1));
  wf.l_Phi = lds(kGroup * x->nop);
  const int tile_end = o;
  o = tile0;
  wf.l_pt = lds(2 * wf.nprim);
  o = std::max(o, tile_end);
  // fused walker kernels: point evaluations, local energy, overlaps
  wf.l_part = lds(std::max(x->nt, 4 * x->nop));
  wf.l_chi = lds(4 * x->Mpad);
  wf.l_v = lds(4 * x->nop);
  wf.l_yb = lds(kGroup * (nPm + 1));
  wf.l_sij = lds(x->nstruct * x->nstruct);
  wf.l_ratio = lds(x->nstruct);
  wf.l_gU = lds(3 * x->N);
  wf.l_lU = lds(x->N);
  wf.l_gD = lds(3 * x->N);
  wf.l_lD = lds(x->N);
  const int full_end = o;
  // adjoint-kernel regions
  o = full_end;
  wf.l_aPhi = lds(5 * x->N * x->nop);
  wf.l_aG0 = lds(x->N * x->nop);
  wf.l_aG = lds(x->N * x->nop);
  wf.l_aA = lds(nmax * nmax);
  wf.l_aP = lds(nmax * nmax);
  wf.l_aM = lds(nmax * nmax);
  wf.l_aU[0] = lds(5 * (int)x->sp[0].sets.size());
  wf.l_aU[1] = lds(5 * (int)x->sp[1].sets.size());
  wf.l_aBS = lds(nmax * nmax);
  wf.l_aT = lds(nmax * nPm);
  wf.l_aXi = lds(nmax * nPm);
  wf.l_aBXi = lds(nmax * nPm);
  wf.l_aW = lds(3 * nPm * nmax);
  wf.l_aV[0] = lds(18 * (int)x->sp[0].sets.size());
  wf.l_aV[1] = lds(18 * (int)x->sp[1].sets.size());
  wf.lds_adj_doubles = o;
  o = full_end;
  wf.lds_doubles = o;
  wf.lds_sweep_doubles = sweep_layout(x).lds_sweep_doubles;
  {
    DevWF a = aux_layout(x);
    wf.lds_finish_doubles = a.lds_finish_doubles;
    wf.lds_tile_doubles = a.lds_tile_doubles;
  }

  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) { delete x; return VBQMC_EHIP; }
  hipDeviceProp_t prop;
  he = hipGetDeviceProperties(&prop, dev);
  if (he != hipSuccess) { delete x; return VBQMC_EHIP; }
  x->lds_limit = (int)prop.sharedMemPerBlock;
  x->dev = dev;
  he = scratch_address(dev, &x->scratch);
  if (he != hipSuccess) {
    std::fprintf(stderr, "vbqmc_create: no address for the scratch array: %s\n", hipGetErrorString(he));
    delete x;
    return VBQMC_EHIP;
  }
  // the adjoint keeps each spin's first-pass B, B S, T and B Xi for its
  // second pass when they fit the LDS beside its own regions and do not
  // take a second resident workgroup per CU away (else the second pass
  // recomputes them)
  {
    int need[2], tot = 0;
    for (int s = 0; s < 2; ++s) {
      const int n = x->sp[s].n, nP = (int)x->sp[s].porb.size();
      // B, B S, T, B Xi, then the pivot column and pivots of its inversion
      need[s] = (2 * n * n + 2 * n * nP + n + (n + 1) / 2 + 1) / 2 * 2;
      tot += need[s];
    }
    wf.adj_save = 0;
    wf.l_aSave[0] = wf.l_aSave[1] = 0;
    const size_t lim = (size_t)x->lds_limit, before = (size_t)wf.lds_adj_doubles * 8,
                 after = (size_t)(wf.lds_adj_doubles + tot) * 8;
    if (after <= lim && (2 * before > lim || 2 * after <= lim)) {
      wf.adj_save = 1;
      wf.l_aSave[0] = wf.lds_adj_doubles;
      wf.l_aSave[1] = wf.lds_adj_doubles + need[0];
      wf.lds_adj_doubles += tot;
    }
  }
  if ((size_t)wf.lds_doubles * 8 > (size_t)x->lds_limit) {
    char b[160];
    std::snprintf(b, sizeof b, "system needs %d bytes of LDS per walker, device allows %d", wf.lds_doubles * 8,
                  x->lds_limit);
    return bad(b);
  }
  // lanes per walker of the single-electron sweep
  {
    const int req = opt ? opt->walker_lanes : 0;
    auto fits = [&](int G) {
      return (size_t)sweepg_layout(x, G).lds_sweepg_doubles * 8 <= (size_t)x->lds_limit;
    };
    const int nmax = std::max(x->nup, x->ndn);
    if (req == 16 || req == 32) {
      if (!fits(req)) return bad("walker_lanes: the walkers of one wavefront do not fit in LDS");
      x->sweep_g = req;
    } else if (req == 64) {
      x->sweep_g = 64;
    } else if (req == 0) {
      // two walkers per wavefront (measured best for 9 and 20 electrons per
      // spin); a workgroup per walker when that does not fit LDS
      x->sweep_g = nmax <= 32 && fits(32) ? 32 : 64;
    } else {
      return bad("walker_lanes must be 0, 16, 32 or 64");
    }
    if (x->sweep_g < 64) wf.lds_sweepg_doubles = sweepg_layout(x, x->sweep_g).lds_sweepg_doubles;
  }
  // kernel of single-electron VMC steps: with no lane count asked for, the
  // row kernel when the system fits it, else the walker-resident kernel when
  // it fits that; else the sweep + local-energy kernels
  // (f_een: single-electron moves and DMC steps only on the walker-resident
  // kernel; without a fit the calls report EINVAL)
  const bool een = !x->een.empty();
  if (een && wf.precision != VBQMC_FP64) return bad("f_een: the FP64 form only");
  {
    const int req = opt ? opt->step_kernel : 0;
    const int lanes = opt ? opt->walker_lanes : 0;
    if (een && (req == 1 || req == 2))
      return bad("f_een: single-electron VMC runs on the walker-resident kernel only (step_kernel 0 or 3)");
    if (req == 2) {
      if (!rows_fit(x)) return bad("step_kernel 2: the system does not fit the row kernel");
      x->step_kernel = 2;
    } else if (req == 3) {
      if (!dmcw_fit(x)) return bad("step_kernel 3: the system does not fit the walker-resident kernel");
      x->step_kernel = 3;
    } else if (req == 1) {
      x->step_kernel = 1;
    } else if (req == 0) {
      if (een) x->step_kernel = dmcw_fit(x) ? 3 : 1;
      else x->step_kernel = lanes != 0 ? 1 : rows_fit(x) ? 2 : dmcw_fit(x) ? 3 : 1;
    } else {
      return bad("step_kernel must be 0, 1, 2 or 3");
    }
    if (x->step_kernel == 2) wf.lds_rows_doubles = rows_layout(x).lds_rows_doubles;
  }
  // kernel of DMC steps: electron-major launches when fewer than four walkers
  // fit a CU in the one-workgroup-per-walker kernel, else that kernel
  {
    const int req = opt ? opt->dmc_kernel : 0;
    if (een && (req == 1 || req == 2))
      return bad("f_een: DMC runs on the walker-resident kernel only (dmc_kernel 0 or 3)");
    if (req == 2) {
      if (!dmcb_fit(x)) return bad("dmc_kernel 2: the system does not fit the electron-major DMC kernels");
      x->dmc_kernel = 2;
    } else if (req == 1) {
      x->dmc_kernel = 1;
    } else if (req == 3) {
      if (!dmcw_fit(x)) return bad("dmc_kernel 3: the system does not fit the walker-resident DMC kernel");
      x->dmc_kernel = 3;
    } else if (req == 0) {
      if (dmcw_fit(x)) x->dmc_kernel = 3;
      else if (een) x->dmc_kernel = 1;
      else x->dmc_kernel = (size_t)wf.lds_doubles * 8 > 40960 && dmcb_fit(x) ? 2 : 1;
    } else {
      return bad("dmc_kernel must be 0, 1, 2 or 3");
    }
  }

  // ---- device tables ----
  size_t bytes = 0;
  auto add = [&](size_t n, size_t sz) { bytes += arena_bytes_for(n, sz); };
  add(x->nuc.size(), 8); add(x->en.size(), 8); add(x->een.size(), 8); add(x->shtab.size(), 4);
  add(x->pexp.size(), 8); add(x->pcoef.size(), 8); add(x->pshell.size(), 4); add(x->fnmap.size(), 4);
  add((size_t)x->Mpad * x->nop, 8); add((size_t)x->Mpad * x->nop, 4); add((size_t)x->Mpad * x->nop, 2);
  for (int s = 0; s < 2; ++s) {
    SpinHost& h = x->sp[s];
    add(h.ref.size(), 4); add(h.porb.size(), 4); add(h.uinfo.size(), 4); add(h.wrow.size(), 4);
    add(h.wother.size(), 4); add(h.wother.size(), 8); add((size_t)x->nop, 4);
  }
  add(x->dw_rs.size(), 4);
  add(x->srow.size(), 4); add(x->slu.size(), 4); add(x->slc.size(), 8); add(sizeof(DevWF), 1); add(sizeof(DevWF), 1);
  add(sizeof(DevWF), 1); add(sizeof(DevWF), 1); add(sizeof(DevWF), 1); add(sizeof(DevWF), 1); add(sizeof(DevWF), 1);
  add((size_t)wf.timg_len, 8);
  he = hipMalloc((void**)&x->dmem, bytes);
  if (he != hipSuccess) { delete x; return VBQMC_ENOMEM; }
  x->dbytes = bytes;
  char* p = x->dmem;
  auto up = [&](const void* src, size_t n, size_t sz, void* dst) {
    if (n && he == hipSuccess) he = hipMemcpy(dst, src, n * sz, hipMemcpyHostToDevice);
  };
  double* d_nuc = carve<double>(p, x->nuc.size()); up(x->nuc.data(), x->nuc.size(), 8, d_nuc);
  x->d_en = carve<double>(p, x->en.size());
  x->d_een = x->een.empty() ? nullptr : carve<double>(p, x->een.size());
  int* d_shtab = carve<int>(p, x->shtab.size()); up(x->shtab.data(), x->shtab.size(), 4, d_shtab);
  double* d_pexp = carve<double>(p, x->pexp.size()); up(x->pexp.data(), x->pexp.size(), 8, d_pexp);
  double* d_pcoef = carve<double>(p, x->pcoef.size()); up(x->pcoef.data(), x->pcoef.size(), 8, d_pcoef);
  int* d_pshell = carve<int>(p, x->pshell.size()); up(x->pshell.data(), x->pshell.size(), 4, d_pshell);
  int* d_fnmap = carve<int>(p, x->fnmap.size()); up(x->fnmap.data(), x->fnmap.size(), 4, d_fnmap);
  x->d_lamT = carve<double>(p, (size_t)x->Mpad * x->nop);
  x->d_lamT32 = carve<float>(p, (size_t)x->Mpad * x->nop);
  x->d_lamT16 = carve<uint16_t>(p, (size_t)x->Mpad * x->nop);
  for (int s = 0; s < 2; ++s) {
    SpinHost& h = x->sp[s];
    SpinTab& t = wf.sp[s];
    t.n = h.n; t.e0 = h.e0; t.nP = (int)h.porb.size(); t.nU = (int)h.sets.size();
    int* a = carve<int>(p, h.ref.size()); up(h.ref.data(), h.ref.size(), 4, a); t.ref = a;
    a = carve<int>(p, h.porb.size()); up(h.porb.data(), h.porb.size(), 4, a); t.porb = a;
    a = carve<int>(p, h.uinfo.size()); up(h.uinfo.data(), h.uinfo.size(), 4, a); t.uinfo = a;
    a = carve<int>(p, h.wrow.size()); up(h.wrow.data(), h.wrow.size(), 4, a); t.wrow = a;
    a = carve<int>(p, h.wother.size()); up(h.wother.data(), h.wother.size(), 4, a); t.wother = a;
    x->d_wcoef[s] = carve<double>(p, h.wother.size());
    t.wcoef = x->d_wcoef[s];
    std::vector<int> om(x->nop, -1);
    for (int j = 0; j < (int)h.ref.size(); ++j) om[h.ref[j]] = j;
    for (int q = 0; q < (int)h.porb.size(); ++q) om[h.porb[q]] = h.n + q;
    a = carve<int>(p, om.size()); up(om.data(), om.size(), 4, a); t.omap = a;
  }
  int* d_srow = carve<int>(p, x->srow.size()); up(x->srow.data(), x->srow.size(), 4, d_srow);
  int* d_slu = carve<int>(p, x->slu.size()); up(x->slu.data(), x->slu.size(), 4, d_slu);
  x->d_slc = carve<double>(p, x->slc.size());
  x->d_wf = (DevWF*)carve<char>(p, sizeof(DevWF));
  x->d_wf_aux = (DevWF*)carve<char>(p, sizeof(DevWF));
  x->d_wf_sweep = (DevWF*)carve<char>(p, sizeof(DevWF));
  x->d_wf_sweepg = (DevWF*)carve<char>(p, sizeof(DevWF));
  x->d_wf_rows = (DevWF*)carve<char>(p, sizeof(DevWF));
  x->d_wf_dmcb = (DevWF*)carve<char>(p, sizeof(DevWF));
  x->d_wf_dmcw = (DevWF*)carve<char>(p, sizeof(DevWF));
  x->d_timg = carve<double>(p, (size_t)wf.timg_len);
  {
    unsigned* a = carve<unsigned>(p, x->dw_rs.size());
    up(x->dw_rs.data(), x->dw_rs.size(), 4, a);
    wf.dw_rs_g = a;
  }
  if (he != hipSuccess) { hipFree(x->dmem); delete x; return VBQMC_EHIP; }
  wf.nuc = d_nuc; wf.en = x->d_en; wf.shtab = d_shtab; wf.pexp = d_pexp;
  wf.neen = x->een.empty() ? 0 : kEenTerms;
  wf.een = x->d_een;
  wf.pcoef = d_pcoef; wf.pshell = d_pshell; wf.fnmap = d_fnmap; wf.lamT = x->d_lamT; wf.lamT32 = x->d_lamT32; wf.lamT16 = x->d_lamT16;
  wf.srow = d_srow; wf.slu = d_slu; wf.slc = x->d_slc; wf.timg = x->d_timg;
  if (upload_lambda(x) || upload_coefficients(x)) {
    hipFree(x->dmem);
    delete x;
    return VBQMC_EHIP;
  }
  *out = x;
  return VBQMC_OK;
}

void vbqmc_destroy(vbqmc_ctx* ctx) {
  if (!ctx) return;
  if (ctx->dmem) (void)hipFree(ctx->dmem);
  if (ctx->d_ecp) (void)hipFree(ctx->d_ecp);
  delete ctx;
}

namespace {
// [c | lambda | b_anti, b_par, b3..b6 | a1..a6 per nucleus | f_een per nucleus]
int n_params(const vbqmc_ctx* x) {
  return x->nstruct + x->norb * x->M + 6 + 6 * x->nnuc + (int)x->een.size();
}
}  // namespace

int vbqmc_get_info(const vbqmc_ctx* x, vbqmc_info_t* o) {
  if (!x || !o) return VBQMC_EINVAL;
  o->n_electrons = x->N; o->n_up = x->nup; o->n_dn = x->ndn; o->n_nuclei = x->nnuc;
  o->n_basis = x->M; o->n_orbitals = x->norb; o->n_structures = x->nstruct;
  o->n_determinants = (int)x->pair_up.size();
  o->n_unique_up = (int)x->sp[0].sets.size();
  o->n_unique_dn = (int)x->sp[1].sets.size();
  o->n_table_up = (int)x->sp[0].porb.size();
  o->n_table_dn = (int)x->sp[1].porb.size();
  o->n_params = n_params(x);
  o->block_threads = x->nt;
  o->sweep_lanes = x->sweep_g;
  o->step_kernel = x->step_kernel;
  o->dmc_kernel = x->dmc_kernel;
  o->walker_state_bytes = (int64_t)x->wf.rec_len * 8;
  o->lds_bytes = (int64_t)x->wf.lds_doubles * 8;
  return VBQMC_OK;
}

int vbqmc_set_params(vbqmc_ctx* x, const double* p) {
  if (!x || !p) return VBQMC_EINVAL;
  // kernels still running on any stream may read the tables replaced below
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hipfail(x, e, "set_params: device synchronisation");
  int k = 0;
  for (int I = 0; I < x->nstruct; ++I) x->c[I] = p[k++];
  for (size_t q = 0; q < x->lam.size(); ++q) x->lam[q] = p[k++];
  x->ee[2] = p[k++];
  x->ee[3] = p[k++];
  for (int j = 4; j < 8; ++j) x->ee[j] = p[k++];
  for (int a = 0; a < x->nnuc; ++a)
    for (int j = 0; j < 6; ++j) x->en[6 * a + j] = p[k++];
  for (double& v : x->een) v = p[k++];
  if (upload_lambda(x)) return VBQMC_EHIP;
  if (upload_coefficients(x)) return VBQMC_EHIP;
  return VBQMC_OK;
}

int vbqmc_set_ecp(vbqmc_ctx* x, const vbqmc_ecp* ecp) {
  if (!x) return VBQMC_EINVAL;
  const int nc = ecp ? ecp->n_centers : 0;
  if (nc < 0 || nc > x->nnuc) return fail(x, VBQMC_EINVAL, "set_ecp: bad number of centres");
  if (nc && (x->wf.precision != VBQMC_FP64 || x->wf.trial_prec != VBQMC_FP64))
    return fail(x, VBQMC_EINVAL, "set_ecp: pseudopotentials need the FP64 precision form");
  if (nc && !x->een.empty()) return fail(x, VBQMC_EINVAL, "set_ecp: not available with f_een");
  if (nc && (!ecp->center || !ecp->n_channels || !ecp->r_cut || !ecp->n_terms || !ecp->terms))
    return fail(x, VBQMC_EINVAL, "set_ecp: arrays missing");
  std::vector<int> info(8 * (size_t)nc, 0);
  std::vector<double> rcut(nc), terms;
  std::vector<char> seen(x->nnuc, 0);
  int k = 0, t = 0;
  for (int c = 0; c < nc; ++c) {
    const int a = ecp->center[c], L = ecp->n_channels[c];
    if (a < 0 || a >= x->nnuc || seen[a]) return fail(x, VBQMC_EINVAL, "set_ecp: bad or repeated centre");
    seen[a] = 1;
    if (L < 0 || L > kEcpMaxL) return fail(x, VBQMC_EINVAL, "set_ecp: at most 4 nonlocal channels");
    if (!(ecp->r_cut[c] >= 0.0) || !std::isfinite(ecp->r_cut[c])) return fail(x, VBQMC_EINVAL, "set_ecp: bad r_cut");
    rcut[c] = ecp->r_cut[c];
    info[8 * c] = a;
    info[8 * c + 1] = L;
    info[8 * c + 2] = (int)(terms.size() / 3);
    for (int q = 0; q <= L; ++q) {
      const int nt = ecp->n_terms[k++];
      if (nt < 0 || nt > 64) return fail(x, VBQMC_EINVAL, "set_ecp: bad term count");
      for (int j = 0; j < nt; ++j, ++t) {
        const double cc = ecp->terms[3 * t], n = ecp->terms[3 * t + 1], al = ecp->terms[3 * t + 2];
        if (!std::isfinite(cc) || !(al >= 0.0) || !std::isfinite(al) || n != std::floor(n) || n < 0 || n > 6)
          return fail(x, VBQMC_EINVAL, "set_ecp: a term needs finite c, integer n in 0..6 and alpha >= 0");
        terms.insert(terms.end(), {cc, n, al});
      }
      info[8 * c + 3 + q] = (int)(terms.size() / 3);
    }
  }
  // kernels still running on any stream may read the tables replaced below
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hipfail(x, e, "set_ecp: device synchronisation");
  if (x->d_ecp) (void)hipFree(x->d_ecp);
  x->d_ecp = nullptr;
  x->ecp = DevEcp{};
  if (!nc) return VBQMC_OK;
  const size_t bi = info.size() * sizeof(int), br = rcut.size() * 8, bt = std::max<size_t>(terms.size(), 1) * 8;
  const size_t oi = 0, orc = (bi + 255) / 256 * 256, ot = orc + (br + 255) / 256 * 256;
  e = hipMalloc((void**)&x->d_ecp, ot + bt);
  if (e != hipSuccess) {
    x->d_ecp = nullptr;
    return fail(x, VBQMC_ENOMEM, "set_ecp: device allocation");
  }
  e = hipMemcpy(x->d_ecp + oi, info.data(), bi, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(x->d_ecp + orc, rcut.data(), br, hipMemcpyHostToDevice);
  if (e == hipSuccess && !terms.empty()) e = hipMemcpy(x->d_ecp + ot, terms.data(), terms.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(x->d_ecp);
    x->d_ecp = nullptr;
    return hipfail(x, e, "set_ecp: upload");
  }
  // scratch of the batched projection (12 points of one electron and centre)
  // beyond the walker kernels' LDS layout, when it fits the device's LDS
  const int K = kEcpPts, C = std::max(1, x->nt / K), nPm = std::max(1, std::max(x->wf.sp[0].nP, x->wf.sp[1].nP));
  const int scr = K * (4 + x->wf.Mpad + x->wf.nop + nPm + 3) + 3 * C * K;
  const bool fits = (size_t)(x->wf.lds_doubles + scr) * 8 <= (size_t)x->lds_limit;
  x->ecp = DevEcp{nc, (const int*)(x->d_ecp + oi), (const double*)(x->d_ecp + orc), (const double*)(x->d_ecp + ot),
                  fits ? x->wf.lds_doubles : -1, fits ? scr : 0, nPm};
  return VBQMC_OK;
}

int vbqmc_get_params(const vbqmc_ctx* x, double* p) {
  if (!x || !p) return VBQMC_EINVAL;
  int k = 0;
  for (int I = 0; I < x->nstruct; ++I) p[k++] = x->c[I];
  for (double v : x->lam) p[k++] = v;
  p[k++] = x->ee[2];
  p[k++] = x->ee[3];
  for (int j = 4; j < 8; ++j) p[k++] = x->ee[j];
  for (int a = 0; a < x->nnuc; ++a)
    for (int j = 0; j < 6; ++j) p[k++] = x->en[6 * a + j];
  for (double v : x->een) p[k++] = v;
  return VBQMC_OK;
}

int vbqmc_evaluate(vbqmc_ctx* x, int64_t W, const double* R, double* logabs, int32_t* sign, double* grad,
                   double* eloc, double* ratio, vbqmc_stream stream) {
  if (!x) return VBQMC_EINVAL;
  if (W < 0 || (W > 0 && (!R || !logabs || !sign))) return fail(x, VBQMC_EINVAL, "evaluate: bad arguments");
  if (W == 0) return VBQMC_OK;
  if (W > (int64_t)INT32_MAX) return fail(x, VBQMC_EINVAL, "evaluate: too many walkers");
  hipError_t e = launch_evaluate(x->wf, x->d_wf, x->nt, W, R, 3 * x->N, logabs, sign, grad, eloc, ratio, nullptr,
                                 x->ecp, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "evaluate");
}

int vbqmc_walkers_init(vbqmc_ctx* x, int64_t W, const double* R, void* state, vbqmc_stream stream) {
  if (!x || W < 0 || (W > 0 && (!R || !state))) return fail(x, VBQMC_EINVAL, "walkers_init: bad arguments");
  if (W == 0) return VBQMC_OK;
  if (W > (int64_t)INT32_MAX) return fail(x, VBQMC_EINVAL, "walkers_init: too many walkers");
  hipError_t e = launch_evaluate(x->wf, x->d_wf, x->nt, W, R, 3 * x->N, nullptr, nullptr, nullptr, nullptr, nullptr, (double*)state,
                                 x->ecp, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "walkers_init");
}

int vbqmc_walkers_positions(vbqmc_ctx* x, int64_t W, const void* state, double* R, vbqmc_stream stream) {
  if (!x || W < 0 || (W > 0 && (!R || !state))) return fail(x, VBQMC_EINVAL, "walkers_positions: bad arguments");
  if (W == 0) return VBQMC_OK;
  hipError_t e = launch_positions(x->wf, x->d_wf, W, (const double*)state, R, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "walkers_positions");
}

int vbqmc_walkers_eloc(vbqmc_ctx* x, int64_t W, const void* state, double* eloc, vbqmc_stream stream) {
  if (!x || W < 0 || (W > 0 && (!eloc || !state))) return fail(x, VBQMC_EINVAL, "walkers_eloc: bad arguments");
  if (W == 0) return VBQMC_OK;
  hipError_t e = launch_record_eloc(x->wf, x->d_wf, W, (const double*)state, eloc, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "walkers_eloc");
}

}  // extern "C"

namespace {
// the sweep + batched local-energy kernels fit the device's LDS
bool split_fits(const vbqmc_ctx* x) {
  return (size_t)std::max(x->wf.lds_sweep_doubles, x->wf.lds_tile_doubles) * 8 <= (size_t)x->lds_limit;
}
}  // namespace

extern "C" {

int vbqmc_vmc_sweep(vbqmc_ctx* x, void* state, int64_t W, uint64_t seed, uint64_t step, double step_size,
                    double* n_accept, vbqmc_stream stream) {
  if (!x || W < 0 || (W > 0 && (!state || !n_accept))) return fail(x, VBQMC_EINVAL, "vmc_sweep: bad arguments");
  if (!(step_size > 0) || !std::isfinite(step_size)) return fail(x, VBQMC_EINVAL, "vmc_sweep: bad step size");
  if (W > (int64_t)INT32_MAX) return fail(x, VBQMC_EINVAL, "vmc_sweep: too many walkers");
  if (!split_fits(x)) return fail(x, VBQMC_EINVAL, "vmc_sweep: system too large for the sweep kernels");
  if (!x->een.empty()) return fail(x, VBQMC_EINVAL, "vmc_sweep: not available with f_een");
  if (x->ecp.ncen) return fail(x, VBQMC_EINVAL, "vmc_sweep: not available with pseudopotentials");
  if (W == 0) return VBQMC_OK;
  hipError_t e = launch_vmc_split(x->wf, x->d_wf_sweep, x->d_wf_sweepg, x->sweep_g, x->d_wf_aux, x->nt, 1,
                                  (double*)state, W, 1, seed, step, step_size, nullptr, nullptr, n_accept, nullptr,
                                  nullptr, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "vmc_sweep");
}

int vbqmc_vmc_measure(vbqmc_ctx* x, void* state, int64_t W, const vbqmc_vmc_acc* acc, vbqmc_stream stream) {
  if (!x || !acc || W < 0 || (W > 0 && !state)) return fail(x, VBQMC_EINVAL, "vmc_measure: bad arguments");
  if (W > (int64_t)INT32_MAX) return fail(x, VBQMC_EINVAL, "vmc_measure: too many walkers");
  if (!split_fits(x)) return fail(x, VBQMC_EINVAL, "vmc_measure: system too large for the local-energy kernels");
  if (!x->een.empty()) return fail(x, VBQMC_EINVAL, "vmc_measure: not available with f_een");
  if (x->ecp.ncen) return fail(x, VBQMC_EINVAL, "vmc_measure: not available with pseudopotentials");
  if (W == 0) return VBQMC_OK;
  if (!acc->e_sum || !acc->e2_sum || !acc->e_last)
    return fail(x, VBQMC_EINVAL, "vmc_measure: accumulator pointers missing");
  hipError_t e = launch_vmc_split(x->wf, x->d_wf_sweep, x->d_wf_sweepg, x->sweep_g, x->d_wf_aux, x->nt, 2,
                                  (double*)state, W, 1, 0, 0, 1.0, acc->e_sum, acc->e2_sum, nullptr, acc->e_last,
                                  acc->sij_sum, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "vmc_measure");
}

int vbqmc_vmc_advance(vbqmc_ctx* x, void* state, int64_t W, int32_t n_steps, uint64_t seed, uint64_t step0,
                      double step_size, int32_t all_electron, const vbqmc_vmc_acc* acc, vbqmc_stream stream) {
  if (!x || !acc || W < 0 || n_steps < 0 || (W > 0 && !state)) return fail(x, VBQMC_EINVAL, "vmc: bad arguments");
  if (!(step_size > 0) || !std::isfinite(step_size)) return fail(x, VBQMC_EINVAL, "vmc: bad step size");
  if (W == 0 || n_steps == 0) return VBQMC_OK;
  if (!acc->e_sum || !acc->e2_sum || !acc->n_accept || !acc->e_last)
    return fail(x, VBQMC_EINVAL, "vmc: accumulator pointers missing");
  if (W > (int64_t)INT32_MAX) return fail(x, VBQMC_EINVAL, "vmc: too many walkers");
  if (!all_electron && !x->een.empty() && x->step_kernel != 3)
    return fail(x, VBQMC_EINVAL,
                "vmc: with f_een, single-electron moves need the walker-resident kernel (a system that fits it)");
  // with pseudopotentials every step runs on the one-workgroup-per-walker kernel
  if (!all_electron && x->step_kernel == 2 && !x->ecp.ncen) {
    // single-electron moves and E_L of every step in one row-kernel launch
    hipError_t e = launch_vmc_rows(x->wf, x->d_wf_rows, (double*)state, W, n_steps, seed, step0, step_size,
                                   acc->e_sum, acc->e2_sum, acc->n_accept, acc->e_last, acc->sij_sum,
                                   (hipStream_t)stream);
    return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "vmc");
  }
  if (!all_electron && x->step_kernel == 3 && (!acc->sij_sum || x->nstruct <= 256) && !x->ecp.ncen) {
    // rebuild the records (orbital-row caches at every electron), then one
    // walker-resident launch per step: moves, refresh and E_L
    DwVmc vm{step_size, W, acc->e_sum, acc->e2_sum, acc->n_accept, acc->e_last, acc->sij_sum};
    const DevWF lay = dmcw_layout(x);
    hipError_t e = launch_dmcw_vmc(lay, x->d_wf_dmcw, (double*)state, seed, 0, 1, vm, (hipStream_t)stream);
    for (int st = 0; st < n_steps && e == hipSuccess; ++st)
      e = launch_dmcw_vmc(lay, x->d_wf_dmcw, (double*)state, seed, (uint32_t)(step0 + st), 0, vm,
                          (hipStream_t)stream);
    return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "vmc");
  }
  if (!all_electron && split_fits(x) && !x->ecp.ncen) {
    // single-electron moves: walker-resident sweep + batched local energy
    hipError_t e = launch_vmc_split(x->wf, x->d_wf_sweep, x->d_wf_sweepg, x->sweep_g, x->d_wf_aux, x->nt, 3,
                                    (double*)state, W, n_steps, seed, step0, step_size, acc->e_sum, acc->e2_sum,
                                    acc->n_accept, acc->e_last, acc->sij_sum, (hipStream_t)stream);
    return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "vmc");
  }
  hipError_t e = launch_vmc(x->wf, x->d_wf, x->nt, (double*)state, W, n_steps, seed, step0, step_size, all_electron ? 1 : 0,
                            acc->e_sum, acc->e2_sum, acc->n_accept, acc->e_last, acc->sij_sum, x->ecp,
                            (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "vmc");
}

// DMC workspace: ctrl (8 doubles) | w, we, wc, ub [cap] | nacc [cap][3] | ncopy [cap] |
// offs [cap+1] | (electron-major kernels) P, V [cap][3], Vp [cap][4][nop], ek, ep [cap]
namespace {
size_t dmc_ws_base(int64_t cap) { return 64 + 7 * (size_t)cap * 8 + (size_t)cap * 4 + ((size_t)cap + 1) * 4; }
}  // namespace

int vbqmc_dmc_workspace_bytes(const vbqmc_ctx* x, int64_t cap, int32_t n_steps, size_t* bytes) {
  if (!x || !bytes || cap < 1) return VBQMC_EINVAL;
  (void)n_steps;
  size_t b = dmc_ws_base(cap) + 256;
  if (x->dmc_kernel == 2) b += (size_t)cap * (8 + 4 * (size_t)x->nop) * 8 + 256;
  *bytes = b;
  return VBQMC_OK;
}

namespace {
int dmc_advance_impl(vbqmc_ctx* x, void* states[2], int64_t* W_io, int64_t cap, int32_t n_steps, uint64_t seed,
                     uint64_t step0, double tau, double* e_trial_io, int64_t W_target, const vbqmc_dmc_log* lg,
                     void* ws, size_t ws_bytes, vbqmc_stream stream);
}  // namespace

int vbqmc_dmc_advance(vbqmc_ctx* x, void* states[2], int64_t* W_io, int64_t cap, int32_t n_steps, uint64_t seed,
                      uint64_t step0, double tau, double* e_trial_io, int64_t W_target, const vbqmc_dmc_log* lg,
                      void* ws, size_t ws_bytes, vbqmc_stream stream) {
  return dmc_advance_impl(x, states, W_io, cap, n_steps, seed, step0, tau, e_trial_io, W_target, lg, ws, ws_bytes,
                          stream);
}

int vbqmc_dmc_advance_noalloc(vbqmc_ctx* x, void* states[2], int64_t* W_io, int64_t cap, int32_t n_steps,
                              uint64_t seed, uint64_t step0, double tau, double* e_trial_io, int64_t W_target,
                              const vbqmc_dmc_log* lg, vbqmc_stream stream) {
  if (!x) return VBQMC_EINVAL;
  if (cap < 1) return fail(x, VBQMC_EINVAL, "dmc_noalloc: bad capacity");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hipfail(x, e, "dmc_noalloc: current device");
  if (dev != x->dev) return fail(x, VBQMC_EINVAL, "dmc_noalloc: the current device is not the context's device");
  size_t need = 0;
  vbqmc_dmc_workspace_bytes(x, cap, n_steps, &need);
  if (need > kNoAllocScratchBytes) {
    char b[200];
    std::snprintf(b, sizeof b,
                  "dmc_noalloc: capacity %lld needs %zu bytes of scratch, above the fixed %zu bytes; lower the "
                  "capacity or pass a workspace to vbqmc_dmc_advance",
                  (long long)cap, need, kNoAllocScratchBytes);
    return fail(x, VBQMC_EWORKSPACE, b);
  }
  if (lg && lg->step_ms) return fail(x, VBQMC_EINVAL, "dmc_noalloc: step timing (log->step_ms) is not available");
  return dmc_advance_impl(x, states, W_io, cap, n_steps, seed, step0, tau, e_trial_io, W_target, lg, x->scratch,
                          kNoAllocScratchBytes, stream);
}

namespace {
int dmc_advance_impl(vbqmc_ctx* x, void* states[2], int64_t* W_io, int64_t cap, int32_t n_steps, uint64_t seed,
                     uint64_t step0, double tau, double* e_trial_io, int64_t W_target, const vbqmc_dmc_log* lg,
                     void* ws, size_t ws_bytes, vbqmc_stream stream) {
  if (!x || !states || !states[0] || !states[1] || !W_io || !e_trial_io || !lg || !ws)
    return fail(x, VBQMC_EINVAL, "dmc: bad arguments");
  if (!lg->pop || !lg->wsum || !lg->wesum || !lg->etrial || !lg->n_accept || !lg->n_prop)
    return fail(x, VBQMC_EINVAL, "dmc: log pointers missing");
  // with pseudopotentials every step runs on the one-workgroup-per-walker kernel
  const int dk = x->ecp.ncen ? 1 : x->dmc_kernel;
  int64_t W = *W_io;
  if (!x->een.empty() && x->dmc_kernel != 3)
    return fail(x, VBQMC_EINVAL, "dmc: with f_een, DMC needs the walker-resident kernel (a system that fits it)");
  if (W < 1 || W > cap || cap > (int64_t)INT32_MAX || W_target < 1 || !(tau > 0) || n_steps < 0)
    return fail(x, VBQMC_EINVAL, "dmc: bad population, capacity or time step");
  size_t need = 0;
  vbqmc_dmc_workspace_bytes(x, cap, n_steps, &need);
  if (ws_bytes < need) return fail(x, VBQMC_EWORKSPACE, "dmc: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  char* p = (char*)ws;
  double* ctrl = (double*)p; p += 64;
  DmcBranch br;
  br.w = (double*)p; p += cap * 8;
  br.we = (double*)p; p += cap * 8;
  br.wc = (double*)p; p += cap * 8;
  br.ub = (double*)p; p += cap * 8;
  // per walker: accepted moves, sum of the proposals' and of the accepted
  // moves' squared displacements
  double* nacc = (double*)p; p += 3 * cap * 8;
  br.nc = (int*)p; p += cap * 4;
  int* offs = (int*)p;
  double h[DC_COUNT] = {0};
  h[DC_W] = (double)W;
  h[DC_ET] = *e_trial_io;
  hipError_t e = hipMemcpyAsync(ctrl, h, sizeof h, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hipfail(x, e, "dmc: control upload");
  double* cur = (double*)states[0];
  double* oth = (double*)states[1];
  // electron-major scratch (8-byte aligned after the integer arrays)
  char* pb = (char*)ws + ((dmc_ws_base(cap) + 255) & ~(size_t)255);
  double* Pw = (double*)pb;
  double* Vw = Pw + 3 * cap;
  double* Vpw = Vw + 3 * cap;
  double* ekw = Vpw + 4 * (size_t)x->nop * cap;
  double* epw = ekw + cap;
  // rebuild every record from its positions (fresh inverses, local energy and
  // the orbital-gradient rows the drift of the first moves reads)
  if (dk == 3)
    e = launch_dmcw(dmcw_layout(x), x->d_wf_dmcw, cur, ctrl, cap, seed, 0, tau, br, nacc, 1, s);
  else if (dk == 2)
    e = launch_dmcb_finish(x->wf, x->d_wf, x->d_wf_dmcb, (size_t)dmcb_layout(x).lds_tile_doubles * 8, cur, ctrl, cap,
                           seed, 0, tau, Vpw, ekw, epw, br, 1, s);
  else
    e = launch_evaluate(x->wf, x->d_wf, x->nt, W, cur + x->wf.r_R, x->wf.rec_len, nullptr, nullptr, nullptr,
                        nullptr, nullptr, cur, x->ecp, s);
  if (e != hipSuccess) return hipfail(x, e, "dmc: record refresh");
  // optional per-step timing of the move-and-energy kernels
  std::vector<hipEvent_t> ev;
  auto drop_events = [&]() {
    for (hipEvent_t v : ev) hipEventDestroy(v);
    ev.clear();
  };
  if (lg->step_ms) {
    ev.resize(2 * (size_t)n_steps, nullptr);
    for (size_t k = 0; k < ev.size() && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
    if (e != hipSuccess) {
      drop_events();
      return hipfail(x, e, "dmc: timing events");
    }
  }
  for (int st = 0; st < n_steps; ++st) {
    uint32_t step = (uint32_t)(step0 + st);
    if (!ev.empty()) e = hipEventRecord(ev[2 * st], s);
    if (e != hipSuccess) {
      drop_events();
      return hipfail(x, e, "dmc: timing event");
    }
    if (dk == 3) {
      e = launch_dmcw(dmcw_layout(x), x->d_wf_dmcw, cur, ctrl, cap, seed, step, tau, br, nacc, 0, s);
    } else if (dk == 2) {
      const size_t rows_lds = (size_t)dmcb_layout(x).lds_tile_doubles * 8;
      for (int i = 0; i < x->N && e == hipSuccess; ++i)
        e = launch_dmcb_move(x->wf, x->d_wf, x->d_wf_dmcb, rows_lds, cur, ctrl, cap, i, seed, step, tau, Pw, Vw,
                             Vpw, nacc, s);
      if (e == hipSuccess)
        e = launch_dmcb_finish(x->wf, x->d_wf, x->d_wf_dmcb, rows_lds, cur, ctrl, cap, seed, step, tau, Vpw, ekw,
                               epw, br, 0, s);
    } else {
      e = launch_dmc_step(x->wf, x->d_wf, x->nt, cur, ctrl, cap, seed, step, tau, br, nacc, x->ecp, s);
    }
    if (e == hipSuccess && !ev.empty()) e = hipEventRecord(ev[2 * st + 1], s);
    if (e != hipSuccess) {
      drop_events();
      return hipfail(x, e, "dmc: step");
    }
    e = launch_dmc_tail(ctrl, br, nacc, offs, cap, x->N, st, tau, (double)W_target, lg->pop, lg->wsum,
                        lg->wesum, lg->wcsum, lg->etrial, lg->n_accept, lg->n_prop, lg->dr2_acc, lg->dr2_prop, cur,
                        oth, x->wf.rec_len, s);
    if (e != hipSuccess) {
      drop_events();
      return hipfail(x, e, "dmc: branching");
    }
    std::swap(cur, oth);
  }
  e = hipMemcpyAsync(h, ctrl, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (int st = 0; st < n_steps && e == hipSuccess && !ev.empty(); ++st) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev[2 * st], ev[2 * st + 1]);
    lg->step_ms[st] = ms;
  }
  drop_events();
  if (e != hipSuccess) return hipfail(x, e, "dmc: control download");
  if (h[DC_ERR] != 0.0) {
    // the failing step's branching did not run: its walkers (after that
    // step's moves) are in the buffer that step worked on
    int64_t Wl = (int64_t)h[DC_W];
    double* held = (double*)states[((int64_t)h[DC_ERRSTEP]) & 1];
    if (held != (double*)states[0]) {
      e = launch_copy_records(held, (double*)states[0], Wl * x->wf.rec_len, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    *W_io = Wl;
    *e_trial_io = h[DC_ET];
    return fail(x, h[DC_ERR] == 1.0 ? VBQMC_ENONFINITE : VBQMC_EPOPULATION,
                h[DC_ERR] == 1.0 ? "dmc: a walker became singular or non-finite"
                                 : "dmc: population empty or above capacity");
  }
  int64_t Wn = (int64_t)h[DC_W];
  if (cur != (double*)states[0]) {
    e = launch_copy_records(cur, (double*)states[0], Wn * x->wf.rec_len, s);
    if (e != hipSuccess) return hipfail(x, e, "dmc: final copy");
  }
  *W_io = Wn;
  *e_trial_io = h[DC_ET];
  return VBQMC_OK;
}
}  // namespace

int vbqmc_param_grad_workspace_bytes(const vbqmc_ctx* x, int64_t W, size_t* bytes) {
  if (!x || !bytes || W < 0) return VBQMC_EINVAL;
  *bytes = param_grad_ws_doubles(x->wf, W) * 8;
  return VBQMC_OK;
}

int vbqmc_param_grad(vbqmc_ctx* x, int64_t W, const double* R, double* dlogpsi, double* deloc, void* ws,
                     size_t ws_bytes, vbqmc_stream stream) {
  if (!x || W < 0 || (W > 0 && (!R || !dlogpsi || !deloc))) return fail(x, VBQMC_EINVAL, "param_grad: bad arguments");
  if (x->ecp.ncen) return fail(x, VBQMC_EINVAL, "param_grad: not available with pseudopotentials");
  if (W == 0) return VBQMC_OK;
  size_t need = param_grad_ws_doubles(x->wf, W) * 8;
  if (need && (!ws || ws_bytes < need)) return fail(x, VBQMC_EWORKSPACE, "param_grad: workspace too small");
  if ((size_t)x->wf.lds_adj_doubles * 8 > (size_t)x->lds_limit)
    return fail(x, VBQMC_EINVAL, "param_grad: system too large for the adjoint kernel's LDS budget");
  if (W > (int64_t)INT32_MAX) return fail(x, VBQMC_EINVAL, "param_grad: too many walkers");
  // a workgroup whose LDS leaves no room for a second one on the CU runs
  // with four wavefronts, one per SIMD
  const int nt = (size_t)x->wf.lds_adj_doubles * 8 * 2 > (size_t)x->lds_limit
                     ? (x->wf.precision == VBQMC_FP64 && x->een.empty() ? 512 : 256)
                     : x->nt;
  hipError_t e = launch_param_grad(x->wf, x->d_wf, nt, W, R, dlogpsi, deloc, (double*)ws, need / 8, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "param_grad");
}

int vbqmc_reduce_walkers(vbqmc_ctx* x, int64_t W, int32_t K, const double* weights, const double* in, double* out,
                         vbqmc_stream stream) {
  if (!x || W < 0 || K < 0 || (K > 0 && (!in || !out))) return fail(x, VBQMC_EINVAL, "reduce: bad arguments");
  if (K == 0) return VBQMC_OK;
  hipError_t e = launch_reduce(W, K, weights, in, out, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "reduce");
}

// ---------------------------------------------------------------------------
// linear optimisation method: sample sums on the device, estimators and the
// step on the host
// ---------------------------------------------------------------------------
int vbqmc_lm_acc_doubles(int32_t P, int64_t* n) {
  if (P < 1 || !n) return VBQMC_EINVAL;
  *n = 3 * (int64_t)(P + 1) * (P + 1);
  return VBQMC_OK;
}

int vbqmc_lm_accumulate(vbqmc_ctx* x, int64_t W, const double* dlogpsi, const double* deloc, const double* eloc,
                        const double* weight, double* acc, vbqmc_stream stream) {
  if (!x || W < 0 || !acc || (W > 0 && (!dlogpsi || !deloc || !eloc)))
    return fail(x, VBQMC_EINVAL, "lm_accumulate: bad arguments");
  if (W == 0) return VBQMC_OK;
  const int P = n_params(x);
  hipError_t e = launch_lm_accumulate(P, W, dlogpsi, deloc, eloc, weight, acc, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "lm_accumulate");
}

int vbqmc_lm_accumulate_cols(int32_t P, int64_t W, const double* dlogpsi, const double* deloc, const double* eloc,
                             const double* weight, double* acc, vbqmc_stream stream) {
  if (P < 1 || W < 0 || !acc || (W > 0 && (!dlogpsi || !deloc || !eloc))) return VBQMC_EINVAL;
  if (W == 0) return VBQMC_OK;
  hipError_t e = launch_lm_accumulate(P, W, dlogpsi, deloc, eloc, weight, acc, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : VBQMC_EHIP;
}

int vbqmc_lm_estimators(int32_t P, const double* acc, double* e0, double* g_l, double* g_r, double* h_bar,
                        double* s_bar, double* var) {
  if (P < 1 || !acc || !e0 || !g_l || !g_r || !h_bar || !s_bar) return VBQMC_EINVAL;
  const int64_t P1 = P + 1;
  const double* S1 = acc;
  const double* H1 = acc + P1 * P1;
  const double* D1 = acc + 2 * P1 * P1;
  const double sw = S1[0];
  if (!(sw > 0)) return VBQMC_EINVAL;
  std::vector<double> mO(P), mOE(P), mD(P);
  const double mE = H1[0] / sw;
  for (int i = 0; i < P; ++i) {
    mO[i] = S1[i + 1] / sw;
    mOE[i] = H1[i + 1] / sw;
    mD[i] = D1[i + 1] / sw;
  }
  *e0 = mE;
  if (var) *var = D1[0] / sw - mE * mE;
  for (int i = 0; i < P; ++i) {
    g_l[i] = 2.0 * (mOE[i] - mO[i] * mE);
    g_r[i] = 2.0 * (mOE[i] - mO[i] * mE + mD[i]);
  }
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) {
      const double oo = S1[(i + 1) * P1 + j + 1] / sw, ooe = H1[(i + 1) * P1 + j + 1] / sw;
      const double od = D1[(i + 1) * P1 + j + 1] / sw;
      h_bar[(int64_t)i * P + j] = ooe - mO[i] * mOE[j] - mO[j] * mOE[i] + mO[i] * mO[j] * mE + od - mO[i] * mD[j];
      s_bar[(int64_t)i * P + j] = oo - mO[i] * mO[j];
    }
  return VBQMC_OK;
}

// LU with partial pivoting of the n x n row-major A in place (row swaps in
// piv); false if a pivot is exactly zero
static bool lu_factor(int n, std::vector<double>& A, std::vector<int>& piv) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      const double v = std::fabs(A[(size_t)r * n + k]);
      if (v > best) { best = v; p = r; }
    }
    piv[k] = p;
    if (!(best > 0)) return false;
    if (p != k)
      for (int c = 0; c < n; ++c) std::swap(A[(size_t)k * n + c], A[(size_t)p * n + c]);
    const double inv = 1.0 / A[(size_t)k * n + k];
    double* rk = &A[(size_t)k * n];
    for (int r = k + 1; r < n; ++r) {
      double* rr = &A[(size_t)r * n];
      const double l = rr[k] * inv;
      rr[k] = l;
      if (l != 0.0)
        for (int c = k + 1; c < n; ++c) rr[c] -= l * rk[c];
    }
  }
  return true;
}

// solve A x = b (trans = false) or A^T x = b (trans = true) from lu_factor
static void lu_solve(int n, const std::vector<double>& A, const std::vector<int>& piv, std::vector<double>& b,
                     bool trans) {
  if (!trans) {
    for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
    for (int r = 0; r < n; ++r) {
      double a = b[r];
      for (int c = 0; c < r; ++c) a -= A[(size_t)r * n + c] * b[c];
      b[r] = a;
    }
    for (int r = n - 1; r >= 0; --r) {
      double a = b[r];
      for (int c = r + 1; c < n; ++c) a -= A[(size_t)r * n + c] * b[c];
      b[r] = a / A[(size_t)r * n + r];
    }
  } else {
    // A = P^T L U: U^T t = b, L^T v = t, x = P^T v
    for (int r = 0; r < n; ++r) {
      double a = b[r];
      for (int c = 0; c < r; ++c) a -= A[(size_t)c * n + r] * b[c];
      b[r] = a / A[(size_t)r * n + r];
    }
    for (int r = n - 1; r >= 0; --r) {
      double a = b[r];
      for (int c = r + 1; c < n; ++c) a -= A[(size_t)c * n + r] * b[c];
      b[r] = a;
    }
    for (int k = n - 1; k >= 0; --k) std::swap(b[k], b[piv[k]]);
  }
}

int vbqmc_lm_solve(int32_t n, double e0, const double* g_l, const double* g_r, const double* h_bar,
                   const double* s_bar, double a_diag, double* dp, double* e_lin) {
  if (n < 1 || !g_l || !g_r || !h_bar || !s_bar || !dp || !e_lin || !(a_diag >= 0)) return VBQMC_EINVAL;
  const size_t nn = (size_t)n * n;
  std::vector<double> A(nn), x(n), y(n);
  std::vector<int> piv;
  // x(E) = (Hbar + a I - E Sbar)^-1 g_L; f(E) = E - E0 + g_R.x / 4; f'(E) = 1 + y^T Sbar x / 4 with
  // y = (Hbar + a I - E Sbar)^-T g_R
  auto build = [&](double E) {
    for (size_t k = 0; k < nn; ++k) A[k] = h_bar[k] - E * s_bar[k];
    for (int i = 0; i < n; ++i) A[(size_t)i * n + i] += a_diag;
    return lu_factor(n, A, piv);
  };
  double E = e0;
  for (int it = 0; it < 100; ++it) {
    if (!build(E)) return VBQMC_ESINGULAR;
    for (int i = 0; i < n; ++i) { x[i] = g_l[i]; y[i] = g_r[i]; }
    lu_solve(n, A, piv, x, false);
    lu_solve(n, A, piv, y, true);
    double gx = 0, ysx = 0;
    for (int i = 0; i < n; ++i) {
      gx += g_r[i] * x[i];
      double a = 0;
      for (int j = 0; j < n; ++j) a += s_bar[(size_t)i * n + j] * x[j];
      ysx += y[i] * a;
    }
    const double f = E - e0 + 0.25 * gx, fp = 1.0 + 0.25 * ysx;
    if (!std::isfinite(f) || !std::isfinite(fp) || fp == 0.0) return VBQMC_ENONFINITE;
    const double En = E - f / fp;
    const bool done = std::fabs(En - E) <= 1e-13 * std::max(1.0, std::fabs(E));
    E = En;
    if (done) {
      if (!build(E)) return VBQMC_ESINGULAR;
      for (int i = 0; i < n; ++i) x[i] = g_l[i];
      lu_solve(n, A, piv, x, false);
      for (int i = 0; i < n; ++i) dp[i] = -0.5 * x[i];
      *e_lin = E;
      return VBQMC_OK;
    }
  }
  return VBQMC_ENONFINITE;
}

// ---------------------------------------------------------------------------
// structure weights (host)
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Orbital rotations (Sec. 2.2, Eq. PsiJVBp and the passage on orbital classes)
// ---------------------------------------------------------------------------

int vbqmc_det_occupancy(const vbqmc_ctx* x, int32_t max_dets, uint8_t* occ, int32_t* n_dets) {
  if (!x || !n_dets) return VBQMC_EINVAL;
  // determinant pairs that some structure holds with a nonzero coefficient
  std::vector<int> live;
  for (size_t k = 0; k < x->pair_up.size(); ++k) {
    bool nz = false;
    for (auto& pr : x->pair_links[k]) nz = nz || pr.second != 0.0;
    if (nz) live.push_back((int)k);
  }
  *n_dets = (int32_t)live.size();
  if (!occ) return VBQMC_OK;
  if (max_dets < (int32_t)live.size()) return VBQMC_EINVAL;
  const size_t no = (size_t)x->norb;
  std::fill(occ, occ + live.size() * 2 * no, (uint8_t)0);
  for (size_t t = 0; t < live.size(); ++t) {
    const int k = live[t];
    for (int o : x->sp[0].sets[x->pair_up[k]]) occ[(t * 2 + 0) * no + o] = 1;
    for (int o : x->sp[1].sets[x->pair_dn[k]]) occ[(t * 2 + 1) * no + o] = 1;
  }
  return VBQMC_OK;
}

namespace {
// E_kl (orbital l -> orbital k, either spin) acting on a determinant gives a
// nonzero determinant iff some spin holds l and not k; on the sum of
// determinants it is taken as nonzero iff that holds for one of them
bool excitation_nonzero(int no, int nd, const uint8_t* occ, int k, int l) {
  for (int t = 0; t < nd; ++t)
    for (int s = 0; s < 2; ++s) {
      const uint8_t* o = occ + ((size_t)t * 2 + s) * no;
      if (o[l] && !o[k]) return true;
    }
  return false;
}
}  // namespace

int vbqmc_rotation_pairs(int32_t n_orb, int32_t n_dets, const uint8_t* occ, const int32_t* loc_class,
                         int32_t max_pairs, int32_t* pairs, int32_t* n_pairs) {
  if (n_orb < 1 || n_dets < 1 || !occ || !n_pairs || max_pairs < 0 || (max_pairs > 0 && !pairs))
    return VBQMC_EINVAL;
  int32_t np = 0;
  for (int l = 0; l < n_orb; ++l)
    for (int k = 0; k < n_orb; ++k) {
      if (k == l || (loc_class && loc_class[k] != loc_class[l])) continue;
      if (!excitation_nonzero(n_orb, n_dets, occ, k, l)) continue;
      // both directions act: two independent parameters, each listed from
      // its own source orbital; one direction only: kappa_lk = -kappa_kl
      const int kind = excitation_nonzero(n_orb, n_dets, occ, l, k) ? 0 : 1;
      if (np < max_pairs) {
        pairs[3 * np] = k;
        pairs[3 * np + 1] = l;
        pairs[3 * np + 2] = kind;
      }
      ++np;
    }
  *n_pairs = np;
  return np <= max_pairs ? VBQMC_OK : VBQMC_EINVAL;
}

int vbqmc_orbital_classes(int32_t n_orb, int32_t M, const double* lam, int32_t* cls) {
  if (n_orb < 1 || M < 1 || !lam || !cls) return VBQMC_EINVAL;
  for (int p = 0; p < n_orb; ++p) {
    cls[p] = p;
    for (int q = 0; q < p; ++q) {
      bool same = true;
      for (int mu = 0; mu < M && same; ++mu)
        same = (lam[(size_t)p * M + mu] != 0.0) == (lam[(size_t)q * M + mu] != 0.0);
      if (same) {
        cls[p] = cls[q];
        break;
      }
    }
  }
  return VBQMC_OK;
}

int vbqmc_rotate_orbitals(int32_t n_orb, int32_t M, const double* lam, int32_t n_pairs, const int32_t* pairs,
                          const double* theta, double* lam_out) {
  if (n_orb < 1 || M < 1 || !lam || !lam_out || n_pairs < 0 || (n_pairs > 0 && (!pairs || !theta)))
    return VBQMC_EINVAL;
  const int n = n_orb;
  // generator K: orbital l gains K[k][l] phi_k
  std::vector<double> K((size_t)n * n, 0.0);
  for (int q = 0; q < n_pairs; ++q) {
    const int k = pairs[3 * q], l = pairs[3 * q + 1], kind = pairs[3 * q + 2];
    if (k < 0 || k >= n || l < 0 || l >= n || k == l || kind < 0 || kind > 1 || !std::isfinite(theta[q]))
      return VBQMC_EINVAL;
    K[(size_t)k * n + l] += theta[q];
    if (kind == 1) K[(size_t)l * n + k] -= theta[q];
  }
  // exp(K) by scaling and squaring: the Taylor series of exp(K / 2^j) with
  // ||K / 2^j||_1 <= 1/2, summed until the terms stop changing the sum
  double nrm = 0.0;
  for (int c = 0; c < n; ++c) {
    double a = 0.0;
    for (int r = 0; r < n; ++r) a += std::fabs(K[(size_t)r * n + c]);
    nrm = std::max(nrm, a);
  }
  int j = 0;
  while (nrm > 0.5 && j < 1000) {
    nrm *= 0.5;
    ++j;
  }
  const double sc = std::ldexp(1.0, -j);
  std::vector<double> A((size_t)n * n), E((size_t)n * n, 0.0), T((size_t)n * n, 0.0), U((size_t)n * n);
  for (size_t i = 0; i < A.size(); ++i) A[i] = K[i] * sc;
  for (int i = 0; i < n; ++i) E[(size_t)i * n + i] = T[(size_t)i * n + i] = 1.0;
  auto matmul = [n](const std::vector<double>& X, const std::vector<double>& Y, std::vector<double>& Z) {
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        double a = 0.0;
        for (int m = 0; m < n; ++m) a += X[(size_t)r * n + m] * Y[(size_t)m * n + c];
        Z[(size_t)r * n + c] = a;
      }
  };
  for (int t = 1; t <= 40; ++t) {
    matmul(T, A, U);  // T = A^t / t!
    double tn = 0.0;
    for (size_t i = 0; i < U.size(); ++i) {
      T[i] = U[i] / t;
      E[i] += T[i];
      tn = std::max(tn, std::fabs(T[i]));
    }
    if (tn == 0.0 || tn < 1e-18) break;
  }
  for (int r = 0; r < j; ++r) {
    matmul(E, E, U);
    E.swap(U);
  }
  // lambda'_l = sum_k exp(K)[k][l] lambda_k
  std::vector<double> out((size_t)n * M, 0.0);
  for (int l = 0; l < n; ++l)
    for (int k = 0; k < n; ++k) {
      const double e = E[(size_t)k * n + l];
      if (e == 0.0) continue;
      for (int mu = 0; mu < M; ++mu) out[(size_t)l * M + mu] += e * lam[(size_t)k * M + mu];
    }
  std::copy(out.begin(), out.end(), lam_out);
  return VBQMC_OK;
}

int vbqmc_rotation_grad(vbqmc_ctx* x, int64_t W, int32_t n_pairs, const int32_t* pairs, const double* dlogpsi,
                        const double* deloc, double* out_dlogpsi, double* out_deloc, vbqmc_stream stream) {
  if (!x || W < 0 || n_pairs < 0) return fail(x, VBQMC_EINVAL, "rotation_grad: bad arguments");
  if (W == 0 || n_pairs == 0) return VBQMC_OK;
  if (!pairs || !dlogpsi || !deloc || !out_dlogpsi || !out_deloc || W > 0x7fffffff)
    return fail(x, VBQMC_EINVAL, "rotation_grad: bad arguments");
  hipError_t e = launch_rotation_grad(n_params(x), x->nstruct, x->M, x->nop, x->norb, W, n_pairs, pairs, x->d_lamT,
                                      dlogpsi, deloc, out_dlogpsi, out_deloc, (hipStream_t)stream);
  return e == hipSuccess ? VBQMC_OK : hipfail(x, e, "rotation_grad");
}

int vbqmc_lm_redundant(int32_t n, const double* s_bar, double tol, int32_t* keep) {
  if (n < 1 || !s_bar || !keep || !(tol >= 0.0) || !std::isfinite(tol)) return VBQMC_EINVAL;
  // Cholesky factor of Sbar over the parameters kept so far (row i of L
  // stored for each kept i, columns in kept order)
  std::vector<int> kept;
  std::vector<double> L;  // kept.size() rows of length n
  std::vector<double> y;
  for (int i = 0; i < n; ++i) {
    const double d = s_bar[(size_t)i * n + i];
    keep[i] = 0;
    if (!(d > 0.0) || !std::isfinite(d)) continue;
    const size_t m = kept.size();
    y.assign(m, 0.0);
    double r = d;
    for (size_t a = 0; a < m; ++a) {
      double v = s_bar[(size_t)i * n + kept[a]];
      for (size_t b = 0; b < a; ++b) v -= L[a * n + b] * y[b];
      y[a] = v / L[a * n + a];
      r -= y[a] * y[a];
    }
    // residual variance of parameter i after its projection on the kept ones
    if (r > tol * d) {
      keep[i] = 1;
      L.resize((m + 1) * n, 0.0);
      for (size_t b = 0; b < m; ++b) L[m * n + b] = y[b];
      L[m * n + m] = std::sqrt(r);
      kept.push_back(i);
    }
  }
  return VBQMC_OK;
}

int vbqmc_weights_chirgwin_coulson(int32_t n, const double* S, const double* c, double* w) {
  if (n < 1 || !S || !c || !w) return VBQMC_EINVAL;
  double tot = 0;
  for (int I = 0; I < n; ++I) {
    double a = 0;
    for (int J = 0; J < n; ++J) a += S[I * n + J] * c[J];
    w[I] = c[I] * a;
    tot += w[I];
  }
  if (!(tot > 0)) return VBQMC_EINVAL;
  for (int I = 0; I < n; ++I) w[I] /= tot;
  return VBQMC_OK;
}

// cyclic Jacobi eigen-decomposition of a symmetric n x n matrix
static void jacobi_eig(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double th = (A[q * n + q] - A[p * n + p]) / (2 * apq);
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        double cs = 1 / std::sqrt(t * t + 1), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = cs * akp - sn * akq;
          A[k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = cs * apk - sn * aqk;
          A[q * n + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = cs * vkp - sn * vkq;
          V[k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
}

int vbqmc_weights_lowdin(int32_t n, const double* S, const double* c, double* w) {
  if (n < 1 || !S || !c || !w) return VBQMC_EINVAL;
  std::vector<double> A(n * n), V;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[i * n + j] = 0.5 * (S[i * n + j] + S[j * n + i]);
  jacobi_eig(n, A, V);
  // S^{1/2} = V diag(sqrt(max(ev,0))) V^T ; cbar = S^{1/2} c
  std::vector<double> tmp(n, 0.0), cb(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double a = 0;
    for (int i = 0; i < n; ++i) a += V[i * n + k] * c[i];
    tmp[k] = a * std::sqrt(std::max(A[k * n + k], 0.0));
  }
  double tot = 0;
  for (int i = 0; i < n; ++i) {
    double a = 0;
    for (int k = 0; k < n; ++k) a += V[i * n + k] * tmp[k];
    cb[i] = a;
    tot += a * a;
  }
  if (!(tot > 0)) return VBQMC_EINVAL;
  for (int i = 0; i < n; ++i) w[i] = cb[i] * cb[i] / tot;
  return VBQMC_OK;
}

}  // extern "C"
