/*
 * vbqmc.h -- C ABI of the MI355X (gfx950) library for the Jastrow-Valence-Bond
 * (JVB) quantum Monte Carlo hot path.
 *
 * Method: Radenkovic, Domin, Toulouse, Braida, "The Valence-Bond Quantum Monte
 * Carlo Method" (2022).  Each entry point below names the passage that defines
 * what it computes.
 *
 * Conventions (all entry points)
 *   - Atomic units: bohr, hartree.
 *   - Electrons 0 .. n_up-1 are spin up, n_up .. N-1 spin down; spins are
 *     fixed (Sec. 2.3.1).
 *   - Device pointers are marked [dev], host pointers [host].  Arrays are
 *     row-major; positions are [walker][electron][xyz] FP64.
 *   - The wave function is reported as ln|Psi| plus a sign, never as Psi.
 *   - Every call is ordered on the given HIP stream (NULL = default stream)
 *     and may return before the device work finishes; asynchronous device
 *     faults surface at the next synchronising call.
 *   - Return value: 0 on success, a negative VBQMC_E* code otherwise; the
 *     message is available from vbqmc_last_error(ctx).  No C++ exception
 *     crosses this interface.
 *   - A context is not re-entrant: use one context per host thread/stream.
 *   - Ownership: the library copies every host array passed to
 *     vbqmc_create / vbqmc_set_params; it never frees caller memory.  Device
 *     memory for walker states, outputs and workspaces is always the
 *     caller's; the library allocates only its own small constant tables at
 *     vbqmc_create (and vbqmc_set_ecp) and frees them at vbqmc_destroy.
 */
#ifndef VBQMC_H
#define VBQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vbqmc_ctx vbqmc_ctx;
typedef struct ihipStream_t* vbqmc_stream; /* a hipStream_t */

enum {
  VBQMC_OK = 0,
  VBQMC_EINVAL = -1,     /* bad argument or unsupported system shape */
  VBQMC_ENOMEM = -2,     /* host or device allocation failed (create only) */
  VBQMC_EWORKSPACE = -3, /* caller buffer too small */
  VBQMC_EHIP = -4,       /* a HIP runtime call failed */
  VBQMC_ESINGULAR = -5,  /* a reference determinant is exactly singular */
  VBQMC_ENONFINITE = -6, /* non-finite input or Psi = 0 */
  VBQMC_EPOPULATION = -7 /* DMC population empty or above capacity */
};

enum { VBQMC_FP64 = 0, VBQMC_FP32 = 1, VBQMC_BF16 = 2, VBQMC_MIXED = 3 };

/* Nuclei and electron counts (Sec. 2.1; Hamiltonian of Sec. 2.3.1). */
typedef struct {
  int32_t n_nuclei;
  const double* charge;   /* [host] [n_nuclei] */
  const double* position; /* [host] [n_nuclei][3] */
  int32_t n_up, n_dn;
} vbqmc_system;

/*
 * The JVB wave function Psi = J * sum_I c_I Phi_I (Sec. 2.1, Eq. PsiJVBSCF).
 *
 * Basis (Sec. 2.1): shells of kind 0 (Gaussian: sum_k c_k exp(-a_k r^2)) or
 * 1 (Slater: sum_k c_k exp(-a_k r)) times the unnormalised angular set
 * l=0: 1; l=1: x, y, z; l=2: xy, yz, zx, x^2-y^2, 3z^2-r^2.  Basis functions
 * are numbered shell by shell in that order (M in total).
 * Orbitals: phi_p = sum_mu lambda[p][mu] chi_mu, lambda is [n_orbitals][M].
 * Structures (Eq. PhiI): structure I is the unit-weight sum of its HLSP
 * terms; a term lists inactive (doubly occupied) orbitals, singlet pairs
 * (i, j) (i == j allowed) and unpaired spin-up orbitals.  term_counts[3t..]
 * = (n_inactive, n_pairs, n_unpaired) and term_orbitals concatenates, per
 * term, inactive[], pairs[2*n_pairs], unpaired[].
 * Jastrow (Sec. 2.1): f_en + f_ee pair terms
 *   u(r) = a R/(1 + b R) + sum_{p=2..5} q_p R^p,  R = r/(1 + kappa r),
 * ee = {a_anti, a_par, b_anti, b_par, b3, b4, b5, b6} (a fixed by the cusp
 * conditions), en = [n_nuclei][6] = {a1, a2, a3, a4, a5, a6}.
 * een (optional, NULL for none): the three-body term f_een, per nucleus 23
 * coefficients c_t; term t adds, for every electron pair i < j,
 *   c_t Rbar_ij^k (Rbar_ia^l + Rbar_ja^l) (Rbar_ia Rbar_ja)^m,  Rbar = 1/(1 + kappa r),
 * with (k, l, m) taken over p = k + l + 2m = 2..5, k < p, l <= p - k
 * (p - k - 2 when k = 0), ordered by p, then k, then l.  Element sharing and
 * the cusp-preserving constraints among the c_t are the caller's.  With
 * f_een, single-electron VMC and DMC run only on the walker-resident kernel
 * (step_kernel / dmc_kernel 3; EINVAL at create for another choice, and at
 * the call when the system does not fit it), vbqmc_vmc_sweep and
 * vbqmc_vmc_measure are EINVAL, and all-electron VMC, evaluation and the
 * parameter derivatives take it everywhere.
 */
typedef struct {
  int32_t n_shells;
  const int32_t* shell_center; /* [host] nucleus index per shell */
  const int32_t* shell_kind;   /* [host] 0 Gaussian, 1 Slater */
  const int32_t* shell_l;      /* [host] 0, 1 or 2 */
  const int32_t* shell_nprim;  /* [host] primitives per shell */
  const double* prim_exp;      /* [host] concatenated exponents */
  const double* prim_coef;     /* [host] concatenated coefficients */
  int32_t n_orbitals;
  const double* lambda;        /* [host] [n_orbitals][M] */
  int32_t n_structures;
  const double* coef;          /* [host] c_I */
  int32_t n_terms;
  const int32_t* term_structure; /* [host] [n_terms] */
  const int32_t* term_counts;    /* [host] [n_terms][3] */
  const int32_t* term_orbitals;  /* [host] concatenated, see above */
  double kappa;
  double ee[8];
  const double* en;              /* [host] [n_nuclei][6] */
  const double* een;             /* [host] [n_nuclei][23] or NULL */
} vbqmc_wavefunction;

/* precision: VBQMC_FP64 (all FP64), VBQMC_FP32 or VBQMC_BF16 (basis values
 * and the basis->orbital contraction in that type with FP32 accumulation;
 * determinants, inverse refresh, determinant and structure sums in FP64),
 * or VBQMC_MIXED: the orbital rows of trial points and DMC proposals in FP32
 * (they decide acceptance and the drift only), while the reference inverse
 * is rebuilt from FP64 rows before every local energy and the local-energy
 * rows are FP64, so E_L is the FP64 value at the sampled configuration.
 * VBQMC_MIXED applies to the row kernel (step_kernel 2), the wavefront
 * sweep (16 or 32 lanes per walker) and electron-major DMC (dmc_kernel 2);
 * every other path runs it in FP64.
 * refresh_every: accepted single-electron updates per spin after which the
 * reference inverse is rebuilt by a fresh factorisation (default 32).  The
 * row step kernel rebuilds the four walkers of a wavefront together as soon
 * as one of them has reached the limit.
 * walker_lanes: lanes of a 64-lane wavefront given to one walker in the
 * single-electron VMC sweep: 16 or 32 (several walkers per wavefront, if
 * their state fits in LDS), 64 (one walker per workgroup), or 0 to let the
 * library choose (32 when a spin has at most 32 electrons and two walkers
 * fit in LDS, else 64).  Results do not depend on it beyond rounding.
 * step_kernel: how vbqmc_vmc_advance runs single-electron steps: 1 = a sweep
 * launch (lanes per walker as walker_lanes) then the batched local-energy
 * launches, per step; 2 = the row kernel: four walkers per wavefront, 16
 * lanes each, moves and E_L of all n_steps steps in one launch (systems with
 * at most 24 electrons and, per spin, at most 16 reference slots plus table
 * orbitals and 16 distinct determinants; EINVAL at create otherwise); 3 =
 * the walker-resident kernel of dmc_kernel 3 in its Metropolis form: each
 * call rebuilds the records from their positions (one launch) and then runs
 * one launch per step (moves, refresh and E_L of four walkers per
 * workgroup), with the same limits as dmc_kernel 3 (EINVAL at create
 * otherwise), S_IJ sums included for up to 256 structures (a call with more
 * runs the sweep and local-energy kernels).  0 = 2 when the system fits it and
 * walker_lanes is 0, else 3 when it fits that and walker_lanes is 0, else 1.
 * Results do not depend on it beyond rounding.
 * dmc_kernel: how vbqmc_dmc_advance runs a step: 1 = one workgroup per walker
 * makes all of the walker's moves, E_L and weight; 2 = electron-major: for
 * each electron a proposal launch, an MFMA launch for the orbital rows at
 * the proposals and an acceptance launch, each over all walkers, then one
 * per-walker launch for refresh, E_L and weight (spins with at most 64
 * reference slots plus table orbitals; EINVAL at create otherwise);
 * 3 = walker-resident: one launch per step in which a workgroup keeps four
 * walkers (one per wavefront) for all their moves, refresh, E_L and weight,
 * with the value and gradient orbital rows of each electron's position kept
 * in the walker record (FP64, at most 32 electrons and 64
 * reference slots plus table orbitals per spin, at most 64 orbitals; EINVAL
 * at create otherwise); 0 = 3 when the system fits it, else 2 when one
 * workgroup per walker would need more than 40 KiB of LDS and the system fits
 * it, else 1.  Results do not depend on it beyond rounding. */
typedef struct {
  int32_t precision;
  int32_t refresh_every;
  int32_t walker_lanes;
  int32_t step_kernel;
  int32_t dmc_kernel;
} vbqmc_options;

typedef struct {
  int32_t n_electrons, n_up, n_dn, n_nuclei;
  int32_t n_basis, n_orbitals, n_structures;
  int32_t n_determinants;        /* distinct (up, down) determinant pairs */
  int32_t n_unique_up, n_unique_dn; /* distinct spin determinants */
  int32_t n_table_up, n_table_dn;   /* orbitals replacing reference columns */
  int32_t n_params;              /* n_structures + n_orbitals*n_basis + 6 + 6*n_nuclei (+ 23*n_nuclei with f_een) */
  int32_t block_threads;         /* threads per walker in the walker kernels */
  int32_t sweep_lanes;           /* lanes per walker in the single-electron sweep */
  int32_t step_kernel;           /* kernel of single-electron VMC steps (vbqmc_options) */
  int32_t dmc_kernel;            /* kernel of DMC steps (vbqmc_options) */
  int64_t walker_state_bytes;    /* bytes per walker record */
  int64_t lds_bytes;             /* LDS bytes per walker block */
} vbqmc_info_t;

/* Build a context: expands the HLSP structures into determinants (Eq. PhiI,
 * N_det,I = 2^{N_pairs}), picks the reference determinant per spin and
 * uploads the constant tables.  The reference of each spin is that spin's
 * determinant in the first product of the expansion (structures, their terms,
 * then the pair orientations, each pair (i, j) first as up i, down j) with no
 * orbital repeated in either spin; every other spin determinant is handled as
 * at most 3 replaced columns of it.  Rounding errors of the determinant ratios
 * grow with the ratio of the largest spin determinant to the reference one.  Errors: EINVAL (inconsistent counts, more than
 * 3 orbitals of a determinant differing from its spin's reference, sizes
 * above the kernel limits: 64 electrons per spin, 1024 basis functions),
 * ENOMEM, EHIP. */
int vbqmc_create(const vbqmc_system* sys, const vbqmc_wavefunction* wf, const vbqmc_options* opt,
                 vbqmc_ctx** out);
void vbqmc_destroy(vbqmc_ctx* ctx);
const char* vbqmc_last_error(const vbqmc_ctx* ctx);
int vbqmc_get_info(const vbqmc_ctx* ctx, vbqmc_info_t* out);
/*
 * Pseudopotentials (Sec. 2.1, basis choice: the valence calculations use
 * energy-consistent pseudopotentials, whose form the paper does not give;
 * this is the usual semilocal form).  For a pseudo-nucleus a, whose charge in
 * vbqmc_system is its effective (valence) charge Z_a, each electron at
 * distance r adds to the potential energy
 *   V_loc(r) + sum_{l < L} V_l(r) P_l-projection,
 *   V(r) = sum_k c_k r^(n_k - 2) exp(-alpha_k r^2)   (each radial part),
 * besides the -Z_a / r of the Hamiltonian.  The projection of channel l is
 * taken in E_L as (2l + 1) times the mean, over the 12 directions u_q to the
 * vertices of an icosahedron (fixed orientation; exact for spherical
 * harmonics to degree 5), of P_l(u_q . (r_i - a) / r) times the ratio
 * Psi(r_i -> a + r u_q) / Psi, and only for r < r_cut.
 * terms: per centre, n_terms[] gives L + 1 counts (local part, then channel
 * 0 .. L-1), and terms[] concatenates their [c, n, alpha] (n an integer
 * 0..6, alpha >= 0).
 */
typedef struct {
  int32_t n_centers;          /* 0 removes the pseudopotentials */
  const int32_t* center;      /* [host] [n_centers] nucleus index, each at most once */
  const int32_t* n_channels;  /* [host] [n_centers] L <= 4 */
  const double* r_cut;        /* [host] [n_centers] bohr */
  const int32_t* n_terms;     /* [host] sum over centres of (L + 1) */
  const double* terms;        /* [host] [sum of n_terms][3] */
} vbqmc_ecp;

/* Attach pseudopotentials to a context (replacing earlier ones; NULL or
 * n_centers = 0 removes them).  Synchronises the device first.  With them,
 * vbqmc_evaluate, vbqmc_walkers_init, vbqmc_vmc_advance (all-electron and
 * single-electron moves) and the DMC entry points include the
 * pseudopotential energy in E_L, all on the one-workgroup-per-walker
 * kernels (step and dmc kernel 1 whatever the options say); in DMC the term
 * is taken with the trial function (the locality approximation: the nonlocal
 * part enters the branching weights through E_L only).  vbqmc_vmc_sweep,
 * vbqmc_vmc_measure and vbqmc_param_grad return EINVAL.  Errors: EINVAL (bad centre, channel count, r_cut or term; a
 * precision form other than FP64; f_een), ENOMEM, EHIP. */
int vbqmc_set_ecp(vbqmc_ctx* ctx, const vbqmc_ecp* ecp);


/* Replace the variational parameters p = [c (n_structures) | lambda
 * (n_orbitals*M, row-major) | b_anti, b_par, b3..b6 | per nucleus a1..a6]
 * (Sec. 2.2, Eq. PsiJVBp with the orbital coefficients varied directly).
 * p is [host][n_params].  The call first waits for all work queued on the
 * device (any stream), then replaces the context's device tables, so work
 * queued before it used the old parameters and work queued after it uses the
 * new ones.  Existing walker states become stale: re-run
 * vbqmc_walkers_init. */
int vbqmc_set_params(vbqmc_ctx* ctx, const double* p);
int vbqmc_get_params(const vbqmc_ctx* ctx, double* p);

/*
 * Evaluate ln|Psi|, sign, grad_i ln|Psi|, the local energy E_L = H Psi / Psi
 * and the structure ratios r_I = Phi_I / sum_J c_J Phi_J for W fixed
 * configurations (Sec. 2.1 for Psi, Sec. 2.3.1 Eq. Elav for E_L,
 * Sec. 2.4 for r_I).  Each determinant ratio is computed from a fresh LU of
 * the reference determinant.  R [dev][W][N][3]; logabs [dev][W];
 * sign [dev][W] (0 where Psi = 0); grad [dev][W][N][3] or NULL;
 * eloc [dev][W] or NULL; ratio [dev][W][n_structures] or NULL.
 */
int vbqmc_evaluate(vbqmc_ctx* ctx, int64_t W, const double* R, double* logabs, int32_t* sign,
                   double* grad, double* eloc, double* ratio, vbqmc_stream stream);

/* Walker records: opaque, walker_state_bytes each, caller-allocated [dev].
 * init fills records from positions R [dev][W][N][3] (fresh factorisations,
 * local energy); positions copies R back out of the records. */
int vbqmc_walkers_init(vbqmc_ctx* ctx, int64_t W, const double* R, void* state, vbqmc_stream stream);
int vbqmc_walkers_positions(vbqmc_ctx* ctx, int64_t W, const void* state, double* R,
                            vbqmc_stream stream);
/* Per-walker local energies of the records [dev][W] (the value at the last
 * init / step). */
int vbqmc_walkers_eloc(vbqmc_ctx* ctx, int64_t W, const void* state, double* eloc, vbqmc_stream stream);

/* VMC accumulators, all [dev] and accumulated into (+=), per walker:
 * e_sum/e2_sum: sums of E_L and E_L^2 over steps; n_accept: accepted moves;
 * e_last: E_L after the last step; sij_sum [W][n_structures]^2 or NULL:
 * sums of r_I r_J (the estimator of S_IJ, Sec. 2.4). */
typedef struct {
  double* e_sum;
  double* e2_sum;
  double* n_accept;
  double* e_last;
  double* sij_sum;
} vbqmc_vmc_acc;

/*
 * Metropolis VMC (Sec. 2.3.1): n_steps steps for W walkers, each step being
 * one all-electron move (all_electron != 0) or N single-electron moves in
 * electron order, followed by E_L.  Proposal r' = r + step_size (2u - 1) per
 * component, accepted iff u' < |Psi'/Psi|^2.  Random numbers: Philox4x32-10,
 * key = seed, counter = (walker, step0 + s, 4*electron + purpose, draw)
 * (purpose 0 proposal, 1 acceptance).  Single-electron moves update the
 * reference inverse and determinant table by Sherman-Morrison; the inverse is
 * rebuilt every refresh_every accepted updates.  state [dev] is updated in
 * place.
 */
int vbqmc_vmc_advance(vbqmc_ctx* ctx, void* state, int64_t W, int32_t n_steps, uint64_t seed,
                      uint64_t step0, double step_size, int32_t all_electron, const vbqmc_vmc_acc* acc,
                      vbqmc_stream stream);

/*
 * The two halves of a single-electron VMC step (Sec. 2.3.1), for callers that
 * measure E_L less often than they move.  vbqmc_vmc_sweep does the N
 * single-electron moves of step `step` for every walker exactly as
 * vbqmc_vmc_advance (same draws, same updates) and adds the accepted moves to
 * n_accept [dev][W]; vbqmc_vmc_measure computes E_L (Eq. Elav) of every
 * walker at its current configuration from its record and accumulates it
 * into acc (e_sum, e2_sum, e_last and, if set, sij_sum; n_accept is not
 * used).  vbqmc_vmc_advance with all_electron = 0 equals, per step, a sweep
 * followed by a measure: bit for bit when it runs the sweep and local-energy
 * kernels (step_kernel 1), with the same moves and E_L to rounding when it
 * runs the row or the walker-resident kernel (step_kernel 2 or 3).  Both need the system to fit the sweep and
 * local-energy kernels (EINVAL otherwise, where vbqmc_vmc_advance still
 * runs); state [dev] is any record written by this library.
 */
int vbqmc_vmc_sweep(vbqmc_ctx* ctx, void* state, int64_t W, uint64_t seed, uint64_t step, double step_size,
                    double* n_accept, vbqmc_stream stream);
int vbqmc_vmc_measure(vbqmc_ctx* ctx, void* state, int64_t W, const vbqmc_vmc_acc* acc, vbqmc_stream stream);

/* DMC per-step records, each [dev][n_steps]: population before branching,
 * sum of weights, sum of weight * E_L, trial energy used, accepted and
 * proposed single-electron moves.  step_ms [host][n_steps] or NULL: when set,
 * each step's move-and-local-energy kernels are bracketed by HIP events on
 * the call's stream and their elapsed milliseconds are written here before
 * the call returns (branching and compaction are not included).  wcsum
 * [dev][n_steps] or NULL: sum of weight * E_L clipped to E_T +- sqrt(N/tau),
 * the estimator the trial-energy feedback uses.  dr2_acc, dr2_prop
 * [dev][n_steps] or NULL: sums over the walkers and their electrons of
 * |r' - r|^2 of the accepted moves and of all proposed moves, so that
 * tau_eff = tau dr2_acc / dr2_prop (the effective time step of the
 * drift-diffusion moves with rejections; the weights use the nominal tau). */
typedef struct {
  double* pop;
  double* wsum;
  double* wesum;
  double* etrial;
  double* n_accept;
  double* n_prop;
  double* step_ms;
  double* wcsum;
  double* dr2_acc;
  double* dr2_prop;
} vbqmc_dmc_log;

/*
 * Fixed-node DMC (Sec. 2.3.2, Eq. E0DMCweights): per step each walker makes N
 * drift-diffusion single-electron moves r' = r + tau v + sqrt(tau) chi with
 * v = grad_i ln|Psi|, accepted with min(1, |Psi'/Psi|^2 G(r<-r')/G(r'<-r)),
 * rejected outright if the sign of Psi changes; then weight
 * w = exp(-tau ((E_L + E_L')/2 - E_T)) with E_L clipped to E_T +- sqrt(N/tau);
 * population control: if the expected next population sum w lies outside
 * [0.95, 1.05] W_target, every weight of the step is scaled by the one factor
 * f that brings the sum to the nearer bound (the step's logged E_T is then
 * E_T + ln(f)/tau); floor(w + u) copies (at most 3, children of weight 1,
 * parents' order kept, compaction on the device); next
 * E_T = E_est - (0.1/tau) ln(W/W_target) with E_est the running weighted mean
 * of the clipped E_L of this call.  Random numbers as VMC plus purpose 2
 * (branching, electron index N); the walker index is the slot after
 * compaction.  states: two [dev] buffers of capacity records; the
 * population lives in states[0] on entry and on return.  W_io [host] in/out;
 * e_trial_io [host] in/out.  workspace [dev] of vbqmc_dmc_workspace_bytes.
 * Error EPOPULATION if the population reaches 0 or exceeds capacity (the
 * states are then left at the last good step).
 */
int vbqmc_dmc_workspace_bytes(const vbqmc_ctx* ctx, int64_t capacity, int32_t n_steps, size_t* bytes);
int vbqmc_dmc_advance(vbqmc_ctx* ctx, void* states[2], int64_t* W_io, int64_t capacity, int32_t n_steps,
                      uint64_t seed, uint64_t step0, double tau, double* e_trial_io, int64_t W_target,
                      const vbqmc_dmc_log* log, void* workspace, size_t workspace_bytes,
                      vbqmc_stream stream);

/*
 * vbqmc_dmc_advance without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, semantics and results
 * as vbqmc_dmc_advance, bit for bit (log->step_ms must be NULL: timing
 * events are not created here), except that the workspace is a fixed
 * 32 MiB device array inside the library (one per device, held until the
 * process ends; its address is taken at vbqmc_create), so the call allocates
 * nothing.  Capacities whose vbqmc_dmc_workspace_bytes exceeds 32 MiB are
 * rejected with EWORKSPACE before any work is queued.  Every call on a device
 * shares that device's array: calls that overlap on one device (other
 * streams, other contexts or host threads) race and must be serialised by the
 * caller.  The current device must be the context's (EINVAL otherwise).
 */
int vbqmc_dmc_advance_noalloc(vbqmc_ctx* ctx, void* states[2], int64_t* W_io, int64_t capacity, int32_t n_steps,
                              uint64_t seed, uint64_t step0, double tau, double* e_trial_io, int64_t W_target,
                              const vbqmc_dmc_log* log, vbqmc_stream stream);

/*
 * Parameter derivatives for W fixed configurations (Sec. 2.2, Eqs. Hi0, H0j):
 * dlogpsi[w][j] = d ln|Psi| / d p_j and deloc[w][j] = d E_L / d p_j, parameter
 * order as vbqmc_set_params.  Computed by a hand-written adjoint (reverse)
 * pass that recomputes every spin-determinant inverse; the orbital part is an
 * MFMA contraction of adjoint orbital rows with basis rows.  R [dev][W][N][3];
 * outputs [dev][W][n_params].  workspace [dev] of vbqmc_param_grad_workspace_bytes.
 */
int vbqmc_param_grad_workspace_bytes(const vbqmc_ctx* ctx, int64_t W, size_t* bytes);
int vbqmc_param_grad(vbqmc_ctx* ctx, int64_t W, const double* R, double* dlogpsi, double* deloc,
                     void* workspace, size_t workspace_bytes, vbqmc_stream stream);

/* Deterministic fixed-order weighted sum over walkers (the sample averages
 * of Sec. 2.3.1 and the contraction of per-walker derivatives with an
 * upstream gradient): out[k] = sum_w weights[w] in[w][k]; weights [dev][W]
 * or NULL for unit weights, in [dev][W][K], out [dev][K]. */
int vbqmc_reduce_walkers(vbqmc_ctx* ctx, int64_t W, int32_t K, const double* weights, const double* in,
                         double* out, vbqmc_stream stream);

/* Structure weights from the overlap estimate S [host][n][n] (Sec. 2.4):
 * Chirgwin-Coulson w_I = c_I (S c)_I / c.S.c and Loewdin
 * w_K = cbar_K^2 / |cbar|^2 with cbar = S^{1/2} c (symmetric square root by a
 * Jacobi eigensolver).  Host-only; EINVAL for n < 1 or a non-positive norm. */
int vbqmc_weights_chirgwin_coulson(int32_t n, const double* S, const double* c, double* w);
int vbqmc_weights_lowdin(int32_t n, const double* S, const double* c, double* w);

/*
 * Linear optimisation method (Sec. 2.2, Eqs. Psiblin, geneigeq; its sampled
 * form Sec. 2.3.1, Eqs. geneigeqM, Hi0, H0j, Hij, Sij).
 *
 * Sample sums.  With O_kj = Psi_j/Psi_0 = d ln|Psi|/dp_j and
 * D_kj = E_L,j = d E_L/dp_j of sample k (vbqmc_param_grad), E_k its local
 * energy and w_k its weight (1 for VMC samples), the accumulator holds three
 * row-major (P+1) x (P+1) matrices, P = n_params, of the augmented rows
 * X_k = [1 | O_k] and Y_k = [E_k^2 | D_k]:
 *   S'[i][j] = sum_k w_k X_ki X_kj,  H'[i][j] = sum_k w_k E_k X_ki X_kj,
 *   D'[i][j] = sum_k w_k X_ki Y_kj
 * (so row 0 holds sum w, sum w O_j, sum w E, sum w E O_j, sum w E^2,
 * sum w D_j).  vbqmc_lm_acc_doubles gives the length 3 (P+1)^2.
 * vbqmc_lm_accumulate adds W samples to acc [dev] (the caller zeroes it
 * before the first call; calls on one stream accumulate in a fixed order,
 * FP64 MFMA products): dlogpsi, deloc [dev][W][P], eloc [dev][W],
 * weight [dev][W] or NULL for unit weights.
 */
int vbqmc_lm_acc_doubles(int32_t n_params, int64_t* n);
int vbqmc_lm_accumulate(vbqmc_ctx* ctx, int64_t W, const double* dlogpsi, const double* deloc, const double* eloc,
                        const double* weight, double* acc, vbqmc_stream stream);
/*
 * The same sums for any parameter set the caller assembles per sample
 * (for instance structure coefficients, orbital-rotation parameters from
 * vbqmc_rotation_grad and Jastrow parameters): P columns, dlogpsi, deloc
 * [dev][W][P], acc [dev] of vbqmc_lm_acc_doubles(P).  EINVAL for P < 1.
 */
int vbqmc_lm_accumulate_cols(int32_t P, int64_t W, const double* dlogpsi, const double* deloc, const double* eloc,
                             const double* weight, double* acc, vbqmc_stream stream);

/*
 * Estimators from an accumulator copied to the host (acc [host], length
 * vbqmc_lm_acc_doubles(P)), all averages weighted by w: E0 = <E_L>,
 *   g_L,i = 2 (<O_i E_L> - <O_i><E_L>)                        (Eq. Hi0)
 *   g_R,j = 2 (<O_j E_L> - <O_j><E_L> + <E_L,j>)              (Eq. H0j)
 *   Hbar_ij = <O_i O_j E_L> - <O_i><O_j E_L> - <O_j><O_i E_L>
 *             + <O_i><O_j><E_L> + <O_i E_L,j> - <O_i><E_L,j>  (Eq. Hij)
 *   Sbar_ij = <O_i O_j> - <O_i><O_j>                          (Eq. Sij)
 * Outputs [host]: e0 (1), g_l, g_r (P), h_bar, s_bar (P x P row-major),
 * var (1, <E_L^2> - <E_L>^2) or NULL.  EINVAL if sum w <= 0.
 */
int vbqmc_lm_estimators(int32_t n_params, const double* acc, double* e0, double* g_l, double* g_r, double* h_bar,
                        double* s_bar, double* var);

/*
 * One linear-method step (Eq. geneigeqM): the eigenvector (1, dp) of
 *   [[E0, g_R^T/2], [g_L/2, Hbar + a_diag I]] v = E_lin [[1, 0], [0, Sbar]] v
 * that continues the current wave function, found as the root of
 * E_lin = E0 - g_R^T (Hbar + a_diag I - E_lin Sbar)^-1 g_L / 4 next to E0
 * (Newton's method on E_lin, one LU with partial pivoting of the n x n
 * matrix per iteration), then dp = -(Hbar + a_diag I - E_lin Sbar)^-1 g_L / 2.
 * a_diag >= 0 is the usual stabilising shift of the diagonal.  Host only:
 * n the number of parameters in the (sub)problem, g_l, g_r [host][n],
 * h_bar, s_bar [host][n][n] row-major; outputs dp [host][n], e_lin [host].
 * ESINGULAR if a matrix becomes singular, ENONFINITE if the iteration does
 * not converge within 100 steps.
 */
int vbqmc_lm_solve(int32_t n, double e0, const double* g_l, const double* g_r, const double* h_bar,
                   const double* s_bar, double a_diag, double* dp, double* e_lin);

/*
 * Orbital rotations (Sec. 2.2, Eq. PsiJVBp, and the partition of the
 * orbitals that follows it).  The rotation exp(kappa) with kappa =
 * sum kappa_kl E_kl, E_kl the singlet excitation from orbital l to orbital
 * k, adds kappa_kl phi_k to orbital l to first order.  Orbital classes come
 * from the determinants: inactive (in both spins of every determinant),
 * active (in some), virtual (in none).  An excitation E_kl is kept iff it
 * acts on the wave function (some determinant holds l and not k in one
 * spin; no cancellation between determinants is looked for) and k, l share a
 * localization class; this keeps exactly inactive -> active, inactive ->
 * virtual, active -> virtual and the acting active -> active excitations.
 * A pair whose reverse excitation E_lk does not act is one parameter with
 * kappa_lk = -kappa_kl (kind 1); when both act, kappa_kl and kappa_lk are
 * two independent parameters (kind 0), each listed once.  Redundancies
 * among the derivatives (between orbital parameters, or with structure
 * coefficients) are found from the samples with vbqmc_lm_redundant.
 *
 * vbqmc_det_occupancy: the context's determinant products (those a
 * structure holds with a nonzero coefficient) as occupancies occ [host]
 * [n][2][n_orbitals] (1 if the orbital is in the spin-up (0) or spin-down
 * (1) determinant).  occ NULL: only *n_dets is written; EINVAL if max_dets
 * is smaller than the count.
 *
 * vbqmc_rotation_pairs (host only): the kept excitations as pairs [host]
 * [n][3] = (k, l, kind), ordered by l, then k; loc_class [host][n_orb] or
 * NULL (one class).  *n_pairs is the count even when it exceeds max_pairs
 * (then EINVAL and only max_pairs are written).
 *
 * vbqmc_orbital_classes (host only): localization classes of the orbitals
 * of lambda [host][n_orb][M]: orbitals expanded on the same set of basis
 * functions (the same nonzero pattern) share a class, numbered by the first
 * orbital of the class.
 *
 * vbqmc_rotate_orbitals (host only): lambda_out = exp(K)^T lambda with
 * K[k][l] = theta_q for each pair q = (k, l, kind) (and K[l][k] = -theta_q
 * for kind 1), so that orbital l becomes sum_k exp(K)[k][l] phi_k (the
 * matrix exponential by scaling and squaring of its Taylor series); all
 * arrays [host], lambda and lambda_out [n_orb][M] (may alias).  EINVAL for
 * an out-of-range or diagonal pair or a non-finite theta.
 *
 * vbqmc_rotation_grad: d/d kappa of ln|Psi| and of E_L from the
 * per-walker outputs of vbqmc_param_grad at the context's current
 * parameters, d/d kappa_kl = sum_mu lambda[k][mu] d/d lambda[l][mu] (minus
 * the same with k and l exchanged for kind 1): dlogpsi, deloc [dev][W][P],
 * pairs [dev][n_pairs][3], outputs [dev][W][n_pairs]; a pair out of range
 * gives NaN in its column.  Stream-ordered, FP64.
 *
 * vbqmc_lm_redundant (host only): with the parameters taken in order, keep
 * [host][n] = 1 for a parameter whose residual variance after projection on
 * the kept earlier ones exceeds tol times its variance Sbar_ii (a Cholesky
 * factorisation of s_bar [host][n][n] in the given order that skips the
 * dropped parameters), 0 otherwise (also for Sbar_ii <= 0).  With the
 * structure coefficients placed first, an orbital parameter whose
 * derivative lies in their span (and the span of the kept orbital
 * parameters before it) is dropped.
 */
int vbqmc_det_occupancy(const vbqmc_ctx* ctx, int32_t max_dets, uint8_t* occ, int32_t* n_dets);
int vbqmc_rotation_pairs(int32_t n_orb, int32_t n_dets, const uint8_t* occ, const int32_t* loc_class,
                         int32_t max_pairs, int32_t* pairs, int32_t* n_pairs);
int vbqmc_orbital_classes(int32_t n_orb, int32_t M, const double* lam, int32_t* cls);
int vbqmc_rotate_orbitals(int32_t n_orb, int32_t M, const double* lam, int32_t n_pairs, const int32_t* pairs,
                          const double* theta, double* lam_out);
int vbqmc_rotation_grad(vbqmc_ctx* ctx, int64_t W, int32_t n_pairs, const int32_t* pairs, const double* dlogpsi,
                        const double* deloc, double* out_dlogpsi, double* out_deloc, vbqmc_stream stream);
int vbqmc_lm_redundant(int32_t n, const double* s_bar, double tol, int32_t* keep);

#ifdef __cplusplus
}
#endif

#endif /* VBQMC_H */
