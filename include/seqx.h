/*
 * seqx.h -- semiempirical (NDDO) CIS / TDHF excited states on one MI355X (gfx950).
 *
 * C ABI of libseqx.  The calls follow the paper's problem statement (PySEQM 2.0,
 * "Theory and implementation"): atomic numbers, coordinates and method
 * parameters in; the closed-shell RHF ground state (Eq. 1, F C = C eps with
 * S = I) built from the NDDO integrals; then the lowest roots of CIS (Eq. 7)
 * or TDHF/RPA (Eq. 2) by a Davidson iteration whose only large operation is
 * the matrix-free product of Eqs. 8-9; excitation energies, amplitudes and
 * oscillator strengths out.
 *
 * Conventions shared by every call
 *  - Status codes only; nothing throws or aborts across the ABI.  On error the
 *    outputs are untouched and seqx_last_error() describes the failure.
 *  - Units: Angstrom and eV at the boundary; bohr and hartree inside
 *    (CODATA 2018: 1 Eh = 27.211386245988 eV, a0 = 0.529177210903 A).
 *  - Host pointers are owned by the caller and never retained after a call
 *    returns.  Device pointers (the *_device calls) must be device memory of
 *    the context's GPU, ordered on the context's stream.
 *  - AOs: H carries s; C and O carry s, px, py, pz, in input atom order.
 *  - MOs ascend in eps.  Amplitudes are row-major [root][i][a], i over the
 *    nocc occupied MOs, a over the nvirt virtual MOs.  Roots ascend in omega;
 *    each root is signed so its largest |X| element is positive (ties: lowest
 *    flat index).
 *  - Results are bitwise reproducible for one device and build (no
 *    floating-point atomics).
 *  - A context is not thread-safe; several contexts may coexist.
 */
#ifndef SEQX_H
#define SEQX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SEQX_ABI_VERSION 5
#define SEQX_NPARAM 11 /* per-element parameters, order below */

typedef struct seqx_ctx seqx_ctx; /* one device + one stream */
typedef struct seqx_job seqx_job; /* molecules after integrals + SCF; owns their device state */

typedef enum {
  SEQX_OK = 0,
  SEQX_E_ARG = 1,         /* bad argument (null pointer, size, enum value)               */
  SEQX_E_ELEMENT = 2,     /* atomic number without parameters (supported: 1, 6, 8)      */
  SEQX_E_OPEN_SHELL = 3,  /* odd electron count                                          */
  SEQX_E_GEOMETRY = 4,    /* non-finite coordinate or two atoms closer than 0.1 Angstrom */
  SEQX_E_NOMEM = 5,       /* device allocation failed                                    */
  SEQX_E_DEVICE = 6,      /* HIP / rocSOLVER error, or no usable device                  */
  SEQX_E_SCF_NOCONV = 7,  /* SCF reached max_iter above tol                              */
  SEQX_E_DAV_NOCONV = 8,  /* Davidson reached max_iter above tol                         */
  SEQX_E_UNSTABLE = 9,    /* A-B (or A+B) not positive definite: imaginary TDHF root     */
  SEQX_E_BUFSIZE = 10,    /* caller buffer too small (see *needed)                       */
  SEQX_E_STATE = 11       /* call out of order (e.g. results before solve)               */
} seqx_status;

typedef enum { SEQX_CIS = 0, SEQX_TDHF = 1 } seqx_theory;

/* Arithmetic of the dense MO<->AO transforms inside the sigma build.  Subspace
 * projection, Gram-Schmidt, the small eigensolves and the SCF stay FP64.
 * SEQX_FP32: C, V and the AO matrices stored in FP32, transforms on the FP32
 * matrix cores with FP32 accumulation; the NDDO contraction sums in FP64 and
 * the (eps_a - eps_i) V term is added in FP64 (mixed-precision mode of the
 * paper's outlook).  A seqx_solve in FP32 restarts from its Ritz vectors with
 * FP64 products once its residuals reach max(tol, the FP32 rounding floor) or
 * stop improving, and converges to tol in FP64, so its roots carry FP64
 * accuracy.  SEQX_BF16X3: the same FP32 storage, each transform as three
 * bfloat16 matrix-core products of the split operands x = hi + lo (hi lo,
 * lo hi, hi hi; FP32 accumulation, at most 3 * 2^-16 relative error per
 * product); a seqx_solve steps through split bfloat16, FP32 and FP64 products,
 * restarting from its Ritz vectors at each step once the residuals reach the
 * floor of the current precision, so its roots too carry FP64 accuracy.
 * SEQX_BF16 (single bfloat16) is reserved and returns SEQX_E_ARG. */
typedef enum { SEQX_FP64 = 0, SEQX_FP32 = 1, SEQX_BF16 = 2, SEQX_BF16X3 = 3 } seqx_precision;

/* Starting space of the Davidson iteration:
 *   GAP         unit vectors at the min(nocc*nvirt, 2K) smallest orbital-energy gaps;
 *   LEARNED     unit vectors at the M pairs the context's network scores highest
 *               (P-space guess; M = seqx_solve_opts.pspace, default 4K);
 *   USER        the caller's vectors (molecule 0);
 *   GAP_PSPACE  unit vectors at the M smallest gaps (the same construction as
 *               LEARNED with the gap as the score: the baseline it is compared to).
 * Ties are broken by the flat pair index i*nvirt + a.  The converged roots do
 * not depend on the guess; the iteration count does. */
typedef enum { SEQX_GUESS_GAP = 0, SEQX_GUESS_LEARNED = 1, SEQX_GUESS_USER = 2, SEQX_GUESS_GAP_PSPACE = 3 } seqx_guess;

/* Parameter order of one row of seqx_set_params (eV, exponents in 1/bohr):
 *   zeta_s, zeta_p, U_ss, U_pp, beta_s, beta_p, g_ss, g_sp, g_pp, g_p2, h_sp
 * Entries that do not apply (p terms of H) are ignored. */

typedef struct {
  double tol;       /* max |F P - P F| in hartree; <= 0 selects 1e-10 */
  int32_t max_iter; /* <= 0 selects 300 */
  int32_t ndiis;    /* DIIS history length; <= 0 selects 8, 1 disables DIIS */
  int32_t integrals_only; /* nonzero: build ERIs and core Hamiltonian only, no SCF
                             (seqx_scf_results, seqx_sigma and seqx_solve then return SEQX_E_STATE) */
} seqx_scf_opts;

typedef struct {
  int32_t theory;       /* seqx_theory */
  int32_t nroots;       /* K >= 1, at most nocc*nvirt of the smallest molecule */
  double tol;           /* residual norm in hartree; <= 0 selects 1e-6 */
  int32_t max_iter;     /* <= 0 selects 100 */
  int32_t max_subspace; /* <= 0: derived from mem_budget_bytes, capped at 20 * nroots + 40 */
  size_t mem_budget_bytes; /* 0: 40 % of free device memory (subspace + sigma scratch) */
  int32_t precision;    /* seqx_precision of the transforms */
  int32_t guess;        /* seqx_guess */
  int32_t n_user_guess; /* SEQX_GUESS_USER: number of host vectors in user_guess */
  const double* user_guess; /* host [n_user_guess][nocc][nvirt], molecule 0 only */
  int32_t batched;      /* nonzero: every molecule of the job in one batched Davidson
                           (CIS, gap guess, 1-16 roots, SEQX_FP32 or SEQX_FP64 products):
                           each iteration forms all (molecule, vector) products in one
                           persistent launch and replays one captured HIP graph.  The
                           subspace cap is min(max_subspace or 8 * nroots, 48) per molecule.
                           Molecules need at most 1536 same-atom AO pairs. */
  int32_t pspace;       /* LEARNED / GAP_PSPACE guesses: number of pairs M; <= 0 selects 4 * nroots */
  int32_t root_batch;   /* 1 .. nroots-1: low-memory solve of the roots in batches of this many
                           (the paper's outlook: find a subset of the states, then shift the
                           ones found out of the search space).  Each batch is a Davidson solve
                           of its lowest roots with the earlier roots locked and shifted up
                           (TDHF: A+B += s U U^T over the locked X-Y rows; CIS: A += s X X^T),
                           so the subspace cap (20 * root_batch + 40, or the memory budget)
                           applies per batch and only the K converged roots are kept beyond
                           it.  Single-molecule solver, gap guess only.  0: all roots at once. */
  int32_t nguard;       /* 0 .. 64 extra roots iterated above the nroots wanted ones (single-molecule
                           solver): their Ritz vectors join the expansion and the restarts, which
                           helps when the wanted roots sit in a dense cluster; only the wanted
                           roots decide convergence and are returned; the default subspace cap
                           counts them (20 * (nroots + nguard) + 40). */
} seqx_solve_opts;

typedef struct {
  int32_t scf_iterations;   /* summed over molecules */
  int32_t dav_iterations;   /* iterations of the last solve (max over molecules) */
  int64_t n_sigma;          /* sigma vectors formed in the last solve */
  double commutator;        /* max |FP-PF| at SCF exit, over molecules */
  double t_integrals_s;     /* device time of ERI + core Hamiltonian build */
  double t_scf_s;           /* device time of the SCF */
  double t_davidson_s;      /* wall time of the last solve, sigma included */
  double t_sigma_s;         /* device time spent in sigma builds during the last solve */
  double time_to_roots_s[64]; /* wall time (s) at which each Davidson iteration ended */
  int32_t n_history;
  /* Sigma-build phases since the last seqx_solve started (device time from HIP
   * events on the context stream): 0 C_occ V, 1 (C_occ V) C_virt^T,
   * 2 NDDO contraction G(R), 3 G C_virt, 4 C_occ^T (G C_virt) + de V.
   * Flops and bytes are algorithmic (what the operation must do), not counters. */
  double phase_ms[5];
  int64_t phase_launches[5];
  double phase_flops[5];
  double phase_bytes[5];
  /* Davidson device time by phase in the last seqx_solve (ms, HIP events):
   * 0 sigma build, 1 projected matrices, 2 subspace eigenproblem, 3 Ritz
   * vectors and residuals, 4 convergence check (host read), 5 preconditioner,
   * 6 subspace collapse, 7 orthonormalisation. */
  double dav_phase_ms[8];
  /* Mixed-precision solves (precision != SEQX_FP64): sigma vectors formed with
   * FP64 transforms, and the iteration at which the solve restarted from its
   * Ritz vectors with FP64 products (0 when it never ran in low precision). */
  int64_t n_sigma_fp64;
  int32_t refine_iteration;
  /* Batched solves: wall time of the tile autotuner (excluded from t_davidson_s;
   * zero once the context has tuned every size bucket), whether the iteration
   * ran as a replayed HIP graph, and the tile variant (0: 16x16, 1: 32x16,
   * 2: 32x32 MFMA tiles per wavefront) chosen for molecules with n < 32, < 64,
   * < 96, < 128 and larger. */
  double t_autotune_s;
  int32_t batched_graph;
  int32_t tile_variant[5];
  double batched_sigma_flops; /* algorithmic transform flops of the batched products, 4 n v (n + o) each */
  /* Single-molecule solves: the largest subspace reached and the subspace cap
   * used (max over molecules), and the number of restarts from the Ritz
   * vectors because the cap was reached (summed over molecules). */
  int32_t max_subspace_used;
  int32_t subspace_cap;
  int32_t n_collapses;
  /* SEQX_BF16X3 solves: the iteration at which the solve restarted from its
   * Ritz vectors with FP32 products (0 when it did not), and the sigma vectors
   * formed with split-bfloat16 transforms. */
  int32_t fp32_iteration;
  int64_t n_sigma_bf16x3;
} seqx_stats;

/* Version of this header the library was built with (SEQX_ABI_VERSION). */
int seqx_abi_version(void);

/* Host-only input check (the same one seqx_prepare runs): Z in {1, 6, 8},
 * even electron count per molecule, finite coordinates, no two atoms of a
 * molecule closer than 0.1 Angstrom.  msg (optional, msglen bytes) receives
 * the reason.  Needs no GPU. */
seqx_status seqx_validate(int32_t nmol, const int32_t* natoms, const int32_t* Z,
                          const double* xyz_angstrom, char* msg, size_t msglen);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to order
 * all work on (e.g. torch's current stream) or NULL for the null stream.
 * Returns SEQX_E_DEVICE when no GPU is usable. */
seqx_status seqx_create(int device, void* hip_stream, seqx_ctx** out);
/* Frees the context's device memory (through the allocators it was made with).
 * Free the context's jobs first: a job uses its context until it is freed. */
void seqx_destroy(seqx_ctx* ctx);
/* Text of the last error on this context (owned by ctx, valid until the next call). */
const char* seqx_last_error(const seqx_ctx* ctx);

/* Element parameters: nelem rows of SEQX_NPARAM values for atomic numbers Z[nelem].
 * The paper runs AM1 for every result; any NDDO parameter set of this form may
 * be given.  Derived multipole lengths and additive terms are computed here. */
seqx_status seqx_set_params(seqx_ctx* ctx, int32_t nelem, const int32_t* Z, const double* values);

/* Parameter sets by method.  SEQX_PARAMS_FILE reads a JSON file
 *   {"elements": {"<Z>": {"zeta_s": .., "zeta_p": .., "U_ss": .., "U_pp": ..,
 *                          "beta_s": .., "beta_p": .., "g_ss": .., "g_sp": ..,
 *                          "g_pp": .., "g_p2": .., "h_sp": ..}, ...}, ...}
 * (eV, exponents in 1/bohr; absent entries, e.g. the p terms of H, are 0) and
 * applies it as seqx_set_params would.  The published MNDO / AM1 / PM3 tables
 * (the paper's AM1 runs, "Theory and implementation") are not bundled: those
 * methods return SEQX_E_ARG.  Errors: SEQX_E_ARG for an unreadable or malformed
 * file, SEQX_E_ELEMENT for an unsupported Z. */
typedef enum { SEQX_MNDO = 0, SEQX_AM1 = 1, SEQX_PM3 = 2, SEQX_PARAMS_FILE = 3 } seqx_method;
seqx_status seqx_load_params(seqx_ctx* ctx, seqx_method method, const char* json_path);

/* Device memory of everything this context and its jobs allocate from now on
 * comes from alloc(bytes, user) and goes back through release(ptr, user)
 * (e.g. a framework's caching allocator), instead of hipMalloc / hipFree.
 * alloc must return device memory of the context's GPU, or NULL (the call then
 * fails with SEQX_E_NOMEM).  Buffers keep the allocator that made them; the
 * device is synchronised before a buffer is handed back, so a stream-ordered
 * allocator may reuse it at once.  Both NULL: back to hipMalloc / hipFree for
 * new buffers.  Exactly one NULL: SEQX_E_ARG.  Jobs must be freed before their
 * context is destroyed. */
seqx_status seqx_set_allocator(seqx_ctx* ctx, void* (*alloc)(size_t bytes, void* user),
                               void (*release)(void* ptr, void* user), void* user);

/* Integrals + RHF SCF (paper: ground-state subsection, Eq. 1 with S = I; the
 * two-centre integrals are computed once before the SCF and kept, as in the
 * GPU-implementation subsection) for nmol molecules given as concatenated arrays:
 * natoms[nmol], Z[sum natoms], xyz_angstrom[sum natoms][3].  opts may be NULL.
 * The job keeps C, eps, the ERI tables and the core Hamiltonian on the device.
 * From four molecules on (and no caller allocator set) the molecules are
 * prepared concurrently by library threads on internal streams, after the
 * context's stream has drained; the call returns once all of them are done.
 * The environment variable SEQX_PREPARE_THREADS (1 .. 64, default 8) sets the
 * number of those threads; 1 prepares on the calling thread. */
seqx_status seqx_prepare(seqx_ctx* ctx, int32_t nmol, const int32_t* natoms, const int32_t* Z,
                         const double* xyz_angstrom, const seqx_scf_opts* opts, seqx_job** out);
void seqx_job_free(seqx_job* job);

seqx_status seqx_dims(const seqx_job* job, int32_t mol, int32_t* nao, int32_t* nocc, int32_t* nvirt);

/* Ground state of molecule `mol`: eps_eV[nao], C[nao][nao] (row mu = AO, column p = MO),
 * P[nao][nao] = 2 C_occ C_occ^T.  Any output may be NULL. */
seqx_status seqx_scf_results(const seqx_job* job, int32_t mol, double* eps_eV, double* C, double* P);

/* Core Hamiltonian H[nao][nao] in hartree (U on the diagonal, core attraction
 * on atom-diagonal blocks, resonance (beta_mu+beta_nu)/2 S_mu,nu between atoms). */
seqx_status seqx_core_hamiltonian(const seqx_job* job, int32_t mol, double* H);

/* Packed ERI matrix W[np][np] (hartree), np = sum over atoms of 10 (C, O) or 1 (H):
 * W[P][Q] = (mu nu | lam sig) with P = (mu <= nu) on one atom and Q = (lam <= sig)
 * on one atom; pairs of an atom ordered ss, s px, s py, s pz, px px, px py,
 * px pz, py py, py pz, pz pz; atoms in input order.  Diagonal atom blocks hold
 * the one-centre integrals.  cap: capacity of out in doubles; *needed = np*np. */
seqx_status seqx_integrals(const seqx_job* job, int32_t mol, double* out, size_t cap, size_t* needed);

/* Matrix-free products (Eqs. 8-9) for k host vectors V[k][nocc][nvirt]:
 *   theory CIS : out1 = A V            (out2 unused, may be NULL)
 *   theory TDHF: out1 = (A+B) V, out2 = (A-B) V
 * in hartree, with the transforms in `precision` (SEQX_FP64 or SEQX_FP32; the
 * others return SEQX_E_ARG).  Blocking host copy. */
seqx_status seqx_sigma(seqx_job* job, int32_t mol, int32_t theory, int32_t k, const double* V,
                       double* out1, double* out2, int32_t precision);
/* Same on device buffers (ordered on the context stream, no host sync). */
seqx_status seqx_sigma_device(seqx_job* job, int32_t mol, int32_t theory, int32_t k, const double* dV,
                              double* dout1, double* dout2, int32_t precision);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the products
 * of seqx_sigma_device with every intermediate (AO matrices, transform
 * intermediates, contraction work arrays) taken from one fixed workspace of
 * SEQX_SIGMA_SCRATCH_BYTES per GPU, a device array of the library that each
 * GPU it runs on holds until the process ends.  No allocator is called (no
 * hipMalloc / hipFree, no caller allocator, no events); the vectors are
 * processed in passes of as many as fit.  The caller passes device inputs and
 * outputs as for seqx_sigma_device, ordered on the context stream.
 * Limit: one vector's intermediates must fit the workspace: for n AOs,
 * v virtual MOs and np same-atom AO pairs about 8 (3 n^2 + 3 n v) + 24 np
 * bytes for TDHF in FP64 (CIS: 8 (2 n^2 + 2 n v) + 24 np) and half of the
 * matrix terms in FP32, so a 1980-AO molecule still runs one vector per pass
 * in FP64.  Beyond it the call returns SEQX_E_BUFSIZE and writes nothing.  Every call on one GPU shares that GPU's
 * workspace, which keeps the last call's contents (every element is written
 * before it is read): calls that overlap in time on one GPU, from any
 * context or stream, race and must be ordered by the caller. */
#define SEQX_SIGMA_SCRATCH_BYTES (128u << 20)
seqx_status seqx_sigma_device_noalloc(seqx_job* job, int32_t mol, int32_t theory, int32_t k, const double* dV,
                                      double* dout1, double* dout2, int32_t precision);

/* Davidson for every molecule of the job (seqx_solve_opts above). */
seqx_status seqx_solve(seqx_job* job, const seqx_solve_opts* opts);

/* Results of molecule `mol` after seqx_solve (the K lowest roots of Eq. 2 or
 * Eq. 7; transition dipoles and oscillator strengths as used for the spectra
 * in the results section): omega_eV[K], X[K][nocc][nvirt],
 * Y[K][nocc][nvirt] (zero for CIS), f[K] oscillator strengths,
 * mu[K][3] transition dipoles (atomic units).  Any output may be NULL. */
seqx_status seqx_results(const seqx_job* job, int32_t mol, double* omega_eV, double* X, double* Y,
                         double* f, double* mu);

/* Absorption spectrum of molecule `mol` after seqx_solve (results section of
 * the paper: oscillator strengths of every state, then Gaussian broadening of
 * width 0.1 eV into a continuous profile):
 *   out[i] = sum_n f_n exp(-(E_i - omega_n)^2 / (2 sigma^2)) / (sigma sqrt(2 pi)),
 *   E_i = e0_eV + i de_eV, i < npts (host out[npts], 1/eV),
 * over the solved roots.  sigma_eV is the standard deviation (the paper's width
 * read as such; full width at half maximum = 2.3548 sigma); the lines have unit
 * area, so the profile integrates to the summed oscillator strength.
 * SEQX_E_ARG for sigma_eV <= 0, de_eV <= 0 or npts <= 0; SEQX_E_STATE before a solve. */
seqx_status seqx_spectrum(const seqx_job* job, int32_t mol, double sigma_eV, double e0_eV, double de_eV,
                          int32_t npts, double* out);
/* The same profile for K caller lines (host omega_eV[K], f[K]), e.g. roots
 * gathered from several solves. */
seqx_status seqx_broaden(seqx_ctx* ctx, int32_t K, const double* omega_eV, const double* f, double sigma_eV,
                         double e0_eV, double de_eV, int32_t npts, double* out);

/* Derivatives of the solved excitation energies of molecule `mol` with respect
 * to every NDDO parameter, for re-optimising the parameters against excited-state
 * data (the paper's machine-learning interface, which its conclusion extends to
 * excited states).  grad[K][3][SEQX_NPARAM] (host, cap values): root, element
 * (H, C, O) and parameter in the seqx_set_params order; eV per eV, or eV per
 * 1/bohr for the exponents; zero for elements absent from the molecule and for
 * the p terms of H.  The orbital response is one linear solve with A+B per root
 * (the CIS and TDHF amplitude equations are stationary, so only the orbitals
 * respond); the integral derivatives are central differences of the library's
 * integral tables (step 1e-5 of each value).  zvector_iterations (optional)
 * receives the largest number of conjugate-gradient steps of that solve.
 * SEQX_E_STATE before a solve; SEQX_E_BUFSIZE when cap is too small. */
seqx_status seqx_param_gradient(seqx_job* job, int32_t mol, double* grad, size_t cap, int32_t* zvector_iterations);

seqx_status seqx_get_stats(const seqx_job* job, seqx_stats* out);

/* Convergence history of molecule `mol` in the last seqx_solve: per Davidson
 * iteration, the wall time since the solve started (t_s[it], seconds) and the
 * K Ritz values (omega_eV[it][K]).  cap: capacity in iterations; *n_iter
 * receives the iteration count (SEQX_E_BUFSIZE if it exceeds cap; t_s and
 * omega_eV may be NULL to query it). */
seqx_status seqx_history(const seqx_job* job, int32_t mol, int32_t cap, int32_t* n_iter, double* t_s,
                         double* omega_eV);

/* ---- Learned starting space -------------------------------------------------
 * The paper's closing outlook lists machine-learned initial guesses for the
 * Davidson iteration; these calls build one.  Per pair i -> a, 12 features (hartree, bohr): gap, eps_HOMO - eps_i,
 * eps_a - eps_LUMO, sum_A q_A^2, the four largest |q_A| (q_A: transition
 * Mulliken charge on atom A), sum_A g_A q_A^2, sum_A g_A p_A^i p_A^a (p: orbital
 * populations, g_A = (s_A s_A|s_A s_A)), the distance of the two orbital
 * centroids, and gap + 2 f8 - f9.  Network: standardise with (mu, sd), then
 * 12 -> 128 -> 128 -> 1 with SiLU; weight matrices used as bfloat16 values,
 * activations and sums in FP32.  Training target of a molecule with K solved
 * CIS roots: w_ia = (1/K) sum_n X[n][i][a]^2; loss: mean over molecules of the
 * softmax cross-entropy of the scores against w; optimiser: Adam. */
#define SEQX_MLP_NFEAT 12
#define SEQX_MLP_WIDTH 128
/* flat FP32 parameters: W1[12][128], b1[128], W2[128][128], b2[128], w3[128], b3 */
#define SEQX_MLP_NWEIGHTS 18305
/* ... then the feature means mu[12] and scales sd[12] */
#define SEQX_MLP_NPARAMS 18329

typedef struct {
  int32_t epochs;   /* passes over the training molecules; <= 0 selects 30 */
  int32_t batch;    /* molecules per optimiser step; <= 0 selects 32 */
  double lr;        /* Adam step size; <= 0 selects 2e-3 */
  uint64_t seed;    /* initial weights and molecule order */
  int32_t init;     /* nonzero: fresh weights and feature standardisation from the training set */
} seqx_train_opts;

typedef struct {
  int32_t n_epochs;
  double seconds;     /* wall time of the training (features, targets, epochs) */
  double loss[256];   /* mean training loss of each epoch (first 256) */
} seqx_train_log;

/* Network parameters of the context (SEQX_MLP_NPARAMS floats, layout above). */
seqx_status seqx_mlp_set_params(seqx_ctx* ctx, const float* params, size_t n);
seqx_status seqx_mlp_get_params(const seqx_ctx* ctx, float* out, size_t cap, size_t* needed);
/* Binary file: 8-byte tag "SEQXMLP1", int32 count, then the FP32 parameters. */
seqx_status seqx_mlp_save(const seqx_ctx* ctx, const char* path);
seqx_status seqx_mlp_load(seqx_ctx* ctx, const char* path);
/* Train the context's network on the job's molecules, which must hold solved
 * CIS roots (seqx_solve with theory CIS); their amplitudes are the targets. */
seqx_status seqx_mlp_train(seqx_job* job, const seqx_train_opts* opts, seqx_train_log* log);
/* Features of molecule `mol` (host out [nocc*nvirt][12], cap in floats). */
seqx_status seqx_features(const seqx_job* job, int32_t mol, float* out, size_t cap);
/* Network scores of every pair of molecule `mol` (host z [nocc*nvirt]). */
seqx_status seqx_mlp_scores(const seqx_job* job, int32_t mol, float* z, size_t cap);
/* Loss and weight gradient (host grad[SEQX_MLP_NWEIGHTS]) of the context's
 * network on host features [npairs][12] and targets w[npairs], molecules given
 * by nmol + 1 pair offsets seg (seg[0] = 0, seg[nmol] = npairs). */
seqx_status seqx_mlp_loss_grad(seqx_ctx* ctx, int64_t npairs, const float* feats, const float* w, int32_t nmol,
                               const int64_t* seg, double* loss, float* grad);

#ifdef __cplusplus
}
#endif

#endif /* SEQX_H */
