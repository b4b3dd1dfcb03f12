/*
 * mgdwf.h -- C ABI of the MI355X library for adaptive multigrid on the
 * Shamir domain-wall fermion operator.
 *
 * Method: S. D. Cohen, R. C. Brower, M. A. Clark, J. C. Osborn, "Multigrid
 * Algorithms for Domain-Wall Fermions" (Lattice 2011).  Section numbers below
 * refer to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 * Canonical arrays are complex128, interleaved (re, im) doubles, C order:
 *   4D site     x4 = ((t*Lz + z)*Ly + y)*Lx + x;  direction mu = 0..3 is x, y, z, t
 *   fermion     ((x4*Ls + s)*4 + spin)*3 + colour          (12*Ls*V4 complex)
 *   gauge       ((x4*4 + mu)*3 + a)*3 + b = U_mu(x)[a][b]   (36*V4 complex)
 *   vector set  [k][fermion]                                 (k = 0..n-1)
 *   coarse site X4 = ((T*LZ + Z)*LY + Y)*LX + X, X = x / block_x, ...
 *   coarse vec  (X4*2 + chi)*Nv + k; chi = 0 spins {0,1} (P+), chi = 1 spins {2,3}
 *   coarse op   Dc[X4][d][row][col], row/col = chi*Nv + k, d = 0 self,
 *               d = 1+2mu neighbour +mu, d = 2+2mu neighbour -mu;
 *               (D_c y)(X) = sum_d Dc[X][d] y(X + delta_d), periodic.
 * Several right-hand sides (nrhs) are stacked along a leading axis.
 *
 * Pointers: every array argument is a DEVICE pointer on the handle's device
 * (for instance a torch tensor's data_ptr()) unless the argument list says
 * otherwise.  The caller owns every buffer it passes; the library copies what
 * it keeps (gauge field, basis, coarse operator) into its own internal layouts
 * and never retains a caller pointer after a call returns.
 *
 * Streams: a handle is bound to the HIP stream given at creation and is not
 * thread safe.  apply/restrict/prolong/apply_coarse are stream ordered and
 * asynchronous; set_gauge, set_nullvecs, build_coarse, setup, solve and the
 * get_* calls return after their work has completed.
 *
 * Errors: every call returns an mgdwf_status; nothing throws across this
 * boundary and nothing aborts.  mgdwf_last_error(h) gives a message for the
 * last failure on h (mgdwf_last_error(NULL) for a failed create).  Arguments
 * are validated before any device work.  On MGDWF_ERR_NOT_CONVERGED the
 * solution buffer holds the best iterate and the report is filled; after any
 * other error outputs are undefined.
 */
#ifndef MGDWF_H
#define MGDWF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgdwf_ctx* mgdwf_handle;

typedef enum {
  MGDWF_OK = 0,
  MGDWF_ERR_INVALID_ARG = 1,  /* bad size, block, precision, null pointer   */
  MGDWF_ERR_OOM = 2,          /* device allocation failed                   */
  MGDWF_ERR_HIP = 3,          /* a HIP runtime call failed                  */
  MGDWF_ERR_NOT_CONVERGED = 4,/* solve hit max iterations / stagnated       */
  MGDWF_ERR_STATE = 5,        /* call out of order, e.g. solve before setup */
  MGDWF_ERR_NUMERIC = 6       /* NaN/Inf, or a rank-deficient block panel   */
} mgdwf_status;

typedef enum { MGDWF_F64 = 0, MGDWF_F32 = 1, MGDWF_F16 = 2, MGDWF_BF16 = 3 } mgdwf_prec;

/* The fine operator (Sec. 2, fifth-dimension paragraph; Sec. 4, stencil of one
 * site plus ten unit neighbours).  Shamir form:
 *   (D psi)(x,s) = (5 - M5) psi(x,s)
 *       - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu,s) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu,s)]
 *       - P_- psi(x,s+1) - P_+ psi(x,s-1),  walls closed by +m_f,
 * gamma matrices in the chiral basis with g5 = diag(1,1,-1,-1).
 * Every extent must be >= 2; bc[mu] is +1 (periodic) or -1 (antiperiodic). */
typedef struct {
  int32_t L[4];
  int32_t Ls;
  double M5;
  double mf;
  int32_t bc[4];
} mgdwf_action;

/* The two-dimensional U(1) test problem of Sec. 3 (Fig. 2): the same Shamir
 * form on a 2D lattice with U(1) links,
 *   (D psi)(x,s) = (3 - M5) psi(x,s)
 *       - 1/2 sum_{mu=x,y} [(1 - g_mu) U_mu(x) psi(x+mu,s) + (1 + g_mu) conj(U_mu(x-mu)) psi(x-mu,s)]
 *       - P_- psi(x,s+1) - P_+ psi(x,s-1),  walls closed by +m_f,
 * g_x = sigma_1, g_y = sigma_2, g5 = sigma_3 (P_+ keeps spin 0).  Canonical
 * arrays of a 2D handle (complex128, C order):
 *   2D site     x2 = y*Lx + x
 *   fermion     (x2*Ls + s)*2 + spin                    (2*Ls*Lx*Ly complex)
 *   gauge       x2*2 + mu = U_mu(x), |U| = 1            (2*Lx*Ly complex)
 *   coarse vec  (X2*2 + chi)*Nv + k, chi = spin; blocks are {bx, by, 1, 1}
 *   coarse op   the squared form of mgdwf_get_coarse_op with LZ = LT = 1
 *               (only the offsets self, +-x, +-y and the four xy diagonals
 *               are nonzero).
 * A 2D handle runs the squared-operator multigrid (squared = 1, which the
 * paper used for this test) and every call of the fine level, the transfer,
 * the coarse operator, the solvers, the third level and the checkpoints;
 * the 9-point coarse operator, low_modes, tune, set_tiling, time_kernel and
 * the network calls return MGDWF_ERR_INVALID_ARG for it.  Every extent must
 * be >= 2. */
typedef struct {
  int32_t L[2];
  int32_t Ls;
  double M5;
  double mf;
  int32_t bc[2];
} mgdwf_action2d;

/* Two-level multigrid parameters (Sec. 2). */
typedef struct {
  int32_t block[4];       /* 4D block; each block spans all of Ls (Sec. 2)       */
  int32_t nvec;           /* Nv: basis columns per chirality (coarse dof = 2 Nv)  */
  int32_t sweeps;         /* adaptive sweeps in mgdwf_setup, including sweep 0    */
  int32_t sweep0_iters;   /* CG iterations on D^+D v = 0 in sweep 0               */
  int32_t sweep_iters;    /* flexible-GCR steps with the current V-cycle on        */
                          /* D x = 0 from each vector, per sweep after sweep 0    */
  int32_t nu_pre;         /* smoother steps before the coarse correction          */
  int32_t nu_post;        /* smoother steps after it                              */
  double coarse_tol;      /* relative residual of the coarse solve                */
  int32_t coarse_maxiter; /* iteration cap of the coarse solve                    */
  mgdwf_prec fine_prec;   /* F64 or F32: precision of the V-cycle's fine level    */
  mgdwf_prec coarse_prec; /* F64, F32, F16 or BF16: storage of D_c in the V-cycle */
  int32_t coarse_graph;   /* 1: after the first 8 coarse iterations, replay each
                             block of 8 as one captured HIP graph; 0: launch
                             every kernel.  Results are bitwise the same.
                             2: the whole coarse solve as one persistent
                             cooperative kernel (FP32 fine level, F16/BF16 D_c,
                             nrhs <= 16): at most one workgroup per CU, each
                             owning every G-th coarse site, with the library's
                             own grid barrier, whose waits are bounded (see
                             mgdwf_set_barrier_timeout; a wait that runs out
                             ends the solve with MGDWF_ERR_HIP).  Elsewhere it
                             runs as 1 and sets bit 3 of the report's flags.
                             Same iterations and tests as 1 (the residual
                             every 8 iterations), its sums in another order:
                             results agree to rounding; it skips the last
                             unused D_c^+ apply.  With 1 and 2 the V-cycle's
                             launches before and after the coarse solve are
                             graph replays too.                               */
  int32_t squared;        /* 0: the 9-point D_c = P^+ D P on the gamma5 R5-
                             closed basis.  1: the paper's own multigrid on the
                             squared operator D^+D (Sec. 3 first paragraph,
                             Sec. 4): nvec adaptive vectors (no reflections),
                             A_c = P^+ D^+D P (33-point stencil, Hermitian),
                             V-cycle on D^+D with minimal-residual smoothing
                             (two applications of D per step), CG on A_c,
                             entered with D^+ r so that it preconditions the
                             same flexible GCR on D x = b.  Needs every block
                             extent >= 2 and an F64 or F32 coarse level; the
                             coarse solve runs as launched kernels.            */
  int32_t sweep0_check;   /* 0: sweep 0 returns its last CG iterate.  k > 0: of
                             the iterates after every k CG iterations and
                             after the last, each vector keeps the one with
                             the smallest |D v| / |v| (the earliest on a tie):
                             the Krylov sweep of Sec. 2 is stopped while the
                             vector holds the slowly removed modes (once CG
                             resolves the lowest modes too, the ratio rises
                             again).  One more application of D per vector
                             every k iterations.                               */
  int32_t smoother_dirs;  /* 9-point smoother: 0 keeps every MR direction of
                             one smoother application and forms x once at the
                             end (nu fields per right-hand side); k > 0 keeps
                             at most k and adds them to x every k steps (less
                             memory, one more pass over x per k steps; the
                             sums are grouped differently, so results agree
                             to rounding).                                     */
} mgdwf_mg_params;

/* Outer flexible GCR (Sec. 3).  Every restart recomputes the true residual
 * b - D x in FP64 and restarts the inner cycle from it (iterative refinement). */
typedef struct {
  double tol;             /* stop at |b - D x| / |b| < tol (true FP64 residual)   */
  int32_t max_outer;      /* cap on outer iterations                              */
  int32_t restart;        /* Krylov vectors kept before a restart                 */
} mgdwf_solve_params;

typedef struct {
  int32_t outer_iters;
  int32_t restarts;
  int64_t fine_applies;   /* applications of D or D^+, the paper's cost measure  */
  int64_t coarse_applies; /* applications of D_c or D_c^+                          */
  double true_relres;     /* |b - D x| / |b| in FP64 at return                    */
  double seconds;         /* wall time of the call                                */
  uint32_t flags;         /* bit 0: NaN/Inf met; bit 1: stagnation; bit 2: a   */
                          /* second Gram-Schmidt pass was needed in the FGCR;   */
                          /* bit 3: the persistent coarse solve was asked for   */
                          /* but did not apply (launched loop used instead)     */
  double phase_seconds[3]; /* device time of the V-cycle's phases summed over   */
                          /* the call, from HIP events on the handle's stream:  */
                          /* [0] pre-smoother + restriction, [1] coarse solve   */
                          /* (with the host's convergence checks), [2]          */
                          /* prolongation + residual + post-smoother.  The rest */
                          /* of `seconds` is the outer FGCR and the FP64 true  */
                          /* residuals.  Zero for mgdwf_cgne.                  */
} mgdwf_solve_report;

/* Setup report: median |D v|/|v| over the adaptive vectors after each sweep. */
typedef struct {
  int32_t sweeps_done;
  double null_residual[8];
  double seconds;
} mgdwf_setup_report;

/* ---- lifetime ---------------------------------------------------------- */

/* Create a handle for one lattice and action, bound to `hip_stream` (a
 * hipStream_t, NULL for the default stream) on the current device. */
mgdwf_status mgdwf_create(const mgdwf_action* action, void* hip_stream, mgdwf_handle* out);
/* A handle for the 2D U(1) problem (Sec. 3, Fig. 2; layouts above). */
mgdwf_status mgdwf_create_2d(const mgdwf_action2d* action, void* hip_stream, mgdwf_handle* out);
mgdwf_status mgdwf_destroy(mgdwf_handle h);
/* Message of the last failure on h, or of the last failed create if h is NULL. */
const char* mgdwf_last_error(mgdwf_handle h);

/* Copy the gauge field (canonical complex128, device) into the internal
 * FP64 and FP32 link layouts.  Invalidates any basis / coarse operator. */
mgdwf_status mgdwf_set_gauge(mgdwf_handle h, const double* U);

/* ---- fine operator (step a1) ------------------------------------------ */

/* out = D in (dagger = 0) or D^+ in (dagger = 1) for nrhs canonical fields.
 * prec = F64 computes in FP64; F32 converts in to FP32, applies the FP32
 * kernel and converts back.  in and out must not overlap. */
mgdwf_status mgdwf_apply_dwf(mgdwf_handle h, const double* in, double* out, int32_t dagger,
                             mgdwf_prec prec, int32_t nrhs);

/* ---- transfer (steps a3-a5): Sec. 1 (R, P, RP = 1) and Sec. 2 --------- */

/* Install nvec near-null vectors (canonical, device) with the given block:
 * split each by chirality, orthonormalise every (block, chirality) panel in
 * FP64 (thin QR, columns in order, positive real diagonal) and keep the basis.
 * Fails with MGDWF_ERR_NUMERIC for a rank-deficient panel and
 * MGDWF_ERR_INVALID_ARG if the block does not divide the lattice or
 * nvec > 6 * Ls * (block volume). */
mgdwf_status mgdwf_set_nullvecs(mgdwf_handle h, const int32_t block[4], const double* V,
                                int32_t nvec);
/* The near-null vectors the installed basis was built from, canonical
 * [n][fermion]: after mgdwf_setup the nvec/2 adaptive vectors (normalised, before
 * they are paired with their reflections), after mgdwf_set_nullvecs the nvec
 * vectors given.  *n receives the count; with V == NULL only the count is
 * written.  MGDWF_ERR_STATE before any setup or set_nullvecs. */
mgdwf_status mgdwf_get_nullvecs(mgdwf_handle h, double* V, int32_t* n);
/* The orthonormal basis, canonical [Nv][fermion] (both chirality columns of
 * vector k in field k). */
mgdwf_status mgdwf_get_basis(mgdwf_handle h, double* Vhat);
/* coarse = R fine  (R = P^+), nrhs canonical fine fields -> coarse vectors.
 * prec F64, or F32: the V-cycle's kernels on FP32 copies of the basis and
 * the fields (inputs rounded to FP32, results returned as complex128). */
mgdwf_status mgdwf_restrict(mgdwf_handle h, const double* fine, double* coarse, int32_t nrhs, mgdwf_prec prec);
/* fine = P coarse, same precisions. */
mgdwf_status mgdwf_prolong(mgdwf_handle h, const double* coarse, double* fine, int32_t nrhs, mgdwf_prec prec);

/* ---- coarse operator (steps a6, a7): Sec. 2 step 3, Sec. 4 ------------ */

/* Build D_c = R D P as the 9-point stencil of dense 2Nv x 2Nv blocks (FP64),
 * plus its FP32, FP16 and BF16 copies with one scale per block. */
mgdwf_status mgdwf_build_coarse(mgdwf_handle h);
/* Build the squared operator's coarse operator A_c = P^+ D^+ D P (Sec. 3,
 * Sec. 4) on the installed basis: a stencil over the 33 offsets o = self,
 * +mu / -mu (index 1 + 2 mu / 2 + 2 mu), then for mu < nu the diagonals
 * (+mu+nu, +mu-nu, -mu+nu, -mu-nu), with (A_c y)(X) = sum_o Ac[X][o] y(X + o).
 * Every block extent must be >= 2 (MGDWF_ERR_INVALID_ARG otherwise).  It
 * replaces the 9-point operator for apply_coarse, get_coarse_op and solves
 * with squared = 1. */
mgdwf_status mgdwf_build_coarse_squared(mgdwf_handle h);
/* Offsets of the coarse operator built last: 9 (D_c), 33 (A_c), -1 if none. */
int32_t mgdwf_coarse_stencil_size(mgdwf_handle h);
/* Copy the FP64 coarse operator out (canonical layout, complex128):
 * [X4][d][row][col] over the 9 or 33 offsets of the operator built last. */
mgdwf_status mgdwf_get_coarse_op(mgdwf_handle h, double* Dc);
/* out = D_c in (dagger 0) or D_c^+ in (dagger 1), nrhs canonical coarse
 * vectors, computed with the operator stored in `prec` (F16/BF16 use MFMA with
 * FP32 accumulation; inputs are converted with one scale per site and RHS). */
mgdwf_status mgdwf_apply_coarse(mgdwf_handle h, const double* in, double* out, int32_t dagger,
                                mgdwf_prec prec, int32_t nrhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation and kernels as mgdwf_apply_coarse, allocating nothing.  Reduced
 * precisions stage the FP32 input and output (and the 16-bit packed input)
 * in a static 16 MiB device array that the library holds on every GPU it
 * runs on until the process ends: 2 x (nrhs Vc 2Nv x 8 B, rounded up to 256 B)
 * plus, for F16/BF16, nrhs Vc (4 Nv x 2 B + 4 B) + 256 B must fit, else
 * MGDWF_ERR_INVALID_ARG (F64 needs no scratch).  Every call on one GPU
 * shares that array: calls that overlap on the same GPU (on different
 * streams or from different threads) race and must be ordered by the
 * caller.  Stream ordered and asynchronous, like mgdwf_apply_coarse. */
mgdwf_status mgdwf_apply_coarse_noalloc(mgdwf_handle h, const double* in, double* out, int32_t dagger,
                                        mgdwf_prec prec, int32_t nrhs);

/* ---- setup and solve (steps a8-a11): Sec. 2, Sec. 3 -------------------- */

/* Adaptive setup (Sec. 2): starting from nvec/2 random vectors V0 (nvec when
 * p->squared; canonical, device; the random numbers are inputs), sweep 0 runs sweep0_iters CG
 * iterations on D^+D v = 0 from each; every later sweep applies the current
 * multigrid to the same problem: sweep_iters flexible-GCR steps with the
 * FP64 V-cycle on D x = 0 starting from x = v, and v becomes the x they leave
 * (what the multigrid fails to remove).  After each sweep every vector is
 * normalised, paired with its fifth-dimension reflection, and the basis and
 * D_c are rebuilt.  report may be NULL. */
mgdwf_status mgdwf_setup(mgdwf_handle h, const mgdwf_mg_params* p, const double* V0,
                         mgdwf_setup_report* report);
/* Set the V-cycle parameters used by mgdwf_solve without a new setup
 * (block and nvec must equal the installed basis). */
mgdwf_status mgdwf_set_mg_params(mgdwf_handle h, const mgdwf_mg_params* p);

/* Solve D x = b for nrhs right-hand sides (canonical, device) with flexible
 * GCR preconditioned by the two-level V-cycle; x holds the initial guess on
 * entry (zero it for a cold start).  reports[nrhs] may be NULL. */
mgdwf_status mgdwf_solve(mgdwf_handle h, const double* b, double* x, int32_t nrhs,
                         const mgdwf_solve_params* p, mgdwf_solve_report* reports);

/* out = M in: one application of the two-level V-cycle (Sec. 2, its five
 * steps: pre-smoothing, restriction, coarse solve, prolongation with the
 * residual update, post-smoothing) in the precisions and counts of the
 * current parameters, to nrhs canonical fields (FP32 fine levels round `in`
 * to FP32 and return the result as complex128).  Returns after completion. */
mgdwf_status mgdwf_apply_vcycle(mgdwf_handle h, const double* in, double* out, int32_t nrhs);

/* ---- a third level (Sec. 2: the coarse solve done by the same multigrid) -- */

/* Under the squared coarse operator A_c = P^+ D^+D P a further level: Nv2
 * near-null vectors of A_c (CG on A_c w = 0, null_iters steps from each
 * start), split by the coarse chirality and orthonormalised per block of
 * coarse sites (R2 = W^+, P2 = W), and A_cc = R2 A_c P2 as a 33-offset
 * stencil.  With gamma > 0 the squared V-cycle's coarse solve becomes gamma
 * sweeps of e <- e + K2(b - A_c e) from e = 0 (gamma = 1: V-cycle, 2:
 * W-cycle), K2 = nu MR steps on A_c, R2, CG on A_cc (coarse_tol,
 * coarse_maxiter; residual tested every 8 iterations), P2, nu MR steps; with
 * gamma = 0 it stays CG on A_c.  Applications of A_cc count as coarse
 * applications in the solve report. */
typedef struct {
  int32_t block[4];       /* coarse sites per level-2 block, x y z t (dividing the coarse lattice) */
  int32_t nvec;           /* Nv2: level-2 basis columns per chirality, 1..32, at most the rows of a panel */
  int32_t null_iters;     /* CG steps on A_c w = 0 per start (>= 0)                 */
  int32_t nu;             /* MR steps on A_c before and after the level-2 correction */
  double coarse_tol;      /* CG on A_cc: stop at |r| <= coarse_tol |b|              */
  int32_t coarse_maxiter; /* CG on A_cc: iteration cap (>= 1)                       */
  int32_t gamma;          /* level-2 cycles per coarse solve: 0 off, 1 V, 2 W (<= 4) */
} mgdwf_level2_params;
/* Needs the squared coarse operator (a squared setup or
 * mgdwf_build_coarse_squared).  W0: nvec starts on the coarse lattice
 * (device, complex128 [k][Vc][2][Nv], the coarse-vector layout of
 * mgdwf_restrict; the random numbers are an input).  null_residual (host,
 * may be NULL): median |A_c w| / |w| of the normalised near-null vectors.
 * A later setup or coarse build removes the level. */
mgdwf_status mgdwf_setup_level2(mgdwf_handle h, const mgdwf_level2_params* p, const double* W0,
                                double* null_residual);
/* Change nu, coarse_tol, coarse_maxiter and gamma without a new level-2
 * setup (block and nvec must be the installed ones). */
mgdwf_status mgdwf_set_level2_params(mgdwf_handle h, const mgdwf_level2_params* p);
/* The level-2 near-null vectors W (nvec coarse vectors), its orthonormal
 * basis What (nvec coarse vectors; column (block, chi, j) of What_j) and
 * A_cc (canonical [B][33][row][col] of 2Nv2 x 2Nv2 blocks, offsets in the
 * order of the squared coarse operator); device pointers, any may be NULL. */
mgdwf_status mgdwf_get_level2(mgdwf_handle h, double* W, double* What, double* Acc);

/* ---- setup checkpoints ------------------------------------------------ */

/* The adaptive setup is paid once per gauge field and reused for every
 * right-hand side (Sec. 2): save it to restart without repeating it.
 * mgdwf_save_setup writes to `path` (host file, overwritten) the installed
 * orthonormal basis (Nv canonical FP64 fields), the near-null vectors it was
 * built from, the block, the coarse operator kind (9-point or squared), the
 * lattice geometry, M5, m_f, the boundary signs and a 64-bit checksum
 * (FNV-1a) of the installed FP64 links.  Needs a built coarse operator.
 * mgdwf_load_setup reads such a file into a handle whose gauge field is set:
 * MGDWF_ERR_STATE if the geometry, the action or the gauge checksum differ,
 * MGDWF_ERR_INVALID_ARG for an unreadable or corrupt file; it installs the
 * basis as saved (no re-orthonormalisation, so the coarse operator and later
 * solves repeat the saved handle's bit for bit), rebuilds the coarse operator
 * of the saved kind and clears the solver parameters (set them with
 * mgdwf_set_mg_params).  A file that fails after its header checks (a
 * truncated one) leaves the handle with no basis.  Files hold Nv + (near-null count) fields of 12 V5
 * complex128 each. */
mgdwf_status mgdwf_save_setup(mgdwf_handle h, const char* path);
mgdwf_status mgdwf_load_setup(mgdwf_handle h, const char* path);

/* ---- low modes and the coarse space (Sec. 2, Fig. 1) ------------------ */

/* Lowest nev eigenpairs of D^+D, by m Lanczos steps (nev <= m <= 256) on
 * (D^+D)^-1 with full reorthogonalisation; each step is two solves of D with
 * the installed multigrid to solve_tol (D^-1 G D^-1 G, G = gamma5 R5, since
 * D^+ = G D G; flexible GCR restarted every 16, at most 2000 iterations;
 * MGDWF_ERR_NOT_CONVERGED if a solve misses solve_tol).  v0: start vector (canonical, device; the random numbers are
 * an input).  evals: host, nev eigenvalues ascending.  evecs: device,
 * canonical [nev][fermion], unit norm, may be NULL.  resid: host,
 * |D^+D y - lambda y| / lambda per pair, may be NULL.  Needs a setup
 * (or set_nullvecs + build + set_mg_params). */
mgdwf_status mgdwf_low_modes(mgdwf_handle h, const double* v0, int32_t nev, int32_t m, double solve_tol,
                             double* evals, double* evecs, double* resid);
/* frac[i] = |P R e_i|^2 / |e_i|^2 (host, n entries) for n fields e (canonical,
 * device): how much of each lies in the coarse space of the installed basis. */
mgdwf_status mgdwf_coarse_coverage(mgdwf_handle h, const double* e, int32_t n, double* frac);

/* Release every workspace the handle has grown (solver, setup and timing
 * buffers); later calls allocate what they need again.  The gauge field, the
 * basis and D_c are kept. */
mgdwf_status mgdwf_trim(mgdwf_handle h);

/* Device bytes the handle holds (fields, basis, D_c, workspaces); -1 if h is NULL. */
int64_t mgdwf_memory_bytes(mgdwf_handle h);

/* Ragged batch: handle hs[i] solves nrhs[i] right-hand sides b[i] -> x[i]
 * (device pointers, as mgdwf_solve), every handle on its own stream and host
 * thread, so solves on lattices of different sizes overlap on the device.
 * Handles must be distinct and each must have its own stream for the overlap.
 * reports: sum(nrhs) entries, handle after handle.  Returns MGDWF_OK, or
 * MGDWF_ERR_NOT_CONVERGED if some solve missed the tolerance (its x holds the
 * best iterate), or the first other error (message on that handle). */
mgdwf_status mgdwf_solve_batch(const mgdwf_handle* hs, int32_t n, const double* const* b, double* const* x,
                               const int32_t* nrhs, const mgdwf_solve_params* p, mgdwf_solve_report* reports);

/* Control solver of Sec. 3: CG on the normal equations (CGNE), FP64. */
mgdwf_status mgdwf_cgne(mgdwf_handle h, const double* b, double* x, const mgdwf_solve_params* p,
                        mgdwf_solve_report* report);

/* ---- learned near-null proposals --------------------------------------- */

/* A gauge-covariant network proposes the 4D part of near-null vectors from
 * the gauge field and seeded noise; the fifth dimension is the free-field
 * wall profile (every low mode shares it: the paper's Sec. 2, last
 * paragraph).  Layer: out_o = sum_{d,i} W[d][o][i] T_d in_i with T_0 = 1,
 * T_{1+2mu} f(x) = U_mu(x) f(x+mu), T_{2+2mu} f(x) = U_mu(x-mu)^+ f(x-mu);
 * gate f |f|^2/(1+|f|^2) after layers 1..3; output channel 4k+alpha = spin
 * alpha of proposal k; lift v_k(x,s) = P+ f_k w^(Ls-1-s) + P- f_k w^s,
 * w = 1 - M5.  FP32 arithmetic, BF16 weights, FP32 Adam master weights. */
typedef struct mgdwf_net_s* mgdwf_net;

typedef struct {
  int32_t channels[5]; /* input, three hidden, output (output = 4 x proposals) */
  double lam;          /* weight of the Gram term of the training loss         */
  uint64_t seed;       /* initial weights of layer l ~ N(0, 1/(9 channels[l])) */
} mgdwf_net_config;

mgdwf_status mgdwf_net_create(const mgdwf_net_config* cfg, mgdwf_net* out);
mgdwf_status mgdwf_net_destroy(mgdwf_net net);
/* Message of the last failed call on net (of the last failed create if NULL);
 * calls that also take a handle store their message on the handle too. */
const char* mgdwf_net_last_error(mgdwf_net net);
/* Weights, HOST float arrays of mgdwf_net_num_weights entries, layer after
 * layer, each layer [d = 0..8][out][in].  Setting them resets Adam. */
int64_t mgdwf_net_num_weights(mgdwf_net net);
mgdwf_status mgdwf_net_set_weights(mgdwf_net net, const float* w);
mgdwf_status mgdwf_net_get_weights(mgdwf_net net, float* w);
/* Lifted proposals V (canonical complex128, channels[4]/4 fine fields) on h's
 * lattice and gauge field; eta: input channels, complex128 [C][x4][colour]. */
mgdwf_status mgdwf_net_propose(mgdwf_net net, mgdwf_handle h, const double* eta, double* V);
/* Training loss against the basis installed on h (set_nullvecs or setup):
 * mean_k |(1 - P R) v_k|^2/|v_k|^2 + lam mean_{j<k} |<f_j,f_k>|^2/(|f_j|^2 |f_k|^2);
 * *loss and the weight gradient (HOST float array, may be NULL). */
mgdwf_status mgdwf_net_grad(mgdwf_net net, mgdwf_handle h, const double* eta, double* loss, float* grad);
/* One Adam step (lr; beta 0.9 / 0.999) on that loss; *loss before the step. */
mgdwf_status mgdwf_net_train_step(mgdwf_net net, mgdwf_handle h, const double* eta, double lr, double* loss);
/* `steps` Adam steps cycling over the n handles (each with its gauge field
 * and the target basis installed): step k trains on hs[k % n] with input
 * draw etas[k] (device pointers, one per step) at learning rate
 * lr (lr_final / lr)^(k / (steps - 1)); losses (HOST, may be NULL) gets each
 * step's loss before its update.  MGDWF_ERR_STATE if a handle lacks its
 * gauge field or basis. */
mgdwf_status mgdwf_net_train(mgdwf_net net, const mgdwf_handle* hs, int32_t n, const double* const* etas,
                             int32_t steps, double lr, double lr_final, double* losses);
/* Network files: the channel counts, lam, the Adam step count, the FP32
 * master weights and both Adam moments (training resumes where it stopped).
 * Load refuses a file of other channel counts (MGDWF_ERR_STATE) or a file
 * that is not a complete network file (MGDWF_ERR_INVALID_ARG). */
mgdwf_status mgdwf_net_save(mgdwf_net net, const char* path);
mgdwf_status mgdwf_net_load(mgdwf_net net, const char* path);

/* ---- measurement ------------------------------------------------------- */

/* Kernel ids for mgdwf_time_kernel. */
typedef enum {
  MGDWF_K_DSLASH = 0,    /* fine operator on internal-layout fields  */
  MGDWF_K_RESTRICT = 1,  /* R                                       */
  MGDWF_K_PROLONG = 2,   /* P                                       */
  MGDWF_K_COARSE = 3     /* D_c apply (A_c after build_coarse_squared) */
} mgdwf_kernel;

/* Autotuning of the FP32 Dslash: every tiling of the t-march kernels that
 * the lattice admits is timed (mgdwf_time_kernel's method, `iters` launches at
 * nrhs right-hand sides, D and D^+ alternating) and the fastest is kept on the
 * handle for every later FP32 fine-operator application, unless it is less
 * than 3 % faster than the first admissible tiling (the default), which is
 * then kept, so timing noise does not flip the choice between runs.  Without
 * a call the default is used.  Results are identical up to FP32 rounding
 * order whatever the tiling. */
#define MGDWF_MAX_TILINGS 32
#define MGDWF_TILE_RELOAD 1      /* kernel that reloads each slice's own spinor          */
#define MGDWF_TILE_FOLDED 2      /* workgroups ordered t-chunk first across all RHS       */
#define MGDWF_TILE_ONE_PER_CU 4  /* LDS reserved so one workgroup runs per CU             */
#define MGDWF_TILE_LDS_LINKS 8   /* each t-slice's links staged in LDS by the workgroup   */
#define MGDWF_TILE_PIPELINED 16  /* next hop's loads issued before this hop's SU(3) work  */
#define MGDWF_TILE_SITE_PAIR 32  /* one wavefront per two sites (x pair) x right-hand     */
                                 /* sides x Ls; links loaded once per site pair; tile =   */
                                 /* brick of (x pairs, y, z) items, 4th = t-slices/chunk  */
#define MGDWF_TILE_LDS_NEIGHBOURS 64 /* the tile's slice, links and fifth-dimension         */
                                     /* neighbours in LDS; only face neighbours from memory */
#define MGDWF_TILE_ASYNC_LINKS 256   /* with 64: the next slice's links copied to LDS      */
                                     /* (global_load_lds) during this slice; results      */
                                     /* stream past L2; 4th = t-slices at the tune's nrhs   */
#define MGDWF_TILE_XCD_UNITS 512     /* workgroups in units of (RHS, z-slab), each unit on  */
                                     /* one XCD (its faces in that XCD's L2) when nrhs and  */
                                     /* the z tiles allow whole rounds of eight units       */
typedef struct {
  int32_t ntilings;                   /* tilings timed                                  */
  int32_t chosen;                     /* index into the arrays below                     */
  int32_t id[MGDWF_MAX_TILINGS];      /* tiling id, for mgdwf_set_tiling                 */
  int32_t tile[MGDWF_MAX_TILINGS][4]; /* x, y, z sites per workgroup, t-slices per one   */
  int32_t flags[MGDWF_MAX_TILINGS];   /* MGDWF_TILE_* bits                               */
  double us[MGDWF_MAX_TILINGS];       /* mean time per launch                           */
  int32_t coarse_chosen;              /* 16-bit D_c apply shape kept: 0 = 16x16x16 MFMA,  */
                                      /* 1 = 16x16x32 MFMA; -1 if no D_c was built        */
  double coarse_us[2];                /* mean time per D_c apply for each shape (FP16)  */
} mgdwf_tune_report;
mgdwf_status mgdwf_tune(mgdwf_handle h, int32_t nrhs, int32_t iters, mgdwf_tune_report* report);

/* MFMA shape of the FP16/BF16 coarse apply: 0 = 16x16x16 tiles, 1 = 16x16x32
 * tiles (gfx950), -1 = the default (0).  mgdwf_tune also times both (4 iters
 * launches each at its nrhs, after the Dslash tilings, when the coarse
 * operator is built) and keeps shape 1 only when it is at least 3 % faster.
 * The two differ only in FP32 summation order. */
mgdwf_status mgdwf_set_coarse_tiling(mgdwf_handle h, int32_t id);
/* Use tiling `id` (from a tune report) for later FP32 applications; -1 restores
 * the default.  MGDWF_ERR_INVALID_ARG if the lattice does not admit it. */
mgdwf_status mgdwf_set_tiling(mgdwf_handle h, int32_t id);

/* Launch kernel `k` `iters` times back to back on the handle's stream on
 * internal buffers and return the mean time per launch in *ms, measured with
 * HIP events recorded on that stream.  On a 2D handle the kernels are the 2D
 * model's (its Dslash, R, P and A_c). */
mgdwf_status mgdwf_time_kernel(mgdwf_handle h, mgdwf_kernel k, mgdwf_prec prec, int32_t nrhs,
                               int32_t iters, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* MGDWF_H */
