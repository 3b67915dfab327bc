/*
 * xlbomd.h -- C ABI of the per-time-step electronic hot path of shadow
 * (KSA-)XL-BOMD for semiempirical sp Hamiltonians on one MI355X (gfx950).
 *
 * Method: Kulichenko et al., "Semi-Empirical Shadow Molecular Dynamics: A
 * PyTorch implementation", arXiv:2303.00689.  Equation numbers below are the
 * paper's.
 *
 * Conventions shared by every call
 *   - Orbital index 4*atom + {0: s, 1: px, 2: py, 3: pz}; n = 4 * n_atoms.
 *   - Matrices are dense, symmetric, n x n, FP64, row-major (equal to
 *     column-major because they are symmetric), owned by the caller, in
 *     DEVICE memory of the current HIP device.  The library never frees them.
 *   - Density matrices at this interface are spin-summed: P = 2 D with the
 *     paper's one-spin D, so Tr P = N_e.  The dynamical variable X and the
 *     kernel result Y use the same scaling.
 *   - Atom pairs (A < B) are enumerated row-major; packed orbital pairs
 *     (mu nu), mu <= nu, run over the row-major upper triangle of a 4x4 block;
 *     a packed symmetric 10 x 10 block stores its upper triangle row-major in
 *     55 values.
 *   - Every call enqueues its work on the stream given at create time.  Calls
 *     that return host scalars (mu, entropy, rank, residual, energies, the MD
 *     report) synchronise that stream before returning.
 *   - No call throws; each returns an xlbomd_status.  The last error message
 *     of a handle is available through xlbomd_last_error().  One handle must
 *     not be used by two host threads at once.
 *   - Units: eV, Angstrom, fs, amu, K.
 */
#ifndef XLBOMD_H
#define XLBOMD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xlbomd_ctx *xlbomd_handle;

typedef enum {
  XLBOMD_OK = 0,
  XLBOMD_E_ARG = -1,       /* invalid argument (null pointer, size, range)        */
  XLBOMD_E_HIP = -2,       /* a HIP runtime call failed                            */
  XLBOMD_E_NOCONV = -3,    /* chemical potential or SCF not converged              */
  XLBOMD_E_NONFINITE = -4, /* a NaN or Inf was detected in a result                */
  XLBOMD_E_STATE = -5,     /* call order violated (e.g. response before fermi_dm)  */
  XLBOMD_E_NOMEM = -6,     /* device allocation failed                             */
  XLBOMD_E_UNSTABLE = -7   /* an MD guard tripped: ||D0 - X|| or T_ion above limit */
} xlbomd_status;

/* Arithmetic of the recursive Fermi-operator and response GEMM chains.  The
 * Fock build, traces, chemical potential, Krylov algebra, forces and energies
 * are FP64 in every mode. */
typedef enum {
  XLBOMD_FP64 = 0,   /* FP64 storage, FP64 MFMA                                    */
  XLBOMD_BF16X3 = 1, /* FP32 storage, two-term BF16 split, 3 products, FP32 acc   */
  XLBOMD_BF16X6 = 2, /* FP32 storage, three-term BF16 split, 6 products, FP32 acc */
  XLBOMD_FP16X3 = 3, /* FP32 storage, two-term FP16 split with 2^11-scaled low   */
                     /* parts, 3 products, FP32 acc                               */
  /* Density matrix (Fermi chain and chemical potential) in FP64, the m response
   * chains of the Krylov kernel in the named split precision.  The forces of
   * eq. 37 depend on R, X and D0[X] only, so they keep FP64 accuracy while the
   * split arithmetic carries the response chains. */
  XLBOMD_DM64_BF16X3 = 4,
  XLBOMD_DM64_BF16X6 = 5,
  XLBOMD_DM64_FP16X3 = 6
} xlbomd_precision;

/* Synthetic NDDO-type sp Hamiltonian (stand-in for AM1/MNDO/PM3, which the
 * method section builds on, eq. 6 with S = I):
 *   h_AA = diag(eps_s, eps_p, eps_p, eps_p) - sum_{B != A} z_core W_AB[:, ss]
 *   h_AB = t(R) {s-s: 1, s_A-p_B: l, p_A-s_B: -l, p_A-p_B: l l^T},
 *          t(R) = t0 exp(-(R - r0_hop)/lam_hop), l = (R_B - R_A)/R
 *   W_AB = coul_k / sqrt(R^2 + coul_a^2) * (J + noise_amp * noise_AB)
 *   V_nn = sum_{A<B} z_core^2 W_AB[ss,ss] + a_rep exp(-(R - r0_rep)/rho_rep) */
typedef struct {
  double eps_s, eps_p;
  double t0, r0_hop, lam_hop;
  double coul_k, coul_a;
  double noise_amp;
  double z_core;
  double a_rep, r0_rep, rho_rep;
  double mass;     /* amu, every atom                                    */
  double j55[55];  /* packed 10 x 10 pattern J of the two-centre blocks  */
} xlbomd_model;

/* One system.  Host arrays are copied at create time (the two-centre noise is
 * repacked into the library's tile-major device layout) and may be freed
 * afterwards. */
typedef struct {
  int n_atoms;               /* 1 .. 8191 (n^2 < 2^30 elements per matrix)           */
  double n_elec;             /* N_e, 0 < N_e < 2n                                     */
  const double *onecenter;   /* host, n_atoms x 5: Gss, Gsp, Gpp, Gp2, Hsp (eV)       */
  const float *noise55;      /* host, n_pair x 55, packed symmetric blocks, pair order */
                             /* A < B row-major; may be NULL when n_atoms == 1         */
  xlbomd_model model;
} xlbomd_system;

/* Integration and chain settings. */
typedef struct {
  xlbomd_precision prec;
  double T_e;         /* electronic temperature, K (beta = 1/(k_B T_e), eq. 7)           */
  int m;              /* Krylov rank used by xlbomd_step (eq. 34), 0 <= m <= 32          */
  double krylov_tol;  /* relative-residual stop for xlbomd_step's kernel, 0 = fixed m    */
  double dt;          /* fs                                                              */
  double kappa;       /* eq. 35 kappa = dt^2 omega^2                                     */
  double alpha;       /* eq. 29/35 damping alpha                                         */
  double c[7];        /* eq. 29/35 damping c_k, k = 0..6                                 */
  double kernel_c;    /* m = 0: the original XL-BOMD kernel K = -c I (scaled identity,   */
                      /* Results, low-gap fullerene test: c = 1, or 0.9 tuned), c > 0    */
  /* Per-step guards of xlbomd_step / xlbomd_step_langevin (0 = off): a step
   * whose ||D0[X] - X||_F exceeds w0_limit, or whose ionic temperature exceeds
   * T_ion_limit (K), ends the call with XLBOMD_E_UNSTABLE after that step
   * (the instability the Results describe: the residual and the temperature
   * run away).  A T_ion guard reads the velocities back every step. */
  double w0_limit;
  double T_ion_limit;
} xlbomd_params;

/* MD state of xlbomd_step, all DEVICE pointers owned by the caller.  The X
 * history is a ring of 7 matrices: X(t - k dt) lives in slot (head + k) % 7.
 * The state is all a trajectory carries from step to step: a copy of it (the
 * buffers and the host fields) resumes the trajectory bit for bit, on the same
 * or on a new handle.  Every call taking a state returns XLBOMD_E_ARG,
 * touching nothing, if a pointer is null or head is outside [0, 7). */
typedef struct {
  double *R;      /* n_atoms x 3, Angstrom                                  */
  double *V;      /* n_atoms x 3, Angstrom/fs                               */
  double *A;      /* n_atoms x 3, Angstrom/fs^2 (force / mass)             */
  double *X;      /* 7 x n x n ring                                         */
  double *Y;      /* n x n, kernel result Y(t) of eq. 34 at the current t   */
  int head;       /* host: ring slot of X(t)                                */
  double mu;      /* host: chemical potential of the last evaluation, eV    */
  double mu_prev; /* host: the one before (NaN: none); the warm start of the */
                  /* next evaluation extrapolates linearly from the two     */
} xlbomd_md_state;

/* Per-step report (host). */
typedef struct {
  double E_tot;   /* KE + U, the constant of motion of eq. 26                 */
  double KE;      /* sum 1/2 M v^2                                            */
  double U;       /* shadow potential, eq. 13 with -2 T_e S                   */
  double TS;      /* 2 T_e S                                                  */
  double T_ion;   /* 2 KE / ((3N - 3) k_B)                                    */
  double mu;      /* chemical potential                                       */
  double W0;      /* ||D0[X] - X||_F, spin-summed                             */
  double relres;  /* relative residual of the rank-m kernel                   */
  int rank;       /* Krylov rank used                                          */
  int status;     /* XLBOMD_OK, or the status that ended the call at this step */
                  /* (XLBOMD_E_UNSTABLE: a guard; XLBOMD_E_NONFINITE: a NaN or */
                  /* Inf in F, the residual or the energies)                  */
  int levels;     /* recursion levels L of the Fermi chain                      */
  int mu_passes;  /* exact chemical-potential shift passes (0: series shift)   */
} xlbomd_report;

/* Create a handle for one system; allocates all device workspace.  `stream`
 * is a hipStream_t (NULL = default stream).  Positions must be set with
 * xlbomd_set_geometry before any other call. */
xlbomd_status xlbomd_create(const xlbomd_system *sys, const xlbomd_params *prm,
                            void *stream, xlbomd_handle *out);
xlbomd_status xlbomd_destroy(xlbomd_handle h);
const char *xlbomd_last_error(xlbomd_handle h);
/* Dimension n = 4 * n_atoms of the handle's matrices (0 on a null handle). */
int xlbomd_n_orb(xlbomd_handle h);

/* Copy positions R (DEVICE, n_atoms x 3) into the handle; h(R), W(R) and V_nn
 * are then evaluated on the fly by the calls below (eq. 17's h and G depend on
 * R only through the pair geometry). */
xlbomd_status xlbomd_set_geometry(xlbomd_handle h, const double *R);

/* dense one-electron matrix h(R) into H (DEVICE n x n), eq. 6. */
xlbomd_status xlbomd_hcore(xlbomd_handle h, double *H);

/* Fock build F = h + G(P) (eq. 6 / eq. 17 with S = I) for a spin-summed P,
 * G(P)_mn = sum_ls P_ls [(mn|ls) - 1/2 (ml|ns)] (eq. 3 at D = P/2) with NDDO
 * integrals.  include_h = 0 returns G(P) only (the F1 = G(V) of eq. 36).
 * P and F are DEVICE n x n and must not alias. */
xlbomd_status xlbomd_fock(xlbomd_handle h, const double *P, double *F, int include_h);

/* finite-temperature density matrix of eq. 19, P = 2 (exp(beta (F - mu0)) + 1)^-1,
 * with mu0 fixed by Tr P = N_e (eq. 8), by a recursive Fermi-operator GEMM chain in
 * the handle's precision and an exact chemical-potential shift.
 *   mu      host in/out: warm-start guess (NaN: none) / converged mu0
 *   P       DEVICE n x n output (must not alias F)
 *   entropy host out, nullable: S/k_B = -sum_i [f ln f + (1-f) ln(1-f)] (eq. 4, one spin)
 * The chain is cached in the handle for xlbomd_dm_response.  Returns
 * XLBOMD_E_NOCONV if |Tr P - N_e| > 1e-9 N_e after the shift; in the pure
 * split modes (FP32 storage of the Fermi chain) the trace is resolved to
 * 8e-7 n (BF16X6, FP16X3) or 8e-6 n (BF16X3) on top of that, and a strongly
 * gapped state, whose mu the electron count fixes only to the gap, takes no
 * shift once the trace is within a quarter of that. */
xlbomd_status xlbomd_fermi_dm(xlbomd_handle h, const double *F, double *mu, double *P,
                              double *entropy);

/* Spectral bounds of F, the step that fixes the chain depth: on return
 * lohi[0] <= every eigenvalue of F <= lohi[1].  Gershgorin discs, tightened by
 * min(32, n) Lanczos steps: the extreme Ritz values widened by their residual
 * bounds beta_k |s_k| and by 1e-3 of the Ritz spread.  F: DEVICE n x n
 * symmetric; lohi: HOST, 2 doubles.  Synchronises the handle's stream.
 * XLBOMD_E_NONFINITE if F holds a non-finite entry. */
xlbomd_status xlbomd_spectral_bounds(xlbomd_handle h, const double *F, double *lohi);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the bounds
 * of xlbomd_spectral_bounds, bit for bit the same, without a handle and
 * without any allocation.  The kernels' scratch (min(32, n) + 1 Lanczos
 * vectors, a product vector, per-row Gershgorin intervals and the reduced
 * scalars, about 4.7 MB) is one file-scope device array of the library, one
 * copy per GPU, held until the process ends.
 *   F       DEVICE n x n symmetric FP64 on the current device
 *   n       1 .. XLBOMD_SPECTRAL_BOUNDS_NOALLOC_MAX_N; larger n returns
 *           XLBOMD_E_ARG before any work
 *   stream  hipStream_t (NULL = default stream); the call synchronises it
 *   lohi    HOST, 2 doubles: lohi[0] <= every eigenvalue of F <= lohi[1]
 * XLBOMD_E_NONFINITE if F holds a non-finite entry.  Every call on a GPU
 * shares that GPU's scratch array, so calls that overlap on one GPU (other
 * host threads, other streams) race and must be serialised by the caller. */
#define XLBOMD_SPECTRAL_BOUNDS_NOALLOC_MAX_N 16384
xlbomd_status xlbomd_spectral_bounds_noalloc(const double *F, int n, void *stream, double *lohi);

/* canonical first-order response P1 = 2 dD/dlambda of D[F + lambda F1] at the
 * state of the last xlbomd_fermi_dm (eq. 36), with mu re-solved (Tr P1 = 0).
 * F1, P1: DEVICE n x n.  XLBOMD_E_STATE if no chain is cached. */
xlbomd_status xlbomd_dm_response(xlbomd_handle h, const double *F1, double *P1);

/* rank-m Krylov approximation (eq. 34, K0 = I) of Y = J^-1 (P0 - X), with
 * J V = P1[G(V)] - V the Jacobian of the residual (eq. 15).  Requires a
 * xlbomd_fermi_dm on F = h + G(X) just before (its chain is reused).
 *   m         requested rank (0 <= m <= 32); tol > 0 stops early once the
 *             relative residual falls below tol.  m = 0 is the original
 *             XL-BOMD kernel K = -c I: Y = -kernel_c (P0 - X), rank 0,
 *             relres 1 (no Jacobian is applied)
 *   Y         DEVICE n x n output
 *   rank      host out: rank used (breakdown is reported here, not as an error)
 *   relres    host out: ||sum W_i M_ij <W_j, W0> - W0|| / ||W0||  */
xlbomd_status xlbomd_krylov_kernel(xlbomd_handle h, const double *X, const double *P0, int m,
                                   double tol, double *Y, int *rank, double *relres);

/* forces -dU/dR_A at fixed X (eq. 24, eq. 37 with S = I) into forces
 * (DEVICE n_atoms x 3, eV/Angstrom) and the parts of U (host, nullable, 4 values):
 *   [0] Tr[h P0], [1] Tr[(P0 - X/2) G(X)], [2] V_nn, [3] Tr[h P0] + Tr[(P0 - X/2)G(X)] + V_nn */
xlbomd_status xlbomd_forces(xlbomd_handle h, const double *P0, const double *X,
                            double *forces, double *energy);

/* ---------------------------------------------------------------------------
 * Non-orthogonal basis (Methods section 3, eqs. 17-21; eqs. 36, 37, 39, 41).
 * Single-point electronic calls for a basis with overlap S != I.  The MD
 * path (xlbomd_step and its integrator) is orthogonal only: with S != I the
 * extended variable X = D S is not symmetric.
 *
 * The overlap is the model's synthetic one: S_AA = I and, for A != B, the
 * angular structure of the hopping block (s-s: s; s_A-p_B: s l;
 * p_A-s_B: -s l; p_A-p_B: s l l^T, l = (R_B - R_A)/R) with
 * s(R) = s0 exp(-(R - r0)/lam). */
typedef struct {
  double s0;   /* overlap at r0 (dimensionless), finite */
  double r0;   /* Angstrom, finite                      */
  double lam;  /* decay length, Angstrom, > 0           */
} xlbomd_overlap_model;

/* S(R) at the handle's positions into S (DEVICE n x n).  XLBOMD_E_ARG for
 * null pointers or constants out of range; XLBOMD_E_STATE before
 * xlbomd_set_geometry. */
xlbomd_status xlbomd_overlap(xlbomd_handle h, const xlbomd_overlap_model *ov, double *S);

/* Z = S^(-1/2), the symmetric (Loewdin) choice of eq. 21 (Z^T S Z = I), by a
 * coupled Newton-Schulz iteration on the FP64 GEMMs.  S: DEVICE n x n,
 * symmetric positive definite; Z: DEVICE n x n output, not aliasing S;
 * iterations: host out, nullable.  XLBOMD_E_ARG if the spectral lower bound
 * of S is not positive, XLBOMD_E_NOCONV after 60 iterations.  The first
 * non-orthogonal call on a handle allocates four FP64 n x n work matrices. */
xlbomd_status xlbomd_lowdin(xlbomd_handle h, const double *S, double *Z, int *iterations);

/* Spin-summed P = 2 Z D0_perp Z^T (eq. 20) with D0_perp the Fermi matrix
 * (eq. 19) of F_perp = Z^T F Z (eq. 18), mu fixed by Tr D0_perp = N_occ
 * (equivalently Tr P S = N_e).  F: DEVICE n x n symmetric; Z: DEVICE n x n,
 * any Z with Z^T S Z = I; mu: host in/out as in xlbomd_fermi_dm; P: DEVICE
 * n x n output, not aliasing F or Z; entropy: host out, nullable.  The
 * chain of F_perp is cached for xlbomd_dm_response_nonorth.  The transforms
 * are FP64; the chain runs in the handle's precision. */
xlbomd_status xlbomd_fermi_dm_nonorth(xlbomd_handle h, const double *F, const double *Z, double *mu, double *P,
                                      double *entropy);

/* Canonical response of eq. 36: P1 = Z P1_perp Z^T, P1_perp the response of
 * the cached chain to Z^T F1 Z (Tr P1 S = 0).  Z must be the one of the last
 * xlbomd_fermi_dm_nonorth.  F1: DEVICE n x n symmetric; P1: DEVICE n x n
 * output, not aliasing F1 or Z.  XLBOMD_E_STATE unless the cached chain is
 * that of an xlbomd_fermi_dm_nonorth (any later density-matrix evaluation on
 * the handle replaces it). */
xlbomd_status xlbomd_dm_response_nonorth(xlbomd_handle h, const double *F1, const double *Z, double *P1);

/* Pulay force term of eq. 41: forces[I] = + Tr[Z Z^T F P S_{R_I}] for the
 * spin-summed P (the gradient term is -2 Tr[Z Z^T F D S_{R_I}], D = P / 2),
 * into forces (DEVICE n_atoms x 3, eV/Angstrom, overwritten).  F, P: DEVICE
 * n x n symmetric; Z: as above.  With xlbomd_forces(P0 = P, X = the density
 * G is built from) it gives the eq. 37 forces for S != I.  Deterministic: one
 * wavefront per atom in a fixed order. */
xlbomd_status xlbomd_pulay_forces(xlbomd_handle h, const xlbomd_overlap_model *ov, const double *F,
                                  const double *P, const double *Z, double *forces);

/* damped X-Verlet of eq. 35 on the ring st->X using st->Y, and the
 * leapfrog position update of eqs. 27-28 (positions and half-step velocities);
 * advances st->head.  Used by xlbomd_step; exposed for testing. */
xlbomd_status xlbomd_integrate(xlbomd_handle h, xlbomd_md_state *st);

/* One or more KSA-XL-BOMD NVE steps (eqs. 27-30, 35, 37): for each step
 * integrate, evaluate F, P0 and the kernel at the new state, forces, and the
 * closing half kick.  rep: host array of n_steps reports (nullable).  A step
 * that fails (a non-finite F or residual, a guard of xlbomd_params) ends the
 * call with that status, written also into that step's report; the state is
 * then that of the failing step, and later reports are untouched. */
xlbomd_status xlbomd_step(xlbomd_handle h, xlbomd_md_state *st, int n_steps,
                          xlbomd_report *rep);

/* Langevin (NVT) variant of xlbomd_step, the thermostat of the paper's
 * Results runs (the paper does not give its scheme): the nuclei follow the
 * BAOAB splitting (Leimkuhler and Matthews 2013): half kick, half drift,
 * v <- c1 v + c2 xi with c1 = exp(-gamma dt), c2 = sqrt(k_B T_ion / M
 * (1 - c1^2)), half drift, forces, half kick; the electronic update (eq. 35)
 * is that of xlbomd_step.
 *   gamma   friction, 1/fs (>= 0; 0 reproduces xlbomd_step exactly)
 *   T_ion   bath temperature, K (>= 0)
 *   xi      DEVICE, n_steps x n_atoms x 3 independent standard normal
 *           numbers drawn by the caller; step k reads xi + 3 n_atoms k
 * E_tot in the reports is not a constant of motion here. */
xlbomd_status xlbomd_step_langevin(xlbomd_handle h, xlbomd_md_state *st, int n_steps, double gamma,
                                   double T_ion, const double *xi, xlbomd_report *rep);

/* Steps of an ensemble of independent trajectories (systems of uneven
 * sizes): member i advances h[i] with st[i] by n_steps exactly as
 * xlbomd_step does, and the members run concurrently, each from a host
 * thread of its own (at most 16 threads, taking members in index order) on
 * its handle's stream.  Create the
 * handles on distinct streams so that their GPU work overlaps.  Streams share
 * the process's hardware queues (HIP's GPU_MAX_HW_QUEUES, 4 by default), and
 * kernels on one queue run in order: set it to 16 before the first HIP call
 * so that the 16 members in flight each have one.
 *   h, st   host arrays of count distinct handles and their states
 *   rep     host, count x n_steps reports, member-major (nullable)
 * Returns XLBOMD_E_ARG for a repeated handle; otherwise the status of the
 * first failing member (its message in that handle's last_error), after
 * every member has run. */
xlbomd_status xlbomd_ensemble_step(xlbomd_handle *h, xlbomd_md_state *st, int count, int n_steps,
                                   xlbomd_report *rep);

/* Initial state for xlbomd_step: evaluates P0, Y and the accelerations at
 * (st->R, X(t0)) with X(t0 - k dt) = X(t0) for all k (Methods, section 5);
 * st->mu_prev is reset to NaN. */
xlbomd_status xlbomd_md_init(xlbomd_handle h, xlbomd_md_state *st);

/* Settings of xlbomd_scf.  Linear mixing X <- X + mix (P0[X] - X) runs first,
 * until the residual ||P0[X] - X||_F is below mix_tol (or tol) or max_mix
 * steps are taken; then Newton-Krylov steps X <- X - lam Y with Y the rank-m
 * kernel of eq. 34 (the paper's KSA SCF, Results: SCF optimisation), lam
 * halved from 1 until the residual decreases (down to 1/16384). */
typedef struct {
  int m;           /* Krylov rank of a Newton step, 1 .. 30                  */
  double tol;      /* stop once the residual is <= tol (spin-summed, F-norm) */
  int max_iter;    /* Newton-Krylov steps, >= 0                              */
  double mix;      /* linear-mixing coefficient, 0 < mix <= 1               */
  double mix_tol;  /* mixing ends below this residual                       */
  int max_mix;     /* at most this many mixing steps, >= 0                   */
} xlbomd_scf_params;

/* What xlbomd_scf did (host). */
typedef struct {
  double residual;   /* final ||P0[X] - X||_F                                  */
  int mix_steps;     /* mixing steps taken                                     */
  int newton_steps;  /* Newton-Krylov steps taken                              */
  int evaluations;   /* Fock builds + density matrices, line-search trials too */
  int responses;     /* density-matrix responses (Krylov directions)           */
} xlbomd_scf_report;

/* Ground state D_min of the self-consistency P0[X] = X (Methods, section 5:
 * the MD history starts from it).  X: DEVICE n x n in/out (initial guess in,
 * D_min out).  history: HOST, nullable, receives the residual after every
 * mixing step and every Newton step, at most history_len values.  rep: HOST,
 * nullable.  Returns XLBOMD_E_NOCONV if the residual is still above tol at
 * the end (X then holds the last iterate and rep is filled). */
xlbomd_status xlbomd_scf(xlbomd_handle h, double *X, const xlbomd_scf_params *p, double *history,
                         int history_len, xlbomd_scf_report *rep);

/* Diagnostic: C = A B (+ optional symmetric-output mode) with the response-chain
 * GEMM of the handle's precision, on DEVICE n x n FP64 matrices (A symmetric, B
 * any; sym_out only where A B is symmetric).  In split modes the operands are
 * rounded to FP32 storage first, exactly as the chains store their matrices
 * (B transposed on the way: the split kernels take their second operand by
 * rows).  For testing and timing the MFMA kernels. */
xlbomd_status xlbomd_matmul(xlbomd_handle h, const double *A, const double *B, double *Cout,
                            int sym_out, int reps);

/* Diagnostic timing: enable != 0 starts recording a pair of HIP events around
 * every GEMM, Fock-build and force launch on the handle's stream (at most
 * 65536 launches; later ones are not recorded); 0 stops.  Either call clears
 * earlier records. */
xlbomd_status xlbomd_profile(xlbomd_handle h, int enable);
/* Sums over the recorded launches, 10 classes x {launches, milliseconds,
 * work} (30 doubles): GEMMs by arithmetic and output kind, [0] FP64 full,
 * [1] FP64 symmetric output, [2] / [3] BF16x3 split full / symmetric, [4] / [5]
 * BF16x6, [6] / [7] FP16x3 (work = executed MFMA flops: 2n^3 per product, n^3
 * for a product with symmetric output, times the 3 or 6 MFMA products a split
 * product runs), [8] Fock build and [9] forces (work = algorithmic HBM bytes:
 * 220 per atom pair of FP32 noise, 128 per atom block on or above the
 * diagonal of each symmetric input read (P; P0 and X), and 8 n^2 for the F
 * the Fock build writes). */
xlbomd_status xlbomd_profile_read(xlbomd_handle h, double *out);

/* GEMM tile table (process-wide): which kernel family runs an n x n product of
 * the Fermi and response chains.  Families: 1 = small tiles (FP64 64 x 64;
 * split 128 x 128), 2 = large tiles (FP64 128 x 128, and 128 x 64 over the
 * upper triangle for symmetric outputs, n % 16 == 0, 128 <= n <= 23170;
 * split 224 x 224, and 160 x 160 for symmetric outputs and for FP16x3,
 * n % 32 == 0, 128 <= n <= 32767), 3 = medium tiles (split only: the
 * large-tile kernel with 128 x 128 tiles at two workgroups per compute unit,
 * n % 4 == 0 (FP16x3: n % 32 == 0), 128 <= n <= 32767), 4 = compact tiles
 * (FP64 32 x 32, n % 4 == 0; split: the large-tile kernel at 64 x 64,
 * n % 4 == 0, 64 <= n <= 32767), 0 = the library's built-in rule.
 *   rows    HOST, count x 4 ints {prec, sym, n_max, family}: prec is the
 *           arithmetic of the product, numbered as the precision enum's first
 *           four values: 0 FP64, 1 BF16x3, 2 BF16x6, 3 FP16x3; sym 0 full / 1
 *           symmetric output; n_max >= 1
 *   count   0..XLBOMD_TILE_TABLE_MAX; 0 clears the table
 * A product of order n uses the family of the row with the smallest n_max >= n
 * among those of its prec and sym (the first given, on ties), when that family
 * can run n; otherwise the built-in rule.  The rows are copied.  In FP64 the
 * families give the same bits on and above the diagonal (a symmetric
 * output's lower triangle is computed by one and mirrored by the other); in
 * split precision each stays within the split arithmetic's error budget.  Set the table before stepping: changing it while
 * other calls run leaves their products to either table.  Returns
 * XLBOMD_E_ARG (table unchanged) for a malformed row or count. */
#define XLBOMD_TILE_TABLE_MAX 256
xlbomd_status xlbomd_set_tile_table(const int *rows, int count);

/* Autotuning: the average time, in microseconds, of reps products C = A B of
 * order n in arithmetic prec (0..3 as above) with output kind sym, run by
 * kernel family `family` (1 to 4) on `stream` (hipStream_t, may be null),
 * after one warm-up product.  Allocates and frees its own operands, filled
 * with one constant byte pattern (for offline tuning, not for a stepping
 * loop); random operands draw more power and run up to ~12% slower, so the
 * times rank the families rather than predict a step.  Returns XLBOMD_E_ARG if the
 * family cannot run n, XLBOMD_E_HIP if an allocation or launch fails. */
xlbomd_status xlbomd_time_gemm(int n, int prec, int sym, int family, int reps, void *stream, double *us);

#ifdef __cplusplus
}
#endif
#endif /* XLBOMD_H */
